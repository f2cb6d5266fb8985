"""Pins of the oracle's launch sampling (Methods, "The SIMTRA model").

* inverse normal (Wichura AS241) against scipy's ndtri;
* racetrack radius: truncated normal against scipy.stats.truncnorm;
* Thompson energy with cut-off: closed-form mean and median, KS test against the
  closed-form CDF, and E_max reached at RN = 1;
* cosine-law emission: <cos> = 2/3, <cos^2> = 1/2, KS against F(mu) = mu^2;
* start point on the target plane, directions into the gas.
"""
import math

import numpy as np
import pytest
from scipy import special, stats

import oracle
import sputter_inputs as si


def test_norm_inv_matches_scipy():
    ps = np.concatenate([np.logspace(-300, -1, 200), np.linspace(0.01, 0.99, 397),
                         1.0 - np.logspace(-16, -1, 100)])
    for p in ps:
        ref = special.ndtri(p)
        got = oracle.norm_inv(p)
        assert abs(got - ref) <= 1e-14 * max(1.0, abs(ref)), (p, got, ref)


def test_norm_cdf_matches_scipy():
    for z in np.linspace(-30, 8, 381):
        ref = special.ndtr(z)
        assert abs(oracle.norm_cdf(z) - ref) <= 1e-15 + 1e-14 * ref


def _thompson_closed_form(U, Emax):
    Y = Emax + U
    norm = Emax**2 / (2.0 * U * Y**2)
    mean = (math.log(Y / U) + 2.0 * U / Y - U**2 / (2.0 * Y**2) - 1.5) / norm
    smax = Emax / Y
    z = smax / math.sqrt(2.0)
    median = U * z / (1.0 - z)
    return mean, median, norm


LAMBDA_EMAX = {  # (Lambda, E_max) for 400 eV Ar+ and k = 1
    "Ni": (0.963906, 381.1225), "Pd": (0.793772, 313.6189),
    "Pt": (0.564343, 219.8971), "Ru": (0.812153, 318.1210),
}


@pytest.mark.parametrize("el", ["Ni", "Pd", "Pt", "Ru"])
def test_thompson_energy(el, params):
    cfg = si.Config(si.Chamber(), si.Grid(), [si.species_cathode(el, n_particles=10)])
    info = oracle.seg_info([cfg], params)
    lam, emax = LAMBDA_EMAX[el]
    assert abs(info["Lambda"] - lam) < 1e-6
    assert abs(info["E_max"] - emax) < 1e-4
    n = 200_000
    s = oracle.launch_batch([cfg], params, seed=3, pid0=0, n=n)
    E = s[:, 6]
    U = cfg.cathodes[0].U_s
    mean, median, norm = _thompson_closed_form(U, info["E_max"])
    # second moment from the pdf E/(E+U)^3 / norm, by quadrature (independent of the sampler)
    m2 = __import__("scipy").integrate.quad(lambda e: e * e * e / (e + U) ** 3 / norm, 0, info["E_max"])[0]
    sd = math.sqrt(m2 - mean**2)
    assert abs(E.mean() - mean) < 4.5 * sd / math.sqrt(n)
    assert abs(np.median(E) - median) < 0.02 * median
    F = lambda e: (e / (e + U)) ** 2 / (info["E_max"] / (info["E_max"] + U)) ** 2
    assert stats.kstest(E, F).pvalue > 1e-4
    assert E.max() <= info["E_max"] * (1 + 1e-12) and E.min() > 0.0


def test_thompson_cutoff_reached_at_rn_one(params):
    # With RN = 1 the inverse CDF returns E_max exactly: E = U s/(1-s), s = E_max/(E_max+U)
    cfg = si.single_ni()
    info = oracle.seg_info([cfg], params)
    s = info["s_max"]
    assert abs(4.44 * s / (1 - s) - info["E_max"]) < 1e-9


def test_racetrack_radius_truncnorm(params):
    cfg = si.single_ni()
    n = 200_000
    s = oracle.launch_batch([cfg], params, seed=5, pid0=0, n=n)
    c = np.array(cfg.cathodes[0].center)
    q = s[:, :3] - c
    nrm = np.array(cfg.cathodes[0].normal)
    assert np.abs(q @ nrm).max() < 1e-12                 # start point on the target plane
    r = np.linalg.norm(q, axis=1)
    a, b = (0 - 15) / 3, (25.4 - 15) / 3
    tn = stats.truncnorm(a, b, loc=15, scale=3)
    assert abs(tn.mean() - 14.997063) < 1e-6 and abs(tn.std() - 2.994885) < 1e-6
    assert abs(r.mean() - tn.mean()) < 4.5 * tn.std() / math.sqrt(n)
    assert abs(r.std() - tn.std()) < 0.01 * tn.std()
    assert stats.kstest(r, tn.cdf).pvalue > 1e-4
    assert r.min() >= 0.0 and r.max() <= 25.4
    # azimuth of the start point uniform on [0, 2 pi)
    u, v = np.array(cfg.cathodes[0].u_axis), np.cross(nrm, cfg.cathodes[0].u_axis)
    psi = np.mod(np.arctan2(q @ v, q @ u), 2 * np.pi)
    assert stats.kstest(psi / (2 * np.pi), "uniform").pvalue > 1e-4


def test_truncated_normal_extreme_draws(params):
    # the CDF end points: Phi(alpha) and 1 - Phi(beta) of N(15, 3) on [0, 25.4]
    info = oracle.seg_info([si.single_ni()], params)
    assert abs(info["PhiA"] - 2.8665e-7) < 1e-10
    assert abs(info["QB"] - 2.6348e-4) < 1e-8
    assert abs(info["dPhi"] - (1 - info["PhiA"] - info["QB"])) < 1e-15


def test_cosine_law(params):
    cfg = si.quaternary(counts=[10, 10, 10, 10])
    for k in range(4):
        n = 100_000
        s = oracle.launch_batch([cfg], params, seed=11, pid0=0, n=n, seg=k)
        d = s[:, 3:6]
        assert np.abs(np.linalg.norm(d, axis=1) - 1).max() < 1e-14
        mu = d @ np.array(cfg.cathodes[k].normal)
        assert mu.min() > 0.0
        assert abs(mu.mean() - 2 / 3) < 4.5 * math.sqrt(1 / 2 - 4 / 9) / math.sqrt(n)
        assert abs((mu**2).mean() - 0.5) < 4.5 * math.sqrt(1 / 3 - 1 / 4) / math.sqrt(n)
        assert stats.kstest(mu, lambda m: m**2).pvalue > 1e-4
