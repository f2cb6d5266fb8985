"""Pins of the oracle's launch with a measured racetrack and a six-coefficient emission law
(Methods, "The SIMTRA model": start position sampled from the measured racetrack; nascent
angular distribution sum_i c_i cos^i theta).

The racetrack profile is a radial erosion depth, linear between nodes; the start radius has a
density proportional to depth(r) r.  The polar angle has cos(theta) with density proportional
to sum c_i mu^i on [0, 1].  Pins: closed forms for a flat and a linear profile and for pure
cos^i laws, evaluated on the same Philox numbers (pinned against rocRAND elsewhere);
independent numeric inversion (scipy quad + brentq) for an irregular profile and a mixed law;
zero-weight node intervals are never sampled; sample moments.
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize, stats

import oracle
import sputter_inputs as si

SEED = 12345


def _u(pid0, n, seed=SEED):
    """The launch block's four RN of particles pid0.. of segment 0 (Philox keyed (pid, 0, 0, 0))."""
    ctr = np.zeros((n, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(pid0, pid0 + n, dtype=np.uint64).astype(np.uint32)
    w = oracle.philox_batch(ctr, [seed & 0xFFFFFFFF, seed >> 32]).astype(np.float64)
    return (np.floor(w / 256.0) + 1.0) / 2.0**24


def _launch(cat, n=4000, pid0=0):
    cfg = si.Config(si.Chamber(pressure=0.0), si.Grid(), [cat])
    out = oracle.launch_batch([cfg], si.Params(), SEED, pid0, n)
    x, d = out[:, :3], out[:, 3:6]
    c, nrm = np.asarray(cat.center), np.asarray(cat.normal)
    rel = x - c
    r = np.sqrt((rel ** 2).sum(1) - (rel @ nrm) ** 2)
    mu = d @ nrm
    return r, mu, rel @ nrm


def test_flat_profile_is_uniform_over_the_disc():
    R = 25.4
    cat = si.species_cathode("Ni", rt_profile=[(0.0, 1.0), (R, 1.0)])
    r, _, h = _launch(cat)
    u0 = _u(0, len(r))[:, 0]
    assert np.abs(h).max() < 1e-12                      # on the target plane
    assert np.abs(r - R * np.sqrt(u0)).max() < 1e-9     # F(r) = (r/R)^2


def test_linear_profile_closed_form():
    R = 20.0
    cat = si.species_cathode("Ni", rt_profile=[(0.0, 0.0), (R, 3.0)])
    r, _, _ = _launch(cat)
    u0 = _u(0, len(r))[:, 0]
    assert np.abs(r - R * np.cbrt(u0)).max() < 1e-9     # density ~ r^2 -> F(r) = (r/R)^3


def test_irregular_profile_against_independent_inversion():
    prof = si.measured_racetrack(seed=3)
    cat = si.species_cathode("Ni", rt_profile=prof)
    r, _, _ = _launch(cat, n=300)
    u0 = _u(0, len(r))[:, 0]
    rr = np.array([p[0] for p in prof]); dd = np.array([p[1] for p in prof])
    f = lambda s: np.interp(s, rr, dd) * s
    edges = [integrate.quad(f, rr[i], rr[i + 1], epsabs=1e-14, epsrel=1e-13)[0] for i in range(len(rr) - 1)]
    cum = np.concatenate([[0.0], np.cumsum(edges)])
    Z = cum[-1]
    for ri, ui in zip(r, u0):
        t = ui * Z
        i = int(np.searchsorted(cum, t)) - 1
        i = min(max(i, 0), len(rr) - 2)
        g = lambda s: cum[i] + integrate.quad(f, rr[i], s, epsabs=1e-14, epsrel=1e-12)[0] - t
        ref = optimize.brentq(g, rr[i], rr[i + 1], xtol=1e-13, rtol=1e-14)
        assert abs(ri - ref) < 1e-8, (ri, ref, ui)


def test_zero_weight_intervals_are_never_sampled():
    # no erosion inside 10 mm and beyond 20 mm: every start radius lies in [10, 20]
    prof = [(0.0, 0.0), (10.0, 0.0), (12.0, 1.0), (18.0, 1.0), (20.0, 0.0), (25.4, 0.0)]
    cat = si.species_cathode("Ni", rt_profile=prof)
    r, _, _ = _launch(cat, n=20000)
    assert r.min() >= 10.0 - 1e-12 and r.max() <= 20.0 + 1e-12
    # and the mean radius is the weighted mean of depth(r) r^2 / depth(r) r
    rr = np.array([p[0] for p in prof]); dd = np.array([p[1] for p in prof])
    num = integrate.quad(lambda s: np.interp(s, rr, dd) * s * s, 0, 25.4, points=rr[1:-1], limit=200)[0]
    den = integrate.quad(lambda s: np.interp(s, rr, dd) * s, 0, 25.4, points=rr[1:-1], limit=200)[0]
    assert abs(r.mean() - num / den) < 5 * r.std() / math.sqrt(len(r))


@pytest.mark.parametrize("i", [0, 2, 5])
def test_pure_power_laws_closed_form(i):
    c = [0.0] * 6
    c[i] = 1.0
    cat = si.species_cathode("Ni", cos_coeff=tuple(c))
    _, mu, _ = _launch(cat)
    u3 = _u(0, len(mu))[:, 3]
    assert np.abs(mu - u3 ** (1.0 / (i + 1))).max() < 1e-12   # density ~ mu^i -> F = mu^(i+1)


def test_mixed_law_against_independent_inversion_and_moments():
    c = np.array(si.UNDER_COSINE)
    cat = si.species_cathode("Ni", cos_coeff=tuple(c))
    _, mu, _ = _launch(cat, n=20000)
    u3 = _u(0, len(mu))[:, 3]
    G = lambda m: sum(c[i] * m ** (i + 1) / (i + 1) for i in range(6))
    for k in range(0, 20000, 997):
        ref = optimize.brentq(lambda m: G(m) - u3[k] * G(1.0), 0.0, 1.0, xtol=1e-15, rtol=1e-15)
        assert abs(mu[k] - ref) < 1e-12
    # <mu> = sum c_i/(i+2) / sum c_i/(i+1); KS against the closed-form CDF
    mean = sum(c[i] / (i + 2) for i in range(6)) / sum(c[i] / (i + 1) for i in range(6))
    assert abs(mu.mean() - mean) < 5 * mu.std() / math.sqrt(len(mu))
    assert stats.kstest(mu, lambda m: G(np.clip(m, 0, 1)) / G(1.0)).pvalue > 1e-4


def test_cosine_law_path_unchanged():
    """The plain cosine keeps cos(theta) = sqrt(RN) exactly."""
    cat = si.species_cathode("Ni")
    _, mu, _ = _launch(cat)
    u3 = _u(0, len(mu))[:, 3]
    assert np.abs(mu - np.sqrt(u3)).max() < 1e-15
