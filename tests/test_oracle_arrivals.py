"""Pins of the oracle's arrival tallies: energy and incidence-angle distributions of the atoms
deposited on the substrate (Introduction: besides the deposition profile, a Monte Carlo model
yields the energy and angular distributions of arriving particles).

* At 0 Pa the atoms fly straight with their launch energy, which is drawn independently of
  position and direction, so the arrival energies follow the Thompson law exactly (closed-form
  CDF over the bins).
* At 0 Pa from a point source on the axis of a parallel square substrate the incidence angle is
  the emission angle; the fraction arriving between angles a1 and a2 is
  int_{a1}^{a2} I(cos a) sin a * arc(h tan a) da, with I the emission intensity per steradian
  and arc(rho) the angle of the circle of radius rho lying on the square (closed form).
* Thermalised arrivals carry at most the thermalisation energy; non-deposits have no angle.
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
import sputter_inputs as si

N = 1_000_000


def _chi2_ok(obs, exp, min_exp=5.0):
    m = exp >= min_exp
    z = (obs[m] - exp[m]) / np.sqrt(exp[m])
    dof = int(m.sum())
    chi2 = float((z ** 2).sum())
    return chi2 < dof + 4.5 * math.sqrt(2 * dof), chi2, dof, m


def _tallies(cfgs, params, seed):
    r = oracle.run(cfgs, params, seed=seed, records=True)
    plan_first = np.cumsum([0] + [c.n_particles for cfg in cfgs for c in cfg.cathodes])
    nbs = [cfg.grid.nu * cfg.grid.nv for cfg in cfgs for _ in cfg.cathodes]
    bo = np.concatenate([[0], np.cumsum(nbs)[:-1]])
    hE, hA, es = oracle.arrival_tallies(r["records"], plan_first, nbs, bo)
    return r, hE, hA, es


def test_zero_pressure_arrival_energy_is_thompson(params):
    cfg = si.single_ni(0.0, N)
    r, hE, hA, es = _tallies([cfg], params, seed=2)
    info = oracle.seg_info([cfg], params)
    U, Emax = si.SPECIES["Ni"]["U_s"], info["E_max"]
    F = lambda E: np.minimum((np.asarray(E) / (np.asarray(E) + U)) ** 2, (Emax / (Emax + U)) ** 2) / (Emax / (Emax + U)) ** 2
    e_edges, _ = oracle.arrival_edges()
    lo = np.concatenate([[0.0], e_edges[1:oracle.N_ARRIVAL_E]])
    hi = np.concatenate([e_edges[1:oracle.N_ARRIVAL_E], [np.inf]])
    p = F(np.minimum(hi, 1e300)) - F(lo)
    n_dep = int(r["counters"][0, 1])
    ok, chi2, dof, m = _chi2_ok(hE[0].astype(np.float64), n_dep * p)
    assert ok, (chi2, dof)
    assert hE[0][~m].sum() <= 5 * max(1.0, (n_dep * p[~m]).sum())
    # every deposit is tallied once in each histogram; the energy sums add up
    assert hE.sum() == hA.sum() == n_dep
    dep = r["records"][r["records"][:, 3] == 1]
    assert es.sum() == np.rint(dep[:, 7] * oracle.ESUM_SCALE).astype(np.uint64).sum()


def _arc(rho, w):
    """Angle of the circle of radius rho (centred on the square's centre) inside the square."""
    if rho <= w:
        return 2 * math.pi
    if rho >= w * math.sqrt(2.0):
        return 0.0
    return 2 * math.pi - 8 * math.acos(w / rho)


@pytest.mark.parametrize("law", [(0, 1, 0, 0, 0, 0), si.UNDER_COSINE])
def test_zero_pressure_point_source_incidence_angles(params, law):
    cfg = si.with_launch(si.single_ni(0.0, N), [(0.0, 1.0), (1e-6, 1.0)], law)
    r, hE, hA, es = _tallies([cfg], params, seed=4)
    h, w = 100.0, 50.0
    c = np.asarray(law, dtype=np.float64)
    norm = 2 * math.pi * sum(c[i] / (i + 1) for i in range(6))
    I = lambda mu: sum(c[i] * mu ** i for i in range(6)) / norm
    f = lambda a: I(math.cos(a)) * math.sin(a) * _arc(h * math.tan(a), w)
    a_brk = [math.atan(w / h), math.atan(w * math.sqrt(2) / h)]
    exp = np.zeros(oracle.N_ARRIVAL_A)
    for j in range(oracle.N_ARRIVAL_A):
        a1, a2 = math.radians(j), math.radians(j + 1)
        pts = [b for b in a_brk if a1 < b < a2]
        exp[j] = integrate.quad(f, a1, a2, points=pts or None, epsabs=1e-13, epsrel=1e-11, limit=200)[0]
    ok, chi2, dof, m = _chi2_ok(hA[0].astype(np.float64), N * exp)
    assert ok, (chi2, dof)
    assert hA[0][exp == 0].sum() == 0                 # nothing beyond the square's corner angle
    assert abs(hA.sum() - N * exp.sum()) < 4.5 * math.sqrt(N * exp.sum())


def test_thermalised_arrivals_and_angles(params):
    cfg = si.single_ni(2.0, 5000)
    r, hE, hA, es = _tallies([cfg], params, seed=6)
    rec = r["records"]
    dep = rec[:, 3] == 1
    info = oracle.seg_info([cfg], params)
    walked = dep & (rec[:, 6] > 0)
    assert walked.sum() > 100
    assert np.all(rec[walked, 7] <= info["E_th"])     # thermalised atoms arrive with E <= E_th
    assert np.all((rec[dep, 8] > 0) & (rec[dep, 8] <= 1.0 + 1e-15))
    assert np.all(rec[~dep, 8] == 0.0)
    be, _ = oracle.arrival_bins(np.array([info["E_th"]]), np.array([1.0]))
    assert hE[0][be[0] + 1:].sum() == (dep & ~walked & (rec[:, 7] >= oracle.arrival_edges()[0][be[0] + 1])).sum()
