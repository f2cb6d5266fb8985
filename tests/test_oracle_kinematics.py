"""Pins of the oracle's binary-collision kinematics and gas model.

* stationary gas: E'/E = 1 - Lambda sin^2(theta/2) (theta the CM angle), head-on
  E'/E = 1 - Lambda, lab deflection <= asin(M_gas/M) for a heavier projectile;
* moving gas: momentum and kinetic energy of the pair conserved (the partner's
  final velocity follows from momentum conservation), relative speed preserved;
* Maxwellian partner: <V_i^2> = kT/M_gas; mean relative speed <|v - V|> against a
  Monte Carlo average (pins the erf formula used for the mean free path).
"""
import math

import numpy as np
import pytest

import oracle
import sputter_inputs as si

ELEMENTS = ["Ni", "Pd", "Pt", "Ru"]


def _cfg(el, **ch):
    return [si.Config(si.Chamber(**ch), si.Grid(), [si.species_cathode(el, n_particles=1)])]


@pytest.mark.parametrize("el", ELEMENTS)
def test_head_on_energy_transfer(el, params):
    cfg = _cfg(el)
    info = oracle.seg_info(cfg, params)
    M, Mg = si.SPECIES[el]["mass"], si.AR_MASS
    lam = 4 * M * Mg / (M + Mg) ** 2
    for E in (381.0, 20.0, 0.5):
        # u_b -> s = sqrt(u_b) = 0: head-on, theta_cm = pi
        E2, d2 = oracle.collide(cfg, params, E, [0.0, 0.0, 1.0], [0, 0, 0], 0.0, 0.3)
        assert abs(E2 / E - (1 - lam)) < 1e-12
        assert abs(info["Lambda"] - lam) < 1e-15


@pytest.mark.parametrize("el", ELEMENTS)
def test_stationary_gas_energy_and_deflection(el, params):
    cfg = _cfg(el)
    info = oracle.seg_info(cfg, params)
    M, Mg = si.SPECIES[el]["mass"], si.AR_MASS
    lam = 4 * M * Mg / (M + Mg) ** 2
    rng = np.random.default_rng(7)
    max_lab = math.asin(Mg / M) if M > Mg else math.pi
    for _ in range(300):
        E = 10 ** rng.uniform(-1, 2.6)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        ub, uphi = rng.uniform(), rng.uniform()
        E2, d2 = oracle.collide(cfg, params, E, d, [0, 0, 0], ub, uphi)
        Er = E * Mg / (M + Mg)
        th = oracle.table_theta(params, info["eps_per_eV"] * Er, math.sqrt(ub))
        assert abs(E2 / E - (1 - lam * math.sin(th / 2) ** 2)) < 1e-12
        assert abs(np.linalg.norm(d2) - 1) < 1e-14
        # lab angle from the CM angle: tan(psi) = sin(th) / (cos(th) + M/Mg)
        psi = math.atan2(math.sin(th), math.cos(th) + M / Mg)
        assert abs(math.acos(max(-1, min(1, float(d @ d2)))) - psi) < 1e-7
        assert psi <= max_lab + 1e-12


@pytest.mark.parametrize("el", ELEMENTS)
def test_moving_gas_conservation(el, params):
    cfg = _cfg(el)
    M, Mg = si.SPECIES[el]["mass"], si.AR_MASS
    rng = np.random.default_rng(11)
    for _ in range(300):
        E = 10 ** rng.uniform(-2, 2.6)
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        V = rng.normal(size=3) * 0.03
        ub, uphi = rng.uniform(), rng.uniform()
        E2, d2 = oracle.collide(cfg, params, E, d, V, ub, uphi)
        v = math.sqrt(2 * E / M) * d
        v2 = math.sqrt(2 * E2 / M) * d2
        V2 = (M * v + Mg * V - M * v2) / Mg            # partner from momentum conservation
        ke0 = 0.5 * M * v @ v + 0.5 * Mg * V @ V
        ke1 = 0.5 * M * v2 @ v2 + 0.5 * Mg * V2 @ V2
        assert abs(ke1 - ke0) <= 1e-12 * ke0
        assert abs(np.linalg.norm(v2 - V2) - np.linalg.norm(v - V)) <= 1e-10 * np.linalg.norm(v - V)


def test_maxwell_partner_and_mean_relative_speed(params):
    cfg = _cfg("Ni")
    info = oracle.seg_info(cfg, params)
    n = 100_000
    rng = np.random.default_rng(3)
    # uniforms on ]0,1] as the transport draws them
    w = (rng.integers(0, 2**24, size=(n, 4)) + 1) / 2**24
    V = np.stack([oracle.gas_velocity(cfg, params, w[i]) for i in range(n)])
    kT_over_M = info["kT"] / si.AR_MASS
    for i in range(3):
        assert abs(V[:, i].mean()) < 5 * math.sqrt(kT_over_M / n)
        assert abs((V[:, i] ** 2).mean() / kT_over_M - 1) < 5 * math.sqrt(2 / n)
    # lambda_m(gas motion) / lambda_m(gas at rest) = v / <|v - V|>
    cfg0 = _cfg("Ni", gas_motion=0)
    for E in (0.05, 0.3, 3.0, 100.0):
        v = math.sqrt(2 * E / si.SPECIES["Ni"]["mass"])
        vv = np.array([0.0, 0.0, v])
        mc = np.linalg.norm(vv[None, :] - V, axis=1).mean()
        ratio = oracle.lambda_m(cfg, params, E) / oracle.lambda_m(cfg0, params, E)
        assert abs(ratio - v / mc) < 5e-3 * (v / mc)


def test_mean_free_path_values(params):
    # n = p / (kB T): 0.5 Pa, 300 K -> 1.2072e20 m^-3; lambda = 1/(n sigma) with gas at rest
    cfg0 = _cfg("Ni", gas_motion=0)
    info = oracle.seg_info(cfg0, params)
    assert abs(info["n_mm3"] * 1e9 / 1.2072e20 - 1) < 1e-4
    for E in (381.0, 10.0, 0.1):
        eps = info["eps_per_eV"] * E * si.AR_MASS / (si.AR_MASS + 58.69)
        bm = oracle.beta_max(eps, params.theta_min)       # direct quadrature, not the table
        sigma = math.pi * (info["a_mm"] * bm) ** 2
        lam = oracle.lambda_m(cfg0, params, E)
        assert abs(lam * info["n_mm3"] * sigma - 1) < 2e-3   # table interpolation of beta_max


def test_flight_lengths_exponential(params):
    from scipy import stats
    cfg = _cfg("Ni")
    for E in (381.0, 2.0):
        lam = oracle.lambda_m(cfg, params, E)
        L = oracle.flights(cfg, params, seed=9, pid0=0, n=200_000, E=E)
        assert abs(L.mean() / lam - 1) < 4.5 / math.sqrt(200_000)
        assert stats.kstest(L / lam, "expon").pvalue > 1e-4
        assert L.max() <= lam * 24 * math.log(2) + 1e-9        # RN_1 >= 2^-24
    vac = _cfg("Ni", pressure=0.0)
    assert np.all(np.isinf(oracle.flights(vac, params, seed=9, pid0=0, n=10, E=10.0)))


def test_diffusive_walk_msd(params):
    cfg = _cfg("Ni", pressure=2.0)
    info = oracle.seg_info(cfg, params)
    lam = info["lam_th"]
    n_walk, steps = 20_000, 50
    X = np.stack([oracle.walk(cfg, params, seed=1, pid=i, n_steps=steps) for i in range(n_walk)])
    msd = (X**2).sum(axis=1).mean()
    # exponential steps of mean lam, isotropic: <|x|^2> = N <l^2> = 2 N lam^2
    assert abs(msd / (2 * steps * lam**2) - 1) < 4.5 * math.sqrt(2 / 3) / math.sqrt(n_walk) + 0.01
    assert abs(X.mean(axis=0)).max() < 5 * math.sqrt(2 * steps * lam**2 / 3 / n_walk)


def test_thermal_mean_free_path(params):
    # lambda_th = 1 / (n sigma(1.5 kT) sqrt(1 + M/M_gas))
    for p, el, ref in ((0.5, "Ni", 8.0), (2.0, "Ni", 2.0), (0.5, "Pt", 6.6)):
        info = oracle.seg_info(_cfg(el, pressure=p), params)
        assert abs(info["lam_th"] / ref - 1) < 0.03
