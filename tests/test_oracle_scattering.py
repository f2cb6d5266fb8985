"""Pins of the oracle's scattering integral, cross-section cut-off and table.

The classical deflection integral is checked where it has closed forms (bare
Coulomb: tan(theta/2) = 1/(2 eps beta); inverse-square: theta = pi (1 - beta /
sqrt(beta^2 + A))), against scipy's adaptive quadrature plus brentq root for the
Moliere potential, and by its invariants (theta(0) = pi, monotone in beta,
theta(beta_max) = theta_min).  Its Gauss-Legendre rule is checked against numpy's.
"""
import math

import numpy as np
import pytest
from scipy import integrate, optimize

import oracle
from oracle import COULOMB, INVERSE_SQUARE, MOLIERE


def test_gauss_legendre_nodes_match_numpy():
    for n in (8, 64, 128):
        t, w = oracle.gauss_legendre01(n)
        x, wx = np.polynomial.legendre.leggauss(n)
        assert np.allclose(t, 0.5 * (x + 1), atol=1e-15, rtol=0)
        assert np.allclose(w, 0.5 * wx, atol=2e-14, rtol=0)
        # exact for polynomials of degree <= 2n - 1
        for k in (0, 1, 5, 2 * n - 1):
            assert abs((w * t**k).sum() - 1.0 / (k + 1)) < 1e-14


@pytest.mark.parametrize("eps,beta", [(1e-3, 0.5), (0.1, 2.0), (1.0, 0.05), (3e-5, 1e3), (10.0, 0.3)])
def test_rutherford_closed_form(eps, beta):
    got = oracle.theta_cm(eps, beta, kind=COULOMB)
    ref = 2.0 * math.atan(1.0 / (2.0 * eps * beta))
    assert abs(got - ref) < 5e-11


@pytest.mark.parametrize("A,beta", [(0.5, 0.2), (2.0, 1.0), (10.0, 3.0), (1e-3, 5.0)])
def test_inverse_square_closed_form(A, beta):
    got = oracle.theta_cm(A, beta, kind=INVERSE_SQUARE)
    ref = math.pi * (1.0 - beta / math.sqrt(beta * beta + A))
    assert abs(got - ref) < 1e-11
    assert abs(oracle.closest_approach(A, beta, kind=INVERSE_SQUARE) - math.sqrt(A + beta * beta)) < 1e-12


def test_moliere_screening_normalised():
    assert abs(oracle.lib().or_moliere(0.0) - 1.0) < 1e-15
    assert oracle.lib().or_moliere(50.0) < 1e-6


def _moliere_scipy(eps, beta):
    phi = lambda x: 0.35 * np.exp(-0.3 * x) + 0.55 * np.exp(-1.2 * x) + 0.10 * np.exp(-6.0 * x)
    f = lambda x: 1.0 - phi(x) / (x * eps) - beta**2 / x**2
    hi = max(beta, 1.0)
    while f(hi) <= 0:
        hi *= 2
    x0 = optimize.brentq(f, max(beta, 1e-12), hi, xtol=1e-15, rtol=1e-15, maxiter=500)

    def g(t):
        u = 1.0 - t * t
        h = 1.0 - u * phi(x0 / u) / (x0 * eps) - beta**2 * u * u / x0**2
        return 2.0 * t / math.sqrt(max(h, 1e-300))

    I, _ = integrate.quad(g, 1e-12, 1.0, epsabs=1e-14, epsrel=1e-13, limit=400)
    return math.pi - 2.0 * beta / x0 * I


@pytest.mark.parametrize("eps", [1e-10, 1e-7, 1e-4, 2.2e-3, 0.1, 1.0])
@pytest.mark.parametrize("beta", [0.05, 0.7, 4.0, 25.0])
def test_moliere_against_scipy_quadrature(eps, beta):
    got = oracle.theta_cm(eps, beta)
    ref = _moliere_scipy(eps, beta)
    assert abs(got - ref) < 2e-9, (got, ref)


def test_theta_invariants():
    for eps in (1e-9, 1e-5, 1e-2, 0.5):
        assert oracle.theta_cm(eps, 0.0) == math.pi
        betas = np.linspace(0.0, 80.0, 161)
        th = np.array([oracle.theta_cm(eps, b) for b in betas])
        assert np.all(np.diff(th) < 0) or np.all(np.diff(th[th > 1e-9]) < 0)
        assert th.min() > -1e-9 and th.max() <= math.pi


@pytest.mark.parametrize("eps", [1e-10, 1e-6, 2.2e-3, 1.0])
def test_beta_max_gives_theta_min(eps):
    bm = oracle.beta_max(eps, 0.1)
    assert abs(oracle.theta_cm(eps, bm) - 0.1) < 1e-10
    assert oracle.theta_cm(eps, 0.99 * bm) > 0.1 > oracle.theta_cm(eps, 1.01 * bm)


def test_table_nodes_and_interpolation(params):
    th, bm = oracle.table(params)
    ne, ns = params.table_ne, params.table_ns
    T = th.reshape(ne, ns)
    assert np.all(T[:, 0] == math.pi)
    assert np.abs(T[:, -1] - 0.1).max() < 1e-10
    assert np.all(np.diff(bm) < 0)        # larger eps: shorter range of deflection
    lo, hi = params.log_eps_lo, params.log_eps_hi
    for i in (0, 17, 128, 255):
        eps = 10 ** (lo + (hi - lo) * i / (ne - 1))
        assert abs(bm[i] - oracle.beta_max(eps, 0.1)) < 1e-9 * bm[i]
        for j in (0, 1, 100, 256):
            assert abs(oracle.table_theta(params, eps, j / (ns - 1)) - T[i, j]) < 1e-12
            if 0 < j < ns - 1:
                assert abs(T[i, j] - oracle.theta_cm(eps, j / (ns - 1) * bm[i])) < 1e-12
    # off-grid: bilinear error well below a milliradian
    rng = np.random.default_rng(0)
    errs = []
    for _ in range(200):
        le = rng.uniform(lo, hi)
        s = rng.uniform(0.02, 1.0)
        eps = 10**le
        b = s * float(np.interp(le, np.linspace(lo, hi, ne), bm))
        errs.append(abs(oracle.table_theta(params, eps, s) - oracle.theta_cm(eps, b)))
    assert max(errs) < 5e-3 and np.median(errs) < 2e-4
    # clamped outside the table range
    assert oracle.table_theta(params, 1e-14, 0.5) == oracle.table_theta(params, 10**lo, 0.5)
    assert oracle.table_theta(params, 10.0, 0.5) == oracle.table_theta(params, 10**hi, 0.5)
