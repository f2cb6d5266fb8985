"""Pins of the oracle's post-processing: power-rate fit, composition map, areas.

* Table S1 (Supporting Information): printed rates equal thickness / time to the
  printed rounding; the least-squares line through each supply's two points is the
  two-point line;
* composition map: sums to 100 at.%, a lone element is 100 %, invariance under a
  common rescaling of an element's profile and its calibration value, a two-element
  hand-worked case, gradients against central finite differences;
* measurement areas: 342 distinct lattice points ordered by distance; the area
  average of constant / linear profiles and against a fine-grid integral.
"""
import csv
import math
import os

import numpy as np
import pytest

import oracle
import sputter_inputs as si

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _table_s1():
    with open(os.path.join(GOLD, "table_s1.csv")) as fh:
        rows = [r for r in csv.DictReader(l for l in fh if not l.startswith("#"))]
    return rows


def test_table_s1_rates_are_thickness_over_time():
    for r in _table_s1():
        rate = float(r["thickness_nm"]) / float(r["time_s"])
        printed = r["rate_nm_per_s"]
        unit = 10.0 ** -len(printed.split(".")[1])         # last printed digit
        off = abs(rate - float(printed)) / unit
        if (r["element"], r["power_type"], r["power_W"]) == ("Ni", "DC", "5"):
            # 165.5 nm / 28800 s = 0.0057465: the paper prints 0.005745 (1.5 digits low);
            # the printed rate is the one used for the fit
            assert 1.0 < off < 2.0
        else:
            assert off <= 0.5, r


def test_power_rate_fit_recovers_two_point_lines():
    rows = _table_s1()
    pairs = {}
    for r in rows:
        pairs.setdefault((r["element"], r["power_type"]), []).append((float(r["power_W"]), float(r["rate_nm_per_s"])))
    expected = {  # two-point slope/intercept from the printed rates
        ("Ni", "DC"): (1.036833e-3, 5.608333e-4), ("Ni", "RF"): (4.555217e-4, 1.343478e-4),
        ("Pd", "DC"): (4.944e-3, -2.0e-5), ("Pd", "RF"): (1.366962e-3, -4.707736e-3),
        ("Pt", "DC"): (3.086333e-3, -1.321667e-3), ("Ru", "DC"): (1.495267e-3, -2.054333e-3),
    }
    for key, pts in pairs.items():
        (p1, r1), (p2, r2) = pts
        a, b = oracle.fit_power_rate([p1, p2], [r1, r2])
        a2 = (r2 - r1) / (p2 - p1)
        assert abs(a - a2) < 1e-14 and abs(b - (r1 - a2 * p1)) < 1e-14
        ea, eb = expected[key]
        assert abs(a - ea) < 1e-9 and abs(b - eb) < 1e-9


def _rand_inputs(B=5, J=7, K=4, seed=0):
    rng = np.random.default_rng(seed)
    f = rng.uniform(0.1, 2.0, (K, J))
    a = rng.uniform(0.5, 2, K)
    b = rng.uniform(0, 0.2, K)
    P = rng.uniform(20, 200, (B, K))
    M = rng.uniform(50, 200, K)
    rho = rng.uniform(8, 22, K)
    fref = f.mean(axis=1)
    return f, a, b, P, M, rho, fref


def test_composition_invariants():
    f, a, b, P, M, rho, fref = _rand_inputs()
    c = oracle.composition(f, a, b, P, M, rho, fref)
    assert c.shape == (5, 7, 4)
    assert np.allclose(c.sum(axis=2), 100.0, atol=1e-12)
    assert (c > 0).all()
    # one element with non-zero rate -> 100 %
    P1 = np.zeros_like(P); P1[:, 2] = 50.0
    b1 = np.zeros_like(b)
    c1 = oracle.composition(f, a, b1, P1, M, rho, fref)
    assert np.allclose(c1[:, :, 2], 100.0) and np.allclose(np.delete(c1, 2, axis=2), 0.0)
    # rescaling an element's profile together with its calibration value changes nothing
    f2, fref2 = f.copy(), fref.copy()
    f2[1] *= 3.7; fref2[1] *= 3.7
    assert np.allclose(oracle.composition(f2, a, b, P, M, rho, fref2), c, atol=1e-12)
    # default calibration value = mean over areas
    assert np.allclose(oracle.composition(f, a, b, P, M, rho), c)


def test_composition_two_element_hand_case():
    # element 1: rate 2 nm/s, rho/M = 0.1; element 2: rate 1 nm/s, rho/M = 0.3, same profile
    f = np.array([[1.0], [1.0]])
    c = oracle.composition(f, np.array([1.0, 1.0]), np.array([0.0, 0.0]), np.array([[2.0, 1.0]]),
                           np.array([10.0, 10.0]), np.array([1.0, 3.0]), np.array([1.0, 1.0]))
    # atoms ~ 2*0.1 = 0.2 and 1*0.3 = 0.3 -> 40 % / 60 %
    assert np.allclose(c[0, 0], [40.0, 60.0])


def test_composition_gradients_finite_differences():
    f, a, b, P, M, rho, fref = _rand_inputs(B=3, J=4, K=3, seed=2)
    ct = oracle.composition(f, a, b, P * 1.1, M, rho, fref) + 0.3
    g = oracle.composition_grads(f, a, b, P, M, rho, fref, ct)

    def loss(**kw):
        args = dict(f=f, a=a, b=b, P=P, M=M, rho=rho, fref=fref)
        args.update(kw)
        return oracle.sq_euclid(oracle.composition(**args), ct).sum()

    for name in ("f", "a", "b", "P", "M", "rho", "fref"):
        base = dict(f=f, a=a, b=b, P=P, M=M, rho=rho, fref=fref)[name]
        it = np.nditer(base, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            h = 1e-6 * max(1.0, abs(base[idx]))
            xp, xm = base.copy(), base.copy()
            xp[idx] += h; xm[idx] -= h
            fd = (loss(**{name: xp}) - loss(**{name: xm})) / (2 * h)
            assert abs(fd - g[name][idx]) < 1e-5 * max(1.0, abs(fd)), (name, idx, fd, g[name][idx])
    assert abs(g["loss"] - loss()) < 1e-9


def test_area_centres():
    c = oracle.area_centres()
    assert c.shape == (342, 2)
    assert len({(round(x, 6), round(y, 6)) for x, y in c}) == 342
    r = np.hypot(c[:, 0], c[:, 1])
    assert np.all(np.diff(r) >= -1e-12)
    assert np.allclose(np.mod(c / 4.5 + 1e-9, 1.0), 0.0, atol=1e-6)
    # every lattice point strictly closer than the farthest chosen one is chosen
    rmax = r.max()
    m = int(rmax / 4.5) + 1
    inner = sum(1 for i in range(-m, m + 1) for j in range(-m, m + 1) if math.hypot(4.5 * i, 4.5 * j) < rmax - 1e-9)
    assert inner < 342 <= inner + sum(1 for i in range(-m, m + 1) for j in range(-m, m + 1)
                                      if abs(math.hypot(4.5 * i, 4.5 * j) - rmax) < 1e-9)
    assert rmax < 50.0


def test_area_gather():
    g = si.Grid(center=(0, 0, 280), normal=(0, 0, -1), u_axis=(1, 0, 0), half_u=50, half_v=50, shape=1,
                nu=200, nv=200)
    cen = oracle.area_centres()
    const = np.full((200, 200), 3.25)
    assert np.allclose(oracle.area_gather(const, g, cen), 3.25)
    uc = -50 + 0.5 * (np.arange(200) + 0.5)
    lin = 2.0 + 0.1 * uc[None, :] - 0.05 * uc[:, None]
    val = oracle.area_gather(lin, g, cen)
    assert np.allclose(val, 2.0 + 0.1 * cen[:, 0] - 0.05 * cen[:, 1], atol=1e-12)
    # against a fine-grid integral of the piecewise-constant profile
    rng = np.random.default_rng(0)
    prof = rng.uniform(0, 1, (200, 200))
    fine = np.kron(prof, np.ones((10, 10)))             # 0.05 mm cells
    for a in (0, 100, 341):
        cu, cv = cen[a]
        x0 = int(round((cu - 2.25 + 50) / 0.05)); y0 = int(round((cv - 2.25 + 50) / 0.05))
        ref = fine[y0:y0 + 90, x0:x0 + 90].mean()
        assert abs(oracle.area_gather(prof, g, cen[a:a + 1])[0] - ref) < 1e-12


def test_normalize_roundtrip():
    g = si.Grid()
    counts = np.random.default_rng(0).integers(0, 100, (50, 50))
    f = oracle.normalize(counts, 12345, g)
    assert abs((f * 12345 * 4.0).sum() - counts.sum()) < 1e-8
