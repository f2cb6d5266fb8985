"""Pins of the oracle's tilt inversion (Results, the cathode-tilt study and Figure 8: the
simulation repeated over cathode tilts, each library compared with the measured one by the
compositional area it covers and by d_e).

* Covered area: the whole diagram (the three pure elements among the points) is 1; any
  triangle of compositions covers |det| of its three compositions (as fractions), the
  barycentric area formula, whatever interior points are added; a regular polygon inscribed in
  the diagram covers its closed-form area; collinear or fewer than three points cover 0; the
  area does not depend on point order or on which element is called 0, 1, 2 (the diagram map
  is an isometry of the simplex); random small sets against a brute-force sum over the hull
  edges found by the all-points-on-one-side test.
* Fits: a sampled parabola gives its vertex on uneven sweeps, unmoved by an offset or scale of
  the misfit and shifted with the sweep; a vertex outside the sweep gives its end; a parabola
  opening downwards or a flat one gives the smallest sample; on noisy samples the vertex is
  unbiased; a sampled line gives its exact crossing, also with residuals orthogonal to lines
  added; a crossing outside the sweep or a flat line gives NaN.
* Sweep compositions: each library sums to 100 at.% at every area, is unchanged when its area
  values are scaled, and a lone element is 100 at.%.
* The ternary library's rate lines are the least-squares lines through Table S1's samples.
"""
import csv
import itertools
import math
from pathlib import Path

import numpy as np
import pytest

import oracle
import sputter_inputs as si

GOLDEN = Path(__file__).parent / "golden"
SIMPLEX = math.sqrt(3.0) / 4.0 * 100.0 * 100.0


def _random_compositions(rng, n, K=3):
    c = rng.dirichlet(np.ones(K), size=n) * 100.0
    return c


def test_whole_diagram_is_one():
    rng = np.random.default_rng(0)
    c = np.vstack([np.eye(3) * 100.0, _random_compositions(rng, 300)])
    rng.shuffle(c)
    assert abs(oracle.hull_area_fraction(c) - 1.0) < 1e-14


@pytest.mark.parametrize("seed", range(5))
def test_triangle_is_barycentric_determinant(seed):
    rng = np.random.default_rng(10 + seed)
    tri = _random_compositions(rng, 3)
    exact = abs(np.linalg.det(tri / 100.0))
    # interior points: convex combinations of the corners
    w = rng.dirichlet(np.ones(3), size=200)
    pts = np.vstack([tri, w @ tri])
    rng.shuffle(pts)
    assert abs(oracle.hull_area_fraction(pts) - exact) < 1e-12 * max(exact, 1e-3)


@pytest.mark.parametrize("n", [3, 4, 7, 50])
def test_regular_polygon_closed_form(n):
    rng = np.random.default_rng(n)
    r = 20.0                                       # diagram units (at.%), inside the triangle
    cx, cy = 50.0, 50.0 / math.sqrt(3.0)           # the equiatomic point
    phi = rng.uniform(0, 2 * math.pi) + 2 * math.pi * np.arange(n) / n
    x, y = cx + r * np.cos(phi), cy + r * np.sin(phi)
    c2 = y * 2.0 / math.sqrt(3.0)
    c1 = x - 0.5 * c2
    c = np.stack([100.0 - c1 - c2, c1, c2], axis=1)
    inner = c.mean(axis=0) + 0.3 * (c[rng.integers(0, n, 100)] - c.mean(axis=0))
    exact = 0.5 * n * r * r * math.sin(2 * math.pi / n) / SIMPLEX
    got = oracle.hull_area_fraction(np.vstack([inner, c]))
    assert abs(got - exact) < 1e-12


def test_degenerate_sets():
    rng = np.random.default_rng(3)
    a, b = _random_compositions(rng, 2)
    line = a[None, :] + rng.uniform(0, 1, (40, 1)) * (b - a)[None, :]
    assert oracle.hull_area_fraction(line) < 1e-13
    assert oracle.hull_area_fraction(a[None, :]) == 0.0
    assert oracle.hull_area_fraction(np.vstack([a, b])) == 0.0
    assert oracle.hull_area_fraction(np.repeat(a[None, :], 10, axis=0)) == 0.0


def test_order_and_element_labels_do_not_matter():
    rng = np.random.default_rng(4)
    c = 20.0 + _random_compositions(rng, 342) * 0.4
    ref = oracle.hull_area_fraction(c)
    for perm in itertools.permutations(range(3)):
        assert abs(oracle.hull_area_fraction(c[:, perm]) - ref) < 1e-13
    assert abs(oracle.hull_area_fraction(c[rng.permutation(len(c))]) - ref) < 1e-15


def _brute_hull_area(c):
    x, y = oracle.ternary_xy(c)
    P = np.stack([x, y], axis=1)
    s = 0.0
    n = len(P)
    for i in range(n):
        for j in range(n):
            if i == j or np.array_equal(P[i], P[j]):
                continue
            d = P[j] - P[i]
            cr = d[0] * (P[:, 1] - P[i, 1]) - d[1] * (P[:, 0] - P[i, 0])
            # directed hull edge: every point on the left or on the segment, none strictly
            # beyond its ends along the line
            if np.all(cr >= -1e-12):
                on = np.abs(cr) <= 1e-12
                t = ((P[on] - P[i]) @ d) / (d @ d)
                if np.all(t >= -1e-12) and np.all(t <= 1 + 1e-12):
                    s += P[i, 0] * P[j, 1] - P[j, 0] * P[i, 1]
    return 0.5 * s / SIMPLEX


@pytest.mark.parametrize("n", [3, 4, 5, 6, 9])
def test_against_brute_force(n):
    rng = np.random.default_rng(100 + n)
    for _ in range(20):
        c = _random_compositions(rng, n)
        assert abs(oracle.hull_area_fraction(c) - _brute_hull_area(c)) < 1e-12


def test_fit_min_parabola_vertex():
    rng = np.random.default_rng(5)
    for _ in range(50):
        x = np.sort(rng.uniform(10, 16, int(rng.integers(3, 12))))
        x0 = rng.uniform(x[0], x[-1])
        y = rng.uniform(0.1, 5.0) * (x - x0) ** 2 + rng.uniform(-3, 3)
        assert abs(oracle.sweep_fit_min(x, y) - x0) < 1e-9
        # a constant or a positive scale of the misfit, or a shift of the sweep, moves nothing
        assert abs(oracle.sweep_fit_min(x, 3.0 * y + 10.0) - x0) < 1e-9
        assert abs(oracle.sweep_fit_min(x + 2.5, y) - (x0 + 2.5)) < 1e-9
    x = np.linspace(11, 14, 7)
    assert oracle.sweep_fit_min(x, (x - 9.0) ** 2) == 11.0          # vertex left of the sweep
    assert oracle.sweep_fit_min(x, (x - 16.0) ** 2) == 14.0         # right of it
    assert oracle.sweep_fit_min(x, -(x - 12.0) ** 2) == 14.0        # opens downwards: smallest sample
    assert oracle.sweep_fit_min(x, np.ones(7)) == 11.0              # flat: the first sample
    assert oracle.sweep_fit_min(x[:2], [2.0, 1.0]) == x[1]


def test_fit_min_averages_noise():
    """Noise on the samples: the least-squares vertex scatters around the true one by about
    sigma_v = sqrt(var), well inside the sample spacing, and without bias."""
    rng = np.random.default_rng(8)
    x = np.linspace(11.0, 14.5, 8)
    x0 = 12.7
    v = np.array([oracle.sweep_fit_min(x, 100.0 * (x - x0) ** 2 + rng.normal(0, 20.0, 8)) for _ in range(400)])
    assert abs(v.mean() - x0) < 0.02 and v.std() < 0.1


def test_fit_match_line_crossing():
    rng = np.random.default_rng(9)
    x = np.array([11.0, 11.7, 12.1, 13.0, 14.2])
    for slope in (0.5, -0.8):
        y = slope * (x - 12.6) + 1.0
        assert abs(oracle.sweep_fit_match(x, y, 1.0) - 12.6) < 1e-12
        assert math.isnan(oracle.sweep_fit_match(x, y, 1.0 + 10 * abs(slope)))      # outside the sweep
    assert math.isnan(oracle.sweep_fit_match(x, np.full(5, 2.0), 2.0))               # flat
    assert math.isnan(oracle.sweep_fit_match(x[:1], [1.0], 1.0))
    # symmetric noise about a line does not move the crossing
    e = rng.normal(0, 0.1, 5)
    e -= np.polynomial.polynomial.polyval(x, np.polynomial.polynomial.polyfit(x, e, 1))
    assert abs(oracle.sweep_fit_match(x, 0.5 * (x - 12.6) + 1.0 + e, 1.0) - 12.6) < 1e-12


def test_sweep_composition_invariants():
    rng = np.random.default_rng(6)
    a, b, P, M, rho = si.ternary_composition_inputs()
    f = rng.uniform(1e-5, 1e-4, (4, 3, 342))
    c = oracle.sweep_composition(f, a, b, P, M, rho)
    assert c.shape == (4, 342, 3)
    assert np.allclose(c.sum(axis=2), 100.0, atol=1e-12)
    f2 = f * rng.uniform(0.5, 2.0, (4, 1, 1))
    assert np.allclose(oracle.sweep_composition(f2, a, b, P, M, rho), c, rtol=1e-13, atol=1e-12)
    f1 = f.copy()
    f1[:, 1:, :] = 0.0
    f1[:, 1:, 0] = 1e-30                                     # keep the calibration value finite
    c1 = oracle.sweep_composition(f1, a, b, P, M, rho)
    assert np.allclose(c1[:, 1:, 0], 100.0, atol=1e-9)


def test_ternary_rate_lines_are_table_s1_fits():
    rows = [r for r in csv.DictReader(l for l in open(GOLDEN / "table_s1.csv") if not l.startswith("#"))]
    for el, sup, a, b in zip(si.TERNARY_ELEMENTS, ("RF", "DC", "DC"), si.TERNARY_RATE_A, si.TERNARY_RATE_B):
        pts = [(float(r["power_W"]), float(r["rate_nm_per_s"])) for r in rows
               if r["element"] == el and r["power_type"] == sup]
        assert len(pts) == 2
        fa, fb = oracle.fit_power_rate([p for p, _ in pts], [q for _, q in pts])
        assert abs(fa - a) < 1e-15 and abs(fb - b) < 1e-15
