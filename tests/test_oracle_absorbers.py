"""Pins of the oracle's absorbing objects (Methods, "The SIMTRA model" and "The SIMTRA Python
wrapper": dummy objects such as masks, shutters and chimneys collect the atoms that reach them;
a multi-cathode system split into single-cathode runs neglects cross deposition, which the
cross_absorb option lifts by letting the other targets absorb).

* The surface test with discs, rectangles and open tubes against a brute-force march along
  the ray (sign changes of each surface's signed distance, bisection), from outside and inside
  a tube.
* 0 Pa, point source on the axis: an atom whose emission angle exceeds the chimney's
  acceptance atan(R/L) ends on the tube, exactly; every other atom is unaffected (its record is
  identical to the run without the chimney).  The same for a disc mask.
* With the other targets absorbing, every particle that does not end on another target has
  exactly the record of the run without: the option only stops paths that cross a target.
"""
import math

import numpy as np
import pytest

import oracle
import sputter_inputs as si


def _crossings(f, t_max, h=0.05):
    """All sign changes of f on (0, t_max] (f vectorised over t), refined by bisection."""
    t = np.concatenate([[1e-9], np.arange(h, t_max, h), [t_max]])
    v = f(t) > 0
    out = []
    for i in np.nonzero(v[1:] != v[:-1])[0]:
        a, b, fa = t[i], t[i + 1], v[i]
        for _ in range(80):
            m = 0.5 * (a + b)
            if (f(np.array([m]))[0] > 0) == fa:
                a = m
            else:
                b = m
        out.append(0.5 * (a + b))
    return out


def _brute_objects(objs, x, d, t_max):
    best = math.inf
    for o in objs:
        c, n, u = (np.asarray(v, dtype=np.float64) for v in (o.center, o.normal, o.u_axis))
        v = np.cross(n, u)
        pts = lambda t: x[None, :] + t[:, None] * d[None, :] - c[None, :]
        if o.kind in ("disc", "rect"):
            for t in _crossings(lambda t: pts(t) @ n, t_max):
                q = x + t * d - c
                ins = ((q @ u) ** 2 + (q @ v) ** 2 <= o.half_u ** 2) if o.kind == "disc" else \
                    (abs(q @ u) <= o.half_u and abs(q @ v) <= o.half_v)
                if ins:
                    best = min(best, t)
                    break
        else:
            def radial(t):
                w = pts(t)
                return np.sqrt(np.maximum((w * w).sum(1) - (w @ n) ** 2, 0.0)) - o.half_u
            for t in _crossings(radial, t_max):
                za = (x + t * d - c) @ n
                if 0.0 <= za <= o.length:
                    best = min(best, t)
                    break
    return best


def _objects_cfg():
    cfg = si.single_ni(0.5, 10)
    cfg.absorbers = [
        si.Absorber("disc", center=(0.0, 0.0, 150.0), normal=(0.0, 0.0, 1.0), half_u=20.0),
        si.Absorber("rect", center=(40.0, -30.0, 160.0), normal=(0.0, math.sin(0.4), math.cos(0.4)),
                    u_axis=(1.0, 0.0, 0.0), half_u=15.0, half_v=8.0),
        si.Absorber("tube", center=(0.0, 0.0, 100.0), normal=(0.0, 0.0, 1.0), half_u=30.0, length=40.0),
        si.Absorber("tube", center=(-120.0, 60.0, 60.0), normal=(math.sin(0.3), 0.0, math.cos(0.3)),
                    u_axis=(math.cos(0.3), 0.0, -math.sin(0.3)), half_u=12.0, length=70.0),
    ]
    return cfg


def test_object_hits_against_ray_march(params):
    cfg = _objects_cfg()
    rng = np.random.default_rng(23)
    hits = 0
    for trial in range(240):
        if trial % 4 == 0:              # start inside the chimney around the target
            x = np.array([rng.uniform(-20, 20), rng.uniform(-20, 20), rng.uniform(101, 139)])
        else:
            while True:
                x = np.array([rng.uniform(-180, 180), rng.uniform(-180, 180), rng.uniform(5, 295)])
                if math.hypot(x[0], x[1]) < 190:
                    break
        tgt = np.array([rng.uniform(-60, 60), rng.uniform(-60, 60), rng.uniform(90, 170)])
        d = tgt - x
        d /= np.linalg.norm(d)
        t_o, st, _ = oracle.hit([cfg], params, x, d)
        t_b = _brute_objects(cfg.absorbers, x, d, 1000.0)
        if t_b < t_o - 1e-7:
            raise AssertionError(("missed object", trial, t_b, t_o))
        if abs(t_b - t_o) < 1e-7:
            hits += 1
            assert st == 2                # objects absorb (WALL)
    assert hits > 40


def _point_source(n, law=(0, 1, 0, 0, 0, 0), absorbers=()):
    cfg = si.with_launch(si.single_ni(0.0, n), [(0.0, 1.0), (1e-6, 1.0)], law)
    cfg.absorbers = list(absorbers)
    return cfg


@pytest.mark.parametrize("law", [(0, 1, 0, 0, 0, 0), si.UNDER_COSINE])
def test_chimney_acceptance_is_exact(params, law):
    n = 200_000
    R, L = 30.0, 40.0
    tube = si.Absorber("tube", center=(0.0, 0.0, 100.0), normal=(0.0, 0.0, 1.0), half_u=R, length=L)
    with_t = oracle.run([_point_source(n, law, [tube])], params, seed=8, records=True)["records"]
    without = oracle.run([_point_source(n, law)], params, seed=8, records=True)["records"]
    mu = oracle.launch_batch([_point_source(n, law)], params, 8, 0, n)[:, 5]     # d_z = cos(theta)
    mu_c = L / math.hypot(L, R)
    on_tube = (np.abs(np.hypot(with_t[:, 0], with_t[:, 1]) - R) < 1e-9) & (with_t[:, 2] >= 100.0) & \
              (with_t[:, 2] <= 100.0 + L)
    assert np.array_equal(on_tube, mu < mu_c)
    assert np.all(with_t[on_tube, 3] == 2)
    assert np.array_equal(with_t[~on_tube], without[~on_tube])


def test_mask_shadow_is_exact(params):
    n = 200_000
    rm, zm = 12.0, 150.0
    mask = si.Absorber("disc", center=(0.0, 0.0, zm), normal=(0.0, 0.0, 1.0), half_u=rm)
    with_m = oracle.run([_point_source(n, absorbers=[mask])], params, seed=9, records=True)["records"]
    without = oracle.run([_point_source(n)], params, seed=9, records=True)["records"]
    L = oracle.launch_batch([_point_source(n)], params, 9, 0, n)
    x0, d = L[:, :3], L[:, 3:6]
    t = (zm - x0[:, 2]) / d[:, 2]
    q = x0 + t[:, None] * d
    hits_mask = np.hypot(q[:, 0], q[:, 1]) <= rm
    on_mask = (np.abs(with_m[:, 2] - zm) < 1e-9) & (np.hypot(with_m[:, 0], with_m[:, 1]) <= rm + 1e-9)
    assert np.array_equal(on_mask, hits_mask)
    assert np.array_equal(with_m[~on_mask], without[~on_mask])
    assert np.all(with_m[on_mask, 3] == 2)


def test_cross_absorption_only_stops_paths_that_cross_a_target(params):
    cfg = si.quaternary(0.5, 25.0, 150.0, [3000, 600, 2000, 1200])
    cross = si.Config(cfg.chamber, cfg.grid, cfg.cathodes, cross_absorb=True)
    a = oracle.run([cross], params, seed=10, records=True)["records"]
    b = oracle.run([cfg], params, seed=10, records=True)["records"]
    first = np.cumsum([0] + [c.n_particles for c in cfg.cathodes])
    n_on_other = 0
    for k, cat in enumerate(cfg.cathodes):
        r = a[first[k]:first[k + 1]]
        on_other = np.zeros(len(r), bool)
        for j, o in enumerate(cfg.cathodes):
            if j == k:
                continue
            c, nn = np.array(o.center), np.array(o.normal)
            w = r[:, :3] - c
            h = w @ nn
            rho = np.sqrt(np.maximum((w * w).sum(1) - h * h, 0.0))
            on_other |= (np.abs(h) < 1e-9) & (rho <= o.radius + 1e-9)
        n_on_other += on_other.sum()
        assert np.all(r[on_other, 3] == 2)
        assert np.array_equal(r[~on_other], b[first[k]:first[k + 1]][~on_other])
    assert n_on_other > 0
