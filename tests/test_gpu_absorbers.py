"""GPU parity of absorbing objects (masks, shutters, chimneys, the other targets) against the
FP64 oracle, through the C-ABI (Methods, "The SIMTRA model" and "The SIMTRA Python wrapper":
dummy objects collect the atoms that reach them; cross_absorb lets the other targets of a
configuration absorb).

Bar: per particle, the batched FP32 path puts >= 99 % of particles in the oracle's terminal
state within 1e-3 mm of its end point, the FP64 path >= 99.9 % within 1e-6 mm; tallies equal
the histogram of the records; tallies are bit-identical across launch shapes.  At 0 Pa from a
point source, the atoms that end on a chimney are exactly those whose polar angle exceeds its
acceptance atan(R/L), and a disc mask takes exactly the atoms whose straight line crosses it,
outside a rounding band around the edge; every other atom's record equals the run without the
object bit for bit.
"""
import math
from dataclasses import replace

import numpy as np
import pytest

import oracle
import sputter_inputs as si
from parity import bin_flips_off_edge, match_stats, records_histogram, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2411_14413_amd as spx  # noqa: E402

PARAMS = si.Params()


def _objects_cfg(pressure, n):
    cfg = si.single_ni(pressure, n)
    cfg.absorbers = [
        si.Absorber("disc", center=(0.0, 0.0, 150.0), normal=(0.0, 0.0, 1.0), half_u=20.0),
        si.Absorber("rect", center=(40.0, -30.0, 160.0), normal=(0.0, math.sin(0.4), math.cos(0.4)),
                    u_axis=(1.0, 0.0, 0.0), half_u=15.0, half_v=8.0),
        si.Absorber("tube", center=(0.0, 0.0, 100.0), normal=(0.0, 0.0, 1.0), half_u=30.0, length=40.0),
        si.Absorber("tube", center=(-120.0, 60.0, 60.0), normal=(math.sin(0.3), 0.0, math.cos(0.3)),
                    u_axis=(math.cos(0.3), 0.0, -math.sin(0.3)), half_u=12.0, length=70.0),
    ]
    return cfg


def _batch():
    return [_objects_cfg(0.5, 20000), _objects_cfg(2.0, 2500),
            si.with_chimneys(si.quaternary(0.5, 25.0, 150.0, [3000, 1000, 2000, 1500])),
            replace(si.quaternary(1.2, 10.0, 95.0, [800, 300, 500, 400]), cross_absorb=True)]


def _first(plan):
    return list(plan.first) + [plan.n_particles]


@pytest.fixture(scope="module")
def batch_ref():
    cfgs = _batch()
    say("oracle: absorbers batch", [c.n_particles for cfg in cfgs for c in cfg.cathodes])
    return cfgs, oracle.run(cfgs, PARAMS, seed=31, records=True)


@pytest.mark.parametrize("precision, tol, need", [(32, 1e-3, 0.99), (64, 1e-6, 0.999)])
def test_absorber_parity(batch_ref, precision, tol, need):
    cfgs, ref = batch_ref
    say(f"absorbers parity, precision {precision}")
    plan = spx.Plan(cfgs, PARAMS, precision=precision)
    out = plan.run(seed=31, records=True)
    torch.cuda.synchronize()
    rec = spx.records_to_numpy(out["records"])
    first = _first(plan)
    wall_o = wall_g = 0
    for k in range(plan.n_segments):
        sl = slice(first[k], first[k + 1])
        m = match_stats(rec[sl], ref["records"][sl], tol)
        say(f"  seg {k}: {m}")
        assert m["frac"] >= need, (k, m)
        grid = [cfg.grid for cfg in cfgs for _ in cfg.cathodes][k]
        assert bin_flips_off_edge(rec[sl], ref["records"][sl], tol, grid) == 0, (k, m)
        wall_o += int((ref["records"][sl, 3] == 2).sum())
        wall_g += int((rec[sl]["state"] == 2).sum())
    assert abs(wall_g - wall_o) <= 0.01 * wall_o + 5
    hist = records_histogram(rec, [nv * nu for nv, nu in plan.shapes], first, plan.n_bins)
    C = out["counters"].cpu().numpy()
    for k in range(plan.n_segments):
        assert np.array_equal(out["counts_seg"][k].cpu().numpy().ravel(), hist[k])
        assert C[k, 0] == C[k, 1] + C[k, 2] + C[k, 3]


def test_absorber_determinism_across_launch_shapes():
    cfgs = [_objects_cfg(0.5, 20000), si.with_chimneys(si.quaternary(0.9, 30.0, 120.0, [2000, 500, 1500, 800]))]
    say("absorbers: determinism across launch shapes")
    plan = spx.Plan(cfgs, PARAMS)
    results = []
    for blocks, threads, refill, bmin, defer in ((0, 256, 4, 4, 8), (0, 1024, 8, 8, 16), (7, 64, 64, 64, 2),
                                                 (300, 512, 4, 16, 32)):
        plan.set_launch(blocks, threads, refill, bmin, defer)
        out = plan.run(seed=12, records=True)
        torch.cuda.synchronize()
        results.append((out["counts"].cpu().numpy(), out["counters"].cpu().numpy(), out["records"].cpu().numpy()))
    for r in results[1:]:
        for a, b in zip(r, results[0]):
            assert np.array_equal(a, b)


def _point_source(n, law=(0, 1, 0, 0, 0, 0), absorbers=()):
    cfg = si.with_launch(si.single_ni(0.0, n), [(0.0, 1.0), (1e-6, 1.0)], law)
    cfg.absorbers = list(absorbers)
    return cfg


def _gpu_records(cfg, seed, precision):
    plan = spx.Plan([cfg], PARAMS, precision=precision)
    out = plan.run(seed=seed, records=True)
    torch.cuda.synchronize()
    return spx.records_to_numpy(out["records"])


def _pos(r):
    return np.stack([r["x"], r["y"], r["z"]], axis=1)


@pytest.mark.parametrize("precision, band", [(32, 2e-5), (64, 1e-9)])
@pytest.mark.parametrize("law", [(0, 1, 0, 0, 0, 0), si.UNDER_COSINE])
def test_chimney_acceptance_is_exact(law, precision, band):
    n = 1_000_000
    R, L = 30.0, 40.0
    say(f"chimney acceptance at 0 Pa: precision {precision}, law {law}")
    tube = si.Absorber("tube", center=(0.0, 0.0, 100.0), normal=(0.0, 0.0, 1.0), half_u=R, length=L)
    with_t = _gpu_records(_point_source(n, law, [tube]), 8, precision)
    without = _gpu_records(_point_source(n, law), 8, precision)
    mu = oracle.launch_batch([_point_source(n, law)], PARAMS, 8, 0, n)[:, 5]     # d_z = cos(theta)
    mu_c = L / math.hypot(L, R)
    p = _pos(with_t)
    tol = 1e-3 if precision == 32 else 1e-9
    on_tube = (np.abs(np.hypot(p[:, 0], p[:, 1]) - R) < tol) & (p[:, 2] >= 100.0 - tol) & (p[:, 2] <= 100.0 + L + tol)
    clear = np.abs(mu - mu_c) > band
    say(f"  on tube {int(on_tube.sum())}, in the rounding band {int((~clear).sum())}")
    assert np.array_equal(on_tube[clear], (mu < mu_c)[clear])
    assert np.all(with_t["state"][on_tube] == 2)
    assert np.array_equal(with_t[~on_tube], without[~on_tube])


@pytest.mark.parametrize("precision, band", [(32, 2e-3), (64, 1e-7)])
def test_mask_shadow_is_exact(precision, band):
    n = 1_000_000
    rm, zm = 12.0, 150.0
    say(f"mask shadow at 0 Pa: precision {precision}")
    mask = si.Absorber("disc", center=(0.0, 0.0, zm), normal=(0.0, 0.0, 1.0), half_u=rm)
    with_m = _gpu_records(_point_source(n, absorbers=[mask]), 9, precision)
    without = _gpu_records(_point_source(n), 9, precision)
    Lb = oracle.launch_batch([_point_source(n)], PARAMS, 9, 0, n)
    x0, d = Lb[:, :3], Lb[:, 3:6]
    t = (zm - x0[:, 2]) / d[:, 2]
    rho = np.hypot(x0[:, 0] + t * d[:, 0], x0[:, 1] + t * d[:, 1])
    p = _pos(with_m)
    tol = 1e-3 if precision == 32 else 1e-9
    on_mask = (np.abs(p[:, 2] - zm) < tol) & (np.hypot(p[:, 0], p[:, 1]) <= rm + tol)
    clear = np.abs(rho - rm) > band
    say(f"  on mask {int(on_mask.sum())}, in the rounding band {int((~clear).sum())}")
    assert np.array_equal(on_mask[clear], (rho <= rm)[clear])
    assert np.all(with_m["state"][on_mask] == 2)
    assert np.array_equal(with_m[~on_mask], without[~on_mask])


def test_cross_absorption_at_zero_pressure_only_stops_paths_that_cross_a_target():
    cfg = si.quaternary(0.0, 25.0, 150.0, [200_000, 50_000, 150_000, 100_000])
    cross = replace(cfg, cross_absorb=True)
    say("cross absorption at 0 Pa")
    plan_a = spx.Plan([cross], PARAMS)
    plan_b = spx.Plan([cfg], PARAMS)
    a = spx.records_to_numpy(plan_a.run(seed=10, records=True)["records"])
    b = spx.records_to_numpy(plan_b.run(seed=10, records=True)["records"])
    torch.cuda.synchronize()
    first = _first(plan_a)
    n_on_other = 0
    for k in range(plan_a.n_segments):
        r, r0 = a[first[k]:first[k + 1]], b[first[k]:first[k + 1]]
        p = _pos(r)
        on_other = np.zeros(len(r), bool)
        for j, o in enumerate(cfg.cathodes):
            if j == k:
                continue
            w = p - np.asarray(o.center)
            h = w @ np.asarray(o.normal)
            rho = np.sqrt(np.maximum((w * w).sum(1) - h * h, 0.0))
            on_other |= (np.abs(h) < 1e-3) & (rho <= o.radius + 1e-3)
        n_on_other += int(on_other.sum())
        assert np.all(r["state"][on_other] == 2)
        assert np.array_equal(r[~on_other], r0[~on_other])
    say(f"  {n_on_other} atoms end on another target")
    assert n_on_other > 0
