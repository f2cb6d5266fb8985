"""GPU parity of the transport path against the FP64 oracle, through the C-ABI.

Bar (per particle, same Philox streams): the batched FP32 path puts >= 99 % of
particles in the oracle's terminal state within 1e-3 mm of the oracle's end point;
the plain FP64 path >= 99.9 % within 1e-6 mm.  Integer work is exact: tallies equal
the histogram of the records, counters equal their record-derived values, and
deposited + wall + escaped = launched; tallies are bit-identical across launch
shapes and graph replays.  Tallies agree with the oracle's within 3 sigma of
counting noise, and the 0 Pa profile with the analytic line-of-sight flux.
"""
import math

import numpy as np
import pytest

import oracle
import sputter_inputs as si
from parity import match_stats, records_histogram, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2411_14413_amd as spx  # noqa: E402

PARAMS = si.Params()


def small_batch():
    return [si.single_ni(0.5, 20000), si.single_ni(0.0, 20000), si.single_ni(2.0, 2500),
            si.quaternary(0.5, 25.0, 150.0, [4000, 1000, 3000, 2000]),
            si.quaternary(1.7, 8.0, 95.0, [700, 300, 500, 400])]


@pytest.fixture(scope="module")
def batch_ref():
    cfgs = small_batch()
    say("oracle: small batch", [c.n_particles for cfg in cfgs for c in cfg.cathodes])
    ref = oracle.run(cfgs, PARAMS, seed=7, records=True)
    return cfgs, ref


def _first(plan):
    return list(plan.first) + [plan.n_particles]


def test_philox_bitwise():
    n = 1 << 20
    rng = np.random.default_rng(3)
    ctr = rng.integers(0, 2**32, size=(n, 4), dtype=np.uint64).astype(np.uint32)
    ctr[:1000, 1] = np.arange(1000)
    seed = 0x0123456789ABCDEF
    say("philox: 2^20 counters")
    got = spx.philox(torch.from_numpy(ctr.view(np.int32)).cuda(), seed).cpu().numpy().view(np.uint32)
    ref = oracle.philox_batch(ctr, [seed & 0xFFFFFFFF, seed >> 32])
    assert np.array_equal(got, ref)


def test_table_matches_oracle():
    say("table: FP64 GPU quadrature vs oracle")
    plan = spx.Plan([si.single_ni(0.5, 10)], PARAMS)
    th, bm = plan.table()
    oth, obm = oracle.table(PARAMS)
    assert np.abs(th.ravel() - oth).max() < 1e-10
    assert np.abs(bm / obm - 1).max() < 1e-10
    assert np.all(th[:, 0] == math.pi)


def test_segment_constants_match_oracle():
    cfgs = si.quaternary_sweep(8, scale=1e-3) + small_batch()
    say("segment constants:", len(cfgs), "configs")
    plan = spx.Plan(cfgs, PARAMS)
    k = 0
    for c, cfg in enumerate(cfgs):
        for j in range(len(cfg.cathodes)):
            g = plan.segment_info(k)
            o = oracle.seg_info(cfgs, PARAMS, seg=k)
            for name in ("Lambda", "E_max", "s_max", "a_mm", "eps_per_eV", "n_mm3", "kT", "E_th", "PhiA", "QB",
                         "dPhi", "mu_red", "vth", "vg"):
                assert abs(g[name] - o[name]) <= 1e-13 * max(1.0, abs(o[name])) + 1e-300, (k, name, g[name], o[name])
            if math.isfinite(o["lam_th"]):
                assert abs(g["lam_th"] / o["lam_th"] - 1) < 1e-9
            k += 1


@pytest.mark.parametrize("precision, tol, need", [(32, 1e-3, 0.99), (64, 1e-6, 0.999)])
def test_per_particle_parity(batch_ref, precision, tol, need):
    cfgs, ref = batch_ref
    say(f"parity: precision {precision}")
    plan = spx.Plan(cfgs, PARAMS, precision=precision)
    out = plan.run(seed=7, records=True)
    torch.cuda.synchronize()
    rec = spx.records_to_numpy(out["records"])
    first = _first(plan)
    for k in range(plan.n_segments):
        sl = slice(first[k], first[k + 1])
        m = match_stats(rec[sl], ref["records"][sl], tol)
        say(f"  seg {k}: {m}")
        assert m["frac"] >= need, (k, m)
        assert m["bin_frac"] >= 0.999, (k, m)
    # integer work is exact: tallies = histogram of records, counters = record sums
    hist = records_histogram(rec, [nv * nu for nv, nu in plan.shapes], first, plan.n_bins)
    C = out["counters"].cpu().numpy()
    for k in range(plan.n_segments):
        assert np.array_equal(out["counts_seg"][k].cpu().numpy().ravel(), hist[k])
        r = rec[first[k]:first[k + 1]]
        assert C[k, 0] == len(r) == plan.seg_particles[k]
        assert C[k, 1] == (r["state"] == 1).sum() and C[k, 2] == (r["state"] == 2).sum()
        assert C[k, 3] == (r["state"] == 3).sum()
        assert C[k, 5] == r["diffusive"].astype(np.int64).sum()
        assert C[k, 0] == C[k, 1] + C[k, 2] + C[k, 3]
        assert abs(int(C[k, 6]) - int(ref["counters"][k, 6])) <= 0.01 * C[k, 0] + 3
        assert int(C[k, 6]) >= int((r["diffusive"] > 0).sum())
    # normalised profiles
    for k in range(plan.n_segments):
        nv, nu = plan.shapes[k]
        g = cfgs[0].grid if k < 3 else cfgs[3].grid
        area = (2 * g.half_u / nu) * (2 * g.half_v / nv)
        prof = out["profiles_seg"][k].cpu().numpy()
        cnt = out["counts_seg"][k].cpu().numpy()
        assert np.allclose(prof, cnt / (plan.seg_particles[k] * area), rtol=1e-15, atol=0)
    # tallies within counting noise of the oracle's (same particles: far inside)
    for k in range(plan.n_segments):
        a = out["counts_seg"][k].cpu().numpy().astype(np.float64)
        b = ref["counts"][k].astype(np.float64)
        z = (a - b) / np.sqrt(np.maximum(a + b, 1.0))
        assert np.abs(z).max() < 3.0, (k, np.abs(z).max())


def test_longest_walks_parity():
    """The longest histories of a 2 Pa run (tens of thousands of diffusive steps, each added to
    the offset from its clearance-ball centre in FP32) end where the FP64 oracle's do: the
    rounding of a walk between two surface tests is relative to the offset, at most the ball
    radius, so N steps drift by about sqrt(N) ulp(r) / sqrt(12), far inside the 1e-3 mm bar."""
    cfg = si.single_ni(2.0, 200_000)
    say("longest walks at 2 Pa: FP32 records vs the oracle on the same particles")
    plan = spx.Plan([cfg], PARAMS)
    rec = spx.records_to_numpy(plan.run(seed=21, records=True)["records"])
    torch.cuda.synchronize()
    pids = np.argsort(rec["events"].astype(np.int64))[-300:]
    ref = oracle.run_list([cfg], PARAMS, 21, np.zeros(len(pids), np.uint32), pids)
    m = match_stats(rec[pids], ref, 1e-3)
    say(f"  events {int(rec['events'][pids].min())}..{int(rec['events'][pids].max())}: {m}")
    assert int(rec["events"][pids].min()) > 5000
    assert m["same_state"] >= 0.99 and m["frac"] >= 0.97, m
    assert m["d_median"] < 2e-4, m


@pytest.mark.parametrize("pressure, n", [(5.0, 3000), (10.0, 1000)])
def test_high_pressure_parity(pressure, n):
    """Above the workloads' pressures the walks grow long (up to ~4e5 events at 10 Pa) and the
    offset walk's rounding drifts as sqrt(N); the FP32 bar still holds for the run."""
    cfg = [si.single_ni(pressure, n)]
    say(f"parity at {pressure} Pa")
    ref = oracle.run(cfg, PARAMS, seed=11, records=True)["records"]
    plan = spx.Plan(cfg, PARAMS)
    rec = spx.records_to_numpy(plan.run(seed=11, records=True)["records"])
    torch.cuda.synchronize()
    m = match_stats(rec, ref, 1e-3)
    say(f"  events up to {int(rec['events'].max())}: {m}")
    assert m["same_state"] >= 0.995 and m["frac"] >= 0.99, m


def test_determinism_across_launch_shapes():
    cfgs = [si.single_ni(0.5, 30000), si.single_ni(2.0, 3000), si.quaternary(0.9, 30.0, 120.0, [2000, 500, 1500, 800])]
    say("determinism: launch shapes")
    plan = spx.Plan(cfgs, PARAMS)
    results = []
    for blocks, threads, refill, bmin, defer in ((0, 256, 1, 1, 8), (0, 1024, 24, 32, 16), (7, 64, 64, 64, 1),
                                                 (300, 512, 8, 3, 64), (0, 512, 1, 64, 5)):
        plan.set_launch(blocks, threads, refill, bmin, defer)
        out = plan.run(seed=11, records=True)
        torch.cuda.synchronize()
        results.append((out["counts"].cpu().numpy(), out["counters"].cpu().numpy(), out["records"].cpu().numpy()))
    for r in results[1:]:
        assert np.array_equal(r[0], results[0][0])
        assert np.array_equal(r[1], results[0][1])
        assert np.array_equal(r[2], results[0][2])


def test_graph_replays_identical():
    cfgs = [si.single_ni(0.5, 50000), si.single_ni(2.0, 2000)]
    say("graph replays")
    plan = spx.Plan(cfgs, PARAMS)
    bufs = plan.allocate(profiles=True)
    outs = []
    for i in range(4):
        plan.run_into(5, bufs)
        junk = torch.randn(1 << 20, device="cuda").sum()   # unrelated eager work in between
        torch.cuda.synchronize()
        outs.append((bufs["counts"].cpu().numpy().copy(), bufs["counters"].cpu().numpy().copy(),
                     bufs["profiles"].cpu().numpy().copy()))
        del junk
    for o in outs[1:]:
        for x, y in zip(o, outs[0]):
            assert np.array_equal(x, y)
    # a different seed changes the tallies; the same seed again restores them
    plan.run_into(6, bufs)
    torch.cuda.synchronize()
    assert not np.array_equal(bufs["counts"].cpu().numpy(), outs[0][0])
    plan.run_into(5, bufs)
    torch.cuda.synchronize()
    assert np.array_equal(bufs["counts"].cpu().numpy(), outs[0][0])


def test_zero_pressure_profile_against_line_of_sight():
    from test_oracle_transport import analytic_bin_fractions
    n = 10_000_000
    cfg = si.single_ni(0.0, n)
    say("0 Pa: 1e7 particles vs analytic view factor")
    plan = spx.Plan([cfg], PARAMS)
    out = plan.run(seed=0)
    torch.cuda.synchronize()
    counts = out["counts_seg"][0].cpu().numpy().astype(np.float64)
    exp = n * analytic_bin_fractions(cfg)
    z = (counts - exp) / np.sqrt(exp)
    dof = counts.size
    chi2 = float((z**2).sum())
    say(f"  chi2/dof = {chi2 / dof:.4f}, max|z| = {np.abs(z).max():.2f}, total {counts.sum():.0f} vs {exp.sum():.0f}")
    assert chi2 < dof + 4.5 * math.sqrt(2 * dof)
    assert np.abs(z).max() < 5.0
    assert abs(counts.sum() - exp.sum()) < 4.5 * math.sqrt(exp.sum())


def test_edge_cases():
    say("edge cases")
    cfgs = [
        si.quaternary(0.5, 25.0, 150.0, [0, 5, 0, 1]),            # empty segments next to tiny ones
        si.single_ni(0.5, 1),                                      # a single particle
        si.Config(si.Chamber(pressure=0.3), si.Grid(nu=1, nv=1), [si.species_cathode("Pt", n_particles=700)]),
        si.Config(si.Chamber(pressure=0.5, gas_motion=0), si.Grid(nu=7, nv=3, half_v=20.0),
                  [si.species_cathode("Ru", n_particles=900)]),
    ]
    ref = oracle.run(cfgs, PARAMS, seed=3, records=True)
    for precision, tol in ((32, 1e-3), (64, 1e-6)):
        plan = spx.Plan(cfgs, PARAMS, precision=precision)
        out = plan.run(seed=3, records=True)
        torch.cuda.synchronize()
        rec = spx.records_to_numpy(out["records"])
        assert len(rec) == len(ref["records"]) == 0 + 5 + 0 + 1 + 1 + 700 + 900
        m = match_stats(rec, ref["records"], tol)
        assert m["frac"] >= 0.99, m
        C = out["counters"].cpu().numpy()
        assert np.array_equal(C[:, 0], [0, 5, 0, 1, 1, 700, 900])
        assert np.array_equal(C[:, 0], C[:, 1] + C[:, 2] + C[:, 3])
    # the event cap turns every long history into ESCAPED, identically on both sides
    p = si.Params(event_cap=3)
    cfg = [si.single_ni(2.0, 3000)]
    ref = oracle.run(cfg, p, seed=9, records=True)
    plan = spx.Plan(cfg, p)
    out = plan.run(seed=9, records=True)
    torch.cuda.synchronize()
    rec = spx.records_to_numpy(out["records"])
    assert (rec["state"] == 3).sum() > 0
    assert rec["events"].max() == 3
    m = match_stats(rec, ref["records"], 1e-3)
    assert m["frac"] >= 0.99, m


def test_event_cap_in_the_walk():
    """A cap that ends most 2 Pa histories in the middle of their diffusive walk: every
    history past it escapes with exactly `cap` events, where the oracle's does, whether the
    step-by-step walk or the wave-cooperative tail (waves left with few walkers) reaches the
    cap; records are bit-identical across launch shapes that move histories between the two."""
    p = si.Params(event_cap=300)
    cfg = [si.single_ni(2.0, 3000)]
    say("event cap 300 at 2 Pa")
    ref = oracle.run(cfg, p, seed=19, records=True)
    plan = spx.Plan(cfg, p)
    recs = []
    for blocks, threads in ((0, 256), (7, 64), (3, 1024)):
        plan.set_launch(blocks, threads, 4, 16, 8)
        recs.append(spx.records_to_numpy(plan.run(seed=19, records=True)["records"]))
        torch.cuda.synchronize()
    for r in recs[1:]:
        assert np.array_equal(r, recs[0])
    rec = recs[0]
    capped = rec["state"] == 3
    say(f"  {int(capped.sum())} of {len(rec)} capped; diffusive steps of the capped {int(rec['diffusive'][capped].sum())}")
    assert capped.mean() > 0.3 and rec["diffusive"][capped].min() > 0
    assert np.all(rec["events"][capped] == 300) and rec["events"].max() == 300
    m = match_stats(rec, ref["records"], 1e-3)
    assert m["same_state"] >= 0.995 and m["frac"] >= 0.99, m


def test_phase_times():
    """The two kernels' device times of the last run (events recorded between them)."""
    say("phase times")
    plan = spx.Plan([si.single_ni(2.0, 20000), si.single_ni(0.0, 20000)], PARAMS)
    with pytest.raises(spx.SpxError):
        plan.phase_times()                      # no run yet
    bufs = plan.allocate(profiles=False)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    plan.run_into(4, bufs)
    ev1.record()
    tb, td = plan.phase_times()
    torch.cuda.synchronize()
    total = ev0.elapsed_time(ev1)
    say(f"  ballistic {tb:.3f} ms, diffusive {td:.3f} ms, step {total:.3f} ms")
    assert tb > 0 and td > 0 and tb + td <= total * 1.001 + 0.05
    # FP64 plans have no batched phases
    p64 = spx.Plan([si.single_ni(0.5, 100)], PARAMS, precision=64)
    p64.run(seed=1)
    with pytest.raises(spx.SpxError):
        p64.phase_times()


def _measured_launch_batch():
    prof = si.measured_racetrack(seed=0)
    return [si.with_launch(si.single_ni(0.5, 20000), prof, si.UNDER_COSINE),
            si.with_launch(si.single_ni(0.0, 20000), [(0.0, 0.0), (10.0, 0.0), (12.0, 1.0), (18.0, 1.0),
                                                     (20.0, 0.0), (25.4, 0.0)], (0, 0, 1, 0, 0, 0)),
            si.with_launch(si.single_ni(2.0, 2000), prof, (1, 0, 0, 0, 0, 0)),
            si.with_launch(si.quaternary(0.5, 25.0, 150.0, [3000, 1000, 2000, 1500]), prof, si.UNDER_COSINE)]


@pytest.mark.parametrize("precision, tol, need", [(32, 1e-3, 0.99), (64, 1e-6, 0.999)])
def test_measured_racetrack_and_emission_law_parity(precision, tol, need):
    """Launch from a measured racetrack profile with six-coefficient emission laws: per-particle
    parity with the oracle, integer identities."""
    cfgs = _measured_launch_batch()
    say(f"measured racetrack / emission law parity, precision {precision}")
    ref = oracle.run(cfgs, PARAMS, seed=21, records=True)
    plan = spx.Plan(cfgs, PARAMS, precision=precision)
    out = plan.run(seed=21, records=True)
    torch.cuda.synchronize()
    rec = spx.records_to_numpy(out["records"])
    first = _first(plan)
    for k in range(plan.n_segments):
        sl = slice(first[k], first[k + 1])
        m = match_stats(rec[sl], ref["records"][sl], tol)
        say(f"  seg {k}: {m}")
        assert m["frac"] >= need, (k, m)
    hist = records_histogram(rec, [nv * nu for nv, nu in plan.shapes], first, plan.n_bins)
    for k in range(plan.n_segments):
        assert np.array_equal(out["counts_seg"][k].cpu().numpy().ravel(), hist[k])


def test_zero_pressure_measured_launch_against_line_of_sight():
    from test_oracle_transport import analytic_bin_fractions_general
    n = 10_000_000
    cfg = si.with_launch(si.single_ni(0.0, n), si.measured_racetrack(seed=0), si.UNDER_COSINE)
    say("0 Pa, measured racetrack, under-cosine law: 1e7 particles vs the integrated line of sight")
    plan = spx.Plan([cfg], PARAMS)
    out = plan.run(seed=0)
    torch.cuda.synchronize()
    counts = out["counts_seg"][0].cpu().numpy().astype(np.float64)
    exp = n * analytic_bin_fractions_general(cfg)
    z = (counts - exp) / np.sqrt(exp)
    dof = counts.size
    chi2 = float((z ** 2).sum())
    say(f"  chi2/dof = {chi2 / dof:.4f}, max|z| = {np.abs(z).max():.2f}")
    assert chi2 < dof + 4.5 * math.sqrt(2 * dof)
    assert np.abs(z).max() < 5.0
    assert abs(counts.sum() - exp.sum()) < 4.5 * math.sqrt(exp.sum())


def test_run_entry_matches_plan():
    """The one-call entry gives the tallies of an explicit plan, bit for bit."""
    cfgs = [si.single_ni(0.5, 20000), si.quaternary(0.9, 30.0, 120.0, [2000, 500, 1500, 800])]
    say("run(): one-call entry vs Plan.run")
    a = spx.run(cfgs, seed=5, params=PARAMS)
    b = spx.Plan(cfgs, PARAMS).run(seed=5)
    torch.cuda.synchronize()
    assert np.array_equal(a["counts"].cpu().numpy(), b["counts"].cpu().numpy())
    assert np.array_equal(a["counters"].cpu().numpy(), b["counters"].cpu().numpy())
    assert a["plan"].n_segments == 5


def test_autotune_leaves_results_unchanged():
    """Timing runs of the autotuner use their own buffers and the chosen launch parameters do
    not change any result: tallies, counters and records equal those of the default launch."""
    cfgs = [si.single_ni(2.0, 20000), si.quaternary(0.5, 25.0, 150.0, [3000, 800, 2000, 1200])]
    say("autotune: results unchanged")
    plan = spx.Plan(cfgs, PARAMS)
    ref = plan.run(seed=9, records=True)
    torch.cuda.synchronize()
    r0 = (ref["counts"].cpu().numpy(), ref["counters"].cpu().numpy(), ref["records"].cpu().numpy())
    launch = plan.autotune()
    say(f"  chosen {launch}")
    out = plan.run(seed=9, records=True)
    torch.cuda.synchronize()
    for a, b in zip(r0, (out["counts"].cpu().numpy(), out["counters"].cpu().numpy(), out["records"].cpu().numpy())):
        assert np.array_equal(a, b)


def test_seeds_share_one_graph():
    """Five seeds, each into fresh output buffers, through one instantiated graph: the seed and
    the buffers are replaced in the graph's kernel nodes, the graph is built once, and every
    run equals a fresh plan's run of the same seed bit for bit."""
    cfgs = [si.single_ni(0.5, 20000), si.single_ni(2.0, 2000), si.quaternary(0.9, 30.0, 120.0, [2000, 500, 1500, 800])]
    say("five seeds through one graph")
    plan = spx.Plan(cfgs, PARAMS)
    outs = []
    for seed in (3, 4, 5, 2**40 + 7, 3):
        o = plan.run(seed=seed, records=True)
        outs.append((seed, o))
    torch.cuda.synchronize()
    inst, upd = plan.graph_info()
    say(f"  instantiations {inst}, node updates {upd}")
    assert inst == 1
    assert upd >= 4 * 3          # at least the zero, ballistic and diffusive nodes of each later run
    for seed, o in outs:
        f = spx.Plan(cfgs, PARAMS).run(seed=seed, records=True)
        torch.cuda.synchronize()
        for key in ("counts", "counters", "records", "profiles"):
            assert torch.equal(o[key], f[key]), (seed, key)
    assert not torch.equal(outs[0][1]["counts"], outs[1][1]["counts"])
    assert torch.equal(outs[0][1]["records"], outs[4][1]["records"])
    # without records the record pointer of the nodes is null: still the same graph
    o = plan.run(seed=4, records=False)
    torch.cuda.synchronize()
    assert plan.graph_info()[0] == 1
    assert torch.equal(o["counts"], outs[1][1]["counts"])
    # arrival tallies run other kernel instances: a graph of their own
    o = plan.run(seed=4, arrivals=True)
    torch.cuda.synchronize()
    assert plan.graph_info()[0] == 2
    assert torch.equal(o["counts"], outs[1][1]["counts"])


def test_runs_on_two_streams_are_ordered():
    """Runs of one plan on two streams, enqueued back to back without host synchronisation,
    share the plan's queue and counters; the library orders them, so each equals the run on
    its own."""
    cfgs = [si.single_ni(2.0, 6000), si.single_ni(0.5, 20000)]
    say("two streams, one plan")
    plan = spx.Plan(cfgs, PARAMS)
    ref = {s: plan.run(seed=s) for s in (1, 2)}
    torch.cuda.synchronize()
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ba, bb = plan.allocate(), plan.allocate()
    for _ in range(3):
        plan.run_into(1, ba, stream=sa)
        plan.run_into(2, bb, stream=sb)
    torch.cuda.synchronize()
    assert torch.equal(ba["counts"], ref[1]["counts"]) and torch.equal(ba["counters"], ref[1]["counters"].view(-1))
    assert torch.equal(bb["counts"], ref[2]["counts"]) and torch.equal(bb["counters"], ref[2]["counters"].view(-1))


def test_tested_step_counter():
    """The work counter of diffusive steps tested against the surfaces: every step on the plain
    FP64 path (steps ended in the gas plus the last one of each thermalised atom), and on the
    batched path only those that left their clearance balls, the first step of each walk
    among them."""
    cfgs = [si.single_ni(2.0, 3000), si.quaternary(0.5, 25.0, 150.0, [3000, 800, 2000, 1200])]
    say("tested-step counter")
    C = {}
    for prec in (32, 64):
        C[prec] = spx.Plan(cfgs, PARAMS, precision=prec).run(seed=17)["counters"].cpu().numpy()
    torch.cuda.synchronize()
    c64, c32 = C[64], C[32]
    assert np.all(c64[:, 3] == 0)
    assert np.array_equal(c64[:, 7], c64[:, 5] + c64[:, 6])
    assert np.all(c32[:, 7] >= c32[:, 6]) and np.all(c32[:, 7] <= c32[:, 5] + c32[:, 6])
    frac = c32[:, 7].sum() / (c32[:, 5] + c32[:, 6]).sum()
    say(f"  batched walk tests {frac:.3%} of its diffusive steps")
    assert 0 < frac < 0.2
