"""Full-size runs in the benchmark's launch configuration (autotuned), checked where
the oracle can follow: sampled particles one by one, exact integer identities at
every size, the analytic 0 Pa profile, and compositions against the oracle run on
the same particles.

* three 1e7-particle chambers of the single-target geometry (0.5 / 0 / 2 Pa);
* the four-cathode Ni/Pd/Pt/Ru system, 2.3e7 particles, 200x200 wafer grid;
* the 64-chamber sweep of that system (~1.4e8 particles) in one launch;
* that system with 2.7e8 particles, more than one round of the batched path holds (2^28
  tickets), so the particles run in two rounds.
"""
import math

import numpy as np
import pytest

import oracle
import sputter_inputs as si
from parity import match_stats, say

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_2411_14413_amd as spx  # noqa: E402

PARAMS = si.Params()


def _run_full(cfgs, seed):
    plan = spx.Plan(cfgs, PARAMS)
    launch = plan.autotune()
    say(f"  launch {launch}, {plan.n_particles} particles, {plan.n_segments} segments")
    out = plan.run(seed=seed, records=True)
    torch.cuda.synchronize()
    return plan, out


def _check_integer_identities(plan, out):
    """Tallies = histogram of the records (on the GPU), counters = record sums, conservation."""
    rec32 = out["records"].view(torch.int32).view(-1, 14)
    st, bn, dif = rec32[:, 8], rec32[:, 9], rec32[:, 11]
    C = out["counters"].cpu().numpy()
    first = list(plan.first) + [plan.n_particles]
    for k in range(plan.n_segments):
        a, b = first[k], first[k + 1]
        s = st[a:b]
        dep = s == 1
        nb = plan.shapes[k][0] * plan.shapes[k][1]
        h = torch.bincount(bn[a:b][dep].long(), minlength=nb)
        assert torch.equal(h, out["counts_seg"][k].reshape(-1)), k
        assert C[k, 0] == b - a == plan.seg_particles[k]
        assert C[k, 1] == int(dep.sum()) and C[k, 2] == int((s == 2).sum()) and C[k, 3] == int((s == 3).sum())
        assert C[k, 5] == int(dif[a:b].to(torch.int64).sum())
    assert np.array_equal(C[:, 0], C[:, 1] + C[:, 2] + C[:, 3])


def _sampled_parity(plan, out, cfgs, seed, per_seg, rng):
    """per_seg: particles sampled per segment (an int, or a list with one count per segment)."""
    first = list(plan.first)
    seg_ids, pids = [], []
    for k, N in enumerate(plan.seg_particles):
        if N == 0:
            continue
        want = per_seg[k] if isinstance(per_seg, (list, tuple)) else per_seg
        p = rng.choice(N, size=min(want, N), replace=False)
        seg_ids += [k] * len(p)
        pids += list(p)
    seg_ids, pids = np.array(seg_ids), np.array(pids)
    ref = oracle.run_list(cfgs, PARAMS, seed, seg_ids, pids)
    idx = torch.as_tensor(np.array(first)[seg_ids] + pids, device="cuda")
    rec = spx.records_to_numpy(out["records"].view(-1, 56)[idx].reshape(-1))
    m = match_stats(rec, ref, 1e-3)
    per = []
    for k in np.unique(seg_ids):
        sel = seg_ids == k
        per.append(match_stats(rec[sel], ref[sel], 1e-3)["frac"])
    return m, np.array(per)


def test_fullsize_single_target_legs():
    say("full size: 3 x 1e7, single target, 0.5 / 0 / 2 Pa")
    cfgs = si.single_ni_legs(10_000_000)
    plan, out = _run_full(cfgs, seed=0)
    _check_integer_identities(plan, out)
    m, per = _sampled_parity(plan, out, cfgs, 0, 300, np.random.default_rng(0))
    say(f"  sampled parity {m}, per leg {per}")
    assert m["frac"] >= 0.99 and per.min() >= 0.97
    # the 0 Pa leg against the analytic line-of-sight profile
    from test_oracle_transport import analytic_bin_fractions
    counts = out["counts_seg"][1].cpu().numpy().astype(np.float64)
    exp = 1e7 * analytic_bin_fractions(cfgs[1])
    z = (counts - exp) / np.sqrt(exp)
    assert (z**2).sum() < z.size + 4.5 * math.sqrt(2 * z.size) and np.abs(z).max() < 5.0


def test_fullsize_quaternary_compositions():
    say("full size: four cathodes, 2.3e7 particles; compositions vs the oracle on the same particles")
    cfg = si.quaternary()
    plan, out = _run_full([cfg], seed=1)
    _check_integer_identities(plan, out)
    m, per = _sampled_parity(plan, out, [cfg], 1, 400, np.random.default_rng(1))
    say(f"  sampled parity {m}, per cathode {per}")
    assert m["frac"] >= 0.99 and per.min() >= 0.97
    # GPU chain: profiles -> 342 areas -> at.% for 16 power vectors
    g = cfg.grid
    cen = spx.area_centres(342, 4.5)
    prof = torch.stack([p for p in out["profiles_seg"]])
    f_gpu = spx.area_gather(prof, g, cen)                           # [4, 342] float64
    ci = si.composition_inputs(batch=16)
    fref = f_gpu.mean(dim=1)
    c_gpu = spx.comp_forward(f_gpu, *[torch.as_tensor(x, device="cuda") for x in (ci.a, ci.b, ci.P, ci.M, ci.rho)],
                             fref).cpu().numpy()
    # oracle chain on the same particles
    say("  oracle: 2.3e7 particles")
    r = oracle.run([cfg], PARAMS, seed=1)
    f_or = np.stack([oracle.area_gather(oracle.normalize(r["counts"][k], cfg.cathodes[k].n_particles, g), g,
                                        oracle.area_centres()) for k in range(4)])
    c_or = oracle.composition(f_or, ci.a, ci.b, ci.P, ci.M, ci.rho, f_or.mean(axis=1))
    err = np.abs(c_gpu - c_or).max()
    say(f"  composition max |diff| = {err:.4f} at.%")
    assert err < 0.1
    # tallies within counting noise of the oracle's
    for k in range(4):
        a = out["counts_seg"][k].cpu().numpy().astype(np.float64)
        b = r["counts"][k].astype(np.float64)
        z = (a - b) / np.sqrt(np.maximum(a + b, 1.0))
        assert np.abs(z).max() < 3.0
    # the hand-written backward at the fit's full size: 1024 power vectors x 342 areas x 4
    # cathodes on these area profiles, target = the composition at the first power vector,
    # against float64 torch autograd (the oracle) on the same float32-rounded inputs
    ci = si.composition_inputs(batch=1024)
    f32 = f_gpu.float()
    fr32 = f32.mean(dim=1)
    ins = [f32.double().cpu().numpy(), ci.a, ci.b, ci.P, ci.M, ci.rho, fr32.double().cpu().numpy()]
    ins = [np.asarray(x, dtype=np.float32).astype(np.float64) for x in ins]
    c_t = oracle.composition(*ins[:3], ins[3][:1], *ins[4:])[0]
    ref = oracle.composition_grads(*ins, c_t[None])
    dev = [torch.as_tensor(x, dtype=torch.float32, device="cuda").contiguous().requires_grad_(True) for x in ins]
    c = spx.CompositionMap.apply(*dev)
    loss = spx.SquaredDistance.apply(c, torch.as_tensor(c_t, dtype=torch.float32, device="cuda")).sum()
    loss.backward()
    torch.cuda.synchronize()
    say(f"  backward at B=1024, J=342, K=4: loss {float(loss.detach()):.6g} (oracle {ref['loss']:.6g})")
    assert abs(float(loss.detach()) / ref["loss"] - 1) < 1e-4
    for name, t in zip(("f", "a", "b", "P", "M", "rho", "fref"), dev):
        gr = t.grad.cpu().numpy().astype(np.float64)
        err = np.abs(gr - ref[name]).max() / np.abs(ref[name]).max()
        say(f"    grad {name}: rel err {err:.2e}")
        assert err < 2e-4, (name, err)


def test_fullsize_sweep():
    cfgs = si.quaternary_sweep(64)
    say(f"full size: 64-chamber sweep, {si.total_particles(cfgs)} particles in one launch")
    plan, out = _run_full(cfgs, seed=2)
    _check_integer_identities(plan, out)
    # 200 particles of every segment, 400 of those at 1 Pa and above, where the walks are
    # longest and the FP32 drift largest
    press = [cfg.chamber.pressure for cfg in cfgs for _ in cfg.cathodes]
    per_seg = [400 if p >= 1.0 else 200 for p in press]
    m, per = _sampled_parity(plan, out, cfgs, 2, per_seg, np.random.default_rng(2))
    hi = np.array([p >= 1.0 for p, N in zip(press, plan.seg_particles) if N > 0])
    say(f"  sampled parity {m}, worst segment {per.min()}, worst at >= 1 Pa {per[hi].min()}")
    assert m["frac"] >= 0.99 and per.min() >= 0.97


def test_fullsize_two_rounds():
    n = (1 << 28) + (1 << 22)
    counts = [n * 5 // 23, n * 2 // 23, n * 7 // 23]
    counts.append(n - sum(counts))
    cfgs = [si.quaternary(counts=counts)]
    say(f"full size: four cathodes, {n} particles (two rounds)")
    plan, out = _run_full(cfgs, seed=4)
    _check_integer_identities(plan, out)
    m, per = _sampled_parity(plan, out, cfgs, 4, 400, np.random.default_rng(4))
    say(f"  sampled parity {m}, per cathode {per}")
    assert m["frac"] >= 0.99 and per.min() >= 0.98
