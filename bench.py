#!/usr/bin/env python3
"""Benchmark: batched FP32 transport vs the plain FP64 per-segment comparator.

Workload (default): the single planar Ni target of the paper's Methods geometry
stand-in, three chambers in one batch -- Ar at 0.5 Pa, 0 Pa (line of sight) and
2 Pa (thermalisation dominated) -- 1e7 particles each (3e7 per step), FP32
transport with integer tallies.  A step is one replay of the plan's HIP graph:
zero tallies, the persistent transport kernel over all three chambers, and the
FP64 normalisation of the tallies to deposition profiles.  Inputs are synthetic
(seeded geometry and gas; every random number is generated on the GPU).

Prints ONE JSON line.  `value` is particles/s of the FP32 path; the FP64 plain
comparator, collisions/s, the matched tally error, the ALU roofline of the
transport kernel and the FP64 CPU oracle timed on this host are reported beside it.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particles/sec (and collisions/sec) at matched tally error, FP32 batched vs FP64 plain"

# VALU issue slots per lane of each unit of work, counted from the formulas the kernel
# evaluates: a 32x32->64 multiply and a native transcendental take 4 slots, any other FP32 or
# 32-bit integer operation 1.  Philox4x32-10 block: 10 rounds x (2 multiplies + 2 three-input
# XORs) = 100 (the key schedule is wave-uniform, scalar); a uniform from a word: 3.
PHILOX, U01 = 100, 3
SURFACE_TEST = 100        # substrate plate, target disc, chamber side and caps (planes: reciprocal 4)
OPS = dict(
    # 2 blocks, 5 uniforms; truncated-normal inverse CDF, Thompson energy, cosine direction, frame
    LAUNCH=2 * PHILOX + 5 * U01 + 95,
    # block, 3 uniforms, lambda_m (table + Maxwellian mean speed) 60, free path 6, surface test,
    # compensated move 15, event bookkeeping 2
    BALLISTIC=PHILOX + 3 * U01 + 60 + 6 + SURFACE_TEST + 15 + 2,
    # gas-velocity block and 4 uniforms, Box-Muller 40, kinematics with the table lookup 130
    COLLIDE=PHILOX + 4 * U01 + 40 + 130,
    # every diffusive step: half a block (two steps per block), 21-bit codes 5 and their 3 RN 6,
    # isotropic direction and exponential length 20 (sqrt, sin, cos, log2 16; 1 - mu^2, two
    # products, the length scale 4), the step added to the offset from the ball centre 3 (fused
    # multiply-adds), clearance-ball test 4, bookkeeping 2
    DIFFUSIVE=PHILOX // 2 + 5 + 6 + 20 + 3 + 4 + 2,
    # a diffusive step that leaves its clearance ball (counted by the kernels): exact
    # renormalisation of the position 18, the surface test, the compensated move 15, the new
    # clearance (point-to-region distances of plate, target and chamber, 3 square roots) 45
    TESTED=18 + SURFACE_TEST + 15 + 45,
)
# per absorbing object of the segment: its part of the surface test (planar: plane crossing
# with a reciprocal and the in-shape test; tube: the quadratic with a square root and a
# reciprocal, both roots' axial tests) and of the clearance (point-to-region distance)
OBJ_TEST = {"disc": 30, "rect": 30, "tube": 50}
OBJ_CLEAR = {"disc": 25, "rect": 22, "tube": 23}
# Peak: the FP32 vector rate of the MI355X, 157.3 TFLOP/s = 78.6e12 FMA/s, i.e. 128 lanes per
# CU per clock (256 CUs, 2.4 GHz); one slot = one full-rate 32-bit lane operation.
PEAK_ALU = 256 * 128 * 2.4e9
QUEUE_RECORD_BYTES = 48   # one thermalised atom handed from the ballistic to the diffusive phase


def segment_objects(cfgs):
    """Absorbing objects of each (config, cathode) run, by kind: the configuration's own plus,
    with cross_absorb, the other targets (discs)."""
    out = []
    for cfg in cfgs:
        own = [a.kind for a in getattr(cfg, "absorbers", []) or []]
        for _ in cfg.cathodes:
            out.append(own + (["disc"] * (len(cfg.cathodes) - 1) if getattr(cfg, "cross_absorb", False) else []))
    return out


def algorithmic_ops(counters, cfgs):
    """ALU slots of one run from its counters [n_seg, 8]: (ballistic phase, diffusive phase)."""
    ops_b = ops_d = 0.0
    for k, objs in enumerate(segment_objects(cfgs)):
        N, coll, diff, therm, tested = (float(counters[k, i]) for i in (0, 4, 5, 6, 7))
        ballistic_flights = coll + (N - therm)   # every collision, plus the last flight of atoms never thermalised
        diffusive_steps = diff + therm           # every diffusive step, plus the last step of thermalised atoms
        o_test = sum(OBJ_TEST[o] for o in objs)
        o_clear = sum(OBJ_CLEAR[o] for o in objs)
        ops_b += N * OPS["LAUNCH"] + ballistic_flights * (OPS["BALLISTIC"] + o_test) + coll * OPS["COLLIDE"]
        ops_d += diffusive_steps * OPS["DIFFUSIVE"] + tested * (OPS["TESTED"] + o_test + o_clear)
    return ops_b, ops_d


# the sources the two transport kernels are compiled from (their device code, launch
# arguments and queue record layout)
TRANSPORT_SOURCES = ("spx_device.hpp", "spx_host.hpp", "transport.hip")


def kernel_source_hash():
    """Digest of the transport kernels' sources: HBM traffic taken with rocprofv3 counters is
    reported only for the kernels it was measured on."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2411_14413_amd", "csrc")
    for name in TRANSPORT_SOURCES:
        h.update(name.encode())
        h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed rocprofv3 counters
    (profiles/hbm_traffic.json), or None when they were taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    table = json.load(open(path))
    e = table.get(workload, {}).get(kernel)
    if not e or e.get("sources") != kernel_source_hash():
        return None
    return e["bytes_per_launch"]


TILT_SWEEP = [11.0, 11.5, 12.0, 12.5, 13.0, 13.5, 14.0, 14.5]
TILT_PLANTED = 12.7


def workload(name, scale=1.0):
    import sputter_inputs as si
    if name == "legs":
        n = int(1e7 * scale)
        return (si.single_ni_legs(n),
                f"single Ni target (50.8 mm), Ar 0.5 / 0 / 2 Pa, 300 K, 100x100 mm substrate at 100 mm, "
                f"50x50 bins, 3 chambers x {n:.0e} particles in one launch")
    if name == "legs_measured":
        n = int(1e7 * scale)
        prof = si.measured_racetrack(seed=0)
        return ([si.with_launch(c, prof, si.UNDER_COSINE) for c in si.single_ni_legs(n)],
                f"single Ni target (50.8 mm) with a measured racetrack profile and an under-cosine "
                f"six-coefficient emission law, Ar 0.5 / 0 / 2 Pa, 300 K, 100x100 mm substrate at 100 mm, "
                f"50x50 bins, 3 chambers x {n:.0e} particles in one launch")
    if name == "quaternary":
        cfg = si.quaternary()
        return [cfg], "four confocal cathodes Ni/Pd/Pt/Ru, tilt 25 deg, 150 mm, Ar 0.5 Pa, 100 mm wafer 200x200 bins, 2.3e7 particles"
    if name == "quaternary_chimneys":
        cfg = si.with_chimneys(si.quaternary())
        return [cfg], ("four confocal cathodes Ni/Pd/Pt/Ru, tilt 25 deg, 150 mm, Ar 0.5 Pa, 100 mm wafer 200x200 bins, "
                       "2.3e7 particles; each target in a 30 mm open chimney (radius + 5 mm), the other targets absorb")
    if name == "tilt_fit":
        n = int(1e8 * scale)
        return (si.tilt_sweep(TILT_SWEEP, n_particles=n),
                f"tilt inversion of a ternary Pd-Pt-Ru library: {len(TILT_SWEEP)} common cathode tilts "
                f"{TILT_SWEEP[0]}-{TILT_SWEEP[-1]} deg x 3 confocal cathodes (200 mm) x {n:.0e} particles at "
                f"Ar 0.5 Pa in one launch, then 342 areas, at.%, d_e^2 and covered area against a library "
                f"simulated at {TILT_PLANTED} deg, and both fits")
    if name == "sweep":
        cfgs = si.quaternary_sweep(64, scale=scale)
        return cfgs, "64 four-cathode chambers: p U(0.1,2) Pa, tilt U(0,40) deg, distance U(80,200) mm, 1e5-1e7 particles each"
    raise SystemExit(f"unknown workload {name}")


def tally_error(counts_seg):
    import numpy as np
    vals = []
    for c in counts_seg:
        c = c[c > 0]
        if c.size:
            vals.append(float(np.median(1.0 / np.sqrt(c))))
    return vals


def time_steps(plan, bufs, seed, steps, warmup, phase_times=True, post=None):
    import torch
    for _ in range(warmup):
        plan.run_into(seed, bufs)
        if post is not None:
            post(bufs)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
    phases = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for a, b in ev:
        a.record(stream)
        plan.run_into(seed, bufs)
        if post is not None:
            post(bufs)
        b.record(stream)
        # per-kernel device times of this step, from the HIP events the plan records between
        # its kernels on this stream (waits for the step: a few microseconds per step)
        if phase_times:
            phases.append(plan.phase_times())
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = [a.elapsed_time(b) for a, b in ev]
    return wall, ms, phases


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfgs, params, seed, target_s, one_thread_s):
    """The FP64 oracle on this host with the benchmark's seed: the first n particles of every
    (config, cathode) on all threads (n sized by a pilot to ~target_s), and a smaller sample on
    one thread.  Returns the report and the all-threads run's records (for the accuracy of the
    GPU run, which must use the same seed)."""
    import oracle
    oracle.table(params)                      # table build is set-up, not timed
    n0 = 500
    t = time.perf_counter()
    oracle.run(cfgs, params, seed=seed, pid_begin=0, pid_end=n0)
    t0 = time.perf_counter() - t
    n = int(min(max(n0, n0 * target_s / max(t0, 1e-3)), 10_000_000))
    t = time.perf_counter()
    r = oracle.run(cfgs, params, seed=seed, pid_begin=0, pid_end=n, records=True)
    dt = time.perf_counter() - t
    launched = int(r["counters"][:, 0].sum())
    rate = launched / dt
    # one thread: a sample of ~one_thread_s from the all-threads rate
    n1 = int(max(50, n * one_thread_s / max(dt * r["threads"], 1e-3)))
    t = time.perf_counter()
    r1 = oracle.run(cfgs, params, seed=seed, pid_begin=0, pid_end=n1, n_threads=1)
    dt1 = time.perf_counter() - t
    l1 = int(r1["counters"][:, 0].sum())
    rep = dict(value=rate, unit="particles/s", cores=int(r["threads"]), kind="oracle",
               sample=f"first {n} particles of each of the {len(r['counters'])} chambers/cathodes "
                      f"({launched} particles, same mix as the workload), {dt:.1f} s, FP64 C, OpenMP",
               single_thread={"value": l1 / dt1, "unit": "particles/s", "cores": int(r1["threads"]),
                              "sample": f"first {n1} particles of each chamber/cathode ({l1} particles), {dt1:.1f} s"},
               cpu_model=cpu_model(), host_cpus=os.cpu_count())
    return rep, r, n


def accuracy(plan, cfgs, seed, ref, n_first, bufs_kw):
    """Error of the benchmarked FP32 run against the FP64 oracle on the particles the oracle
    leg simulated (the first n_first of every segment; same Philox streams): one more run of
    the same plan with records, untimed."""
    import numpy as np
    import torch
    import paper_2411_14413_amd as spx
    bufs = plan.allocate(records=True, **bufs_kw)
    plan.run_into(seed, bufs)
    torch.cuda.synchronize()
    rec_all = bufs["records"].view(-1, 56)
    idx = np.concatenate([np.arange(f, f + min(n_first, N)) for f, N in zip(plan.first, plan.seg_particles)])
    rec = spx.records_to_numpy(rec_all[torch.as_tensor(idx, device="cuda")].reshape(-1).cpu())
    o_rec = ref["records"]                   # x, y, z, state, bin, events, diffusive, E
    d = np.linalg.norm(np.stack([rec["x"], rec["y"], rec["z"]], axis=1) - o_rec[:, :3], axis=1)
    same = rec["state"].astype(np.int64) == o_rec[:, 3].astype(np.int64)
    close = same & (d < 1e-3)
    dep = close & (rec["state"] == 1)
    m = {"same_state": float(same.mean()), "frac": float(close.mean()), "d_median": float(np.median(d)),
         "bin_frac": float((rec["bin"][dep].astype(np.int64) == o_rec[dep, 4].astype(np.int64)).mean())
         if dep.any() else 1.0}
    # tallies of the same particles, GPU records binned vs the oracle's counts: |z| per bin
    zmax, chi2, dof = 0.0, 0.0, 0
    off = 0
    for k, ((nv, nu), N) in enumerate(zip(plan.shapes, plan.seg_particles)):
        n = min(n_first, N)
        r = rec[off:off + n]
        off += n
        g = np.bincount(r["bin"][r["state"] == 1].astype(np.int64), minlength=nv * nu).astype(np.float64)
        o = ref["counts"][k].reshape(-1).astype(np.float64)
        z = (g - o) / np.sqrt(np.maximum(g + o, 1.0))
        zmax = max(zmax, float(np.abs(z).max()))
        chi2 += float((z ** 2).sum())
        dof += int(((g + o) > 0).sum())
    del bufs
    return {"particles": int(len(rec)), "same_state": m["same_state"], "within_1e-3_mm": m["frac"],
            "median_distance_mm": m["d_median"], "deposits_same_bin": m["bin_frac"],
            "tally_max_abs_z": zmax, "tally_chi2_per_bin": chi2 / max(dof, 1),
            "note": "GPU records of the benchmarked FP32 run (same seed and plan, one more untimed run) against "
                    "the FP64 oracle's records of the same particles (the cpu_baseline sample); z = per-bin "
                    "tally difference of those particles over sqrt(sum)"}


def run_workload(name, args, params, n_steps, n_warmup, with_phases=True):
    """Plan, autotune and time one workload; returns (plan, cfgs, bufs, report)."""
    import numpy as np
    import paper_2411_14413_amd as spx
    cfgs, desc = workload(name)
    t = time.perf_counter()
    plan = spx.Plan(cfgs, params, precision=32)
    setup_s = time.perf_counter() - t
    t = time.perf_counter()
    if args.launch and name == args.workload:
        launch = plan.set_launch(*(int(x) for x in args.launch.split(",")))
    else:
        launch = plan.launch if args.no_autotune else plan.autotune()
    tune_s = time.perf_counter() - t
    bufs = plan.allocate(profiles=True, arrivals=args.arrivals and name == args.workload)
    wall, ms, phases = time_steps(plan, bufs, args.seed, n_steps, n_warmup, phase_times=with_phases)
    counters = bufs["counters"].view(plan.n_segments, spx._native.N_COUNTERS).cpu().numpy().astype(np.float64)
    n_part = float(counters[:, 0].sum())
    assert n_part == plan.n_particles
    assert np.array_equal(counters[:, 0], counters[:, 1] + counters[:, 2] + counters[:, 3])
    ms_step = wall * 1e3 / n_steps
    ops_b, ops_d = algorithmic_ops(counters, cfgs)
    ms_b = float(np.mean([p[0] for p in phases]))
    ms_d = float(np.mean([p[1] for p in phases]))
    kern = {"k_ballistic32": (ops_b, ms_b), "k_diffusive32": (ops_d, ms_d)}
    coll, diff, therm, tested = (float(counters[:, i].sum()) for i in (4, 5, 6, 7))
    rep = {"workload": desc, "particles_per_step": int(n_part), "segments": plan.n_segments, "launch": launch,
           "ms_per_step": ms_step, "particles_per_s": n_part / (ms_step * 1e-3),
           "collisions_per_s": (coll + diff) / (ms_step * 1e-3),
           "ballistic_collisions_per_s": coll / (ms_step * 1e-3), "diffusive_steps_per_s": diff / (ms_step * 1e-3),
           "tested_step_fraction": tested / max(diff + therm, 1.0),
           # each thermalised atom is one 48-byte queue record, written by the ballistic kernel
           # and read by the diffusive one: the bulk of either kernel's algorithmic HBM bytes
           "thermalized_per_step": int(therm), "queue_bytes_per_launch": int(QUEUE_RECORD_BYTES * therm),
           "step_ms_events": {"median": float(np.median(ms)), "min": float(min(ms)), "max": float(max(ms))},
           "setup_s": {"plan_and_table": setup_s, "autotune": tune_s},
           "kernels": {k: {"ops": o, "ms": t, "achieved_TOPs": o / (t * 1e-3) / 1e12 if t > 0 else None,
                           "frac": o / (t * 1e-3) / PEAK_ALU if t > 0 else None,
                           "traffic": None if args.arrivals else measured_traffic(k, name)}
                       for k, (o, t) in kern.items()}}
    return plan, cfgs, bufs, counters, kern, rep


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="legs", choices=["legs", "legs_measured", "quaternary", "quaternary_chimneys", "sweep", "tilt_fit"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparator leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg (and the accuracy check)")
    ap.add_argument("--no-workloads", action="store_true",
                    help="skip timing the four-cathode and 64-chamber workloads beside the default one")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=20.0,
                    help="target of the CPU pilot-based sizing (the measured run usually takes about half)")
    ap.add_argument("--cpu-one-thread-seconds", type=float, default=8.0)
    ap.add_argument("--launch", default="", help="blocks,threads,refill_min,refill_ballistic[,defer_min] instead of autotuning")
    ap.add_argument("--arrivals", action="store_true",
                    help="also tally arrival energy and angle histograms and per-bin energy sums")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device copy of this size first (HBM counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the tally reduce across GPUs "
              "is designed but not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2411_14413_amd as spx
    import sputter_inputs as si

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    params = si.Params()
    if args.workload == "tilt_fit":
        return tilt_fit_main(args, params)
    plan, cfgs, bufs, counters, kern, rep = run_workload(args.workload, args, params, args.steps, args.warmup)
    ms_step = rep["ms_per_step"]
    value = rep["particles_per_s"]
    counts32 = [bufs["counts"][o:o + nv * nu].cpu().numpy() for o, (nv, nu) in zip(plan.bin_off, plan.shapes)]
    eps32 = tally_error(counts32)
    dominant = max(kern, key=lambda k: kern[k][1])
    ops, ms_k = kern[dominant]
    achieved = ops / (ms_k * 1e-3)
    roofline = dict(bound="alu", kernel=dominant, achieved=achieved / 1e12, peak=PEAK_ALU / 1e12,
                    unit="TOP/s", frac=achieved / PEAK_ALU,
                    traffic=None if args.arrivals else measured_traffic(dominant, args.workload),
                    ops_per_launch=ops, launch_ms=ms_k,
                    phases={k: dict(ops=o, ms=t, achieved=o / (t * 1e-3) / 1e12 if t > 0 else None,
                                    frac=o / (t * 1e-3) / PEAK_ALU if t > 0 else None,
                                    traffic=None if args.arrivals else measured_traffic(k, args.workload))
                            for k, (o, t) in kern.items()},
                    note="VALU issue slots per lane counted from the algorithm (a 32x32->64 multiply or a native "
                         "transcendental = 4 slots; surface tests and absorbing objects charged to the flights and "
                         "to the diffusive steps the kernels report as tested); peak = 256 CU x 128 lanes x 2.4 GHz "
                         "(the FP32 vector rate); kernel time = mean over the timed steps of HIP events recorded "
                         "between the kernels; traffic = rocprofv3 HBM bytes per launch when taken on these sources, "
                         "against queue_bytes_per_launch, the algorithmic bytes of either phase")

    result = {
        "metric": METRIC, "value": value, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": rep["workload"], "particles_per_step": rep["particles_per_step"],
                   "segments": plan.n_segments, "launch": rep["launch"], "seed": args.seed,
                   "arrival_tallies": bool(args.arrivals)},
        "collisions_per_s": rep["collisions_per_s"],
        "ballistic_collisions_per_s": rep["ballistic_collisions_per_s"],
        "diffusive_steps_per_s": rep["diffusive_steps_per_s"],
        "tested_step_fraction": rep["tested_step_fraction"],
        "thermalized_per_step": rep["thermalized_per_step"],
        "queue_bytes_per_launch": rep["queue_bytes_per_launch"],
        "step_ms_events": rep["step_ms_events"],
        "setup_s": rep["setup_s"],
        "roofline": roofline,
    }

    if not args.no_fp64:
        plan64 = spx.Plan(cfgs, params, precision=64)
        bufs64 = plan64.allocate(profiles=True)
        wall64, ms64, _ = time_steps(plan64, bufs64, args.seed, 2, 1, phase_times=False)
        c64 = bufs64["counters"].view(plan.n_segments, spx._native.N_COUNTERS).cpu().numpy().astype(np.float64)
        counts64 = [bufs64["counts"][o:o + nv * nu].cpu().numpy() for o, (nv, nu) in zip(plan64.bin_off, plan64.shapes)]
        eps64 = tally_error(counts64)
        v64 = float(c64[:, 0].sum()) / (wall64 / 2)
        result["fp64_plain"] = {"value": v64, "unit": "particles/s", "ms_per_step": wall64 * 1e3 / 2,
                                "collisions_per_s": float(c64[:, 4].sum() + c64[:, 5].sum()) / (wall64 / 2)}
        result["speedup_vs_fp64_plain"] = value / v64
        result["tally_error"] = {"fp32_batched": eps32, "fp64_plain": eps64,
                                 "max_rel_diff": max(abs(a / b - 1) for a, b in zip(eps32, eps64)),
                                 "definition": "median over non-empty bins of 1/sqrt(count), per chamber/cathode"}
        del plan64, bufs64
    else:
        result["tally_error"] = {"fp32_batched": eps32}

    if not args.no_cpu:
        cfgs_cpu, _ = workload(args.workload)
        cb, ref, n_first = cpu_baseline(cfgs_cpu, params, args.seed, args.cpu_seconds, args.cpu_one_thread_seconds)
        result["cpu_baseline"] = cb
        result["accuracy"] = accuracy(plan, cfgs, args.seed, ref, n_first,
                                      dict(profiles=False, arrivals=bool(args.arrivals)))
    del bufs
    if not args.no_workloads and args.workload == "legs":
        # the paper's four-cathode condition and the 64-chamber sweep, timed in the same run
        ws = {}
        for name in ("quaternary", "sweep"):
            p2, _, b2, _, _, r2 = run_workload(name, args, params, 3, 1)
            r2["roofline_frac"] = {k: v["frac"] for k, v in r2["kernels"].items()}
            ws[name] = r2
            del p2, b2
            torch.cuda.empty_cache()
        result["workloads"] = ws
    result["paper_context"] = ("pySIMTRA/SIMTRA: ~20 min per 4-cathode library of ~1e8 particles per cathode on an "
                               "AMD Ryzen 7 5800X (8 cores, 3.8 GHz), i.e. ~3.3e5 particles/s aggregate")
    print(json.dumps(result), flush=True)


def tilt_fit_main(args, params):
    """The tilt-inversion workload: the timed step is the sweep's transport plus the inversion."""
    import numpy as np
    import torch
    import paper_2411_14413_amd as spx
    import sputter_inputs as si
    cfgs, desc = workload("tilt_fit")
    plan = spx.Plan(cfgs, params, precision=32)
    launch = plan.autotune() if not args.no_autotune else plan.launch
    bufs = plan.allocate(profiles=True)
    # the measured library: the same ternary system simulated at the planted tilt with other
    # random numbers (set-up, not timed)
    n = cfgs[0].cathodes[0].n_particles
    mplan = spx.Plan(si.tilt_sweep([TILT_PLANTED], n_particles=n), params)
    mout = mplan.run(seed=args.seed + 1000)
    cen = torch.as_tensor(spx.area_centres(), device="cuda")
    comp = [torch.as_tensor(v, device="cuda") for v in si.ternary_composition_inputs()]
    f_m = spx.area_gather(torch.stack(mout["profiles_seg"]), cfgs[0].grid, cen).view(1, 3, -1)
    c_m = spx.sweep_composition(f_m, *comp)[0]
    del mplan, mout
    inversion = {}
    post = lambda b: inversion.update(spx.invert_sweep(plan, b, TILT_SWEEP, comp, c_m, centres=cen))
    wall, ms, phases = time_steps(plan, bufs, args.seed, args.steps, args.warmup, post=post)
    counters = bufs["counters"].view(plan.n_segments, spx._native.N_COUNTERS).cpu().numpy().astype(np.float64)
    n_part = float(counters[:, 0].sum())
    ms_step = wall * 1e3 / args.steps
    ops_b, ops_d = algorithmic_ops(counters, cfgs)
    ms_b = float(np.mean([p[0] for p in phases]))
    ms_d = float(np.mean([p[1] for p in phases]))
    kern = {"k_ballistic32": (ops_b, ms_b), "k_diffusive32": (ops_d, ms_d)}
    dominant = max(kern, key=lambda k: kern[k][1])
    ops, ms_k = kern[dominant]
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(10):
        post(bufs)
    ev[1].record()
    torch.cuda.synchronize()
    result = {
        "metric": METRIC, "value": n_part / (ms_step * 1e-3), "unit": "particles/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "particles_per_step": int(n_part), "segments": plan.n_segments,
                   "launch": launch, "seed": args.seed},
        "roofline": dict(bound="alu", kernel=dominant, achieved=ops / (ms_k * 1e-3) / 1e12, peak=PEAK_ALU / 1e12,
                         unit="TOP/s", frac=ops / (ms_k * 1e-3) / PEAK_ALU, traffic=None,
                         phases={k: dict(ms=t, frac=o / (t * 1e-3) / PEAK_ALU) for k, (o, t) in kern.items()}),
        "inversion": {
            "tilts_deg": TILT_SWEEP, "planted_deg": TILT_PLANTED,
            "fit_d_e_deg": float(inversion["x_min_de"].cpu()[0]),
            "fit_covered_area_deg": float(inversion["x_match_area"].cpu()[0]),
            "covered_area": [round(float(v), 6) for v in inversion["area"].cpu()],
            "covered_area_measured": float(inversion["area_measured"].cpu()[0]),
            "d_e2": [round(float(v), 3) for v in inversion["loss"].cpu()],
            "chain_ms": ev[0].elapsed_time(ev[1]) / 10,
            "note": "chain = area gather, sweep compositions, d_e^2, covered areas and both fits, after the "
                    "transport (inside the timed step)"},
    }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
