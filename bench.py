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
OPS = dict(
    # 2 blocks, 5 uniforms; truncated-normal inverse CDF, Thompson energy, cosine direction, frame
    LAUNCH=2 * PHILOX + 5 * U01 + 95,
    # block, 3 uniforms, lambda_m (table + Maxwellian mean speed) 60, free path 6, surface test
    # 100, compensated move 15, event bookkeeping 2
    BALLISTIC=PHILOX + 3 * U01 + 60 + 6 + 100 + 15 + 2,
    # gas-velocity block and 4 uniforms, Box-Muller 40, kinematics with the table lookup 130
    COLLIDE=PHILOX + 4 * U01 + 40 + 130,
    # half a block (two steps per block), 21-bit codes 5 and their 3 RN 6, isotropic direction
    # and exponential length 20 (sqrt, sin, cos, log2 16; 1 - mu^2, two products, the length
    # scale 4), the step added to the offset from the ball centre 3 (fused multiply-adds),
    # clearance-ball test 4, bookkeeping 2, plus 2 for the ~1.3 % of steps that leave the ball
    # and take the surface test and a new clearance (~150 slots)
    DIFFUSIVE=PHILOX // 2 + 5 + 6 + 20 + 3 + 4 + 2 + 2,
)
# Peak: the FP32 vector rate of the MI355X, 157.3 TFLOP/s = 78.6e12 FMA/s, i.e. 128 lanes per
# CU per clock (256 CUs, 2.4 GHz); one slot = one full-rate 32-bit lane operation.
PEAK_ALU = 256 * 128 * 2.4e9
# HBM bytes per launch of each kernel on the default workload from rocprofv3: FETCH_SIZE x 2.000
# + WRITE_SIZE x 1.000 (KiB per dispatch; factors from a 1 GiB copy and fill).  Valid for the
# kernels and the workload they were taken on (reported for that workload only); set to None
# when a kernel changes.
TRAFFIC = {"k_diffusive32": 323_322 * 1024 * 2.000 + 42_186 * 1024 * 1.000,
           "k_ballistic32": 1_420 * 1024 * 2.000 + 692_952 * 1024 * 1.000}


def algorithmic_ops(counters):
    """ALU slots of one run from its counters [n_seg, 7]: (ballistic phase, diffusive phase)."""
    N = counters[:, 0].sum()
    coll = counters[:, 4].sum()
    diff = counters[:, 5].sum()
    therm = counters[:, 6].sum()
    ballistic_flights = coll + (N - therm)     # every collision, plus the last flight of atoms never thermalised
    diffusive_steps = diff + therm             # every diffusive step, plus the last step of thermalised atoms
    return (float(N * OPS["LAUNCH"] + ballistic_flights * OPS["BALLISTIC"] + coll * OPS["COLLIDE"]),
            float(diffusive_steps * OPS["DIFFUSIVE"]))


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


def cpu_baseline(cfgs, params, target_s):
    import oracle
    oracle.table(params)                      # table build is set-up, not timed
    n0 = 500
    t = time.perf_counter()
    oracle.run(cfgs, params, seed=0, pid_begin=0, pid_end=n0)
    t0 = time.perf_counter() - t
    n = int(min(max(n0, n0 * target_s / max(t0, 1e-3)), 10_000_000))
    t = time.perf_counter()
    r = oracle.run(cfgs, params, seed=0, pid_begin=0, pid_end=n)
    dt = time.perf_counter() - t
    launched = int(r["counters"][:, 0].sum())
    return dict(value=launched / dt, unit="particles/s", cores=int(r["threads"]), kind="oracle",
                sample=f"first {n} particles of each of the {len(r['counters'])} chambers/cathodes "
                       f"({launched} particles, same mix as the workload), {dt:.1f} s, FP64 C, OpenMP")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="legs", choices=["legs", "legs_measured", "quaternary", "quaternary_chimneys", "sweep", "tilt_fit"])
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-fp64", action="store_true", help="skip the FP64 comparator leg")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=25.0,
                    help="target of the CPU pilot-based sizing (the measured run usually takes about half)")
    ap.add_argument("--launch", default="", help="blocks,threads,refill_min,refill_ballistic[,defer_min] instead of autotuning")
    ap.add_argument("--arrivals", action="store_true",
                    help="also tally arrival energy and angle histograms and per-bin energy sums")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one device copy of this size first (HBM counter calibration under rocprofv3)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path (the tally reduce across GPUs "
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
    cfgs, desc = workload(args.workload)
    t = time.perf_counter()
    plan = spx.Plan(cfgs, params, precision=32)
    setup_s = time.perf_counter() - t
    t = time.perf_counter()
    if args.launch:
        launch = plan.set_launch(*(int(x) for x in args.launch.split(",")))
    else:
        launch = plan.launch if args.no_autotune else plan.autotune()
    tune_s = time.perf_counter() - t
    bufs = plan.allocate(profiles=True, arrivals=args.arrivals)
    post, inversion = None, None
    if args.workload == "tilt_fit":
        # the measured library: the same ternary system simulated at the planted tilt with other
        # random numbers (set-up, not timed); the timed step is the sweep plus the inversion
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
    assert n_part == plan.n_particles
    assert np.array_equal(counters[:, 0], counters[:, 1] + counters[:, 2] + counters[:, 3])
    ms_step = wall * 1e3 / args.steps
    ms_med = float(np.median(ms))
    value = n_part / (ms_step * 1e-3)
    coll = float(counters[:, 4].sum())
    diff = float(counters[:, 5].sum())
    counts32 = [bufs["counts"][o:o + nv * nu].cpu().numpy() for o, (nv, nu) in zip(plan.bin_off, plan.shapes)]
    eps32 = tally_error(counts32)

    ops_b, ops_d = algorithmic_ops(counters)
    ms_b = float(np.mean([p[0] for p in phases]))
    ms_d = float(np.mean([p[1] for p in phases]))
    kern = {"k_ballistic32": (ops_b, ms_b), "k_diffusive32": (ops_d, ms_d)}
    dominant = max(kern, key=lambda k: kern[k][1])
    ops, ms_k = kern[dominant]
    achieved = ops / (ms_k * 1e-3)
    roofline = dict(bound="alu", kernel=dominant, achieved=achieved / 1e12, peak=PEAK_ALU / 1e12,
                    unit="TOP/s", frac=achieved / PEAK_ALU,
                    traffic=TRAFFIC.get(dominant) if args.workload == "legs" and not args.arrivals else None,
                    ops_per_launch=ops, launch_ms=ms_k,
                    phases={k: dict(ops=o, ms=t, achieved=o / (t * 1e-3) / 1e12 if t > 0 else None,
                                    frac=o / (t * 1e-3) / PEAK_ALU if t > 0 else None) for k, (o, t) in kern.items()},
                    note="VALU issue slots per lane counted from the algorithm (a 32x32->64 multiply or a native "
                         "transcendental = 4 slots); peak = 256 CU x 128 lanes x 2.4 GHz (the FP32 vector rate); "
                         "kernel time = mean over the timed steps of HIP events recorded between the kernels")

    result = {
        "metric": METRIC, "value": value, "unit": "particles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "particles_per_step": int(n_part), "segments": plan.n_segments,
                   "launch": launch, "seed": args.seed, "arrival_tallies": bool(args.arrivals)},
        "collisions_per_s": (coll + diff) / (ms_step * 1e-3),
        "ballistic_collisions_per_s": coll / (ms_step * 1e-3),
        "diffusive_steps_per_s": diff / (ms_step * 1e-3),
        "step_ms_events": {"median": ms_med, "min": float(min(ms)), "max": float(max(ms))},
        "setup_s": {"plan_and_table": setup_s, "autotune": tune_s},
        "roofline": roofline,
    }

    if inversion is not None:
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        for _ in range(10):
            post(bufs)
        ev[1].record()
        torch.cuda.synchronize()
        result["inversion"] = {
            "tilts_deg": TILT_SWEEP, "planted_deg": TILT_PLANTED,
            "fit_d_e_deg": float(inversion["x_min_de"].cpu()[0]),
            "fit_covered_area_deg": float(inversion["x_match_area"].cpu()[0]),
            "covered_area": [round(float(v), 6) for v in inversion["area"].cpu()],
            "covered_area_measured": float(inversion["area_measured"].cpu()[0]),
            "d_e2": [round(float(v), 3) for v in inversion["loss"].cpu()],
            "chain_ms": ev[0].elapsed_time(ev[1]) / 10,
            "note": "chain = area gather, sweep compositions, d_e^2, covered areas and both fits, after the "
                    "transport (inside the timed step)"}

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
    else:
        result["tally_error"] = {"fp32_batched": eps32}

    if not args.no_cpu:
        cfgs_cpu, _ = workload(args.workload)
        result["cpu_baseline"] = cpu_baseline(cfgs_cpu, params, args.cpu_seconds)
    result["paper_context"] = ("pySIMTRA/SIMTRA: ~20 min per 4-cathode library of ~1e8 particles per cathode on an "
                               "AMD Ryzen 7 5800X (8 cores, 3.8 GHz), i.e. ~3.3e5 particles/s aggregate")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
