"""The FP64 oracle under the host sanitizers: its table build, transport and particle-list entry
points run in a process built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host
code only) on a small mix of configurations that reaches every code path of the transport
(pressures 0 / 0.5 / 2 Pa, gas at rest, a measured racetrack with a six-coefficient emission law,
chimneys and masks, cross absorption, the event cap).  Any invalid access or undefined
operation aborts the run; the outputs must equal those of the ordinary build, bit for bit."""
import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

import oracle
import sputter_inputs as si

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)

pytestmark = pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is required")


def _sanitizers_work(tmp):
    src = os.path.join(tmp, "probe.c")
    open(src, "w").write("int main(void) { return 0; }\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined", src, "-o", os.path.join(tmp, "probe")],
                       capture_output=True)
    return r.returncode == 0


def _configs():
    prof = si.measured_racetrack(seed=0)
    base = [si.single_ni(0.5, 300), si.single_ni(0.0, 200), si.single_ni(2.0, 60),
            si.single_ni(0.5, 150, gas_motion=0)]
    measured = [si.with_launch(si.single_ni(0.5, 150), prof, si.UNDER_COSINE)]
    quat = si.quaternary(0.5, 25.0, 150.0, [80, 30, 60, 40])
    return base + measured + [quat, si.with_chimneys(quat)]


def test_oracle_under_host_sanitizers():
    with tempfile.TemporaryDirectory() as tmp:
        if not _sanitizers_work(tmp):
            pytest.skip("this gcc cannot link the address and undefined-behaviour sanitizers")
        exe = os.path.join(tmp, "driver")
        subprocess.run(["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fopenmp",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                        os.path.join(HERE, "oracle_sanitize_driver.c"), os.path.join(ROOT, "oracle", "spx_oracle.c"),
                        "-lm", "-o", exe], check=True, capture_output=True)
        # a small table keeps the sanitized build fast; the reference uses the same parameters
        params = si.Params(table_ne=40, table_ns=41, event_cap=4000)
        cfgs = _configs()
        S = np.ascontiguousarray(oracle.segments(cfgs), dtype=np.float64)
        prm = np.ascontiguousarray(oracle.params_array(params), dtype=np.float64)
        n_seg, n_cols = S.shape
        shapes = [(cfg.grid.nv, cfg.grid.nu) for cfg in cfgs for _ in cfg.cathodes]
        n_bins = sum(a * b for a, b in shapes)
        seed, pid_end = 5, 1 << 40
        S.tofile(os.path.join(tmp, "segs.f64"))
        prm.tofile(os.path.join(tmp, "prm.f64"))
        np.array([oracle.MOLIERE, params.theta_min, params.log_eps_lo, params.log_eps_hi],
                 dtype=np.float64).tofile(os.path.join(tmp, "table.f64"))
        rng = np.random.default_rng(0)
        seg_ids = rng.integers(0, n_seg, 64).astype(np.uint32)
        pids = np.array([rng.integers(0, int(S[k, 43])) for k in seg_ids], dtype=np.uint32)
        seg_ids.tofile(os.path.join(tmp, "list_seg.u32"))
        pids.tofile(os.path.join(tmp, "list_pid.u32"))
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([exe, tmp, str(n_seg), str(n_cols), str(prm.size), str(params.table_ne),
                            str(params.table_ns), str(n_bins), str(seed), str(pid_end), str(seg_ids.size)],
                           capture_output=True, text=True, timeout=600, env=env)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, r.stderr[-4000:]

        # the ordinary build on the same inputs
        th, bm = oracle.table(params)
        assert np.array_equal(np.fromfile(os.path.join(tmp, "theta.f64")), th)
        assert np.array_equal(np.fromfile(os.path.join(tmp, "betamax.f64")), bm)
        ref = oracle.run(cfgs, params, seed=seed, records=True)
        counts = np.fromfile(os.path.join(tmp, "counts.u64"), dtype=np.uint64)
        assert np.array_equal(counts, np.concatenate([c.reshape(-1) for c in ref["counts"]]))
        counters = np.fromfile(os.path.join(tmp, "counters.u64"), dtype=np.uint64).reshape(n_seg, 7)
        assert np.array_equal(counters, ref["counters"])
        assert (counters[:, 3] > 0).any()          # the event cap was reached somewhere
        rec = np.fromfile(os.path.join(tmp, "records.f64")).reshape(-1, oracle.REC)
        assert np.array_equal(rec, ref["records"])
        lst = np.fromfile(os.path.join(tmp, "list.f64")).reshape(-1, oracle.REC)
        assert np.array_equal(lst, oracle.run_list(cfgs, params, seed, seg_ids, pids))
