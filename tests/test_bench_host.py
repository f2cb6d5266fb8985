"""Host-side logic of bench.py (no GPU): the work model that gives the roofline's algorithmic
slots, the HBM-traffic lookup that must go null when the transport kernels' sources change, and
the refusal of more than one GPU."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import sputter_inputs as si  # noqa: E402


def _counters(N, coll, diff, therm, tested):
    c = np.zeros((1, 8))
    c[0, 0], c[0, 4], c[0, 5], c[0, 6], c[0, 7] = N, coll, diff, therm, tested
    return c


def test_work_model_by_hand():
    """Slots of a run without absorbing objects, counted by hand from the per-unit figures."""
    cfgs = [si.single_ni(0.5, 1000)]
    N, coll, diff, therm, tested = 1000.0, 7000.0, 50000.0, 400.0, 900.0
    ob, od = bench.algorithmic_ops(_counters(N, coll, diff, therm, tested), cfgs)
    O = bench.OPS
    # every collision ends a flight, and so does the last flight of each atom never thermalised
    assert ob == N * O["LAUNCH"] + (coll + N - therm) * O["BALLISTIC"] + coll * O["COLLIDE"]
    # every diffusive step, plus the last (terminal) step of each thermalised atom
    assert od == (diff + therm) * O["DIFFUSIVE"] + tested * O["TESTED"]


def test_work_model_charges_objects():
    """Absorbing objects add their surface-test share to every flight and their test and
    clearance shares to every tested diffusive step; the other targets count as discs when
    they absorb."""
    cfg = si.with_chimneys(si.quaternary(counts=[100, 100, 100, 100]))
    objs = bench.segment_objects([cfg])
    assert len(objs) == 4
    kinds = objs[0]
    assert kinds.count("tube") >= 1 and kinds.count("disc") == 3
    c = np.zeros((4, 8))
    c[:, 0], c[:, 4], c[:, 5], c[:, 6], c[:, 7] = 100, 300, 2000, 50, 80
    ob, od = bench.algorithmic_ops(c, [cfg])
    plain_b, plain_d = bench.algorithmic_ops(c, [si.quaternary(counts=[100, 100, 100, 100])])
    t = sum(bench.OBJ_TEST[k] for k in kinds)
    cl = sum(bench.OBJ_CLEAR[k] for k in kinds)
    assert ob - plain_b == pytest.approx(4 * (300 + 100 - 50) * t)
    assert od - plain_d == pytest.approx(4 * 80 * (t + cl))


def test_traffic_only_for_the_measured_sources(tmp_path, monkeypatch):
    """profiles/hbm_traffic.json gives bytes per launch only while the transport sources hash to
    the digest recorded with them."""
    h = bench.kernel_source_hash()
    assert len(h) == 16 and h == bench.kernel_source_hash()
    prof = tmp_path / "profiles"
    prof.mkdir()
    (prof / "hbm_traffic.json").write_text(json.dumps(
        {"legs": {"k_diffusive32": {"sources": h, "bytes_per_launch": 123},
                  "k_ballistic32": {"sources": "0" * 16, "bytes_per_launch": 456}}}))
    real = bench.kernel_source_hash
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_source_hash", lambda: h)
    assert bench.measured_traffic("k_diffusive32", "legs") == 123
    assert bench.measured_traffic("k_ballistic32", "legs") is None      # other sources
    assert bench.measured_traffic("k_diffusive32", "sweep") is None     # not measured
    monkeypatch.setattr(bench, "kernel_source_hash", real)


def test_committed_traffic_table():
    """The committed table covers both transport kernels on the three benchmarked workloads with
    plausible bytes per launch; entries taken on other sources than this tree's are only
    reported as stale (bench.py then reports traffic as null until they are taken again)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    table = json.load(open(path))
    h = bench.kernel_source_hash()
    stale = []
    for wl in ("legs", "quaternary", "sweep"):
        for k in ("k_ballistic32", "k_diffusive32"):
            e = table[wl][k]
            assert len(e["sources"]) == 16
            # HBM bytes per launch: at least the 48-byte queue records the phases hand over
            # (hundreds of MB on every one of these workloads), far below 10 GB
            assert 1e8 < e["bytes_per_launch"] < 1e10
            if e["sources"] != h:
                stale.append(f"{wl}/{k}")
    if stale:
        pytest.skip(f"traffic taken on other transport sources for {stale}: bench.py reports traffic null")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr or "--gpus 1" in r.stderr
