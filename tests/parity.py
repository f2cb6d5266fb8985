"""Helpers shared by the GPU parity tests (no test functions here)."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_positions(rec):
    return np.stack([rec["x"], rec["y"], rec["z"]], axis=1)


def match_stats(rec, ref, tol):
    """Fraction of particles with the same terminal state and end points within tol (mm);
    also whether deposited matches share the bin."""
    st_g = rec["state"].astype(np.int64)
    st_o = ref[:, 3].astype(np.int64)
    d = np.linalg.norm(gpu_positions(rec) - ref[:, :3], axis=1)
    same = st_g == st_o
    close = same & (d < tol)
    dep = close & (st_g == 1)
    bin_same = np.all(rec["bin"][dep].astype(np.int64) == ref[dep, 4].astype(np.int64)) if dep.any() else True
    return dict(frac=float(close.mean()), same_state=float(same.mean()), n=len(rec),
                bin_frac=float((rec["bin"][dep].astype(np.int64) == ref[dep, 4].astype(np.int64)).mean())
                if dep.any() else 1.0, bin_all=bool(bin_same), d_max_matched=float(d[same].max()) if same.any() else 0.0,
                d_median=float(np.median(d)))


def records_histogram(rec, n_bins_seg, first, counts_len):
    """Tally rebuilt from per-particle records, per segment (exact integer check)."""
    out = []
    for k, (off, n, nb) in enumerate(zip(first[:-1], np.diff(first), n_bins_seg)):
        r = rec[off:off + n]
        dep = r[r["state"] == 1]
        out.append(np.bincount(dep["bin"].astype(np.int64), minlength=nb))
    return out
