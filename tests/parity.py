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


def bin_flips_off_edge(rec, ref, tol, grid):
    """Matched deposits (same state, end points within tol) whose bins differ although the
    oracle's end point lies farther than tol from every bin edge of the substrate grid: such a
    flip cannot come from rounding of the end point.  Returns their count."""
    st_g = rec["state"].astype(np.int64)
    d = np.linalg.norm(gpu_positions(rec) - ref[:, :3], axis=1)
    dep = (st_g == 1) & (ref[:, 3].astype(np.int64) == 1) & (d < tol)
    flip = dep & (rec["bin"].astype(np.int64) != ref[:, 4].astype(np.int64))
    if not flip.any():
        return 0
    c, n, u = (np.asarray(v, dtype=np.float64) for v in (grid.center, grid.normal, grid.u_axis))
    v = np.cross(n, u)
    q = ref[flip, :3] - c
    du, dv = 2 * grid.half_u / grid.nu, 2 * grid.half_v / grid.nv
    fu = (q @ u + grid.half_u) / du
    fv = (q @ v + grid.half_v) / dv
    edge = np.minimum(np.abs(fu - np.rint(fu)) * du, np.abs(fv - np.rint(fv)) * dv)
    return int((edge > tol).sum())
