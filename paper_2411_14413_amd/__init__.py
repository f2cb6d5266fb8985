"""MI355X-native Monte Carlo transport of sputtered atoms (arXiv 2411.14413).

Python binding of libspx (include/spx.h).  Argument marshalling only: the
transport, tallies, normalisation, area average and composition map all run in
hand-written gfx950 HIP kernels.  PyTorch provides device memory and streams.

    import paper_2411_14413_amd as spx
    plan = spx.Plan(configs)                 # objects with chamber / grid / cathodes
    out = plan.run(seed=0)                   # dict of torch tensors on the GPU
    c = spx.CompositionMap.apply(f, a, b, P, M, rho, fref)   # at.%, differentiable
"""
from __future__ import annotations

import ctypes
from typing import Dict, List, Optional, Sequence

import numpy as np

from . import _native as N
from ._native import COUNTER_NAMES, DEPOSITED, ESCAPED, N_COUNTERS, WALL, SpxError, check, lib

__all__ = ["Plan", "philox", "area_centres", "area_gather", "comp_forward", "comp_backward", "comp_sqdist",
           "CompositionMap", "SquaredDistance", "records_to_numpy", "COUNTER_NAMES", "DEPOSITED", "WALL",
           "ESCAPED", "SpxError", "version", "arrival_edges"]


def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def version() -> int:
    return int(lib().spx_version())


def _vec(v):
    return N.d3(*[float(x) for x in v])


def _params(params, precision: int) -> N.Params:
    p = N.Params()
    p.theta_min = getattr(params, "theta_min", 0.1) if params is not None else 0.1
    p.E_th_kT = getattr(params, "E_th_kT", 3.0) if params is not None else 3.0
    p.event_cap = getattr(params, "event_cap", 1 << 20) if params is not None else 1 << 20
    p.table_ne = getattr(params, "table_ne", 256) if params is not None else 256
    p.table_ns = getattr(params, "table_ns", 257) if params is not None else 257
    p.log_eps_lo = getattr(params, "log_eps_lo", -10.0) if params is not None else -10.0
    p.log_eps_hi = getattr(params, "log_eps_hi", 0.0) if params is not None else 0.0
    p.precision = int(precision)
    return p


class Plan:
    """A validated, device-resident plan for a batch of sputter systems.

    ``configs``: sequence of objects with ``chamber`` (radius, z_lo, z_hi,
    pressure, T, gas_mass, gas_Z, gas_motion), ``grid`` (center, normal, u_axis,
    half_u, half_v, shape, nu, nv) and ``cathodes`` (each: center, normal, u_axis,
    radius, rt_mu, rt_sigma, rt_lo, rt_hi, U_s, E_i, k_cut, mass, Z, cos_coeff,
    n_particles, optionally rt_profile: [(r, depth), ...] of a measured racetrack).  ``precision`` 32 = batched FP32 transport (one persistent
    launch), 64 = plain FP64 comparator (one launch per segment).
    """

    def __init__(self, configs: Sequence, params=None, precision: int = 32):
        L = lib()
        self.configs = list(configs)
        self.precision = int(precision)
        n = len(self.configs)
        carr = (N.Config * max(n, 1))()
        self._keep = []
        for i, cfg in enumerate(self.configs):
            ch, g = cfg.chamber, cfg.grid
            C = carr[i]
            C.chamber = N.Chamber(ch.radius, ch.z_lo, ch.z_hi, ch.pressure, ch.T, ch.gas_mass, int(ch.gas_Z),
                                  int(ch.gas_motion))
            C.grid = N.Grid(_vec(g.center), _vec(g.normal), _vec(g.u_axis), g.half_u, g.half_v, int(g.shape),
                            int(g.nu), int(g.nv), 0)
            cats = (N.Cathode * len(cfg.cathodes))()
            for k, c in enumerate(cfg.cathodes):
                K = cats[k]
                K.center, K.normal, K.u_axis = _vec(c.center), _vec(c.normal), _vec(c.u_axis)
                K.radius, K.rt_mu, K.rt_sigma, K.rt_lo, K.rt_hi = c.radius, c.rt_mu, c.rt_sigma, c.rt_lo, c.rt_hi
                K.U_s, K.E_i, K.k_cut, K.mass, K.Z = c.U_s, c.E_i, c.k_cut, c.mass, int(c.Z)
                K.cos_coeff = (ctypes.c_double * 6)(*[float(x) for x in c.cos_coeff])
                K.n_particles = int(c.n_particles)
                prof = getattr(c, "rt_profile", None)
                if prof is not None:
                    flat = [float(v) for pt in prof for v in pt]
                    arr = (ctypes.c_double * len(flat))(*flat)
                    self._keep.append(arr)
                    K.rt_n = len(flat) // 2
                    K.rt_profile = ctypes.cast(arr, ctypes.POINTER(ctypes.c_double))
                else:
                    K.rt_n = 0
            self._keep.append(cats)
            C.n_cathodes = len(cfg.cathodes)
            C.cathodes = ctypes.cast(cats, ctypes.POINTER(N.Cathode))
            C.cross_absorb = 1 if getattr(cfg, "cross_absorb", False) else 0
            absorbers = list(getattr(cfg, "absorbers", []) or [])
            kinds = {"disc": 0, "rect": 1, "tube": 2}
            if absorbers:
                objs = (N.Object * len(absorbers))()
                for j, a in enumerate(absorbers):
                    O = objs[j]
                    O.kind = kinds[a.kind]
                    O.center, O.normal, O.u_axis = _vec(a.center), _vec(a.normal), _vec(a.u_axis)
                    O.half_u, O.half_v, O.length = a.half_u, a.half_v, a.length
                self._keep.append(objs)
                C.n_objects = len(absorbers)
                C.objects = ctypes.cast(objs, ctypes.POINTER(N.Object))
            else:
                C.n_objects = 0
        self._p = _params(params, precision)
        h = ctypes.c_void_p()
        check(L.spx_plan_create(carr, n, ctypes.byref(self._p), ctypes.byref(h)), "spx_plan_create")
        self._h = h
        self._keep = None          # the plan holds deep copies
        nb, nc, npart, ns = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_int32()
        check(L.spx_plan_query(h, ctypes.byref(nb), ctypes.byref(nc), ctypes.byref(npart), ctypes.byref(ns)),
              "spx_plan_query")
        self.n_bins, self.n_counters, self.n_particles, self.n_segments = nb.value, nc.value, npart.value, ns.value
        bo = (ctypes.c_uint64 * self.n_segments)()
        fi = (ctypes.c_uint64 * self.n_segments)()
        check(L.spx_plan_layout(h, bo, fi), "spx_plan_layout")
        self.bin_off = list(bo)
        self.first = list(fi)
        self.shapes = [(cfg.grid.nv, cfg.grid.nu) for cfg in self.configs for _ in cfg.cathodes]
        self.seg_particles = [int(c.n_particles) for cfg in self.configs for c in cfg.cathodes]

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                lib().spx_plan_destroy(h)
            except Exception:
                pass
            self._h = None

    # -- running ---------------------------------------------------------------------------
    def allocate(self, profiles: bool = True, records: bool = False, arrivals: bool = False,
                 device=None) -> Dict[str, object]:
        torch = _torch()
        dev = device or torch.device("cuda", torch.cuda.current_device())
        out = dict(
            counts=torch.empty(self.n_bins, dtype=torch.int64, device=dev),
            counters=torch.empty(self.n_counters, dtype=torch.int64, device=dev),
            profiles=torch.empty(self.n_bins, dtype=torch.float64, device=dev) if profiles else None,
            records=torch.empty(self.n_particles * N.RECORD_BYTES, dtype=torch.uint8, device=dev) if records else None,
        )
        if arrivals:
            out["arrival_energy"] = torch.empty(self.n_segments * N.ARRIVAL_E_BINS, dtype=torch.int64, device=dev)
            out["arrival_angle"] = torch.empty(self.n_segments * N.ARRIVAL_A_BINS, dtype=torch.int64, device=dev)
            out["energy_sum"] = torch.empty(self.n_bins, dtype=torch.int64, device=dev)
        return out

    def run_into(self, seed: int, bufs: Dict[str, object], stream=None) -> None:
        """Enqueue one run writing into pre-allocated buffers (see allocate)."""
        if bufs.get("arrival_energy") is not None:
            o = N.Outputs(_ptr(bufs["counts"]), _ptr(bufs["counters"]), _ptr(bufs.get("profiles")),
                          _ptr(bufs.get("records")), _ptr(bufs["arrival_energy"]), _ptr(bufs["arrival_angle"]),
                          _ptr(bufs["energy_sum"]))
            check(lib().spx_run_ex(self._h, int(seed) & (2**64 - 1), ctypes.byref(o), _stream(stream)), "spx_run_ex")
            return
        check(lib().spx_run(self._h, int(seed) & (2**64 - 1), _ptr(bufs["counts"]), _ptr(bufs["counters"]),
                            _ptr(bufs.get("profiles")), _ptr(bufs.get("records")), _stream(stream)), "spx_run")

    def run_noalloc_into(self, seed: int, bufs: Dict[str, object], stream=None) -> None:
        """As run_into, through the entry point that allocates nothing (queue and counters in
        the library's static scratch array; calls on one GPU must not overlap)."""
        o = N.Outputs(_ptr(bufs["counts"]), _ptr(bufs["counters"]), _ptr(bufs.get("profiles")),
                      _ptr(bufs.get("records")), _ptr(bufs.get("arrival_energy")), _ptr(bufs.get("arrival_angle")),
                      _ptr(bufs.get("energy_sum")))
        check(lib().spx_run_noalloc(self._h, int(seed) & (2**64 - 1), ctypes.byref(o), _stream(stream)),
              "spx_run_noalloc")

    def run(self, seed: int = 0, profiles: bool = True, records: bool = False, arrivals: bool = False,
            stream=None) -> Dict[str, object]:
        bufs = self.allocate(profiles=profiles, records=records, arrivals=arrivals)
        self.run_into(seed, bufs, stream)
        out = dict(bufs)
        out["counters"] = bufs["counters"].view(self.n_segments, N_COUNTERS)
        if arrivals:
            out["arrival_energy"] = bufs["arrival_energy"].view(self.n_segments, N.ARRIVAL_E_BINS)
            out["arrival_angle"] = bufs["arrival_angle"].view(self.n_segments, N.ARRIVAL_A_BINS)
        out["counts_seg"] = [bufs["counts"][o:o + nv * nu].view(nv, nu) for o, (nv, nu) in
                             zip(self.bin_off, self.shapes)]
        if profiles:
            out["profiles_seg"] = [bufs["profiles"][o:o + nv * nu].view(nv, nu) for o, (nv, nu) in
                                   zip(self.bin_off, self.shapes)]
        return out

    # -- tuning ----------------------------------------------------------------------------
    def autotune(self, stream=None):
        check(lib().spx_autotune(self._h, _stream(stream)), "spx_autotune")
        return self.launch

    @property
    def launch(self):
        b, t, r, m, d = (ctypes.c_int32() for _ in range(5))
        check(lib().spx_get_launch(self._h, ctypes.byref(b), ctypes.byref(t), ctypes.byref(r), ctypes.byref(m),
                                   ctypes.byref(d)), "spx_get_launch")
        return dict(blocks=b.value, threads=t.value, refill_min=r.value, refill_ballistic=m.value, defer_min=d.value)

    def set_launch(self, blocks: int = 0, threads: int = 256, refill_min: int = 8, refill_ballistic: int = 8,
                   defer_min: int = 8):
        check(lib().spx_set_launch(self._h, int(blocks), int(threads), int(refill_min), int(refill_ballistic),
                                   int(defer_min)), "spx_set_launch")
        return self.launch

    def graph_info(self):
        """(graph instantiations, kernel-node argument updates) of this plan so far."""
        i, u = ctypes.c_uint64(), ctypes.c_uint64()
        check(lib().spx_graph_info(self._h, ctypes.byref(i), ctypes.byref(u)), "spx_graph_info")
        return i.value, u.value

    def phase_times(self):
        """(ballistic ms, diffusive ms) of the last FP32 run (waits for it)."""
        b, d = ctypes.c_float(), ctypes.c_float()
        check(lib().spx_phase_times(self._h, ctypes.byref(b), ctypes.byref(d)), "spx_phase_times")
        return b.value, d.value

    # -- introspection ---------------------------------------------------------------------
    def table(self):
        ne, ns = self._p.table_ne, self._p.table_ns
        th = np.empty(ne * ns)
        bm = np.empty(ne)
        dp = ctypes.POINTER(ctypes.c_double)
        check(lib().spx_get_table(self._h, th.ctypes.data_as(dp), bm.ctypes.data_as(dp)), "spx_get_table")
        return th.reshape(ne, ns), bm

    def segment_info(self, seg: int = 0) -> Dict[str, float]:
        out = (ctypes.c_double * 16)()
        check(lib().spx_segment_info(self._h, int(seg), out), "spx_segment_info")
        names = ("Lambda", "E_max", "s_max", "a_mm", "eps_per_eV", "n_mm3", "kT", "E_th", "lam_th", "PhiA", "QB",
                 "dPhi", "mu_red", "vth", "vg", "z_mid")
        return dict(zip(names, list(out)))


RECORD_DTYPE = np.dtype([("x", "<f8"), ("y", "<f8"), ("z", "<f8"), ("E", "<f8"), ("state", "<u4"),
                         ("bin", "<u4"), ("events", "<u4"), ("diffusive", "<u4"), ("cos_in", "<f8")])


def run(configs: Sequence, seed: int = 0, precision: int = 32, params=None, records: bool = False,
        arrivals: bool = False, autotune: bool = False, stream=None) -> Dict[str, object]:
    """One transport run of ``configs`` with a plan made for the call: the outputs of
    Plan.run, plus the plan under "plan" (reuse a Plan to run a sweep several times)."""
    plan = Plan(configs, params, precision=precision)
    if autotune and precision == 32:
        plan.autotune(stream)
    out = plan.run(seed=seed, records=records, arrivals=arrivals, stream=stream)
    out["plan"] = plan
    return out


def arrival_edges():
    """Bin edges of the arrival tallies: (energy [61] f64, cos [91] f64, energy f32, cos f32)."""
    e64 = np.empty(N.ARRIVAL_E_BINS + 1)
    c64 = np.empty(N.ARRIVAL_A_BINS + 1)
    e32 = np.empty(N.ARRIVAL_E_BINS + 1, dtype=np.float32)
    c32 = np.empty(N.ARRIVAL_A_BINS + 1, dtype=np.float32)
    fp = ctypes.POINTER(ctypes.c_float)
    check(lib().spx_arrival_edges(e64.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  c64.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  e32.ctypes.data_as(fp), c32.ctypes.data_as(fp)), "spx_arrival_edges")
    return e64, c64, e32, c32


def records_to_numpy(rec_bytes) -> np.ndarray:
    """Host structured array (x, y, z, E, state, bin, events, diffusive, cos_in) from a record buffer."""
    a = rec_bytes.detach().cpu().numpy() if hasattr(rec_bytes, "detach") else np.asarray(rec_bytes)
    return a.view(RECORD_DTYPE)


def philox(ctr, seed: int, stream=None):
    """Philox4x32-10 blocks of an [n, 4] int32/uint32 CUDA tensor of counters."""
    torch = _torch()
    c = ctr.contiguous()
    out = torch.empty_like(c)
    check(lib().spx_philox(_ptr(c), int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF, _ptr(out), c.shape[0],
                           _stream(stream)), "spx_philox")
    return out


def area_centres(n_areas: int = 342, pitch: float = 4.5) -> np.ndarray:
    out = np.empty(2 * n_areas)
    check(lib().spx_area_centres(int(n_areas), float(pitch), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
          "spx_area_centres")
    return out.reshape(n_areas, 2)


def area_gather(profiles, grid, centres, half_width: float = 2.25, stream=None):
    """Area averages [n_prof, n_areas] of float64 CUDA profiles [n_prof, nv, nu] (or [nv, nu])."""
    torch = _torch()
    p = profiles.contiguous()
    if p.dim() == 2:
        p = p.unsqueeze(0)
    cen = (centres.to(device=p.device, dtype=torch.float64).contiguous() if isinstance(centres, torch.Tensor)
           else torch.as_tensor(np.asarray(centres, dtype=np.float64), device=p.device).contiguous())
    out = torch.empty(p.shape[0], cen.shape[0], dtype=torch.float64, device=p.device)
    check(lib().spx_area_gather(_ptr(p), p.shape[0], int(grid.nu), int(grid.nv), float(grid.half_u),
                                float(grid.half_v), _ptr(cen), cen.shape[0], float(half_width), _ptr(out),
                                _stream(stream)), "spx_area_gather")
    return out


def _f32(t):
    return t.detach().contiguous().float() if t.dtype != _torch().float32 else t.detach().contiguous()


def comp_forward(f, a, b, P, M, rho, fref, stream=None):
    torch = _torch()
    f, a, b, P, M, rho, fref = (_f32(x) for x in (f, a, b, P, M, rho, fref))
    K, J = f.shape
    B = P.shape[0]
    c = torch.empty(B, J, K, dtype=torch.float32, device=f.device)
    check(lib().spx_comp_forward(_ptr(f), _ptr(a), _ptr(b), _ptr(P), _ptr(M), _ptr(rho), _ptr(fref), _ptr(c), B, J,
                                 K, _stream(stream)), "spx_comp_forward")
    return c


def comp_backward(f, a, b, P, M, rho, fref, gc, stream=None):
    torch = _torch()
    f, a, b, P, M, rho, fref, gc = (_f32(x) for x in (f, a, b, P, M, rho, fref, gc))
    K, J = f.shape
    B = P.shape[0]
    g = {k: torch.empty_like(v) for k, v in dict(f=f, a=a, b=b, P=P, M=M, rho=rho, fref=fref).items()}
    check(lib().spx_comp_backward(_ptr(f), _ptr(a), _ptr(b), _ptr(P), _ptr(M), _ptr(rho), _ptr(fref), _ptr(gc),
                                  _ptr(g["f"]), _ptr(g["a"]), _ptr(g["b"]), _ptr(g["P"]), _ptr(g["M"]),
                                  _ptr(g["rho"]), _ptr(g["fref"]), B, J, K, _stream(stream)), "spx_comp_backward")
    return g


def comp_sqdist(c, ct, gloss=None, want_grad: bool = False, stream=None):
    """Per-row squared Euclidean distance sum_{j,k} (c - ct)^2 and optionally 2 (c - ct) gloss."""
    torch = _torch()
    c, ct = _f32(c), _f32(ct)
    if ct.dim() == 2:
        ct = ct.unsqueeze(0)
    B, J, K = c.shape
    loss = torch.empty(B, dtype=torch.float32, device=c.device)
    gc = torch.empty_like(c) if want_grad else None
    gl = _f32(gloss) if gloss is not None else None
    check(lib().spx_comp_sqdist(_ptr(c), _ptr(ct), ct.shape[0], _ptr(gl), _ptr(loss), _ptr(gc), B, J, K,
                                _stream(stream)), "spx_comp_sqdist")
    return (loss, gc) if want_grad else loss


# -- inversion over a sweep (Results, cathode-tilt study) --------------------------------------
FIT_MIN, FIT_MATCH = 0, 1


def _f64(t):
    return t.detach().contiguous().double() if t.dtype != _torch().float64 else t.detach().contiguous()


def sweep_composition(f, a, b, P, M, rho, stream=None):
    """at.% [T, J, K] (float32) of the T libraries of a sweep: f [T, K, J] float64 area values
    (each library normalised by the mean of its own areas); a, b, P, M, rho [K]."""
    torch = _torch()
    f = _f64(f)
    dev = f.device
    a, b, P, M, rho = (_f64(torch.as_tensor(np.asarray(v, dtype=np.float64), device=dev)) if not
                       isinstance(v, torch.Tensor) else _f64(v) for v in (a, b, P, M, rho))
    T, K, J = f.shape
    c = torch.empty(T, J, K, dtype=torch.float32, device=dev)
    check(lib().spx_sweep_composition(_ptr(f), _ptr(a), _ptr(b), _ptr(P), _ptr(M), _ptr(rho), _ptr(c), T, J, K,
                                      _stream(stream)), "spx_sweep_composition")
    return c


def hull_area(c, stream=None):
    """Covered fraction of the ternary diagram [B] (float32) of libraries c [B, J, 3] or [J, 3]."""
    torch = _torch()
    c = _f32(c)
    if c.dim() == 2:
        c = c.unsqueeze(0)
    if c.shape[2] != 3:
        raise ValueError("hull_area needs ternary compositions [B, J, 3]")
    out = torch.empty(c.shape[0], dtype=torch.float32, device=c.device)
    check(lib().spx_hull_area(_ptr(c), c.shape[0], c.shape[1], _ptr(out), _stream(stream)), "spx_hull_area")
    return out


def sweep_fit(x, y, mode: int, target=None, stream=None):
    """Fitted sweep values [B] (float64): y [B, T] or [T] float32 curves over the host sweep
    values x [T]; mode FIT_MIN (minimiser) or FIT_MATCH (where y reaches target [B])."""
    torch = _torch()
    y = _f32(y)
    if y.dim() == 1:
        y = y.unsqueeze(0)
    hx = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if hx.shape != (y.shape[1],):
        raise ValueError("sweep_fit: x must have one value per column of y")
    tg = _f32(target).reshape(-1) if target is not None else None
    out = torch.empty(y.shape[0], dtype=torch.float64, device=y.device)
    check(lib().spx_sweep_fit(hx.ctypes.data_as(ctypes.c_void_p), _ptr(y), y.shape[0], y.shape[1], int(mode),
                              _ptr(tg), _ptr(out), _stream(stream)), "spx_sweep_fit")
    return out


def invert_sweep(plan, out, x, comp, measured, centres=None, half_width: float = 2.25, stream=None):
    """Finish the inversion of a sweep run: ``plan`` holds one configuration per sweep value
    x [T] (same grid, K cathodes each) and ``out`` its run with profiles; ``comp`` = (a, b, P,
    M, rho) of the library; ``measured`` the measured compositions [J, K] (CUDA); ``centres``
    the area centres [J, 2] (numpy or CUDA; default the 342 areas).  Every step is
    a library call: area gather, compositions, d_e^2 against the measured library, covered
    areas (K = 3) and the two fits."""
    torch = _torch()
    T = len(x)
    K = plan.n_segments // T
    nv, nu = plan.shapes[0]
    if K * T != plan.n_segments or any(o != k * nv * nu for k, o in enumerate(plan.bin_off)) or \
            any(sh != (nv, nu) for sh in plan.shapes):
        raise ValueError("invert_sweep: the plan must hold T configurations of K cathodes on one grid")
    grid = plan.configs[0].grid
    cen = area_centres() if centres is None else centres
    prof = out["profiles"][:plan.n_segments * nv * nu].view(plan.n_segments, nv, nu)
    f = area_gather(prof, grid, cen, half_width, stream).view(T, K, -1)
    c = sweep_composition(f, *comp, stream=stream)
    meas = _f32(measured).reshape(1, c.shape[1], K)
    loss = comp_sqdist(c, meas, stream=stream)
    res = dict(f=f, c=c, loss=loss, x_min_de=sweep_fit(x, loss, FIT_MIN, stream=stream))
    if K == 3:
        area = hull_area(c, stream)
        area_m = hull_area(meas, stream)
        res.update(area=area, area_measured=area_m,
                   x_match_area=sweep_fit(x, area, FIT_MATCH, target=area_m, stream=stream))
    return res


def _autograd_classes():
    torch = _torch()

    class CompositionMap(torch.autograd.Function):
        """at.% [B, J, K] from arrival fractions f [K, J], rates a P + b, masses M,
        densities rho and calibration values fref; backward by spx_comp_backward."""

        @staticmethod
        def forward(ctx, f, a, b, P, M, rho, fref):
            ctx.save_for_backward(f, a, b, P, M, rho, fref)
            return comp_forward(f, a, b, P, M, rho, fref)

        @staticmethod
        def backward(ctx, gc):
            f, a, b, P, M, rho, fref = ctx.saved_tensors
            g = comp_backward(f, a, b, P, M, rho, fref, gc)
            outs = []
            for name, t in zip(("f", "a", "b", "P", "M", "rho", "fref"), (f, a, b, P, M, rho, fref)):
                outs.append(g[name].to(t.dtype) if ctx.needs_input_grad[len(outs)] else None)
            return tuple(outs)

    class SquaredDistance(torch.autograd.Function):
        """Per-row d_e^2 summed over areas: sum_{j,k} (c - c*)^2; c* is a constant target."""

        @staticmethod
        def forward(ctx, c, ct):
            ctx.save_for_backward(c, ct)
            return comp_sqdist(c, ct)

        @staticmethod
        def backward(ctx, gloss):
            c, ct = ctx.saved_tensors
            _, gc = comp_sqdist(c, ct, gloss=gloss, want_grad=True)
            return gc.to(c.dtype), None

    return CompositionMap, SquaredDistance


def __getattr__(name):
    if name in ("CompositionMap", "SquaredDistance"):
        cm, sd = _autograd_classes()
        globals()["CompositionMap"], globals()["SquaredDistance"] = cm, sd
        return globals()[name]
    raise AttributeError(name)
