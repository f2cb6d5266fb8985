"""ctypes view of libspx.so (the C-ABI declared in include/spx.h).

Argument marshalling only: every step of the transport, normalisation, area
average and composition map runs in the HIP kernels of libspx.  There is no
fallback: if the library is missing or cannot be loaded, this module raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libspx.so")

SPX_OK, SPX_EINVAL, SPX_ENOMEM, SPX_EDEVICE, SPX_ESTATE = 0, -1, -2, -3, -4
DEPOSITED, WALL, ESCAPED = 1, 2, 3
N_COUNTERS = 8
COUNTER_NAMES = ("launched", "deposited", "wall", "escaped", "collisions", "diffusive_steps", "thermalized",
                 "tested_steps")

d3 = ctypes.c_double * 3


class Cathode(ctypes.Structure):
    _fields_ = [("center", d3), ("normal", d3), ("u_axis", d3), ("radius", ctypes.c_double),
                ("rt_mu", ctypes.c_double), ("rt_sigma", ctypes.c_double), ("rt_lo", ctypes.c_double),
                ("rt_hi", ctypes.c_double), ("U_s", ctypes.c_double), ("E_i", ctypes.c_double),
                ("k_cut", ctypes.c_double), ("mass", ctypes.c_double), ("Z", ctypes.c_int32),
                ("rt_n", ctypes.c_int32), ("cos_coeff", ctypes.c_double * 6), ("n_particles", ctypes.c_uint64),
                ("rt_profile", ctypes.POINTER(ctypes.c_double))]


class Chamber(ctypes.Structure):
    _fields_ = [("radius", ctypes.c_double), ("z_lo", ctypes.c_double), ("z_hi", ctypes.c_double),
                ("pressure", ctypes.c_double), ("T", ctypes.c_double), ("gas_mass", ctypes.c_double),
                ("gas_Z", ctypes.c_int32), ("gas_motion", ctypes.c_int32)]


class Grid(ctypes.Structure):
    _fields_ = [("center", d3), ("normal", d3), ("u_axis", d3), ("half_u", ctypes.c_double),
                ("half_v", ctypes.c_double), ("shape", ctypes.c_int32), ("nu", ctypes.c_int32),
                ("nv", ctypes.c_int32), ("reserved0", ctypes.c_int32)]


class Object(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved0", ctypes.c_int32), ("center", ctypes.c_double * 3),
                ("normal", ctypes.c_double * 3), ("u_axis", ctypes.c_double * 3), ("half_u", ctypes.c_double),
                ("half_v", ctypes.c_double), ("length", ctypes.c_double)]


class Config(ctypes.Structure):
    _fields_ = [("chamber", Chamber), ("grid", Grid), ("n_cathodes", ctypes.c_int32),
                ("cross_absorb", ctypes.c_int32), ("cathodes", ctypes.POINTER(Cathode)),
                ("n_objects", ctypes.c_int32), ("reserved1", ctypes.c_int32), ("objects", ctypes.POINTER(Object))]


class Params(ctypes.Structure):
    _fields_ = [("theta_min", ctypes.c_double), ("E_th_kT", ctypes.c_double), ("event_cap", ctypes.c_uint32),
                ("table_ne", ctypes.c_int32), ("table_ns", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("log_eps_lo", ctypes.c_double), ("log_eps_hi", ctypes.c_double)]


class Record(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double), ("y", ctypes.c_double), ("z", ctypes.c_double), ("E", ctypes.c_double),
                ("state", ctypes.c_uint32), ("bin", ctypes.c_uint32), ("events", ctypes.c_uint32),
                ("diffusive", ctypes.c_uint32), ("cos_in", ctypes.c_double)]


RECORD_BYTES = ctypes.sizeof(Record)
assert RECORD_BYTES == 56

ARRIVAL_E_BINS, ARRIVAL_A_BINS = 60, 90
ESUM_SCALE = 2.0 ** 24


class Outputs(ctypes.Structure):
    _fields_ = [("counts", ctypes.c_void_p), ("counters", ctypes.c_void_p), ("profiles", ctypes.c_void_p),
                ("records", ctypes.c_void_p), ("arrival_energy", ctypes.c_void_p), ("arrival_angle", ctypes.c_void_p),
                ("energy_sum", ctypes.c_void_p)]

# Every entry point of include/spx.h: name -> (restype, argtypes)
_vp = ctypes.c_void_p
_u64 = ctypes.c_uint64
_i32 = ctypes.c_int32
_dbl = ctypes.c_double
SIGNATURES = {
    "spx_plan_create": (ctypes.c_int, [ctypes.POINTER(Config), _i32, ctypes.POINTER(Params), ctypes.POINTER(_vp)]),
    "spx_plan_query": (ctypes.c_int, [_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64), ctypes.POINTER(_u64),
                                      ctypes.POINTER(_i32)]),
    "spx_plan_layout": (ctypes.c_int, [_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "spx_run": (ctypes.c_int, [_vp, _u64, _vp, _vp, _vp, _vp, _vp]),
    "spx_run_ex": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(Outputs), _vp]),
    "spx_run_noalloc": (ctypes.c_int, [_vp, _u64, ctypes.POINTER(Outputs), _vp]),
    "spx_graph_info": (ctypes.c_int, [_vp, ctypes.POINTER(_u64), ctypes.POINTER(_u64)]),
    "spx_arrival_edges": (ctypes.c_int, [ctypes.POINTER(_dbl), ctypes.POINTER(_dbl), ctypes.POINTER(ctypes.c_float),
                                         ctypes.POINTER(ctypes.c_float)]),
    "spx_autotune": (ctypes.c_int, [_vp, _vp]),
    "spx_get_launch": (ctypes.c_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                                      ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "spx_set_launch": (ctypes.c_int, [_vp, _i32, _i32, _i32, _i32, _i32]),
    "spx_phase_times": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(ctypes.c_float)]),
    "spx_get_table": (ctypes.c_int, [_vp, ctypes.POINTER(_dbl), ctypes.POINTER(_dbl)]),
    "spx_segment_info": (ctypes.c_int, [_vp, _i32, ctypes.POINTER(_dbl)]),
    "spx_philox": (ctypes.c_int, [_vp, ctypes.c_uint32, ctypes.c_uint32, _vp, _u64, _vp]),
    "spx_area_centres": (ctypes.c_int, [_i32, _dbl, ctypes.POINTER(_dbl)]),
    "spx_area_gather": (ctypes.c_int, [_vp, _i32, _i32, _i32, _dbl, _dbl, _vp, _i32, _dbl, _vp, _vp]),
    "spx_comp_forward": (ctypes.c_int, [_vp] * 8 + [_i32, _i32, _i32, _vp]),
    "spx_comp_backward": (ctypes.c_int, [_vp] * 15 + [_i32, _i32, _i32, _vp]),
    "spx_comp_sqdist": (ctypes.c_int, [_vp, _vp, _i32, _vp, _vp, _vp, _i32, _i32, _i32, _vp]),
    "spx_sweep_composition": (ctypes.c_int, [_vp] * 7 + [_i32, _i32, _i32, _vp]),
    "spx_hull_area": (ctypes.c_int, [_vp, _i32, _i32, _vp, _vp]),
    "spx_sweep_fit": (ctypes.c_int, [_vp, _vp, _i32, _i32, _i32, _vp, _vp, _vp]),
    "spx_plan_destroy": (None, [_vp]),
    "spx_last_error": (ctypes.c_char_p, []),
    "spx_version": (ctypes.c_int32, []),
}

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libspx (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                               "(python -m paper_2411_14413_amd.build or __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class SpxError(RuntimeError):
    def __init__(self, code: int, where: str):
        msg = lib().spx_last_error()
        super().__init__(f"{where} failed ({code}): {msg.decode() if msg else ''}")
        self.code = code


def check(code: int, where: str) -> None:
    if code != SPX_OK:
        raise SpxError(code, where)
