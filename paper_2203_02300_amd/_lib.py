"""ctypes loader of ``libdco_stereo.so`` (the gfx950 HIP library).

The library is built in-tree by ``paper_2203_02300_amd.build``.  There is no
fallback: if it is missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdco_stereo.so")

# Symbols the C ABI exports (include/dco_stereo.h).
EXPORTS = (
    "dco_default_params", "dco_stereo_create", "dco_stereo_destroy", "dco_stereo_set_stream",
    "dco_census", "dco_cost_volume", "dco_aggregate", "dco_wta_lrcheck", "dco_stereo_match",
    "dco_stereo_last_disparities", "dco_stereo_profile", "dco_stereo_stage_times",
    "dco_batch_create", "dco_batch_destroy", "dco_batch_match",
    "dco_batch_tile", "dco_soft_forward", "dco_soft_backward", "dco_soft_backward_reuse",
    "dco_vote_refine",
    "dco_stereo_match_half", "dco_densify_default_params", "dco_densify_create",
    "dco_densify_destroy", "dco_densify_run", "dco_densify_stats",
    "dco_contour_default_params", "dco_contour_create", "dco_contour_destroy",
    "dco_contour_run", "dco_contour_launches",
    "dco_status_string", "dco_last_error", "dco_stereo_agg_slices", "dco_debug_fail_alloc",
    "dco_debug_live_allocations", "dco_stereo_match_noalloc",
)

DCO_OK = 0
STATUS = {0: "DCO_OK", -1: "DCO_ERR_ARG", -2: "DCO_ERR_SHAPE", -3: "DCO_ERR_HIP",
          -4: "DCO_ERR_OOM", -5: "DCO_ERR_STATE"}


class DcoError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("census_w", C.c_int), ("census_h", C.c_int),
        ("arm_L1", C.c_int), ("arm_tau1", C.c_int),
        ("lambda_ad", C.c_float), ("lambda_census", C.c_float),
        ("gamma_L", C.c_float), ("eps", C.c_float),
        ("agg_iters", C.c_int), ("lr_max_diff", C.c_int), ("subpixel", C.c_int),
        ("vote_iters", C.c_int),
    ]


class DensifyParams(C.Structure):
    _fields_ = [
        ("lambda_d", C.c_float), ("lambda_s", C.c_float), ("lambda_s2", C.c_float),
        ("tol", C.c_double), ("max_iters", C.c_int), ("iters_per_launch", C.c_int),
    ]


class ContourParams(C.Structure):
    _fields_ = [
        ("T_high", C.c_float), ("T_low", C.c_float), ("T_depth", C.c_float),
        ("box_radius", C.c_int),
    ]


_lib = None


def lib():
    """Load the library (once).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2203_02300_amd.build` (no CPU fallback exists)")
    L = C.CDLL(LIB_PATH)
    P, i, st = C.c_void_p, C.c_int, C.c_int
    sigs = {
        "dco_default_params": (st, [C.POINTER(Params)]),
        "dco_stereo_create": (st, [C.POINTER(P), i, i, i, C.POINTER(Params), P]),
        "dco_stereo_destroy": (None, [P]),
        "dco_stereo_set_stream": (st, [P, P]),
        "dco_census": (st, [P, P, P, P]),
        "dco_cost_volume": (st, [P, i, P, P, P, P, P, P]),
        "dco_aggregate": (st, [P, P, P, P]),
        "dco_wta_lrcheck": (st, [P, P, P, P, P, P, P]),
        "dco_stereo_match": (st, [P, P, P, P, P]),
        "dco_stereo_last_disparities": (st, [P, P, P]),
        "dco_stereo_profile": (st, [P, i]),
        "dco_stereo_stage_times": (st, [P, P, i, P]),
        "dco_batch_create": (st, [C.POINTER(P), i, P, P, P, C.POINTER(Params), P]),
        "dco_batch_destroy": (None, [P]),
        "dco_batch_match": (st, [P, P, P, P, P]),
        "dco_batch_tile": (st, [P, i, P, P, P]),
        "dco_soft_forward": (st, [P, i, P, P, P, P, P]),
        "dco_soft_backward": (st, [P, i, P, P, P, P, P, P, P]),
        "dco_soft_backward_reuse": (st, [P, i, P, P, P, P, P, P, P]),
        "dco_vote_refine": (st, [P, P, P, P, P, i, P, P, P]),
        "dco_stereo_match_half": (st, [P, P, P, i, i, C.c_float, P, P, P]),
        "dco_stereo_match_noalloc": (st, [i, i, i, C.POINTER(Params), P, P, P, P, P]),
        "dco_densify_default_params": (st, [C.POINTER(DensifyParams)]),
        "dco_densify_create": (st, [C.POINTER(P), i, i, C.POINTER(DensifyParams), P]),
        "dco_densify_destroy": (None, [P]),
        "dco_densify_run": (st, [P, P, P, P, P, P, P]),
        "dco_densify_stats": (st, [P, C.POINTER(C.c_int), C.POINTER(C.c_double)]),
        "dco_contour_default_params": (st, [C.POINTER(ContourParams)]),
        "dco_contour_create": (st, [C.POINTER(P), i, i, C.POINTER(ContourParams), P]),
        "dco_contour_destroy": (None, [P]),
        "dco_contour_run": (st, [P, P, P, P, P, P, P]),
        "dco_contour_launches": (st, [P, C.POINTER(C.c_int)]),
        "dco_status_string": (C.c_char_p, [st]),
        "dco_last_error": (C.c_char_p, []),
        "dco_stereo_agg_slices": (st, [P, i, i, i, P]),
        "dco_debug_fail_alloc": (None, [i]),
        "dco_debug_live_allocations": (C.c_long, []),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(status):
    if status != DCO_OK:
        msg = lib().dco_last_error().decode(errors="replace")
        raise DcoError(status, msg)
    return status
