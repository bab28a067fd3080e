"""CPU oracle of the adaptive AD-census stereo matcher -- TEST INFRASTRUCTURE.

Plain single-threaded C (``dco_oracle.c``) behind numpy wrappers.  Only the
tests, the smoke check and the benchmark's CPU-baseline leg may import this
package; the product library never does, and shares no code with it.

Each wrapper takes and returns numpy arrays in the layouts of the C file:
images ``H x W x 3`` uint8, per-pixel maps ``H x W``, arms ``H x W x 4``
(left, right, up, down), volumes ``D x H x W``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dco_oracle.c")
_SO = os.path.join(_HERE, "libdco_oracle.so")
_lib = None

DEFAULTS = dict(cw=9, ch=7, L1=17, tau1=20, gamma=1.0, eps=0.8, lam_ad=10.0, lam_c=40.0,
                iters=2, maxdiff=0, subpixel=1, vote_iters=0)


def build(force: bool = True) -> str:
    """Compile the oracle with the host compiler (no fused multiply-add)."""
    if force or not os.path.exists(_SO):
        tmp = _SO + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-std=c99", "-fPIC",
                               "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _SO)
    return _SO


def swap_library(path):
    """Load the oracle from another build of ``dco_oracle.c`` (the mutation
    tests load deliberately broken copies); ``None`` returns to the default
    build.  Returns the path that was in use before."""
    global _lib, _override
    prev, _override, _lib = _override, path, None
    return prev


_override = None


def lib():
    global _lib
    if _lib is None:
        so = _override
        if so is None:
            so = _SO
            if not os.path.exists(_SO) or os.path.getmtime(_SO) < os.path.getmtime(_SRC):
                build(force=True)
        L = C.CDLL(so)
        P = C.c_void_p
        i, f, dbl = C.c_int, C.c_float, C.c_double
        sig = {
            "orc_grey": [P, i, i, P],
            "orc_census": [P, i, i, i, i, P],
            "orc_arms": [P, i, i, i, i, P],
            "orc_tables": [i, f, f, f, f, P, P, P, P],
            "orc_cost": [i, P, P, P, P, P, i, i, i, i, f, f, f, f, P],
            "orc_aggregate": [P, P, i, i, i, i, P],
            "orc_wta": [P, i, i, i, P, P],
            "orc_lrcheck": [P, P, P, i, i, i, i, P, P],
            "orc_match": [P, P, i, i, i, i, i, i, i, f, f, f, f, i, i, i, i, P, P, P, P],
            "orc_vote": [P, P, P, i, i, i, i, P],
            "orc_vote_finish": [P, P, i, i, i, i, P, P],
            "orc_downscale2": [P, i, i, P],
            "orc_flow_fuse": [P, P, i, i, i, P],
            "orc_flow_terms": [P, i, i, P, P],
            "orc_contour": [P, i, i, P, i, i, f, f, f, P, P],
            "orc_depth_half": [P, P, i, i, f, P, P],
            "orc_soft_forward": [P, P, P, P, P, i, i, i, dbl, dbl, dbl, dbl, dbl, P, P],
            "orc_soft_grad": [P, P, P, P, P, i, i, i, dbl, dbl, dbl, dbl, dbl, P, P],
            "orc_soft_grad_mag": [P, P, P, P, P, i, i, i, dbl, dbl, dbl, dbl, dbl, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = None
        _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def grey(rgb):
    rgb = _c(rgb, np.uint8)
    H, W = rgb.shape[:2]
    out = np.empty((H, W), np.uint8)
    lib().orc_grey(_p(rgb), W, H, _p(out))
    return out


def census(Y, cw=9, ch=7):
    Y = _c(Y, np.uint8)
    H, W = Y.shape
    out = np.empty((H, W), np.uint64)
    lib().orc_census(_p(Y), W, H, cw, ch, _p(out))
    return out


def arms(rgb, L1=17, tau1=20):
    rgb = _c(rgb, np.uint8)
    H, W = rgb.shape[:2]
    out = np.empty((H, W, 4), np.uint8)
    lib().orc_arms(_p(rgb), W, H, L1, tau1, _p(out))
    return out


def tables(L1=17, gamma=1.0, eps=0.8, lam_ad=10.0, lam_c=40.0):
    a = np.empty(L1 + 1, np.float32)
    b = np.empty(L1 + 1, np.float32)
    ta = np.empty(766, np.float32)
    tc = np.empty(65, np.float32)
    lib().orc_tables(L1, gamma, eps, lam_ad, lam_c, _p(a), _p(b), _p(ta), _p(tc))
    return a, b, ta, tc


def cost_q(ref, L, R, cL, cR, arms_ref, D, L1=17, gamma=1.0, eps=0.8, lam_ad=10.0, lam_c=40.0):
    """Integer raw costs q (D x H x W int32); the cost is q * 2^-20."""
    L = _c(L, np.uint8)
    R = _c(R, np.uint8)
    cL = _c(cL, np.uint64)
    cR = _c(cR, np.uint64)
    arms_ref = _c(arms_ref, np.uint8)
    H, W = L.shape[:2]
    q = np.empty((D, H, W), np.int32)
    lib().orc_cost(ref, _p(L), _p(R), _p(cL), _p(cR), _p(arms_ref), W, H, D, L1, gamma, eps,
                   lam_ad, lam_c, _p(q))
    return q


def aggregate(q, arms_ref, iters=2):
    q = _c(q, np.int32)
    arms_ref = _c(arms_ref, np.uint8)
    D, H, W = q.shape
    out = np.empty((D, H, W), np.float32)
    lib().orc_aggregate(_p(q), _p(arms_ref), W, H, D, iters, _p(out))
    return out


def wta(agg):
    agg = _c(agg, np.float32)
    D, H, W = agg.shape
    d = np.empty((H, W), np.int16)
    dl = np.empty((H, W), np.float32)
    lib().orc_wta(_p(agg), W, H, D, _p(d), _p(dl))
    return d, dl


def lrcheck(dL, deltaL, dR, maxdiff=0, subpixel=1):
    dL = _c(dL, np.int16)
    dR = _c(dR, np.int16)
    deltaL = _c(deltaL, np.float32)
    H, W = dL.shape
    disp = np.empty((H, W), np.float32)
    valid = np.empty((H, W), np.uint8)
    lib().orc_lrcheck(_p(dL), _p(deltaL), _p(dR), W, H, maxdiff, subpixel, _p(disp), _p(valid))
    return disp, valid


def match(L, R, D, cw=9, ch=7, L1=17, tau1=20, gamma=1.0, eps=0.8, lam_ad=10.0, lam_c=40.0,
          iters=2, maxdiff=0, subpixel=1, vote_iters=0):
    """Full plain matcher: returns (disp, valid, dL, dR).  With vote_iters > 0
    the LR-valid left disparities go through the Eq. 4 vote (dL stays the
    WTA map)."""
    L = _c(L, np.uint8)
    R = _c(R, np.uint8)
    H, W = L.shape[:2]
    disp = np.empty((H, W), np.float32)
    valid = np.empty((H, W), np.uint8)
    dL = np.empty((H, W), np.int16)
    dR = np.empty((H, W), np.int16)
    lib().orc_match(_p(L), _p(R), W, H, D, cw, ch, L1, tau1, gamma, eps, lam_ad, lam_c, iters,
                    maxdiff, subpixel, vote_iters, _p(disp), _p(valid), _p(dL), _p(dR))
    return disp, valid, dL, dR


def flow_fuse(past, future, R=2):
    """Eq. 6-12 with the box filter and normalisation of Sec. 5.2-5.3.2:
    the normalised fused amplitude on the flows' grid (h x w float32)."""
    past = _c(past, np.float32)
    future = _c(future, np.float32)
    h, w = past.shape[:2]
    out = np.empty((h, w), np.float32)
    lib().orc_flow_fuse(_p(past), _p(future), w, h, R, _p(out))
    return out


def flow_terms(F):
    """Amplitude M (Eq. 6-8) and score (Eq. 9-11) of one flow field, h x w."""
    F = _c(F, np.float32)
    h, w = F.shape[:2]
    M = np.empty((h, w), np.float32)
    S = np.empty((h, w), np.float32)
    lib().orc_flow_terms(_p(F), w, h, _p(M), _p(S))
    return M, S


def contour(Y, Mn, Thigh=0.06, Tlow=0.03, Tdepth=0.03):
    """Depth-gated Canny (Sec. 5.3): (B uint8 0/1, MI float32), H x W."""
    Y = _c(Y, np.uint8)
    Mn = _c(Mn, np.float32)
    H, W = Y.shape
    h, w = Mn.shape
    B = np.empty((H, W), np.uint8)
    MI = np.empty((H, W), np.float32)
    lib().orc_contour(_p(Y), W, H, _p(Mn), w, h, Thigh, Tlow, Tdepth, _p(B), _p(MI))
    return B, MI


def depth_contour(rgb, past, future, R=2, Thigh=0.06, Tlow=0.03, Tdepth=0.03):
    """The whole Sec. 5 filter given the flows: (B, MI, Mn)."""
    Mn = flow_fuse(past, future, R)
    B, MI = contour(grey(rgb), Mn, Thigh, Tlow, Tdepth)
    return B, MI, Mn


def downscale2(rgb):
    """2 x 2 block mean (rounded half up) of an H x W x 3 image."""
    rgb = _c(rgb, np.uint8)
    H, W = rgb.shape[:2]
    out = np.empty((H // 2, W // 2, 3), np.uint8)
    lib().orc_downscale2(_p(rgb), W, H, _p(out))
    return out


def depth_half(disp, valid, fB):
    """(full-scale disparity, depth) of a quarter-size match."""
    disp = _c(disp, np.float32)
    valid = _c(valid, np.uint8)
    H, W = disp.shape
    dfull = np.empty((H, W), np.float32)
    depth = np.empty((H, W), np.float32)
    lib().orc_depth_half(_p(disp), _p(valid), W, H, fB, _p(dfull), _p(depth))
    return dfull, depth


def match_half(L, R, D, fB, **kw):
    """The quarter-size front end: reduce both images, match with D
    quarter-size disparities, double the disparity and convert to depth.
    Returns (dfull, depth, valid) on the (H / 2) x (W / 2) grid."""
    l2, r2 = downscale2(L), downscale2(R)
    disp, valid, _, _ = match(l2, r2, D, **kw)
    dfull, depth = depth_half(disp, valid, fB)
    return dfull, depth, valid


def vote(d, valid, arms, D, iters):
    """Eq. 4 region vote: returns the H x W int16 map (-1 where invalid)."""
    d = _c(d, np.int16)
    valid = _c(valid, np.uint8)
    arms = _c(arms, np.uint8)
    H, W = d.shape
    out = np.empty((H, W), np.int16)
    lib().orc_vote(_p(d), _p(valid), _p(arms), W, H, D, iters, _p(out))
    return out


def vote_finish(agg, dv, subpixel=1):
    """Disparity output of a voted map: (disp, valid)."""
    agg = _c(agg, np.float32)
    dv = _c(dv, np.int16)
    D, H, W = agg.shape
    disp = np.empty((H, W), np.float32)
    valid = np.empty((H, W), np.uint8)
    lib().orc_vote_finish(_p(agg), _p(dv), W, H, D, subpixel, _p(disp), _p(valid))
    return disp, valid


def stages(L, R, D, cw=9, ch=7, L1=17, tau1=20, gamma=1.0, eps=0.8, lam_ad=10.0, lam_c=40.0,
           iters=2, maxdiff=0, subpixel=1):
    """Every intermediate of the plain matcher, stage by stage, as a dict."""
    out = {}
    out["cenL"] = census(grey(L), cw, ch)
    out["cenR"] = census(grey(R), cw, ch)
    out["armsL"] = arms(L, L1, tau1)
    out["armsR"] = arms(R, L1, tau1)
    for ref, tag in ((0, "L"), (1, "R")):
        q = cost_q(ref, L, R, out["cenL"], out["cenR"], out["arms" + tag], D, L1, gamma, eps,
                   lam_ad, lam_c)
        out["q" + tag] = q
        out["agg" + tag] = aggregate(q, out["arms" + tag], iters)
        out["d" + tag], out["delta" + tag] = wta(out["agg" + tag])
    out["disp"], out["valid"] = lrcheck(out["dL"], out["deltaL"], out["dR"], maxdiff, subpixel)
    return out


def soft_forward(L, R, cL, cR, armsL, D, gamma=1.0, eps=0.8, lam_ad=10.0, lam_c=30.0, T=1.0,
                 want_volume=False):
    """FP64 soft-argmin forward: returns dhat (and the aggregated volume)."""
    L = _c(L, np.uint8)
    R = _c(R, np.uint8)
    H, W = L.shape[:2]
    dhat = np.empty((H, W), np.float64)
    vol = np.empty((D, H, W), np.float64) if want_volume else None
    lib().orc_soft_forward(_p(L), _p(R), _p(_c(cL, np.uint64)), _p(_c(cR, np.uint64)),
                           _p(_c(armsL, np.uint8)), W, H, D, gamma, eps, lam_ad, lam_c, T,
                           _p(dhat), _p(vol))
    return (dhat, vol) if want_volume else dhat


def soft_grad(L, R, cL, cR, armsL, D, gdhat, gamma=1.0, eps=0.8, lam_ad=10.0, lam_c=30.0,
              T=1.0):
    """FP64 gradient of sum(gdhat * dhat) w.r.t. (lambda_ad, lambda_census, T)."""
    L = _c(L, np.uint8)
    R = _c(R, np.uint8)
    H, W = L.shape[:2]
    g = np.empty(3, np.float64)
    lib().orc_soft_grad(_p(L), _p(R), _p(_c(cL, np.uint64)), _p(_c(cR, np.uint64)),
                        _p(_c(armsL, np.uint8)), W, H, D, gamma, eps, lam_ad, lam_c, T,
                        _p(_c(gdhat, np.float64)), _p(g))
    return g


def soft_grad_mag(L, R, cL, cR, armsL, D, gdhat, gamma=1.0, eps=0.8, lam_ad=10.0, lam_c=30.0,
                  T=1.0):
    """Per component, the sum of the magnitudes of the terms of soft_grad (a
    bound on the sum of absolute contributions): the scale for the rounding
    error of a float evaluation of the same gradient."""
    L = _c(L, np.uint8)
    R = _c(R, np.uint8)
    H, W = L.shape[:2]
    g = np.empty(3, np.float64)
    lib().orc_soft_grad_mag(_p(L), _p(R), _p(_c(cL, np.uint64)), _p(_c(cR, np.uint64)),
                            _p(_c(armsL, np.uint8)), W, H, D, gamma, eps, lam_ad, lam_c, T,
                            _p(_c(gdhat, np.float64)), _p(g))
    return g
