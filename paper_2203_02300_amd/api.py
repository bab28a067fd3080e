"""Torch-facing binding of the gfx950 stereo library.

Argument marshalling only: shape/dtype/device checks, pointers and the
current HIP stream go to the C ABI (include/dco_stereo.h); every step of the
method runs in the library's kernels.  PyTorch supplies device memory and
streams.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib
from ._lib import Params, check, lib

PARAM_NAMES = tuple(n for n, _ in Params._fields_)


def default_params(**overrides) -> Params:
    p = Params()
    check(lib().dco_default_params(C.byref(p)))
    for k, v in overrides.items():
        if k not in PARAM_NAMES:
            raise TypeError(f"unknown matcher parameter {k!r}")
        setattr(p, k, v)
    return p


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, name, dtype, shape):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be a GPU tensor (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)} (got {tuple(t.shape)})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class StereoMatcher:
    """Plain matcher for W x H pairs and disparities 0 .. D-1.

    ``match(L, R)`` runs the whole path in one call; ``census``,
    ``cost_volume``, ``aggregate`` and ``wta_lrcheck`` expose each stage.
    Images are ``H x W x 3`` uint8 GPU tensors; census codes are returned as
    int64 tensors holding the uint64 bit patterns.
    """

    def __init__(self, W, H, D, device=None, **params):
        self.W, self.H, self.D = int(W), int(H), int(D)
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        self.params = default_params(**params)
        self._h = C.c_void_p()
        with torch.cuda.device(self.device):
            check(lib().dco_stereo_create(C.byref(self._h), self.W, self.H, self.D,
                                          C.byref(self.params), _stream()))

    # -- plumbing --
    def _begin(self):
        if not self._h:
            raise _lib.DcoError(-5, "matcher is closed")
        check(lib().dco_stereo_set_stream(self._h, _stream()))

    def _empty(self, shape, dtype):
        return torch.empty(shape, dtype=dtype, device=self.device)

    @property
    def img_shape(self):
        return (self.H, self.W, 3)

    # -- stages --
    def census(self, rgb):
        """Census codes (H x W int64 = uint64 bits) and arms (H x W x 4 uint8)."""
        _need(rgb, "rgb", torch.uint8, self.img_shape)
        self._begin()
        codes = self._empty((self.H, self.W), torch.int64)
        arms = self._empty((self.H, self.W, 4), torch.uint8)
        check(lib().dco_census(self._h, _ptr(rgb), _ptr(codes), _ptr(arms)))
        return codes, arms

    def cost_volume(self, ref, L, R, cenL, cenR, arms_ref, out=None):
        for t, n in ((L, "L"), (R, "R")):
            _need(t, n, torch.uint8, self.img_shape)
        for t, n in ((cenL, "cenL"), (cenR, "cenR")):
            _need(t, n, torch.int64, (self.H, self.W))
        _need(arms_ref, "arms_ref", torch.uint8, (self.H, self.W, 4))
        if out is None:
            out = self._empty((self.D, self.H, self.W), torch.float32)
        _need(out, "out", torch.float32, (self.D, self.H, self.W))
        self._begin()
        check(lib().dco_cost_volume(self._h, int(ref), _ptr(L), _ptr(R), _ptr(cenL), _ptr(cenR),
                                    _ptr(arms_ref), _ptr(out)))
        return out

    def aggregate(self, cost, arms_ref, out=None):
        _need(cost, "cost", torch.float32, (self.D, self.H, self.W))
        _need(arms_ref, "arms_ref", torch.uint8, (self.H, self.W, 4))
        if out is None:
            out = self._empty((self.D, self.H, self.W), torch.float32)
        _need(out, "out", torch.float32, (self.D, self.H, self.W))
        self._begin()
        check(lib().dco_aggregate(self._h, _ptr(cost), _ptr(arms_ref), _ptr(out)))
        return out

    def wta_lrcheck(self, aggL, aggR):
        """Returns (disp, valid, dL, dR)."""
        for t, n in ((aggL, "aggL"), (aggR, "aggR")):
            _need(t, n, torch.float32, (self.D, self.H, self.W))
        self._begin()
        disp = self._empty((self.H, self.W), torch.float32)
        valid = self._empty((self.H, self.W), torch.uint8)
        dL = self._empty((self.H, self.W), torch.int16)
        dR = self._empty((self.H, self.W), torch.int16)
        check(lib().dco_wta_lrcheck(self._h, _ptr(aggL), _ptr(aggR), _ptr(disp), _ptr(valid),
                                    _ptr(dL), _ptr(dR)))
        return disp, valid, dL, dR

    def match(self, L, R, disp=None, valid=None):
        """The whole matcher in one call: returns (disp, valid)."""
        _need(L, "L", torch.uint8, self.img_shape)
        _need(R, "R", torch.uint8, self.img_shape)
        if disp is None:
            disp = self._empty((self.H, self.W), torch.float32)
        if valid is None:
            valid = self._empty((self.H, self.W), torch.uint8)
        _need(disp, "disp", torch.float32, (self.H, self.W))
        _need(valid, "valid", torch.uint8, (self.H, self.W))
        self._begin()
        check(lib().dco_stereo_match(self._h, _ptr(L), _ptr(R), _ptr(disp), _ptr(valid)))
        return disp, valid

    def match_half(self, L2, R2, fB=0.0, want_depth=True):
        """Quarter-size front end on full images of (2H or 2H+1) x (2W or
        2W+1) x 3: returns (disp2, valid, depth) on this handle's W x H grid
        (depth is None when not requested)."""
        H2, W2 = L2.shape[:2]
        _need(L2, "L2", torch.uint8, (H2, W2, 3))
        _need(R2, "R2", torch.uint8, (H2, W2, 3))
        self._begin()
        disp = self._empty((self.H, self.W), torch.float32)
        valid = self._empty((self.H, self.W), torch.uint8)
        depth = self._empty((self.H, self.W), torch.float32) if want_depth else None
        check(lib().dco_stereo_match_half(self._h, _ptr(L2), _ptr(R2), W2, H2, float(fB),
                                          _ptr(disp), _ptr(valid), _ptr(depth)))
        return disp, valid, depth

    def vote_refine(self, armsL, aggL, dL, valid, iters):
        """Eq. 4 region vote on the left integer map: returns (disp, valid, dvote)."""
        _need(armsL, "armsL", torch.uint8, (self.H, self.W, 4))
        _need(aggL, "aggL", torch.float32, (self.D, self.H, self.W))
        _need(dL, "dL", torch.int16, (self.H, self.W))
        _need(valid, "valid", torch.uint8, (self.H, self.W))
        self._begin()
        disp = self._empty((self.H, self.W), torch.float32)
        vout = self._empty((self.H, self.W), torch.uint8)
        dvote = self._empty((self.H, self.W), torch.int16)
        check(lib().dco_vote_refine(self._h, _ptr(armsL), _ptr(aggL), _ptr(dL), _ptr(valid),
                                    int(iters), _ptr(disp), _ptr(vout), _ptr(dvote)))
        return disp, vout, dvote

    def last_disparities(self):
        """Integer (dL, dR) of the last ``match`` call."""
        self._begin()
        dL = self._empty((self.H, self.W), torch.int16)
        dR = self._empty((self.H, self.W), torch.int16)
        check(lib().dco_stereo_last_disparities(self._h, _ptr(dL), _ptr(dR)))
        return dL, dR

    def agg_slices(self, view, d0=0, n=None):
        """Aggregated costs of disparities d0 .. d0 + n - 1 of one view (0 =
        left, 1 = right) left in the scratch by the last ``match``:
        an n x H x W float tensor."""
        self._begin()
        n = self.D - d0 if n is None else n
        out = self._empty((n, self.H, self.W), torch.float32)
        check(lib().dco_stereo_agg_slices(self._h, int(view), int(d0), int(n), _ptr(out)))
        return out

    def match_staged(self, L, R):
        """The same result through the four staged calls (volumes in memory)."""
        cL, aL = self.census(L)
        cR, aR = self.census(R)
        aggs = []
        for ref, arms in ((0, aL), (1, aR)):
            cost = self.cost_volume(ref, L, R, cL, cR, arms)
            aggs.append(self.aggregate(cost, arms))
            del cost
        return self.wta_lrcheck(aggs[0], aggs[1])

    def close(self):
        if self._h:
            lib().dco_stereo_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
