"""Torch-facing binding of the depth contour extraction (Sec. 5).

Argument marshalling only: every step runs in the library's kernels
(``dco_contour_*`` in include/dco_stereo.h).
"""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import ContourParams, check, lib
from .api import _need, _ptr, _stream

PARAM_NAMES = tuple(n for n, _ in ContourParams._fields_)


class ContourFilter:
    """Depth contour of W x H frames from the frame and its past and future
    optical flows on the (H // 2) x (W // 2) grid."""

    def __init__(self, W, H, **params):
        p = ContourParams()
        check(lib().dco_contour_default_params(C.byref(p)))
        for k, v in params.items():
            if k not in PARAM_NAMES:
                raise TypeError(f"unknown contour parameter {k!r}")
            setattr(p, k, v)
        self.W, self.H = W, H
        self._h = C.c_void_p()
        check(lib().dco_contour_create(C.byref(self._h), W, H, C.byref(p), _stream()))

    def run(self, rgb, past, future):
        """Returns (B uint8, MI float32, Mn float32)."""
        H, W, h, w = self.H, self.W, self.H // 2, self.W // 2
        _need(rgb, "rgb", torch.uint8, (H, W, 3))
        _need(past, "past", torch.float32, (h, w, 2))
        _need(future, "future", torch.float32, (h, w, 2))
        B = torch.empty((H, W), dtype=torch.uint8, device=rgb.device)
        MI = torch.empty((H, W), dtype=torch.float32, device=rgb.device)
        Mn = torch.empty((h, w), dtype=torch.float32, device=rgb.device)
        check(lib().dco_contour_run(self._h, _ptr(rgb), _ptr(past), _ptr(future), _ptr(B),
                                    _ptr(MI), _ptr(Mn)))
        return B, MI, Mn

    def launches(self):
        n = C.c_int()
        check(lib().dco_contour_launches(self._h, C.byref(n)))
        return n.value

    def close(self):
        if self._h:
            lib().dco_contour_destroy(self._h)
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
