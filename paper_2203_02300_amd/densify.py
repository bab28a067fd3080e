"""Torch-facing binding of the depth densification (Sec. 6, Eq. 13-20).

Argument marshalling only: the solve runs in the library's kernels
(``dco_densify_*`` in include/dco_stereo.h).
"""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import DensifyParams, check, lib
from .api import _need, _ptr, _stream

PARAM_NAMES = tuple(n for n, _ in DensifyParams._fields_)


class Densifier:
    """Dense depth of an H x W grid from a sparse depth map, the previous
    frame's depth, the depth contour and the two texture maps of Eq. 16-17."""

    def __init__(self, W, H, **params):
        p = DensifyParams()
        check(lib().dco_densify_default_params(C.byref(p)))
        for k, v in params.items():
            if k not in PARAM_NAMES:
                raise TypeError(f"unknown densification parameter {k!r}")
            setattr(p, k, v)
        self.W, self.H = W, H
        self._h = C.c_void_p()
        check(lib().dco_densify_create(C.byref(self._h), W, H, C.byref(p), _stream()))

    def run(self, Ds, Bdp, Mfuse, MI, Dpre=None, out=None):
        shape = (self.H, self.W)
        for t, n in ((Ds, "Ds"), (Mfuse, "Mfuse"), (MI, "MI")):
            _need(t, n, torch.float32, shape)
        _need(Bdp, "Bdp", torch.uint8, shape)
        if Dpre is not None:
            _need(Dpre, "Dpre", torch.float32, shape)
        if out is None:
            out = torch.empty(shape, dtype=torch.float32, device=Ds.device)
        _need(out, "out", torch.float32, shape)
        check(lib().dco_densify_run(self._h, _ptr(Ds), _ptr(Dpre), _ptr(Bdp), _ptr(Mfuse),
                                    _ptr(MI), _ptr(out)))
        return out

    def stats(self):
        """(iterations, final relative residual) of the last solve."""
        it = C.c_int()
        rel = C.c_double()
        check(lib().dco_densify_stats(self._h, C.byref(it), C.byref(rel)))
        return it.value, rel.value

    def close(self):
        if self._h:
            lib().dco_densify_destroy(self._h)
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
