"""Batched matcher binding: many pairs of uneven size and disparity range in
one persistent kernel launch replayed from a HIP graph (dco_batch_*)."""
from __future__ import annotations

import ctypes as C

import torch

from ._lib import check, lib
from .api import _need, _stream, default_params


class BatchMatcher:
    """Matches len(shapes) pairs per call; shapes = [(W, H, D), ...].

    The launch is captured on the current stream at construction and replayed
    on it by ``match``; creation runs the tile autotuner (or reads its cache).
    """

    def __init__(self, shapes, **params):
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        n = len(self.shapes)
        arr = C.c_int * n
        self._W = arr(*[s[0] for s in self.shapes])
        self._H = arr(*[s[1] for s in self.shapes])
        self._D = arr(*[s[2] for s in self.shapes])
        self.params = default_params(**params)
        self._h = C.c_void_p()
        check(lib().dco_batch_create(C.byref(self._h), n, self._W, self._H, self._D,
                                     C.byref(self.params), _stream()))

    def tile(self, i):
        """(strip output columns, band rows, disparities per item) of pair i."""
        a, b, c = C.c_int(), C.c_int(), C.c_int()
        check(lib().dco_batch_tile(self._h, int(i), C.byref(a), C.byref(b), C.byref(c)))
        return a.value, b.value, c.value

    def match(self, lefts, rights, disps=None, valids=None):
        n = len(self.shapes)
        if len(lefts) != n or len(rights) != n:
            raise ValueError(f"expected {n} left and right images")
        if disps is None:
            disps = [torch.empty((H, W), dtype=torch.float32, device=lefts[i].device)
                     for i, (W, H, D) in enumerate(self.shapes)]
        if valids is None:
            valids = [torch.empty((H, W), dtype=torch.uint8, device=lefts[i].device)
                      for i, (W, H, D) in enumerate(self.shapes)]
        P = C.c_void_p * n
        tabs = [P(), P(), P(), P()]
        for i, (W, H, D) in enumerate(self.shapes):
            for k, (t, name, dt, shp) in enumerate(((lefts[i], "L", torch.uint8, (H, W, 3)),
                                                    (rights[i], "R", torch.uint8, (H, W, 3)),
                                                    (disps[i], "disp", torch.float32, (H, W)),
                                                    (valids[i], "valid", torch.uint8, (H, W)))):
                _need(t, f"{name}[{i}]", dt, shp)
                tabs[k][i] = t.data_ptr()
        check(lib().dco_batch_match(self._h, *tabs))
        return disps, valids

    def close(self):
        if self._h:
            lib().dco_batch_destroy(self._h)
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
