"""Helpers shared by the GPU tests (seeded cases, device transfer, crops)."""
from __future__ import annotations

import functools

import numpy as np

import oracle
from paper_2203_02300_amd import synth


def dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def host(t):
    return t.cpu().numpy()


@functools.lru_cache(maxsize=None)
def case(name):
    """Seeded input pairs of the parity tests: (left, right, D)."""
    if name == "c1":
        p = synth.config_c1()
        return p["left"], p["right"], 16
    if name == "ragged":       # 3 column strips, ragged tail, rows not a multiple of the chunk
        p = synth.make_slanted_pair(437, 93, 40, 7, n_planes=4, dmin=3.0, dmax=36.0,
                                    noise_sigma=2.0, occl_strip_frac=0.03)
        return p["left"], p["right"], 40
    if name == "patches":      # long arms everywhere
        p = synth.make_shift_pair(300, 77, 9, 5, texture="patches")
        return p["left"], p["right"], 24
    if name == "c2":
        p = synth.config_c2()
        return p["left"], p["right"], 64
    if name == "c3":
        p = synth.config_c3()
        return p["left"], p["right"], 128
    raise KeyError(name)


@functools.lru_cache(maxsize=None)
def oracle_stages(name, **kw):
    L, R, D = case(name)
    return oracle.stages(L, R, D, **kw)


def crop_windows(W, H, D, n, seed, interior=(96, 32)):
    """Crop windows whose interior is unaffected by the crop.

    A matcher output at (x, y) depends on pixels within 2*L1 (region) + L1
    (arms of region pixels) + 4 (census) columns of x and of its partners
    x - d .. x + d, and within 2*L1 + L1 + 3 rows of y.  The margins below
    cover that; where the crop meets the image border no margin is needed.
    """
    rng = np.random.default_rng(seed)
    mx, my = D + 60, 60
    iw, ih = interior
    out = []
    for _ in range(n):
        x0 = int(rng.integers(0, W - iw + 1))
        y0 = int(rng.integers(0, H - ih + 1))
        cx0, cx1 = max(0, x0 - mx), min(W, x0 + iw + mx)
        cy0, cy1 = max(0, y0 - my), min(H, y0 + ih + my)
        out.append(((cx0, cx1, cy0, cy1), (x0, x0 + iw, y0, y0 + ih)))
    return out
