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


# Rows of context a band of the oracle needs so that its own rows equal the
# whole-frame result: 2 L1 for the two vertical aggregation stages plus L1
# for the vertical arms of the pixels in those ranges; every Eq. 4 vote pass
# reads the pass before it over a further L1 rows.
BAND_HALO = 51


def oracle_banded(L, R, D, nbands=None, threads=None, **kw):
    """The whole-frame oracle match computed in row bands on host threads
    (the oracle's C calls release the GIL): (disp, valid, dL, dR)."""
    import concurrent.futures as cf
    import os
    H, W = L.shape[:2]
    threads = threads or max(1, min(16, len(os.sched_getaffinity(0))))
    nbands = nbands or threads
    halo = BAND_HALO + 17 * kw.get("vote_iters", 0)
    edges = np.linspace(0, H, nbands + 1).round().astype(int)
    disp = np.empty((H, W), np.float32)
    valid = np.empty((H, W), np.uint8)
    dL = np.empty((H, W), np.int16)
    dR = np.empty((H, W), np.int16)

    def run(i):
        y0, y1 = int(edges[i]), int(edges[i + 1])
        a, b = max(0, y0 - halo), min(H, y1 + halo)
        d, v, l, r = oracle.match(L[a:b], R[a:b], D, **kw)
        disp[y0:y1], valid[y0:y1] = d[y0 - a:y1 - a], v[y0 - a:y1 - a]
        dL[y0:y1], dR[y0:y1] = l[y0 - a:y1 - a], r[y0 - a:y1 - a]

    with cf.ThreadPoolExecutor(threads) as ex:
        list(ex.map(run, range(nbands)))
    return disp, valid, dL, dR


def thread_map(fn, items, threads=None):
    """fn over items on host threads (for oracle calls, which release the GIL)."""
    import concurrent.futures as cf
    import os
    threads = threads or max(1, min(16, len(os.sched_getaffinity(0))))
    with cf.ThreadPoolExecutor(threads) as ex:
        return list(ex.map(fn, items))
