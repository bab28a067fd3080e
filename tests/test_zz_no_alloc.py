"""The allocation-free one-call match (dco_stereo_match_noalloc) called through
the C ABI gives the same bits as dco_stereo_match on a handle: two calls in a
row on one GPU, the second with a smaller input, then other parameters.  The
static scratch is shared by every call, so each call must clear and rewrite
all it reads."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import dev, host

pytestmark = pytest.mark.gpu


def _noalloc(L, R, D, **params):
    import torch
    from paper_2203_02300_amd import _lib
    from paper_2203_02300_amd.api import default_params
    H, W = L.shape[:2]
    p = default_params(**params)
    disp = torch.empty((H, W), dtype=torch.float32, device="cuda")
    valid = torch.empty((H, W), dtype=torch.uint8, device="cuda")
    st = _lib.lib().dco_stereo_match_noalloc(
        W, H, D, C.byref(p), C.c_void_p(torch.cuda.current_stream().cuda_stream),
        C.c_void_p(L.data_ptr()), C.c_void_p(R.data_ptr()), C.c_void_p(disp.data_ptr()),
        C.c_void_p(valid.data_ptr()))
    _lib.check(st)
    torch.cuda.synchronize()
    return host(disp), host(valid)


def _handle(L, R, D, **params):
    import torch
    from paper_2203_02300_amd import StereoMatcher
    H, W = L.shape[:2]
    with StereoMatcher(W, H, D, **params) as m:
        disp, valid = m.match(L, R)
        torch.cuda.synchronize()
        return host(disp), host(valid)


def _same(a, b):
    (da, va), (db, vb) = a, b
    return (np.array_equal(va, vb) and
            np.array_equal(da.view(np.uint32), db.view(np.uint32)))


def _pair(W, H, D, seed):
    from paper_2203_02300_amd import synth
    p = synth.make_slanted_pair(W=W, H=H, D=D, seed=seed)
    return dev(p["left"]), dev(p["right"])


def test_two_calls_in_a_row_second_smaller():
    cases = [(640, 360, 64, 31), (333, 101, 37, 32)]
    for W, H, D, seed in cases:
        print(f"noalloc vs handle: {W}x{H} D={D} seed {seed}", flush=True)
        L, R = _pair(W, H, D, seed)
        got, want = _noalloc(L, R, D), _handle(L, R, D)
        assert _same(got, want), (W, H, D)
        assert 0.3 < want[1].mean() < 1.0


def test_parameters_apply():
    L, R = _pair(320, 240, 48, 33)
    for kw in (dict(vote_iters=2), dict(agg_iters=1), dict(lr_max_diff=1, subpixel=0)):
        print(f"noalloc vs handle: 320x240 D=48 {kw}", flush=True)
        assert _same(_noalloc(L, R, 48, **kw), _handle(L, R, 48, **kw)), kw


def test_too_large_is_rejected_before_any_launch():
    import torch
    from paper_2203_02300_amd import _lib
    from paper_2203_02300_amd.api import default_params
    p = default_params()
    x = torch.zeros(1, dtype=torch.uint8, device="cuda")
    st = _lib.lib().dco_stereo_match_noalloc(1280, 720, 128, C.byref(p), None,
                                              C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()),
                                              C.c_void_p(x.data_ptr()), C.c_void_p(x.data_ptr()))
    assert st == -2
    assert b"static scratch" in _lib.lib().dco_last_error()
