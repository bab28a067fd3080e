"""Allocation failures leave nothing behind.

dco_debug_fail_alloc(k) makes the k-th allocation from then on fail as if
device memory were exhausted.  For every create entry point, k runs from 1
until the create succeeds: each failing create must return DCO_ERR_OOM with
*out cleared and free exactly what it allocated (the library's count of live
allocations returns to where it was), and the successful handle must free
everything on destroy.  A double free would drive the count below its
starting value and fail the same check.  The soft path's lazily allocated
scratch is covered the same way, followed by a working call."""
import ctypes as C

import numpy as np
import pytest

from gpu_util import dev

pytestmark = pytest.mark.gpu

OOM = -4


def _lib():
    from paper_2203_02300_amd import _lib
    return _lib


def _create(what):
    m = _lib()
    L = m.lib()
    h = C.c_void_p()
    if what == "stereo":
        p = m.Params()
        L.dco_default_params(C.byref(p))
        st = L.dco_stereo_create(C.byref(h), 96, 40, 16, C.byref(p), None)
        return st, h, (lambda: L.dco_stereo_destroy(h))
    if what == "batch":
        p = m.Params()
        L.dco_default_params(C.byref(p))
        arr = C.c_int * 2
        st = L.dco_batch_create(C.byref(h), 2, arr(96, 64), arr(40, 32), arr(16, 8), C.byref(p),
                                None)
        return st, h, (lambda: L.dco_batch_destroy(h))
    if what == "densify":
        p = m.DensifyParams()
        L.dco_densify_default_params(C.byref(p))
        st = L.dco_densify_create(C.byref(h), 64, 48, C.byref(p), None)
        return st, h, (lambda: L.dco_densify_destroy(h))
    if what == "contour":
        p = m.ContourParams()
        L.dco_contour_default_params(C.byref(p))
        st = L.dco_contour_create(C.byref(h), 64, 48, C.byref(p), None)
        return st, h, (lambda: L.dco_contour_destroy(h))
    raise KeyError(what)


@pytest.mark.parametrize("what", ["stereo", "batch", "densify", "contour"])
def test_failed_create_frees_what_it_allocated(monkeypatch, what):
    import torch
    monkeypatch.setenv("DCO_AUTOTUNE", "0")   # the batch create's tuner would allocate too
    L = _lib().lib()
    torch.cuda.synchronize()
    base = L.dco_debug_live_allocations()
    print(f"injected allocation failures: {what}", flush=True)
    k = 1
    try:
        while True:
            L.dco_debug_fail_alloc(k)
            st, h, destroy = _create(what)
            if st == 0:
                L.dco_debug_fail_alloc(0)
                assert L.dco_debug_live_allocations() > base
                destroy()
                assert L.dco_debug_live_allocations() == base
                break
            assert st == OOM, (what, k, st)
            assert b"injected" in L.dco_last_error() or b"pinned" in L.dco_last_error()
            assert not h.value, (what, k)
            assert L.dco_debug_live_allocations() == base, (what, k)
            k += 1
            assert k < 400
    finally:
        L.dco_debug_fail_alloc(0)
    assert k > 3, f"{what} made only {k - 1} allocations"


def test_soft_scratch_failure_then_success():
    import torch
    from paper_2203_02300_amd import StereoMatcher
    from paper_2203_02300_amd.soft import soft_forward
    L = _lib().lib()
    base = L.dco_debug_live_allocations()
    rng = np.random.default_rng(1)
    W, H, D = 64, 24, 8
    Ls = rng.integers(0, 256, (1, H, W, 3), dtype=np.uint8)
    Rs = np.roll(Ls, -2, axis=2)
    theta = torch.tensor([10.0, 30.0, 1.0], dtype=torch.float32, device="cuda")
    with StereoMatcher(W, H, D) as m:
        inner = L.dco_debug_live_allocations()
        for k in (1, 3, 7):
            L.dco_debug_fail_alloc(k)
            try:
                with pytest.raises(RuntimeError, match="DCO_ERR_OOM"):
                    soft_forward(m, dev(Ls), dev(Rs), theta)
            finally:
                L.dco_debug_fail_alloc(0)
        dhat, _ = soft_forward(m, dev(Ls), dev(Rs), theta)
        torch.cuda.synchronize()
        assert torch.isfinite(dhat).all()
        assert L.dco_debug_live_allocations() > inner
    assert L.dco_debug_live_allocations() == base
