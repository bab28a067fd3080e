"""GPU parity of the Eq. 4 region vote (Sec. 4.3) against the CPU oracle.

The voted integer maps, validity and the sub-pixel disparities are compared
bit for bit: the vote counts integers, and the output step repeats the WTA
parabola in the same float operations.  Inputs come from the oracle's own
stages.  Calls go through the C ABI.
"""
import numpy as np
import pytest

import oracle
from gpu_util import case, dev, host, oracle_stages

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


@pytest.mark.parametrize("name", ["c1", "ragged", "patches", "c2"])
def test_vote_refine_bit_exact(torch_mod, name):
    from paper_2203_02300_amd import StereoMatcher
    L, R, D = case(name)
    H, W = L.shape[:2]
    st = oracle_stages(name)
    print(f"vote_refine {name} {W}x{H} D={D}", flush=True)
    with StereoMatcher(W, H, D) as m:
        args = (dev(st["armsL"]), dev(st["aggL"]), dev(st["dL"]), dev(st["valid"]))
        for iters in (0, 1, 2, 3):
            disp, valid, dv = m.vote_refine(*args, iters)
            want_dv = oracle.vote(st["dL"], st["valid"], st["armsL"], D, iters)
            want_disp, want_valid = oracle.vote_finish(st["aggL"], want_dv)
            assert np.array_equal(host(dv), want_dv), iters
            assert np.array_equal(host(valid), want_valid), iters
            assert np.array_equal(host(disp).view(np.uint32), want_disp.view(np.uint32)), iters


@pytest.mark.parametrize("name,iters", [("c1", 1), ("c1", 2), ("ragged", 2), ("c2", 2)])
def test_match_with_vote_bit_exact(torch_mod, name, iters):
    from paper_2203_02300_amd import StereoMatcher
    L, R, D = case(name)
    H, W = L.shape[:2]
    print(f"match+vote {name} {W}x{H} D={D} iters={iters}", flush=True)
    want_disp, want_valid, want_dL, _ = oracle.match(L, R, D, vote_iters=iters)
    with StereoMatcher(W, H, D, vote_iters=iters) as m:
        disp, valid = m.match(dev(L), dev(R))
        dL, _ = m.last_disparities()
        assert np.array_equal(host(dL), want_dL)
        assert np.array_equal(host(valid), want_valid)
        assert np.array_equal(host(disp).view(np.uint32), want_disp.view(np.uint32))


def test_vote_on_degenerate_maps(torch_mod):
    """All pixels invalid, all equal, and a map with out-of-range values."""
    from paper_2203_02300_amd import StereoMatcher
    L, R, D = case("c1")
    H, W = L.shape[:2]
    st = oracle_stages("c1")
    rng = np.random.default_rng(3)
    maps = [
        (st["dL"], np.zeros((H, W), np.uint8)),
        (np.full((H, W), 5, np.int16), np.ones((H, W), np.uint8)),
        (rng.integers(-3, D + 3, (H, W)).astype(np.int16), (rng.random((H, W)) < 0.7).astype(np.uint8)),
    ]
    with StereoMatcher(W, H, D) as m:
        for dmap, vmap in maps:
            disp, valid, dv = m.vote_refine(dev(st["armsL"]), dev(st["aggL"]), dev(dmap), dev(vmap), 2)
            want_dv = oracle.vote(dmap, vmap, st["armsL"], D, 2)
            want_disp, want_valid = oracle.vote_finish(st["aggL"], want_dv)
            assert np.array_equal(host(dv), want_dv)
            assert np.array_equal(host(valid), want_valid)
            assert np.array_equal(host(disp).view(np.uint32), want_disp.view(np.uint32))


def test_vote_full_size_1280x720_crops(torch_mod):
    """1280x720, D=128, two passes in the one-call path: validity unchanged by
    the vote, determinism, the staged call equal to the one call, and
    bit-exact agreement with the oracle on crop interiors (margins widened by
    two region radii for the two passes)."""
    from paper_2203_02300_amd import StereoMatcher
    L, R, D = case("c3")
    H, W = L.shape[:2]
    print("match+vote c3 1280x720 D=128 iters=2", flush=True)
    with StereoMatcher(W, H, D) as plain:
        pdisp, pvalid = plain.match(dev(L), dev(R))
        pvalid = host(pvalid)
    with StereoMatcher(W, H, D, vote_iters=2) as m:
        gL, gR = dev(L), dev(R)
        disp, valid = m.match(gL, gR)
        disp2, valid2 = m.match(gL, gR)
        disp, valid = host(disp), host(valid)
        assert np.array_equal(disp.view(np.uint32), host(disp2).view(np.uint32))
        assert np.array_equal(valid, host(valid2))
        assert np.array_equal(valid, pvalid)
        assert np.all(disp[valid == 0] == 0)
        # the vote changes some pixels but keeps most
        changed = np.count_nonzero((disp != host(pdisp)) & (valid == 1))
        assert 0 < changed < 0.5 * valid.sum()
    rng = np.random.default_rng(11)
    mx, my, iw, ih = D + 100, 100, 96, 32
    for _ in range(2):
        x0 = int(rng.integers(0, W - iw + 1))
        y0 = int(rng.integers(0, H - ih + 1))
        cx0, cx1 = max(0, x0 - mx), min(W, x0 + iw + mx)
        cy0, cy1 = max(0, y0 - my), min(H, y0 + ih + my)
        want_disp, want_valid, _, _ = oracle.match(L[cy0:cy1, cx0:cx1], R[cy0:cy1, cx0:cx1], D,
                                                   vote_iters=2)
        sl = (slice(y0 - cy0, y0 - cy0 + ih), slice(x0 - cx0, x0 - cx0 + iw))
        assert np.array_equal(want_valid[sl], valid[y0:y0 + ih, x0:x0 + iw])
        assert np.array_equal(want_disp[sl].view(np.uint32),
                              disp[y0:y0 + ih, x0:x0 + iw].view(np.uint32))


def test_batch_rejects_vote(torch_mod):
    import ctypes as C
    from paper_2203_02300_amd import _lib
    L = _lib.lib()
    p = _lib.Params()
    L.dco_default_params(C.byref(p))
    p.vote_iters = 2
    W, H, D = (C.c_int * 1)(64), (C.c_int * 1)(48), (C.c_int * 1)(16)
    b = C.c_void_p()
    assert L.dco_batch_create(C.byref(b), 1, W, H, D, C.byref(p), None) == -1
    assert b"vote" in L.dco_last_error()


@pytest.mark.parametrize("W,H,D", [(9, 7, 1), (33, 7, 8), (190, 9, 60)])
def test_vote_edge_shapes(torch_mod, W, H, D):
    from paper_2203_02300_amd import StereoMatcher, synth
    p = synth.make_shift_pair(W, H, min(3, D - 1) if D > 1 else 0, 40 + W, texture="patches")
    want_disp, want_valid, _, _ = oracle.match(p["left"], p["right"], D, vote_iters=2)
    with StereoMatcher(W, H, D, vote_iters=2) as m:
        disp, valid = m.match(dev(p["left"]), dev(p["right"]))
        assert np.array_equal(host(valid), want_valid)
        assert np.array_equal(host(disp).view(np.uint32), want_disp.view(np.uint32))
