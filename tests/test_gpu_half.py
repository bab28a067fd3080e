"""GPU parity of the quarter-size front end (Sec. 4.4): reduction of the
full pair, the one-call match on the reduced pair, doubling and depth, bit
for bit against the CPU oracle.  Calls go through the C ABI."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _pair(name):
    from paper_2203_02300_amd import synth
    if name == "small":
        p = synth.make_slanted_pair(128, 96, 32, 21, n_planes=3, dmin=2.0, dmax=28.0,
                                    noise_sigma=2.0, occl_strip_frac=0.03)
        return p["left"], p["right"], 16
    if name == "odd":  # odd full sizes: the last column and row are dropped
        p = synth.make_slanted_pair(131, 99, 32, 22, n_planes=3, dmin=2.0, dmax=28.0,
                                    noise_sigma=2.0, occl_strip_frac=0.03)
        return p["left"], p["right"], 16
    if name == "paper":  # the paper's operating point: 1280x720 reduced to 640x360
        p = synth.config_c3()
        return p["left"], p["right"], 64
    raise KeyError(name)


@pytest.mark.parametrize("name,vote", [("small", 0), ("odd", 0), ("small", 2), ("paper", 0),
                                       ("paper", 2)])
def test_match_half_bit_exact(torch_mod, name, vote):
    from paper_2203_02300_amd import StereoMatcher
    L, R, D = _pair(name)
    H2, W2 = L.shape[:2]
    W, H = W2 // 2, H2 // 2
    fB = 1234.5
    print(f"match_half {name} {W2}x{H2} -> {W}x{H} D={D} vote={vote}", flush=True)
    want_d, want_depth, want_valid = oracle.match_half(L, R, D, fB, vote_iters=vote)
    with StereoMatcher(W, H, D, vote_iters=vote) as m:
        d2, valid, depth = m.match_half(dev(L), dev(R), fB)
        assert np.array_equal(host(valid), want_valid)
        assert np.array_equal(host(d2).view(np.uint32), want_d.view(np.uint32))
        assert np.array_equal(host(depth).view(np.uint32), want_depth.view(np.uint32))
        # the reduced pair itself
        d2b, validb, none = m.match_half(dev(L), dev(R), want_depth=False)
        assert none is None and np.array_equal(host(d2b), host(d2))


def test_match_half_rejects_mismatched_sizes(torch_mod):
    import ctypes as C
    from paper_2203_02300_amd import StereoMatcher, _lib
    L, R, D = _pair("small")
    with StereoMatcher(60, 48, 16) as m:
        with pytest.raises(RuntimeError, match="reduce"):
            m.match_half(dev(L), dev(R), 1.0)
    with StereoMatcher(64, 48, 16) as m:
        disp = dev(np.zeros((48, 64), np.float32))
        valid = dev(np.zeros((48, 64), np.uint8))
        depth = dev(np.zeros((48, 64), np.float32))
        st = _lib.lib().dco_stereo_match_half(m._h, C.c_void_p(dev(L).data_ptr()),
                                              C.c_void_p(dev(R).data_ptr()), 128, 96, 0.0,
                                              C.c_void_p(disp.data_ptr()),
                                              C.c_void_p(valid.data_ptr()),
                                              C.c_void_p(depth.data_ptr()))
        assert st == -1 and b"fB" in _lib.lib().dco_last_error()


@pytest.mark.parametrize("W2,H2,D", [(19, 15, 2), (67, 17, 8)])
def test_match_half_edge_shapes(torch_mod, W2, H2, D):
    from paper_2203_02300_amd import StereoMatcher, synth
    p = synth.make_shift_pair(W2, H2, 2, 7 + W2, texture="patches")
    want_d, want_depth, want_valid = oracle.match_half(p["left"], p["right"], D, 10.0)
    with StereoMatcher(W2 // 2, H2 // 2, D) as m:
        d2, valid, depth = m.match_half(dev(p["left"]), dev(p["right"]), 10.0)
        assert np.array_equal(host(valid), want_valid)
        assert np.array_equal(host(d2).view(np.uint32), want_d.view(np.uint32))
        assert np.array_equal(host(depth).view(np.uint32), want_depth.view(np.uint32))
