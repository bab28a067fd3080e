"""GPU parity: every stage of the HIP path against the CPU oracle.

Integer outputs (census codes, arms, WTA indices, validity) and the
fixed-point cost and aggregated volumes are compared bit for bit; the
sub-pixel disparities are compared bit for bit as well (the float operations
follow the same prescribed order on both sides).  Calls go through the C ABI.
"""
import numpy as np
import pytest

import oracle
from gpu_util import case, crop_windows, dev, host, oracle_stages

pytestmark = pytest.mark.gpu

CASES = ["c1", "ragged", "patches", "c2"]


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def matcher(name, **kw):
    from paper_2203_02300_amd import StereoMatcher
    L, R, D = case(name)
    H, W = L.shape[:2]
    return StereoMatcher(W, H, D, **kw)


def u64(t):
    return host(t).view(np.uint64)


@pytest.mark.parametrize("name", CASES)
def test_census_and_arms_bit_exact(torch_mod, name):
    L, R, D = case(name)
    st = oracle_stages(name)
    with matcher(name) as m:
        for img, tag in ((L, "L"), (R, "R")):
            codes, arms = m.census(dev(img))
            assert np.array_equal(u64(codes), st["cen" + tag])
            assert np.array_equal(host(arms), st["arms" + tag])


@pytest.mark.parametrize("name", CASES)
def test_cost_volume_bit_exact(torch_mod, name):
    L, R, D = case(name)
    st = oracle_stages(name)
    with matcher(name) as m:
        dL, dR = dev(L), dev(R)
        cL = dev(st["cenL"].view(np.int64))
        cR = dev(st["cenR"].view(np.int64))
        for ref, tag in ((0, "L"), (1, "R")):
            cost = m.cost_volume(ref, dL, dR, cL, cR, dev(st["arms" + tag]))
            want = (st["q" + tag].astype(np.float64) * 2.0 ** -20).astype(np.float32)
            got = host(cost)
            assert np.array_equal(got, want), (tag, np.argwhere(got != want)[:5])


@pytest.mark.parametrize("name", CASES)
def test_aggregate_bit_exact(torch_mod, name):
    st = oracle_stages(name)
    with matcher(name) as m:
        for tag in ("L", "R"):
            cost = dev((st["q" + tag].astype(np.float64) * 2.0 ** -20).astype(np.float32))
            agg = host(m.aggregate(cost, dev(st["arms" + tag])))
            want = st["agg" + tag]
            bad = np.argwhere(agg != want)
            assert bad.size == 0, (tag, bad[:5], agg[tuple(bad[0])], want[tuple(bad[0])])


@pytest.mark.parametrize("D", [1, 2, 37])
def test_aggregate_odd_and_small_ranges_bit_exact(torch_mod, D):
    """The staged two-stage aggregation takes two slices per workgroup: with
    an odd range the last workgroup has one slice (it reads that slice twice
    and stores one), and D = 1 has only that workgroup."""
    from paper_2203_02300_amd import StereoMatcher
    L, R, _ = case("ragged")
    H, W = L.shape[:2]
    print(f"staged aggregation, ragged {W}x{H} D={D}", flush=True)
    st = oracle.stages(L, R, D)
    with StereoMatcher(W, H, D) as m:
        for tag in ("L", "R"):
            cost = dev((st["q" + tag].astype(np.float64) * 2.0 ** -20).astype(np.float32))
            agg = host(m.aggregate(cost, dev(st["arms" + tag])))
            bad = np.argwhere(agg != st["agg" + tag])
            assert bad.size == 0, (D, tag, bad[:5])


@pytest.mark.parametrize("name", CASES)
def test_wta_lrcheck_bit_exact(torch_mod, name):
    st = oracle_stages(name)
    with matcher(name) as m:
        disp, valid, dL, dR = m.wta_lrcheck(dev(st["aggL"]), dev(st["aggR"]))
        assert np.array_equal(host(dL), st["dL"])
        assert np.array_equal(host(dR), st["dR"])
        assert np.array_equal(host(valid), st["valid"])
        assert np.array_equal(host(disp), st["disp"])


@pytest.mark.parametrize("name", CASES)
def test_one_call_match_bit_exact(torch_mod, name):
    L, R, D = case(name)
    st = oracle_stages(name)
    with matcher(name) as m:
        disp, valid = m.match(dev(L), dev(R))
        dL, dR = m.last_disparities()
        assert np.array_equal(host(dL), st["dL"])
        assert np.array_equal(host(dR), st["dR"])
        assert np.array_equal(host(valid), st["valid"])
        assert np.array_equal(host(disp), st["disp"])


@pytest.mark.parametrize("kw", [
    dict(agg_iters=1),
    dict(arm_L1=5, arm_tau1=12),
    dict(census_w=5, census_h=5, lr_max_diff=1, subpixel=0),
    dict(lambda_ad=7.5, lambda_census=25.0, gamma_L=2.0, eps=0.5, arm_L1=11),
])
def test_parameter_variants_bit_exact(torch_mod, kw):
    L, R, D = case("ragged")
    okw = dict(cw=kw.get("census_w", 9), ch=kw.get("census_h", 7), L1=kw.get("arm_L1", 17),
               tau1=kw.get("arm_tau1", 20), iters=kw.get("agg_iters", 2),
               maxdiff=kw.get("lr_max_diff", 0), subpixel=kw.get("subpixel", 1),
               lam_ad=kw.get("lambda_ad", 10.0), lam_c=kw.get("lambda_census", 40.0),
               gamma=kw.get("gamma_L", 1.0), eps=kw.get("eps", 0.8))
    st = oracle.stages(L, R, D, **okw)
    with matcher("ragged", **kw) as m:
        disp, valid = m.match(dev(L), dev(R))
        dL, dR = m.last_disparities()
        assert np.array_equal(host(dL), st["dL"])
        assert np.array_equal(host(dR), st["dR"])
        assert np.array_equal(host(valid), st["valid"])
        assert np.array_equal(host(disp), st["disp"])
        sdisp, svalid, sdL, sdR = m.match_staged(dev(L), dev(R))
        assert np.array_equal(host(sdisp), st["disp"])
        assert np.array_equal(host(sdL), st["dL"])


@pytest.mark.parametrize("shape", [(9, 7, 1), (9, 7, 8), (33, 7, 32), (190, 9, 60), (260, 41, 5)])
def test_edge_shapes(torch_mod, shape):
    from paper_2203_02300_amd import StereoMatcher
    from paper_2203_02300_amd import synth
    W, H, D = shape
    p = synth.make_shift_pair(W, H, min(3, D - 1) if D > 1 else 0, 40 + W, texture="patches")
    st = oracle.stages(p["left"], p["right"], D)
    with StereoMatcher(W, H, D) as m:
        disp, valid = m.match(dev(p["left"]), dev(p["right"]))
        dL, dR = m.last_disparities()
        assert np.array_equal(host(dL), st["dL"]) and np.array_equal(host(dR), st["dR"])
        assert np.array_equal(host(disp), st["disp"])
        assert np.array_equal(host(valid), st["valid"])


def test_full_size_1280x720_properties_and_crops(torch_mod):
    """1280x720, D=128 in the launch configuration the benchmark times:
    LR invariant, zero fill, staged == one call, run-to-run determinism, and
    bit-exact agreement with the oracle on crop interiors."""
    L, R, D = case("c3")
    H, W = L.shape[:2]
    from paper_2203_02300_amd import StereoMatcher
    with StereoMatcher(W, H, D) as m:
        gL, gR = dev(L), dev(R)
        disp, valid = m.match(gL, gR)
        dL, dR = m.last_disparities()
        disp2, valid2 = m.match(gL, gR)
        disp, valid, dL, dR = host(disp), host(valid), host(dL), host(dR)
        assert np.array_equal(disp, host(disp2)) and np.array_equal(valid, host(valid2))
        # LR invariant and zero fill
        xs = np.arange(W)[None, :].repeat(H, 0)
        ys = np.arange(H)[:, None].repeat(W, 1)
        xr = xs - dL.astype(int)
        ok = xr >= 0
        want = np.zeros((H, W), np.uint8)
        want[ok] = dL[ok] == dR[ys[ok], xr[ok]]
        assert np.array_equal(valid, want)
        assert np.all(disp[valid == 0] == 0)
        assert valid.mean() > 0.5
        sd, sv, sdl, sdr = m.match_staged(gL, gR)
        assert np.array_equal(host(sd), disp) and np.array_equal(host(sdl), dL)
        assert np.array_equal(host(sdr), dR)
    for (cx0, cx1, cy0, cy1), (x0, x1, y0, y1) in crop_windows(W, H, D, 2, seed=5):
        st = oracle.stages(L[cy0:cy1, cx0:cx1], R[cy0:cy1, cx0:cx1], D)
        sl = (slice(y0 - cy0, y1 - cy0), slice(x0 - cx0, x1 - cx0))
        assert np.array_equal(st["dL"][sl], dL[y0:y1, x0:x1])
        assert np.array_equal(st["valid"][sl], valid[y0:y1, x0:x1])
        assert np.array_equal(st["disp"][sl], disp[y0:y1, x0:x1])


def _crop_check(L, R, D, disp, valid, x0, y0, iw=96, ih=32):
    """Oracle on a crop around [x0, x0 + iw) x [y0, y0 + ih) with margins wide
    enough that the interior equals the whole-frame result."""
    H, W = L.shape[:2]
    mx, my = D + 60, 60
    cx0, cx1 = max(0, x0 - mx), min(W, x0 + iw + mx)
    cy0, cy1 = max(0, y0 - my), min(H, y0 + ih + my)
    st = oracle.stages(L[cy0:cy1, cx0:cx1], R[cy0:cy1, cx0:cx1], D)
    sl = (slice(y0 - cy0, y0 - cy0 + ih), slice(x0 - cx0, x0 - cx0 + iw))
    assert np.array_equal(st["valid"][sl], valid[y0:y0 + ih, x0:x0 + iw])
    assert np.array_equal(st["disp"][sl].view(np.uint32),
                          disp[y0:y0 + ih, x0:x0 + iw].view(np.uint32))


@pytest.mark.parametrize("W,H,D", [(16384, 8, 4), (2050, 8, 2048)])
def test_maximum_width_and_range(torch_mod, W, H, D):
    """The widest frame the library takes, and a disparity range near the
    width, against the whole-frame oracle."""
    from paper_2203_02300_amd import StereoMatcher
    rng = np.random.default_rng(W + D)
    L = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
    R = np.roll(L, -3, axis=1)
    print(f"maximum sizes {W}x{H} D={D}", flush=True)
    st = oracle.stages(L, R, D)
    with StereoMatcher(W, H, D) as m:
        disp, valid = m.match(dev(L), dev(R))
        assert np.array_equal(host(valid), st["valid"])
        assert np.array_equal(host(disp).view(np.uint32), st["disp"].view(np.uint32))


def test_maximum_area(torch_mod):
    """16384 x 8192 (W * H = 2^27, the largest area the library takes), D = 2:
    the largest 32-bit buffer offsets of the aggregation kernels.  Crops at
    the four corners and the centre against the oracle."""
    from paper_2203_02300_amd import StereoMatcher
    W, H, D = 16384, 8192, 2
    rng = np.random.default_rng(7)
    L = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
    R = np.roll(L, -1, axis=1)
    print(f"maximum area {W}x{H} D={D}", flush=True)
    with StereoMatcher(W, H, D) as m:
        disp, valid = m.match(dev(L), dev(R))
        disp, valid = host(disp), host(valid)
    for x0, y0 in ((0, 0), (W - 96, 0), (0, H - 32), (W - 96, H - 32), (W // 2, H // 2)):
        _crop_check(L, R, D, disp, valid, x0, y0)
    # a pure shift by one: every pixel whose partner is inside matches d = 1
    assert valid[:, 1:].mean() > 0.99
