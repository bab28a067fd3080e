"""GPU parity of the depth contour filter (Sec. 5) against the CPU oracle:
the fused amplitude Mn and the normalised magnitude MI bit for bit (the same
IEEE operations in the same order, correctly rounded roots), the contour B
bit for bit.  Calls go through the C ABI."""
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


def _check(rgb, past, future, **kw):
    from paper_2203_02300_amd import ContourFilter
    H, W = rgb.shape[:2]
    R = kw.pop("box_radius", 2)
    names = {"Thigh": "T_high", "Tlow": "T_low", "Tdepth": "T_depth"}
    want_B, want_MI, want_Mn = oracle.depth_contour(rgb, past, future, R=R, **kw)
    with ContourFilter(W, H, box_radius=R, **{names[k]: v for k, v in kw.items()}) as f:
        B, MI, Mn = f.run(dev(rgb), dev(past), dev(future))
        n = f.launches()
    assert np.array_equal(host(Mn).view(np.uint32), want_Mn.view(np.uint32))
    assert np.array_equal(host(MI).view(np.uint32), want_MI.view(np.uint32))
    assert np.array_equal(host(B), want_B)
    return host(B), n


@pytest.mark.parametrize("W,H,seed", [(64, 48, 1), (131, 99, 2), (640, 360, 3), (1280, 720, 11)])
def test_contour_bit_exact(torch_mod, W, H, seed):
    from paper_2203_02300_amd import synth
    d = synth.contour_inputs(W, H, seed)
    print(f"contour {W}x{H} seed={seed}", flush=True)
    B, _ = _check(d["rgb"], d["past"], d["future"])
    assert B.any()


@pytest.mark.parametrize("kw", [dict(box_radius=0), dict(box_radius=5), dict(Thigh=0.1, Tlow=0.1),
                                dict(Tdepth=0.0), dict(Thigh=0.5, Tlow=0.01)])
def test_contour_parameters(torch_mod, kw):
    from paper_2203_02300_amd import synth
    d = synth.contour_inputs(200, 120, 4)
    _check(d["rgb"], d["past"], d["future"], **kw)


def test_contour_degenerate_inputs(torch_mod):
    from paper_2203_02300_amd import synth
    d = synth.contour_inputs(96, 64, 5)
    z = np.zeros_like(d["past"])
    B, _ = _check(d["rgb"], z, z)                        # no motion: the gate drops all
    assert not B.any()
    flat = np.full_like(d["rgb"], 90)
    B, _ = _check(flat, d["past"], d["future"])          # no gradient anywhere
    assert not B.any()


def test_long_weak_chain_needs_several_launches(torch_mod):
    # a horizontal step edge whose contrast grows slowly from left to right:
    # with T_high = 0.95 only its right end is strong and with T_low = 0.2
    # the rest is weak, so hysteresis has to cross four 64-wide tiles
    H, W = 160, 256
    Y = np.full((H, W), 50, np.uint8)
    Y[80:] = 50 + 20 + np.arange(W) // 4
    rgb = np.repeat(Y[:, :, None], 3, axis=2)
    past = np.zeros((H // 2, W // 2, 2), np.float32)
    past[..., 0] = np.arange(W // 2, dtype=np.float32)[None, :] * 0.1  # gate open everywhere
    B, n = _check(rgb, past, past, Thigh=0.95, Tlow=0.2)
    assert n > 2 and (B[79] | B[80]).sum() > 0.9 * W


def test_contour_repeated_runs_are_identical(torch_mod):
    from paper_2203_02300_amd import ContourFilter, synth
    d = synth.contour_inputs(320, 180, 6)
    with ContourFilter(320, 180) as f:
        a = [host(t) for t in f.run(dev(d["rgb"]), dev(d["past"]), dev(d["future"]))]
        b = [host(t) for t in f.run(dev(d["rgb"]), dev(d["past"]), dev(d["future"]))]
    for x, y in zip(a, b):
        assert np.array_equal(x.view(np.uint8), y.view(np.uint8))


@pytest.mark.parametrize("W,H", [(2, 2), (3, 5), (70, 17)])
def test_contour_small_and_odd_frames(torch_mod, W, H):
    rng = np.random.default_rng(W * 31 + H)
    rgb = rng.integers(0, 256, (H, W, 3), dtype=np.uint8)
    past = rng.normal(0, 2, (H // 2, W // 2, 2)).astype(np.float32)
    future = rng.normal(0, 2, (H // 2, W // 2, 2)).astype(np.float32)
    _check(rgb, past, future)


def test_hysteresis_over_several_launch_groups(torch_mod):
    """A weak chain across twelve 64-wide tiles: hysteresis needs more than
    one group of launches, and the final state comes from the right buffer."""
    H, W = 96, 768
    Y = np.full((H, W), 50, np.uint8)
    Y[48:] = 50 + 20 + np.arange(W) // 12
    rgb = np.repeat(Y[:, :, None], 3, axis=2)
    past = np.zeros((H // 2, W // 2, 2), np.float32)
    past[..., 0] = np.arange(W // 2, dtype=np.float32)[None, :] * 0.1
    B, n = _check(rgb, past, past, Thigh=0.95, Tlow=0.2)
    assert n > 8 and (B[47] | B[48]).sum() > 0.9 * W
    # the ridge zig-zags across the boundary of two tile rows, which costs a
    # launch per crossing: the count equals the host model's
    Mn = oracle.flow_fuse(past, past, R=2)
    grey = oracle.grey(rgb)
    strong, _ = oracle.contour(grey, Mn, Thigh=0.95, Tlow=0.95)
    cand, _ = oracle.contour(grey, Mn, Thigh=0.2, Tlow=0.2)
    assert n == _launch_model(cand.astype(np.uint8) + strong.astype(np.uint8))


def _launch_model(state, tw=64, th=16):
    """Launch count of the tiled hysteresis: each launch grows strong pixels
    into 8-connected weak ones inside every 64 x 16 tile until the tile is
    stable, reading the tile's one-pixel halo from the launch's input; the
    launches stop after the first one that changes nothing (counted)."""
    H, W = state.shape
    s = state.copy()
    n = 0
    while True:
        n += 1
        pad = np.pad(s, 1)
        new = s.copy()
        for y0 in range(0, H, th):
            for x0 in range(0, W, tw):
                T = pad[y0:y0 + th + 2, x0:x0 + tw + 2].copy()
                h, w = T.shape[0] - 2, T.shape[1] - 2
                while True:
                    strong = T == 2
                    near = np.zeros_like(strong)
                    for dy in (-1, 0, 1):
                        for dx in (-1, 0, 1):
                            near[1:-1, 1:-1] |= strong[1 + dy:1 + dy + h, 1 + dx:1 + dx + w]
                    grow = (T[1:-1, 1:-1] == 1) & near[1:-1, 1:-1]
                    if not grow.any():
                        break
                    T[1:-1, 1:-1][grow] = 2
                new[y0:y0 + h, x0:x0 + w] = T[1:-1, 1:-1]
        if np.array_equal(new, s):
            return n
        s = new


@pytest.mark.parametrize("tiles", [5, 6, 7, 8])
def test_hysteresis_stop_position_in_a_later_group(torch_mod, tiles):
    """Weak chains across 5 .. 8 tiles of 64 columns, seeded strong only in
    the last tile: the launch count n (groups of four launches, the first
    unchanged launch of a group ends it) takes all four values of n mod 4
    above one group, and each n equals the count of a host model of the
    tiled growth; B is bit-exact against the oracle (in _check)."""
    H, W = 96, 64 * tiles
    Y = np.full((H, W), 50, np.uint8)
    Y[41:] = 50 + 20 + np.arange(W) // 12      # ridge on rows 40 / 41: one tile row
    rgb = np.repeat(Y[:, :, None], 3, axis=2)
    past = np.zeros((H // 2, W // 2, 2), np.float32)
    past[..., 0] = np.arange(W // 2, dtype=np.float32)[None, :] * 0.1
    print(f"hysteresis chain across {tiles} tiles", flush=True)
    B, n = _check(rgb, past, past, Thigh=0.95, Tlow=0.2)
    Mn = oracle.flow_fuse(past, past, R=2)
    grey = oracle.grey(rgb)
    strong, _ = oracle.contour(grey, Mn, Thigh=0.95, Tlow=0.95)
    cand, _ = oracle.contour(grey, Mn, Thigh=0.2, Tlow=0.2)
    assert strong[:, : W - 64].sum() == 0 and strong.any()   # seeds in the last tile only
    want = _launch_model(cand.astype(np.uint8) + strong.astype(np.uint8))
    assert n == want == tiles + 1, (n, want)   # 6, 7, 8, 9: every n mod 4
    assert (B[40] | B[41]).sum() > 0.9 * W
