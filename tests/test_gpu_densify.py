"""GPU densification (Sec. 6, Eq. 13-20) against the oracle's direct FP64
solve.  The GPU runs FP64 preconditioned conjugate gradients to a relative
residual of 1e-9; the error of such a solution is at most the condition
number times that, so the tests ask for 1e-5 of the largest depth (the
prototype solves reach ~1e-8).  Calls go through the C ABI."""
import numpy as np
import pytest

from gpu_util import dev, host
from oracle import densify as dz

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _inputs(W, H, seed, keep=0.7, pre=True):
    from paper_2203_02300_amd import synth
    d = synth.densify_inputs(W, H, seed, keep=keep)
    if not pre:
        d["Dpre"] = np.zeros_like(d["Dpre"])
    return d


@pytest.mark.parametrize("W,H,seed,keep,pre", [(37, 23, 1, 0.7, True), (160, 90, 2, 0.7, True),
                                               (160, 90, 3, 0.05, False),
                                               (320, 180, 4, 0.3, True)])
def test_densify_matches_the_direct_solve(torch_mod, W, H, seed, keep, pre):
    from paper_2203_02300_amd import Densifier
    d = _inputs(W, H, seed, keep, pre)
    print(f"densify {W}x{H} seed={seed} keep={keep} pre={pre}", flush=True)
    want = dz.densify(d["Ds"], d["Dpre"], d["Bdp"], d["Mfuse"], d["MI"])
    with Densifier(W, H) as z:
        D = z.run(dev(d["Ds"]), dev(d["Bdp"]), dev(d["Mfuse"]), dev(d["MI"]),
                  Dpre=dev(d["Dpre"]) if pre else None)
        it, rel = z.stats()
        D = host(D)
    assert rel <= 1e-9 and 0 < it < 4000
    assert np.abs(D - want).max() <= 1e-5 * np.abs(want).max()
    assert np.all(D[want == 0] == 0)  # unanchored regions stay without depth


def test_densify_is_deterministic_and_reusable(torch_mod):
    from paper_2203_02300_amd import Densifier
    d = _inputs(200, 120, 5)
    e = _inputs(200, 120, 6, keep=0.2)
    with Densifier(200, 120, iters_per_launch=4) as z:
        args = (dev(d["Ds"]), dev(d["Bdp"]), dev(d["Mfuse"]), dev(d["MI"]))
        a = host(z.run(*args, Dpre=dev(d["Dpre"])))
        other = host(z.run(dev(e["Ds"]), dev(e["Bdp"]), dev(e["Mfuse"]), dev(e["MI"])))
        b = host(z.run(*args, Dpre=dev(d["Dpre"])))
        assert np.array_equal(a.view(np.uint32), b.view(np.uint32))
        want = dz.densify(e["Ds"], None, e["Bdp"], e["Mfuse"], e["MI"])
        assert np.abs(other - want).max() <= 1e-5 * np.abs(want).max()


def test_densify_degenerate_inputs(torch_mod):
    from paper_2203_02300_amd import Densifier
    W, H = 33, 17
    z0 = np.zeros((H, W), np.float32)
    with Densifier(W, H) as z:
        # no data at all: nothing to solve, depth 0 everywhere
        D = host(z.run(dev(z0), dev(z0.astype(np.uint8)), dev(z0), dev(z0)))
        assert np.all(D == 0) and z.stats()[0] == 0
        # constant data on a few pixels, no contour: constant everywhere
        Ds = z0.copy()
        Ds[3, 4] = Ds[10, 30] = 2.5
        D = host(z.run(dev(Ds), dev(z0.astype(np.uint8)), dev(z0), dev(z0)))
        assert np.allclose(D, 2.5, rtol=1e-6)
    with Densifier(W, H, max_iters=0) as z:
        D = host(z.run(dev(Ds), dev(z0.astype(np.uint8)), dev(z0), dev(z0)))
        assert np.all(D == 0)


@pytest.mark.parametrize("W,H", [(1, 1), (1, 37), (53, 1), (3, 2)])
def test_densify_thin_grids(torch_mod, W, H):
    from paper_2203_02300_amd import Densifier
    rng = np.random.default_rng(W * 100 + H)
    Ds = np.where(rng.random((H, W)) < 0.4, rng.uniform(1, 5, (H, W)), 0).astype(np.float32)
    Ds.flat[0] = 2.0
    B = (rng.random((H, W)) < 0.2).astype(np.uint8)
    Mf = rng.random((H, W)).astype(np.float32)
    MI = rng.random((H, W)).astype(np.float32)
    want = dz.densify(Ds, None, B, Mf, MI)
    with Densifier(W, H) as z:
        D = host(z.run(dev(Ds), dev(B), dev(Mf), dev(MI)))
    assert np.abs(D - want).max() <= 1e-5 * max(np.abs(want).max(), 1e-30)
