"""GPU parity of the differentiable soft-argmin form against the FP64 oracle.

The oracle's forward is pinned against a numpy region-enumeration shadow and
its analytic gradient against central finite differences (CPU tests).  Here
the GPU float path is compared with it: dhat within 1e-3 absolute and each
gradient component within 1e-3 of the largest component (float32 sums of at
most 35 terms per range and float32 softmax).
"""
import numpy as np
import pytest

import oracle
from gpu_util import dev, host
from paper_2203_02300_amd import synth

pytestmark = pytest.mark.gpu


def pairs(seed, W, H, D, n):
    return [synth.make_slanted_pair(W, H, D, seed + i, n_planes=3, dmin=2.0, dmax=D - 3.0,
                                    noise_sigma=2.0, occl_strip_frac=0.03) for i in range(n)]


def oracle_inputs(p):
    L, R = p["left"], p["right"]
    return L, R, oracle.census(oracle.grey(L)), oracle.census(oracle.grey(R)), oracle.arms(L)


def l1_seed(dhat, gt, occ):
    """d loss / d dhat of loss = mean over non-occluded pixels of |dhat - gt|."""
    m = ~occ
    g = np.sign(dhat - gt) * m / max(1, m.sum())
    return g


@pytest.fixture(scope="module")
def torch_mod():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("T", [1.0, 0.1])
def test_soft_forward_and_gradient_match_oracle(torch_mod, T):
    torch = torch_mod
    from paper_2203_02300_amd import StereoMatcher
    from paper_2203_02300_amd.soft import soft_argmin_disparity, soft_forward
    W, H, D, B = 160, 48, 24, 2
    ps = pairs(300, W, H, D, B)
    theta_np = np.array([10.0, 30.0, T])
    with StereoMatcher(W, H, D) as m:
        L = dev(np.stack([p["left"] for p in ps]))
        R = dev(np.stack([p["right"] for p in ps]))
        theta = torch.tensor(theta_np, dtype=torch.float32, device="cuda", requires_grad=True)
        dhat = soft_argmin_disparity(m, L, R, theta)
        gt = torch.from_numpy(np.stack([p["disp"] for p in ps])).cuda()
        occ = torch.from_numpy(np.stack([p["occluded"] for p in ps])).cuda()
        loss = ((dhat - gt).abs() * (~occ)).sum() / (~occ).sum()
        loss.backward()
        g_gpu = host(theta.grad).astype(np.float64)
        _, lse = soft_forward(m, L, R, theta.detach())
        dh_gpu, lse_gpu = host(dhat.detach()), host(lse)
    g_ref = np.zeros(3)
    for b, p in enumerate(ps):
        Lb, Rb, cL, cR, aL = oracle_inputs(p)
        dh, vol = oracle.soft_forward(Lb, Rb, cL, cR, aL, D, lam_ad=10.0, lam_c=30.0, T=T,
                                      want_volume=True)
        assert np.abs(dh_gpu[b] - dh).max() < 1e-3
        z = -vol / T
        mx = z.max(axis=0)
        lse_ref = mx + np.log(np.exp(z - mx).sum(axis=0))
        assert np.abs(lse_gpu[b] - lse_ref).max() < 1e-3 * max(1.0, np.abs(lse_ref).max())
    # the loss normalises over both pairs together
    occ_all = np.stack([p["occluded"] for p in ps])
    nvalid = (~occ_all).sum()
    for b, p in enumerate(ps):
        Lb, Rb, cL, cR, aL = oracle_inputs(p)
        gd = np.sign(dh_gpu[b] - p["disp"]) * (~p["occluded"]) / nvalid
        g_ref += oracle.soft_grad(Lb, Rb, cL, cR, aL, D, gd, lam_ad=10.0, lam_c=30.0, T=T)
    scale = np.abs(g_ref).max()
    assert scale > 0
    assert np.all(np.abs(g_gpu - g_ref) <= 1e-3 * scale), (g_gpu, g_ref)


def test_soft_backward_reuse_is_bit_identical(torch_mod):
    """dco_soft_backward_reuse right after its forward (the held aggregation
    is used), twice in a row, after a forward on another theta (recomputed),
    and after a recomputing backward: the same bits as dco_soft_backward."""
    torch = torch_mod
    from paper_2203_02300_amd import StereoMatcher
    from paper_2203_02300_amd.soft import soft_backward, soft_forward
    W, H, D, B = 160, 48, 24, 2
    ps = pairs(320, W, H, D, B)
    rng = np.random.default_rng(7)
    with StereoMatcher(W, H, D) as m:
        L = dev(np.stack([p["left"] for p in ps]))
        R = dev(np.stack([p["right"] for p in ps]))
        th1 = torch.tensor([10.0, 30.0, 1.0], dtype=torch.float32, device="cuda")
        th2 = torch.tensor([12.0, 25.0, 0.5], dtype=torch.float32, device="cuda")
        gd = dev(rng.normal(0, 1e-3, (B, H, W)).astype(np.float32))
        dh1, lse1 = soft_forward(m, L, R, th1)
        g_ref = host(soft_backward(m, L, R, th1, dh1, lse1, gd))
        dh1, lse1 = soft_forward(m, L, R, th1)
        g1 = host(soft_backward(m, L, R, th1, dh1, lse1, gd, reuse=True))
        g2 = host(soft_backward(m, L, R, th1, dh1, lse1, gd, reuse=True))
        dh2, lse2 = soft_forward(m, L, R, th2)  # replaces the held aggregation
        g3 = host(soft_backward(m, L, R, th1, dh1, lse1, gd, reuse=True))
        g4 = host(soft_backward(m, L, R, th2, dh2, lse2, gd))
        g5 = host(soft_backward(m, L, R, th2, dh2, lse2, gd, reuse=True))
    for g in (g1, g2, g3):
        assert np.array_equal(g.view(np.int32), g_ref.view(np.int32)), (g, g_ref)
    assert np.array_equal(g5.view(np.int32), g4.view(np.int32)), (g5, g4)
    assert not np.array_equal(g4, g_ref)


def test_soft_small_temperature_approaches_wta(torch_mod):
    torch = torch_mod
    from paper_2203_02300_amd import StereoMatcher
    from paper_2203_02300_amd.soft import soft_forward
    W, H, D = 128, 40, 16
    p = pairs(310, W, H, D, 1)[0]
    Lb, Rb, cL, cR, aL = oracle_inputs(p)
    _, vol = oracle.soft_forward(Lb, Rb, cL, cR, aL, D, lam_c=30.0, T=1.0, want_volume=True)
    srt = np.sort(vol, axis=0)
    clear = (srt[1] - srt[0]) > 0.02
    with StereoMatcher(W, H, D) as m:
        theta = torch.tensor([10.0, 30.0, 1e-3], dtype=torch.float32, device="cuda")
        dh, _ = soft_forward(m, dev(Lb), dev(Rb), theta)
        dh = host(dh)[0]
    assert clear.sum() > 100
    assert np.abs(dh[clear] - vol.argmin(axis=0)[clear]).max() < 1e-3


def test_soft_full_size_batch(torch_mod):
    """8 pairs of 640x480, D=64 (the benchmarked configuration): deterministic
    gradients, batch gradient = sum of single-pair gradients, and pair 0
    against the oracle."""
    torch = torch_mod
    from paper_2203_02300_amd import StereoMatcher
    from paper_2203_02300_amd.soft import soft_backward, soft_forward
    ps = synth.config_c5()
    W, H, D = 640, 480, 64
    theta = torch.tensor([10.0, 30.0, 1.0], dtype=torch.float32, device="cuda")
    with StereoMatcher(W, H, D) as m:
        L = dev(np.stack([p["left"] for p in ps]))
        R = dev(np.stack([p["right"] for p in ps]))
        dhat, lse = soft_forward(m, L, R, theta)
        gt = np.stack([p["disp"] for p in ps])
        occ = np.stack([p["occluded"] for p in ps])
        gd = l1_seed(host(dhat), gt, occ).astype(np.float32)
        gdt = dev(gd)
        g1 = host(soft_backward(m, L, R, theta, dhat, lse, gdt)).astype(np.float64)
        g2 = host(soft_backward(m, L, R, theta, dhat, lse, gdt)).astype(np.float64)
        assert np.array_equal(g1, g2)
        gsum = np.zeros(3)
        for b in range(len(ps)):
            d1, l1 = soft_forward(m, L[b:b + 1], R[b:b + 1], theta)
            assert np.array_equal(host(d1)[0], host(dhat)[b])
            gb = soft_backward(m, L[b:b + 1], R[b:b + 1], theta, d1, l1, gdt[b:b + 1].contiguous())
            gsum += host(gb).astype(np.float64)
            if b == 0:
                g0 = host(gb).astype(np.float64)
        assert np.all(np.abs(gsum - g1) <= 1e-4 * np.abs(g1).max())
    Lb, Rb, cL, cR, aL = oracle_inputs(ps[0])
    dh_ref = oracle.soft_forward(Lb, Rb, cL, cR, aL, D, lam_ad=10.0, lam_c=30.0, T=1.0)
    assert np.abs(host(dhat)[0] - dh_ref).max() < 1e-3
    g_ref = oracle.soft_grad(Lb, Rb, cL, cR, aL, D, gd[0].astype(np.float64), lam_ad=10.0,
                             lam_c=30.0, T=1.0)
    assert np.all(np.abs(g0 - g_ref) <= 1e-3 * np.abs(g_ref).max()), (g0, g_ref)


def test_soft_rejects_oversized_batches(torch_mod):
    """B * D above the column passes' grid limit is refused before any work."""
    from paper_2203_02300_amd import StereoMatcher, _lib
    L = _lib.lib()
    with StereoMatcher(64, 48, 16) as m:
        assert L.dco_soft_forward(m._h, 5000, None, None, None, None, None) == -2
        assert b"B*D" in L.dco_last_error()
        assert L.dco_soft_forward(m._h, 0, None, None, None, None, None) == -1
    with StereoMatcher(2100, 8, 4) as m:  # wider than the row passes' LDS allows
        assert L.dco_soft_forward(m._h, 1, None, None, None, None, None) == -2
        assert b"W <= 2048" in L.dco_last_error()
        assert L.dco_soft_backward(m._h, 1, None, None, None, None, None, None, None) == -2


@pytest.mark.parametrize("W,H,D,B", [(2048, 9, 6, 1), (23, 11, 5, 3), (333, 53, 9, 2)])
def test_soft_widest_and_smallest_frames(torch_mod, W, H, D, B):
    """The widest frame the row passes' LDS takes (W = 2048), a small ragged
    batch, and rows that end inside a 256-column chunk with W not a multiple
    of 4 over more rows than one turn of the column passes' ring: dhat, lse
    and the theta gradient against the FP64 oracle."""
    torch = torch_mod
    from paper_2203_02300_amd import StereoMatcher
    from paper_2203_02300_amd.soft import soft_backward, soft_forward
    rng = np.random.default_rng(W + B)
    Ls = rng.integers(0, 256, (B, H, W, 3), dtype=np.uint8)
    Rs = np.roll(Ls, -2, axis=2)
    theta_np = np.array([10.0, 30.0, 1.0])
    print(f"soft {B} x {W}x{H} D={D}", flush=True)
    gd = rng.normal(0, 1e-3, (B, H, W)).astype(np.float32)
    with StereoMatcher(W, H, D) as m:
        L, R = dev(Ls), dev(Rs)
        theta = torch.tensor(theta_np, dtype=torch.float32, device="cuda")
        dhat, lse = soft_forward(m, L, R, theta)
        g = soft_backward(m, L, R, theta, dhat, lse, dev(gd))
        dh_gpu, lse_gpu, g_gpu = host(dhat), host(lse), host(g).astype(np.float64)
    g_ref = np.zeros(3)
    for b in range(B):
        cL, cR = oracle.census(oracle.grey(Ls[b])), oracle.census(oracle.grey(Rs[b]))
        aL = oracle.arms(Ls[b])
        dh, vol = oracle.soft_forward(Ls[b], Rs[b], cL, cR, aL, D, lam_ad=10.0, lam_c=30.0,
                                      T=1.0, want_volume=True)
        assert np.abs(dh_gpu[b] - dh).max() < 1e-3
        z = -vol
        mx = z.max(axis=0)
        lse_ref = mx + np.log(np.exp(z - mx).sum(axis=0))
        assert np.abs(lse_gpu[b] - lse_ref).max() < 1e-3 * max(1.0, np.abs(lse_ref).max())
        g_ref += oracle.soft_grad(Ls[b], Rs[b], cL, cR, aL, D, gd[b].astype(np.float64),
                                  lam_ad=10.0, lam_c=30.0, T=1.0)
    scale = np.abs(g_ref).max()
    assert scale > 0
    assert np.all(np.abs(g_gpu - g_ref) <= 1e-3 * scale), (g_gpu, g_ref)


def test_soft_every_pair_of_the_benchmark_batch(torch_mod):
    """All 8 pairs of 640x480, D = 64 (the benchmarked differentiable
    workload): dhat of every pair against the FP64 oracle, and the batch
    gradient per component against the oracle's within 1e-4 of that
    component's magnitude sum M_k (oracle.soft_grad_mag: the same chain with
    every term replaced by its absolute value, so M_k bounds the sum of the
    absolute contributions).  A float32 evaluation keeps each of those terms
    to a few float32 roundings (~1e-6 relative: A2 from FP64 prefix sums,
    float softmax, FP64 adjoints), so its error is a small multiple of
    1e-6 M_k; cancellation between contributions (the lambda_census
    component is ~1 % of its M_k) cannot inflate it."""
    torch = torch_mod
    from paper_2203_02300_amd import StereoMatcher
    from paper_2203_02300_amd.soft import soft_backward, soft_forward
    from gpu_util import thread_map
    ps = synth.config_c5()
    W, H, D = 640, 480, 64
    print("soft, 8 pairs of 640x480 D=64: GPU forward and backward", flush=True)
    theta = torch.tensor([10.0, 30.0, 1.0], dtype=torch.float32, device="cuda")
    with StereoMatcher(W, H, D) as m:
        L = dev(np.stack([p["left"] for p in ps]))
        R = dev(np.stack([p["right"] for p in ps]))
        dhat, lse = soft_forward(m, L, R, theta)
        gt = np.stack([p["disp"] for p in ps])
        occ = np.stack([p["occluded"] for p in ps])
        dh_gpu = host(dhat)
        gd = l1_seed(dh_gpu, gt, occ).astype(np.float32)
        g_gpu = host(soft_backward(m, L, R, theta, dhat, lse, dev(gd))).astype(np.float64)

    def ref(b):
        Lb, Rb, cL, cR, aL = oracle_inputs(ps[b])
        kw = dict(lam_ad=10.0, lam_c=30.0, T=1.0)
        dh = oracle.soft_forward(Lb, Rb, cL, cR, aL, D, **kw)
        g = oracle.soft_grad(Lb, Rb, cL, cR, aL, D, gd[b].astype(np.float64), **kw)
        M = oracle.soft_grad_mag(Lb, Rb, cL, cR, aL, D, gd[b].astype(np.float64), **kw)
        return dh, g, M

    print("soft, 8 pairs: FP64 oracle on host threads", flush=True)
    refs = thread_map(ref, range(len(ps)))
    for b, (dh, _, _) in enumerate(refs):
        err = np.abs(dh_gpu[b] - dh).max()
        print(f"pair {b}: max |dhat - oracle| = {err:.3g} px", flush=True)
        assert err < 1e-3, b
    g_ref = sum(r[1] for r in refs)
    M = sum(r[2] for r in refs)
    ratio = np.abs(g_gpu - g_ref) / M
    print(f"grad gpu {g_gpu}, oracle {g_ref}, M {M}, |diff| / M {ratio}", flush=True)
    assert np.all(M > 0) and np.all(ratio <= 1e-4), (g_gpu, g_ref, M)
