"""GPU tests of the batched matcher: one persistent launch replayed from a
HIP graph must give, for every pair, the same bits as the one-call matcher
(and, for small pairs, as the CPU oracle)."""
import numpy as np
import pytest

import oracle
from gpu_util import dev, host
from paper_2203_02300_amd import synth

pytestmark = pytest.mark.gpu

SMALL = [(160, 96, 24, 400), (300, 77, 40, 401), (200, 150, 16, 402), (96, 64, 8, 403),
         (437, 93, 40, 404)]


def small_pairs():
    out = []
    for W, H, D, seed in SMALL:
        p = synth.make_slanted_pair(W, H, D, seed, n_planes=3, dmin=2.0, dmax=D - 3.0,
                                    noise_sigma=2.0, occl_strip_frac=0.03)
        out.append((p["left"], p["right"], D))
    return out


@pytest.fixture
def tune_cache(tmp_path, monkeypatch):
    path = tmp_path / "autotune.txt"
    monkeypatch.setenv("DCO_AUTOTUNE_CACHE", str(path))
    return path


def plain(L, R, D):
    from paper_2203_02300_amd import StereoMatcher
    H, W = L.shape[:2]
    with StereoMatcher(W, H, D) as m:
        d, v = m.match(dev(L), dev(R))
        return host(d), host(v)


def test_batch_matches_one_call_and_oracle(tune_cache):
    import torch
    from paper_2203_02300_amd import BatchMatcher
    pairs = small_pairs()
    shapes = [(L.shape[1], L.shape[0], D) for L, R, D in pairs]
    with BatchMatcher(shapes) as bm:
        Ls = [dev(L) for L, R, D in pairs]
        Rs = [dev(R) for L, R, D in pairs]
        disps, valids = bm.match(Ls, Rs)
        torch.cuda.synchronize()
        for i, (L, R, D) in enumerate(pairs):
            pd, pv = plain(L, R, D)
            assert np.array_equal(host(disps[i]), pd), i
            assert np.array_equal(host(valids[i]), pv), i
            if i < 2:
                st = oracle.stages(L, R, D)
                assert np.array_equal(host(disps[i]), st["disp"])
        for i, s in enumerate(shapes):
            sw, band, dc = bm.tile(i)
            assert sw > 0 and 1 <= band <= s[1] and 1 <= dc <= s[2]
    assert tune_cache.exists()


def test_graph_replays_with_eager_work_between(tune_cache):
    import torch
    from paper_2203_02300_amd import BatchMatcher
    pairs = small_pairs()
    shapes = [(L.shape[1], L.shape[0], D) for L, R, D in pairs]
    want = [plain(L, R, D) for L, R, D in pairs]
    with BatchMatcher(shapes) as bm:
        Ls = [dev(L) for L, R, D in pairs]
        Rs = [dev(R) for L, R, D in pairs]
        disps = [torch.full((s[1], s[0]), -7.0, device="cuda") for s in shapes]
        valids = [torch.full((s[1], s[0]), 9, dtype=torch.uint8, device="cuda") for s in shapes]
        for rep in range(4):
            junk = torch.randn(1 << 20, device="cuda").sum()  # eager work between replays
            bm.match(Ls, Rs, disps, valids)
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
            for i in range(len(pairs)):
                assert np.array_equal(host(disps[i]), want[i][0]), (rep, i)
                assert np.array_equal(host(valids[i]), want[i][1]), (rep, i)
            for d in disps:
                d.fill_(-7.0)


def test_row_bands_and_disparity_chunks(tune_cache):
    """Force banded, chunked aggregation items through the tuner cache."""
    from paper_2203_02300_amd import BatchMatcher
    L, R, D = small_pairs()[2]
    H, W = L.shape[:2]
    import torch
    arch = torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]
    # an odd chunk: the last pass of each item stores one of its two slices
    tune_cache.write_text(f"{W}x{H}x{D}:{arch}:iters2:s2 37 3\n")
    with BatchMatcher([(W, H, D)]) as bm:
        assert bm.tile(0)[1:] == (37, 3)
        d, v = bm.match([dev(L)], [dev(R)])
        pd, pv = plain(L, R, D)
        assert np.array_equal(host(d[0]), pd) and np.array_equal(host(v[0]), pv)


def test_full_batch_of_32_pairs(tune_cache):
    """The benchmarked batch: 32 pairs of mixed sizes and disparity ranges,
    every pair bit-identical to the one-call matcher."""
    import torch
    from paper_2203_02300_amd import BatchMatcher
    pairs = synth.config_c4()
    shapes = [(p["W"], p["H"], p["D"]) for p in pairs]
    with BatchMatcher(shapes) as bm:
        Ls = [dev(p["left"]) for p in pairs]
        Rs = [dev(p["right"]) for p in pairs]
        disps, valids = bm.match(Ls, Rs)
        torch.cuda.synchronize()
        for i, p in enumerate(pairs):
            pd, pv = plain(p["left"], p["right"], p["D"])
            assert np.array_equal(host(disps[i]), pd), i
            assert np.array_equal(host(valids[i]), pv), i


@pytest.mark.skip(reason="removed design: a single persistent launch whose workgroups waited "
                         "on per-pair completion counters went silent twice on the GPU (the "
                         "counter increment is issued without the L2-bypass bit while the "
                         "waiting load bypasses L2, so on a multi-XCD GPU the update can stay "
                         "in the producer's L2); the batch now runs one work-list kernel per "
                         "stage inside one graph and has no inter-workgroup waits")
def test_single_launch_with_stage_waits():
    pass
