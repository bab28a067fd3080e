"""Whole-frame GPU parity at the benchmarked sizes.

* The 1280x720 D = 128 pair: every pixel of disp, valid, dL and dR from the
  one-call match against the oracle (computed in row bands on the host
  threads, which equal the whole-frame oracle bit for bit); the same with two
  Eq. 4 vote passes.
* The aggregated volumes the one-call match leaves in its scratch (Eq. 2 as
  two stages, cost fused into the aggregation), element by element: every
  slice of both views at 640x480 D = 64 and at 437x93 with an odd D = 37,
  and bands of rows at 1280x720 D = 128 (top, middle, bottom) against the
  oracle run on the band.
* All 32 pairs of the batched workload against the oracle (not only against
  the one-call match).
Tolerance 0 everywhere: the parity contract of this path is bit-exact.
"""
import numpy as np
import pytest

import oracle
from gpu_util import BAND_HALO, case, dev, host, oracle_banded, thread_map

pytestmark = pytest.mark.gpu


def _bits(a):
    return np.ascontiguousarray(a, np.float32).view(np.uint32)


def _diff(a, b):
    return int(np.count_nonzero(a != b))


@pytest.fixture(scope="module")
def c3_gpu():
    import torch
    from paper_2203_02300_amd import StereoMatcher
    L, R, D = case("c3")
    H, W = L.shape[:2]
    print(f"c3 whole frame {W}x{H} D={D}: GPU match", flush=True)
    with StereoMatcher(W, H, D) as m:
        disp, valid = m.match(dev(L), dev(R))
        dL, dR = m.last_disparities()
        torch.cuda.synchronize()
        out = dict(disp=host(disp), valid=host(valid), dL=host(dL), dR=host(dR))
    return out


def test_c3_whole_frame_matches_oracle(c3_gpu):
    L, R, D = case("c3")
    print("c3 whole frame: oracle in row bands", flush=True)
    od, ov, odL, odR = oracle_banded(L, R, D)
    g = c3_gpu
    assert _diff(g["dL"], odL) == 0, "dL"
    assert _diff(g["dR"], odR) == 0, "dR"
    assert _diff(g["valid"], ov) == 0, "valid"
    assert _diff(_bits(g["disp"]), _bits(od)) == 0, "disp"
    assert 0.5 < ov.mean() < 0.99


def test_c3_whole_frame_with_two_vote_passes():
    import torch
    from paper_2203_02300_amd import StereoMatcher
    L, R, D = case("c3")
    H, W = L.shape[:2]
    print("c3 whole frame, vote_iters = 2: GPU match", flush=True)
    with StereoMatcher(W, H, D, vote_iters=2) as m:
        disp, valid = m.match(dev(L), dev(R))
        torch.cuda.synchronize()
        gd, gv = host(disp), host(valid)
    print("c3 whole frame, vote_iters = 2: oracle in row bands", flush=True)
    od, ov, _, _ = oracle_banded(L, R, D, vote_iters=2)
    assert _diff(gv, ov) == 0
    assert _diff(_bits(gd), _bits(od)) == 0


def test_fused_volume_c2_every_slice():
    import torch
    from paper_2203_02300_amd import StereoMatcher
    L, R, D = case("c2")
    H, W = L.shape[:2]
    print(f"fused volume {W}x{H} D={D}: GPU", flush=True)
    with StereoMatcher(W, H, D) as m:
        m.match(dev(L), dev(R))
        aL, aR = host(m.agg_slices(0)), host(m.agg_slices(1))
        torch.cuda.synchronize()
    print(f"fused volume {W}x{H} D={D}: oracle", flush=True)
    st = oracle.stages(L, R, D)
    assert _diff(_bits(aL), _bits(st["aggL"])) == 0
    assert _diff(_bits(aR), _bits(st["aggR"])) == 0


def test_fused_volume_odd_range_every_slice():
    """An odd disparity range: the last slice has no partner in the paired
    slice order of the scratch volumes.  Every slice of both views (decoded by
    the slice export), dL, dR, disp and valid against the oracle."""
    import torch
    from paper_2203_02300_amd import StereoMatcher
    L, R, _ = case("ragged")
    H, W = L.shape[:2]
    D = 37
    print(f"fused volume {W}x{H} D={D}: GPU", flush=True)
    with StereoMatcher(W, H, D) as m:
        disp, valid = m.match(dev(L), dev(R))
        dL, dR = m.last_disparities()
        aL, aR = host(m.agg_slices(0)), host(m.agg_slices(1))
        last = host(m.agg_slices(0, D - 1, 1))
        torch.cuda.synchronize()
        gd, gv, gdl, gdr = host(disp), host(valid), host(dL), host(dR)
    print(f"fused volume {W}x{H} D={D}: oracle", flush=True)
    st = oracle.stages(L, R, D)
    assert _diff(_bits(aL), _bits(st["aggL"])) == 0
    assert _diff(_bits(aR), _bits(st["aggR"])) == 0
    assert _diff(_bits(last[0]), _bits(st["aggL"][D - 1])) == 0
    assert _diff(gdl, st["dL"]) == 0 and _diff(gdr, st["dR"]) == 0
    assert _diff(gv, st["valid"]) == 0
    assert _diff(_bits(gd), _bits(st["disp"])) == 0


def test_fused_volume_c3_bands():
    import torch
    from paper_2203_02300_amd import StereoMatcher
    L, R, D = case("c3")
    H, W = L.shape[:2]
    bands = [(0, 24), (348, 372), (H - 24, H)]
    print(f"fused volume {W}x{H} D={D}: GPU", flush=True)
    with StereoMatcher(W, H, D) as m:
        m.match(dev(L), dev(R))
        gpu = []
        for y0, y1 in bands:
            gpu.append(tuple(host(m.agg_slices(v)[:, y0:y1]) for v in (0, 1)))
        torch.cuda.synchronize()

    def ref(band):
        y0, y1 = band
        a, b = max(0, y0 - BAND_HALO), min(H, y1 + BAND_HALO)
        st = oracle.stages(L[a:b], R[a:b], D)
        return st["aggL"][:, y0 - a:y1 - a], st["aggR"][:, y0 - a:y1 - a]

    print(f"fused volume {W}x{H} D={D}: oracle on {len(bands)} bands", flush=True)
    refs = thread_map(ref, bands)
    for (gL, gR), (rL, rR) in zip(gpu, refs):
        assert _diff(_bits(gL), _bits(rL)) == 0
        assert _diff(_bits(gR), _bits(rR)) == 0


def test_batched_workload_every_pair_matches_oracle():
    import torch
    from paper_2203_02300_amd import BatchMatcher, synth
    pairs = synth.config_c4()
    shapes = [(p["W"], p["H"], p["D"]) for p in pairs]
    print(f"batched workload: {len(pairs)} pairs on the GPU", flush=True)
    with BatchMatcher(shapes) as bm:
        disps, valids = bm.match([dev(p["left"]) for p in pairs],
                                 [dev(p["right"]) for p in pairs])
        torch.cuda.synchronize()
        got = [(host(d), host(v)) for d, v in zip(disps, valids)]
    print("batched workload: oracle, every pair in row bands", flush=True)
    bad = []
    for i, p in enumerate(pairs):
        od, ov, _, _ = oracle_banded(p["left"], p["right"], p["D"])
        gd, gv = got[i]
        if _diff(gv, ov) or _diff(_bits(gd), _bits(od)):
            bad.append((i, shapes[i], _diff(gv, ov), _diff(_bits(gd), _bits(od))))
    assert not bad, bad
