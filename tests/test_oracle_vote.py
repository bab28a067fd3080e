"""Pins of the oracle's Eq. 4 region vote (Sec. 4.3) against facts fixed
outside the oracle: hand-built regions with known modes, an independent
set-and-counter brute force on tiny inputs, the sub-pixel step of Eq. 3 and
the composition of passes.  CPU only."""
from __future__ import annotations

import collections

import numpy as np
import pytest

import oracle


def _arms_full(H, W, L1=17):
    """Arms of a uniform-colour image: every arm reaches L1 or the border."""
    a = np.empty((H, W, 4), np.uint8)
    for y in range(H):
        for x in range(W):
            a[y, x] = (min(L1, x), min(L1, W - 1 - x), min(L1, y), min(L1, H - 1 - y))
    return a


def _random_arms(rng, H, W, L1):
    """Arbitrary arms that stop at the border (the only property the region
    definition relies on)."""
    a = np.empty((H, W, 4), np.uint8)
    for y in range(H):
        for x in range(W):
            a[y, x] = (rng.integers(0, min(L1, x) + 1), rng.integers(0, min(L1, W - 1 - x) + 1),
                       rng.integers(0, min(L1, y) + 1), rng.integers(0, min(L1, H - 1 - y) + 1))
    return a


def _brute_vote(d, valid, arms, D, iters):
    """Eq. 4 written independently: the region as a set of coordinates, the
    histogram as a Counter, the winner as the least value of maximal count."""
    H, W = d.shape
    cur = {(y, x): int(d[y, x]) for y in range(H) for x in range(W)
           if valid[y, x] and 0 <= d[y, x] < D}
    for _ in range(iters):
        nxt = {}
        for (y, x) in cur:
            l, r, u, dn = (int(v) for v in arms[y, x])
            region = set()
            for yy in range(y - u, y + dn + 1):
                ll, rr = int(arms[yy, x, 0]), int(arms[yy, x, 1])
                region.update((yy, xx) for xx in range(x - ll, x + rr + 1))
            votes = collections.Counter(cur[q] for q in region if q in cur)
            top = max(votes.values())
            nxt[(y, x)] = min(v for v, c in votes.items() if c == top)
        cur = nxt
    out = np.full((H, W), -1, np.int16)
    for (y, x), v in cur.items():
        out[y, x] = v
    return out


def test_vote_keeps_a_constant_field():
    H, W, D = 12, 15, 16
    rng = np.random.default_rng(1)
    d = np.full((H, W), 7, np.int16)
    out = oracle.vote(d, np.ones((H, W), np.uint8), _random_arms(rng, H, W, 17), D, 2)
    assert np.array_equal(out, d)


def test_vote_removes_an_isolated_outlier():
    H, W, D = 20, 20, 16
    d = np.full((H, W), 5, np.int16)
    d[9, 11] = 12
    out = oracle.vote(d, np.ones((H, W), np.uint8), _arms_full(H, W), D, 1)
    assert np.all(out == 5)


def test_vote_tie_goes_to_the_smaller_disparity():
    # two pixels, each region is both pixels: one vote for 5, one for 3
    d = np.array([[5, 3]], np.int16)
    arms = np.array([[[0, 1, 0, 0], [1, 0, 0, 0]]], np.uint8)
    out = oracle.vote(d, np.ones((1, 2), np.uint8), arms, 8, 1)
    assert out.tolist() == [[3, 3]]


def test_invalid_pixels_neither_vote_nor_change():
    d = np.array([[2, 9, 9, 2, 2]], np.int16)
    valid = np.array([[1, 0, 0, 1, 1]], np.uint8)
    arms = _arms_full(1, 5)
    out = oracle.vote(d, valid, arms, 16, 1)
    assert out.tolist() == [[2, -1, -1, 2, 2]]
    # the same map with the 9s valid: three votes for 2 against two for 9,
    # so every pixel takes 2
    out = oracle.vote(d, np.ones((1, 5), np.uint8), arms, 16, 1)
    assert out.tolist() == [[2, 2, 2, 2, 2]]


def test_out_of_range_values_count_as_invalid():
    d = np.array([[4, 40, 4]], np.int16)
    out = oracle.vote(d, np.ones((1, 3), np.uint8), _arms_full(1, 3), 16, 1)
    assert out.tolist() == [[4, -1, 4]]


def test_region_is_the_stage_one_cross():
    # 3 x 3, centre arms reach up and down only; the rows above and below
    # reach right only, so the centre's region is {(0,1),(0,2),(1,1),(2,1),(2,2)}
    arms = np.zeros((3, 3, 4), np.uint8)
    arms[1, 1] = (0, 0, 1, 1)
    arms[0, 1] = (0, 1, 0, 0)
    arms[2, 1] = (0, 1, 0, 0)
    d = np.array([[6, 1, 1], [6, 2, 6], [6, 3, 3]], np.int16)
    out = oracle.vote(d, np.ones((3, 3), np.uint8), arms, 8, 1)
    # centre: votes 1, 1, 2, 3, 3 -> tie between 1 and 3 -> 1
    assert out[1, 1] == 1
    # (1, 0) and (1, 2) have empty arms: their region is themselves
    assert out[1, 0] == 6 and out[1, 2] == 6


@pytest.mark.parametrize("seed", range(6))
def test_vote_matches_an_independent_brute_force(seed):
    rng = np.random.default_rng(100 + seed)
    H, W, D, L1 = 7, 9, 6, 4
    d = rng.integers(0, D, (H, W)).astype(np.int16)
    valid = (rng.random((H, W)) < 0.8).astype(np.uint8)
    arms = _random_arms(rng, H, W, L1)
    for iters in (1, 2, 3):
        assert np.array_equal(oracle.vote(d, valid, arms, D, iters),
                              _brute_vote(d, valid, arms, D, iters))


def test_passes_compose():
    rng = np.random.default_rng(7)
    H, W, D = 16, 20, 10
    d = rng.integers(0, D, (H, W)).astype(np.int16)
    valid = (rng.random((H, W)) < 0.9).astype(np.uint8)
    arms = _random_arms(rng, H, W, 6)
    one = oracle.vote(d, valid, arms, D, 1)
    two = oracle.vote(one, (one >= 0).astype(np.uint8), arms, D, 1)
    assert np.array_equal(oracle.vote(d, valid, arms, D, 2), two)


def test_finish_without_vote_reproduces_the_lr_output():
    from paper_2203_02300_amd import synth
    p = synth.config_c1()
    st = oracle.stages(p["left"], p["right"], 16)
    dv = np.where(st["valid"] == 1, st["dL"], -1).astype(np.int16)
    disp, valid = oracle.vote_finish(st["aggL"], dv)
    assert np.array_equal(valid, st["valid"])
    assert np.array_equal(disp.view(np.uint32), st["disp"].view(np.uint32))
    # zero passes of the vote leave the map as it was
    assert np.array_equal(oracle.vote(st["dL"], st["valid"], st["armsL"], 16, 0), dv)


def test_match_with_vote_is_the_stages_composed():
    from paper_2203_02300_amd import synth
    p = synth.config_c1()
    st = oracle.stages(p["left"], p["right"], 16)
    dv = oracle.vote(st["dL"], st["valid"], st["armsL"], 16, 2)
    want_disp, want_valid = oracle.vote_finish(st["aggL"], dv)
    disp, valid, dL, _ = oracle.match(p["left"], p["right"], 16, vote_iters=2)
    assert np.array_equal(valid, want_valid)
    assert np.array_equal(disp.view(np.uint32), want_disp.view(np.uint32))
    assert np.array_equal(dL, st["dL"])
    # the vote only ever removes disagreement: no valid pixel is dropped
    assert np.array_equal(valid, st["valid"])
