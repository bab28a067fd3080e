"""Pins of the oracle's depth contour filter (Sec. 5, Eq. 6-12 and the gated
Canny of Sec. 5.3): closed forms on ramps and steps, the fusion rule on
hand-built flows, the box filter against a library window mean, the gate,
and hysteresis against connected-component labelling.  CPU only."""
from __future__ import annotations

import numpy as np
import pytest

import oracle


def _flow(U, V=None):
    U = np.asarray(U, np.float32)
    V = np.zeros_like(U) if V is None else np.asarray(V, np.float32)
    return np.stack([U, V], axis=-1)


def test_uniform_flow_has_no_amplitude():
    f = _flow(np.full((6, 9), 3.0), np.full((6, 9), 4.0))
    assert np.all(oracle.flow_fuse(f, f) == 0.0)


def test_amplitude_of_a_linear_speed_ramp():
    # r = x: |r(x+1) - r(x)| = 1 inside, 0 in the last column (no neighbour)
    h, w = 5, 8
    f = _flow(np.tile(np.arange(w, dtype=np.float32), (h, 1)))
    M = oracle.flow_fuse(f, f, R=0)
    want = np.ones((h, w), np.float32)
    want[:, -1] = 0.0
    assert np.array_equal(M, want)


def test_fusion_keeps_the_field_whose_projection_grows():
    # past: U = x^2 / 10 grows along its own direction (score > 0);
    # future: U = 100 - x^2 / 5 shrinks (score < 0) -> Eq. 12 keeps M_past,
    # M_past(x) = (2x + 1) / 10, normalised by its largest value
    h, w = 4, 12
    x = np.arange(w, dtype=np.float64)
    past = _flow(np.tile(x * x / 10.0, (h, 1)))
    future = _flow(np.tile(100.0 - x * x / 5.0, (h, 1)))
    M = oracle.flow_fuse(past, future, R=0)
    want = np.zeros(w)
    want[:-1] = (2 * x[:-1] + 1) / (2 * (w - 2) + 1)
    assert np.allclose(M, np.tile(want, (h, 1)), rtol=2e-6, atol=1e-7)
    # swapped roles: the future field now grows and is kept
    M2 = oracle.flow_fuse(future, past, R=0)
    assert np.array_equal(M, M2)


def test_zero_flow_scores_zero_and_ties_keep_the_larger_amplitude():
    h, w = 3, 6
    x = np.arange(w, dtype=np.float64)
    past = _flow(np.zeros((h, w)))                       # no direction: score 0
    future = _flow(np.tile(3.0 * x, (h, 1)), None)       # U = 3x: score 6 > 0
    assert np.allclose(oracle.flow_fuse(past, future, R=0)[:, :-1], 1.0)
    # a constant flow scores 0 like a zero flow: the tie keeps max(M_past, M_future)
    const = _flow(np.full((h, w), 2.0))
    bump = np.zeros((h, w))
    bump[1, 2] = 5.0
    M = oracle.flow_fuse(const, _flow(bump), R=0)
    assert M.max() == 1.0 and M[1, 2] == 1.0


def test_box_filter_is_the_clipped_window_mean():
    from scipy import ndimage
    rng = np.random.default_rng(3)
    h, w, R = 9, 13, 2
    U = rng.normal(size=(h, w)).astype(np.float32)
    f = _flow(U, rng.normal(size=(h, w)))
    raw = oracle.flow_fuse(f, f, R=0) * 1.0           # normalised M of one field
    # undo the normalisation: flow_fuse(R=0) / its max is M / max M, and the
    # box of the normalised map normalised again equals the box of M normalised
    k = 2 * R + 1
    s = ndimage.uniform_filter(raw.astype(np.float64), size=k, mode="constant") * k * k
    n = ndimage.uniform_filter(np.ones((h, w)), size=k, mode="constant") * k * k
    box = s / np.round(n)
    want = box / box.max()
    assert np.allclose(oracle.flow_fuse(f, f, R=R), want, rtol=1e-5, atol=1e-6)


def _step(H, W, x0, lo=50, hi=200):
    Y = np.full((H, W), lo, np.uint8)
    Y[:, x0:] = hi
    return Y


def test_step_edge_is_one_column():
    H, W, x0 = 12, 16, 7
    B, MI = oracle.contour(_step(H, W, x0), np.ones((H // 2, W // 2), np.float32))
    want = np.zeros((H, W), np.uint8)
    want[:, x0 - 1] = 1  # both columns have G2 = 600^2; the first one survives
    assert np.array_equal(B, want)
    assert np.all(MI[:, x0 - 1] == 1.0) and np.all(MI[:, x0] == 1.0)
    assert np.all(MI[:, : x0 - 1] == 0.0)


def test_gate_drops_edges_outside_the_depth_filter():
    H, W, x0 = 12, 16, 7
    Y = _step(H, W, x0)
    B, _ = oracle.contour(Y, np.zeros((H // 2, W // 2), np.float32))
    assert not B.any()
    Mn = np.zeros((H // 2, W // 2), np.float32)
    Mn[:3] = 1.0  # full-size rows 0..5
    B, _ = oracle.contour(Y, Mn)
    assert B[:6, x0 - 1].all() and not B[6:].any()
    # the gate compares with T_depth: just below drops, equal keeps
    B, _ = oracle.contour(Y, np.full((H // 2, W // 2), 0.0299, np.float32))
    assert not B.any()
    B, _ = oracle.contour(Y, np.full((H // 2, W // 2), np.float32(0.03), np.float32))
    assert B.any()


def test_isolated_weak_edges_are_dropped():
    # two vertical steps: contrast 150 at x = 5 (strong) and 6 at x = 12
    # (normalised 0.04: weak, not touching the strong one)
    H, W = 12, 18
    Y = np.full((H, W), 50, np.uint8)
    Y[:, 5:] = 200
    Y[:, 12:] = 206
    Mn = np.ones((H // 2, W // 2), np.float32)
    B, MI = oracle.contour(Y, Mn)
    want = np.zeros((H, W), np.uint8)
    want[:, 4] = 1
    assert np.array_equal(B, want)
    assert np.allclose(MI[:, 11], 24.0 / 600.0, rtol=1e-6)
    # with T_low above the weak edge and T_high above both, nothing is kept
    B, _ = oracle.contour(Y, Mn, Thigh=1.5, Tlow=0.05)
    assert not B.any()
    # with both thresholds below the weak edge, both edges are strong
    B, _ = oracle.contour(Y, Mn, Thigh=0.02, Tlow=0.01)
    assert B[:, 4].all() and B[:, 11].all() and B.sum() == 2 * H


@pytest.mark.parametrize("seed", range(4))
def test_hysteresis_equals_connected_components(seed):
    from scipy import ndimage
    rng = np.random.default_rng(seed)
    H, W = 40, 52
    Y = (rng.random((H // 4 + 1, W // 4 + 1)) * 255).astype(np.uint8)
    Y = np.kron(Y, np.ones((4, 4), np.uint8))[:H, :W]
    Y = np.clip(Y.astype(int) + rng.integers(-3, 4, (H, W)), 0, 255).astype(np.uint8)
    Mn = rng.random((H // 2, W // 2)).astype(np.float32)
    B, _ = oracle.contour(Y, Mn, Thigh=0.3, Tlow=0.1)
    # candidates (strong or weak) from two runs: with T_high = T_low every
    # candidate is strong; with T_high = 2 (none strong) hysteresis keeps none
    strong, _ = oracle.contour(Y, Mn, Thigh=0.3, Tlow=0.3)
    cand, _ = oracle.contour(Y, Mn, Thigh=0.1, Tlow=0.1)
    lab, n = ndimage.label(cand, structure=np.ones((3, 3)))
    keep = np.zeros(n + 1, bool)
    keep[np.unique(lab[strong == 1])] = True
    keep[0] = False
    assert np.array_equal(B, keep[lab].astype(np.uint8))
    none, _ = oracle.contour(Y, Mn, Thigh=2.0, Tlow=0.1)
    assert not none.any()
