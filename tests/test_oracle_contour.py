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


# ---------------------------------------------------------------------------
# Flows with a vertical component, hand-computed scores, a fusion case whose
# two amplitude fields are not proportional, every suppression sector, and an
# independent array formulation of the whole filter.
# ---------------------------------------------------------------------------

def test_amplitude_of_a_vertical_speed_ramp():
    # r = 5y (U = 3y, V = 4y): |r(y+1) - r(y)| = 5 in every row but the last,
    # and no horizontal change.  Kills: the vertical neighbour taken as the
    # next column (gv from i + 1 instead of i + w).
    h, w = 6, 5
    y = np.arange(h, dtype=np.float32)[:, None] * np.ones((1, w), np.float32)
    M, _ = oracle.flow_terms(_flow(3.0 * y, 4.0 * y))
    want = np.full((h, w), 5.0, np.float32)
    want[-1] = 0.0
    assert np.array_equal(M, want)


def test_amplitude_takes_the_larger_of_the_two_directions():
    # r = 2x + 7y: horizontal change 2, vertical 7 -> 7; last row keeps the
    # horizontal 2; the bottom-right pixel has neither.
    h, w = 4, 5
    ys, xs = np.mgrid[0:h, 0:w].astype(np.float32)
    M, _ = oracle.flow_terms(_flow(2.0 * xs + 7.0 * ys))
    want = np.full((h, w), 7.0, np.float32)
    want[-1, :] = 2.0
    want[-1, -1] = 0.0
    assert np.array_equal(M, want)


def test_score_of_a_vertical_flow():
    # V = y^2 (U = 0): e = (0, 1) wherever V > 0, p1 / p0 one row down / up,
    # score = V(y+1) - V(y-1) = 4y inside; clamped at the last row:
    # V(h-1) - V(h-2).  Row 0 has V = 0: no direction, score 0.
    # Kills: the step of the vertical direction taken from ex (sy = rint(ex)).
    h, w = 6, 3
    V = (np.arange(h, dtype=np.float32) ** 2)[:, None] * np.ones((1, w), np.float32)
    _, S = oracle.flow_terms(_flow(np.zeros((h, w)), V))
    want = np.array([0, 4, 8, 12, 16, 25 - 16], np.float32)[:, None] * np.ones((1, w))
    assert np.array_equal(S, want.astype(np.float32))


def test_score_projects_on_the_flow_direction_at_p():
    # At p = (2, 2) the flow is (3, 2): e = (3, 2) / sqrt(13), which rounds to
    # the step (1, 1).  p1 = (3, 3) carries (0, 10) and p0 = (1, 1) carries
    # (4, 0), so score = 10 ey - 4 ex = (20 - 12) / sqrt(13) > 0.  With the
    # components of e swapped it would be (30 - 8) / sqrt(13).
    # Kills: ex and ey swapped in the projection; the step taken with the
    # wrong sign (p1 = p - rint(e)).
    F = np.zeros((5, 5, 2), np.float32)
    F[2, 2] = (3.0, 2.0)
    F[3, 3] = (0.0, 10.0)
    F[1, 1] = (4.0, 0.0)
    _, S = oracle.flow_terms(F)
    r = np.float32(np.sqrt(np.float32(13.0)))
    ex, ey = np.float32(3.0) / r, np.float32(2.0) / r
    want = (np.float32(0.0) * ex + np.float32(10.0) * ey) - (np.float32(4.0) * ex +
                                                             np.float32(0.0) * ey)
    assert S[2, 2] == want and want > 0
    assert abs(float(S[2, 2]) - 8.0 / np.sqrt(13.0)) < 1e-6


def test_score_direction_with_a_negative_component():
    # flow (2, -3) at p = (2, 2): step (1, -1), p1 = (3, 1), p0 = (1, 3);
    # score = F(p1).e - F(p0).e with e = (2, -3) / sqrt(13).
    # Kills: the sign of the vertical step dropped (|rint(ey)|).
    F = np.zeros((5, 5, 2), np.float32)
    F[2, 2] = (2.0, -3.0)
    F[1, 3] = (0.0, -6.0)    # row 1, column 3 = p1
    F[3, 1] = (5.0, 0.0)     # row 3, column 1 = p0
    _, S = oracle.flow_terms(F)
    assert abs(float(S[2, 2]) - (18.0 - 10.0) / np.sqrt(13.0)) < 1e-6


def test_fusion_with_amplitudes_of_different_shape():
    # past: V = y^2 / 10, growing along its direction (score 0.4 y > 0),
    # amplitude (2y + 1) / 10; future: V = 60 - 2y, shrinking (score -4),
    # amplitude 2 everywhere.  Eq. 12 keeps the past amplitude, a ramp; the
    # inverted rule would keep the future's constant map.
    # Kills: Eq. 12 inverted (the smaller score kept).
    h, w = 10, 4
    y = np.arange(h, dtype=np.float64)[:, None] * np.ones((1, w))
    past = _flow(np.zeros((h, w)), y * y / 10.0)
    future = _flow(np.zeros((h, w)), 60.0 - 2.0 * y)
    M = oracle.flow_fuse(past, future, R=0)
    ramp = (2.0 * y[:, 0] + 1.0) / 10.0
    ramp[-1] = 0.0
    want = np.tile((ramp / ramp.max())[:, None], (1, w))
    assert np.allclose(M, want, rtol=2e-6, atol=1e-7)
    assert M[0, 0] < 0.1      # the constant map of the future would give 1.0 here


def _diag_step(H, W, k, anti=False, lo=40, hi=190):
    ys, xs = np.mgrid[0:H, 0:W]
    s = xs - ys if anti else xs + ys
    return np.where(s >= k, hi, lo).astype(np.uint8)


def test_horizontal_step_edge_is_one_row():
    # a step between rows y0 - 1 and y0: the gradient is vertical (vertical
    # sector), both rows have G2 = 600^2 and the first one survives.
    # Kills: the vertical sector's step along x instead of y.
    H, W, y0 = 14, 12, 6
    Y = np.full((H, W), 50, np.uint8)
    Y[y0:] = 200
    B, MI = oracle.contour(Y, np.ones((H // 2, W // 2), np.float32))
    want = np.zeros((H, W), np.uint8)
    want[y0 - 1] = 1
    assert np.array_equal(B, want)
    assert np.all(MI[y0 - 1] == 1.0) and np.all(MI[y0] == 1.0)


@pytest.mark.parametrize("anti", [False, True])
def test_diagonal_step_edge_keeps_its_two_central_diagonals(anti):
    # Y steps where x + y >= k (45 deg) or x - y >= k (135 deg).  With
    # c = hi - lo, Sobel gives |gx| = |gy| = c, 3c, 3c, c on the diagonals
    # s = k-2 .. k+1 (0 elsewhere), so G2 = 2c^2, 18c^2, 18c^2, 2c^2; the
    # diagonal sector compares s with s - 2 and s + 2, which keeps exactly the
    # two 18c^2 diagonals (both strong).  Checked away from the border, where
    # the replicated edge changes the gradients.
    # Kills: the diagonal sector's sign flipped (then each pixel meets two
    # equal neighbours along the edge and nothing survives).
    H, W, k = 24, 24, 20 if not anti else 2
    Y = _diag_step(H, W, k, anti)
    B, MI = oracle.contour(Y, np.ones((H // 2, W // 2), np.float32))
    ys, xs = np.mgrid[0:H, 0:W]
    s = xs - ys if anti else xs + ys
    inner = (xs >= 2) & (xs < W - 2) & (ys >= 2) & (ys < H - 2)
    want = ((s == k - 1) | (s == k)).astype(np.uint8)
    assert np.array_equal(B[inner], want[inner])
    assert want[inner].sum() > 20
    # MI is normalised by the grid's largest G2 (found at the border), so
    # compare the ratio of the s = k-2 and s = k-1 diagonals: sqrt(2 / 18)
    ratio = MI[inner & (s == k - 2)] / MI[inner & (s == k - 1)][0]
    assert np.allclose(ratio, 1.0 / 3.0, rtol=1e-6)


def test_weak_chain_touching_a_strong_pixel_diagonally_is_kept():
    # hand-set states through the public thresholds: a vertical strong edge in
    # rows 0..5 (column 4) and a weak one in rows 6..11 one column to the right
    # (column 5), whose first pixel touches the strong chain's last one only
    # diagonally.  8-connected hysteresis keeps the weak chain.
    # Kills: 4-connected growth.
    H, W = 12, 12
    Y = np.full((H, W), 50, np.uint8)
    Y[:6, 5:] = 200          # strong step, ridge at column 4 of rows 0..5
    Y[6:, 6:] = 62           # weak step (contrast 12), ridge at column 5
    Mn = np.ones((H // 2, W // 2), np.float32)
    B, MI = oracle.contour(Y, Mn, Thigh=0.5, Tlow=0.02)
    from brute_ref import contour_ref
    Br, _ = contour_ref(Y, Mn, Thigh=0.5, Tlow=0.02)
    assert np.array_equal(B, Br)
    assert B[8:, 5].all() and B[:4, 4].all()
    # the same weak chain with no strong pixel near it is dropped
    Y2 = np.full((H, W), 50, np.uint8)
    Y2[:, 6:] = 62
    Y2[:3, 0] = 200          # a strong corner far away
    B2, _ = oracle.contour(Y2, Mn, Thigh=0.5, Tlow=0.02)
    assert not B2[:, 5].any()


@pytest.mark.parametrize("seed", range(4))
def test_flow_fusion_matches_the_array_formulation(seed):
    from brute_ref import flow_fuse_ref, flow_terms_ref
    rng = np.random.default_rng(100 + seed)
    h, w = 11, 14
    # piecewise flows with both components, zero patches and sign changes
    def field():
        base = rng.normal(0, 3, (h // 3 + 1, w // 3 + 1, 2))
        F = np.kron(base, np.ones((3, 3, 1)))[:h, :w] + rng.normal(0, 0.3, (h, w, 2))
        F[rng.random((h, w)) < 0.1] = 0.0
        return F.astype(np.float32)
    past, future = field(), field()
    for F in (past, future):
        M, S = oracle.flow_terms(F)
        Mr, Sr = flow_terms_ref(F)
        assert np.array_equal(M, Mr) and np.array_equal(S, Sr)
    assert np.allclose(oracle.flow_fuse(past, future, R=2), flow_fuse_ref(past, future, R=2),
                       rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("seed", range(4))
def test_contour_matches_the_array_formulation(seed):
    # blocky random images put gradients in every sector with both signs
    from brute_ref import contour_ref
    rng = np.random.default_rng(200 + seed)
    H, W = 36, 44
    Y = (rng.random((H // 3 + 1, W // 3 + 1)) * 255).astype(np.uint8)
    Y = np.kron(Y, np.ones((3, 3), np.uint8))[:H, :W]
    Y = np.clip(Y.astype(int) + rng.integers(-4, 5, (H, W)), 0, 255).astype(np.uint8)
    Mn = rng.random((H // 2, W // 2)).astype(np.float32)
    for th, tl in ((0.06, 0.03), (0.3, 0.1)):
        B, MI = oracle.contour(Y, Mn, Thigh=th, Tlow=tl)
        Br, MIr = contour_ref(Y, Mn, Thigh=th, Tlow=tl)
        assert np.array_equal(B, Br)
        assert np.array_equal(MI, MIr)
