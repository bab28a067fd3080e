"""Pins of the densification oracle (Sec. 6, Eq. 13-20): a chain with a closed
form at the paper's coefficients, the decoupled case, constant data, contour
isolation, and optimality of the solution for the printed objective summed
term by term.  CPU only."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import densify as dz


def _maps(H, W, seed, contour=False):
    rng = np.random.default_rng(seed)
    Ds = np.where(rng.random((H, W)) < 0.6, rng.uniform(1.0, 5.0, (H, W)), 0.0)
    Dpre = np.where(rng.random((H, W)) < 0.5, rng.uniform(1.0, 5.0, (H, W)), 0.0)
    B = (rng.random((H, W)) < (0.15 if contour else 0.0)).astype(np.uint8)
    return Ds, Dpre, B, rng.random((H, W)), rng.random((H, W))


def test_chain_closed_form_at_the_paper_coefficients():
    # 1 x 5 chain, every edge weight 1, data 1 at x = 0 and 6 at x = 4:
    # E = 0.8 ((D0-1)^2 + (D4-6)^2) + 2 * 1.2 * sum of squared steps, so the
    # interior is linear and D4 - D0 = 0.8 * 5 / (0.8 + 1.2) = 2, D0 + D4 = 7
    Ds = np.array([[1.0, 0, 0, 0, 6.0]])
    z = np.zeros((1, 5))
    D = dz.densify(Ds, None, z.astype(np.uint8), z, z)
    assert np.allclose(D, [[2.5, 3.0, 3.5, 4.0, 4.5]], atol=1e-12)


def test_without_smoothness_the_data_is_returned():
    Ds, Dpre, B, Mf, MI = _maps(9, 11, 1)
    D = dz.densify(Ds, None, B, Mf, MI, lam_s=0.0)
    assert np.allclose(D[Ds > 0], Ds[Ds > 0], atol=1e-12)
    assert np.all(D[Ds == 0] == 0.0)  # unanchored single pixels


def test_stability_blends_with_the_data():
    # one pixel, both terms: D = (0.8 * 2 + 0.02 * 7) / 0.82
    D = dz.densify(np.array([[2.0]]), np.array([[7.0]]), np.zeros((1, 1), np.uint8),
                   np.zeros((1, 1)), np.zeros((1, 1)))
    assert abs(D[0, 0] - (0.8 * 2 + 0.02 * 7) / 0.82) < 1e-12


def test_constant_data_gives_a_constant_field():
    H, W = 8, 10
    rng = np.random.default_rng(2)
    Ds = np.where(rng.random((H, W)) < 0.2, 3.25, 0.0)
    Ds[0, 0] = 3.25
    D = dz.densify(Ds, None, np.zeros((H, W), np.uint8), rng.random((H, W)) * 0.5,
                   rng.random((H, W)))
    assert np.allclose(D, 3.25, atol=1e-10)


def test_a_closed_contour_isolates_its_inside():
    H, W = 9, 9
    B = np.zeros((H, W), np.uint8)
    B[2, 2:7] = B[6, 2:7] = B[2:7, 2] = B[2:7, 6] = 1  # ring around 3..5 x 3..5
    Ds = np.zeros((H, W))
    Ds[0, :] = 4.0                                      # data outside only
    z = np.zeros((H, W))
    D = dz.densify(Ds, None, B, z, z)
    assert np.all(D[3:6, 3:6] == 0.0)                   # no data inside: no depth
    assert np.allclose(D[0, :], 4.0) and np.allclose(D[8, :], 4.0)
    # the ring itself is cut from the outside as well (exactly one end on it)
    assert np.all(D[2:7, 2][1:-1] == 0.0)


@pytest.mark.parametrize("seed", range(3))
def test_solution_minimises_the_printed_objective(seed):
    Ds, Dpre, B, Mf, MI = _maps(6, 7, 10 + seed, contour=True)
    D = dz.densify(Ds, Dpre, B, Mf, MI)
    e0 = dz.energy(D, Ds, Dpre, B, Mf, MI)
    rng = np.random.default_rng(seed)
    A, b, anchor, _ = dz.system(Ds, Dpre, B, Mf, MI)
    for _ in range(5):
        step = rng.normal(size=D.shape) * 1e-3
        assert dz.energy(D + step, Ds, Dpre, B, Mf, MI) >= e0 - 1e-12
    # central differences of the objective vanish at the solution (on pixels
    # that the system determines)
    live = np.abs(D) > 0
    g = np.zeros(D.shape)
    h = 1e-5
    for y, x in zip(*np.nonzero(live)):
        e = np.zeros(D.shape)
        e[y, x] = h
        g[y, x] = (dz.energy(D + e, Ds, Dpre, B, Mf, MI) -
                   dz.energy(D - e, Ds, Dpre, B, Mf, MI)) / (2 * h)
    scale = np.abs(b).max()
    assert np.abs(g).max() < 1e-6 * max(scale, 1.0)


# ---------------------------------------------------------------------------
# Edge weights with s = M_fuse * M_I != 0, solved by hand
# ---------------------------------------------------------------------------

def _pair_solution(a, b, w, lam_d=0.8, lam_s=1.2):
    # two pixels with data a and b joined by one edge of weight w:
    # E = lam_d ((D0 - a)^2 + (D1 - b)^2) + 2 lam_s w (D0 - D1)^2 (the double
    # sum visits the pair twice).  With D0 = m - t, D1 = m + t, m = (a + b) / 2,
    # dE/dt = 0 gives t = lam_d (b - a) / (2 lam_d + 8 lam_s w).
    m = 0.5 * (a + b)
    t = lam_d * (b - a) / (2 * lam_d + 8 * lam_s * w)
    return m - t, m + t


@pytest.mark.parametrize("vertical", [False, True])
def test_pair_weight_uses_the_smaller_product(vertical):
    # s0 = 0.5 * 0.5 = 0.25, s1 = 1.0 * 0.75 = 0.75: w = 1 - min = 0.75.
    # D0, D1 = 3.5 -/+ 0.8 * 5 / (1.6 + 7.2).
    # Kills: min swapped for max (w = 0.25 gives 2.5, 4.5); s as a sum
    # (M_fuse + M_I > 1 gives w = 0); the right / down weight taken from the
    # wrong neighbour.
    Ds = np.array([[1.0, 6.0]])
    Mf = np.array([[0.5, 1.0]])
    MI = np.array([[0.5, 0.75]])
    B = np.zeros((1, 2), np.uint8)
    if vertical:
        Ds, Mf, MI, B = Ds.T.copy(), Mf.T.copy(), MI.T.copy(), B.T.copy()
    D = dz.densify(Ds, None, B, Mf, MI).ravel()
    want = _pair_solution(1.0, 6.0, 0.75)
    assert np.allclose(D, want, atol=1e-12)
    assert abs(want[0] - (3.5 - 4.0 / 8.8)) < 1e-15


def test_pair_weight_is_clamped_at_zero():
    # s = 2 on both pixels: 1 - min(s) < 0 is clamped to 0, the pixels
    # decouple and keep their data.  Kills: the clamp removed (a negative
    # weight pushes the two depths apart).
    D = dz.densify(np.array([[1.0, 6.0]]), None, np.zeros((1, 2), np.uint8),
                   np.array([[2.0, 2.0]]), np.array([[1.0, 1.0]]))
    assert np.allclose(D, [[1.0, 6.0]], atol=1e-12)


def test_pair_on_the_contour_stays_coupled():
    # both pixels on B_dp: the edge is not cut (only a pixel pair with exactly
    # one end on the contour is).  Kills: cutting every edge that touches B.
    Mf = np.array([[0.5, 1.0]])
    MI = np.array([[0.5, 0.75]])
    D = dz.densify(np.array([[1.0, 6.0]]), None, np.ones((1, 2), np.uint8), Mf, MI)
    assert np.allclose(D.ravel(), _pair_solution(1.0, 6.0, 0.75), atol=1e-12)
    D1 = dz.densify(np.array([[1.0, 6.0]]), None, np.array([[1, 0]], np.uint8), Mf, MI)
    assert np.allclose(D1, [[1.0, 6.0]], atol=1e-12)


def test_two_by_two_grid_with_every_weight_different():
    # s = M_fuse * M_I = [[0.1, 0.6], [0.3, 0.9]] (M_I = 1).  Edge weights by
    # hand: top (0,0)-(0,1): 1 - 0.1 = 0.9; bottom (1,0)-(1,1): 1 - 0.3 = 0.7;
    # left (0,0)-(1,0): 1 - 0.1 = 0.9; right (0,1)-(1,1): 1 - 0.6 = 0.4.
    # Data on the diagonal only.  The normal equations written out from
    # Eq. 20: 2 lam_d w_sp (D_p - Ds_p) + 4 lam_s sum_e w_e (D_p - D_q) = 0.
    # Kills: the weights of the down edges computed with the transposed s
    # (they become 0.9 / 0.4 / 0.7 in other places).
    s = np.array([[0.1, 0.6], [0.3, 0.9]])
    Ds = np.array([[2.0, 0.0], [0.0, 7.0]])
    edges = {(0, 1): 0.9, (2, 3): 0.7, (0, 2): 0.9, (1, 3): 0.4}   # pixels 0..3 row-major
    lam_d, lam_s = 0.8, 1.2
    A = np.zeros((4, 4))
    rhs = np.zeros(4)
    for p, v in enumerate(Ds.ravel()):
        if v > 0:
            A[p, p] += 2 * lam_d
            rhs[p] += 2 * lam_d * v
    for (p, q), w in edges.items():
        for a, b in ((p, q), (q, p)):
            A[a, a] += 4 * lam_s * w
            A[a, b] -= 4 * lam_s * w
    want = np.linalg.solve(A, rhs).reshape(2, 2)
    D = dz.densify(Ds, None, np.zeros((2, 2), np.uint8), s, np.ones((2, 2)))
    assert np.allclose(D, want, atol=1e-12)
    wr, wd = dz.edge_weights(np.zeros((2, 2), np.uint8), s, np.ones((2, 2)))
    assert np.allclose(wr, [[0.9, 0.0], [0.7, 0.0]]) and np.allclose(wd, [[0.9, 0.4], [0.0, 0.0]])
