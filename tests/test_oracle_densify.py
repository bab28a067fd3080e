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
