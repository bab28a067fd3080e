"""Pins of the oracle's quarter-size front end (Sec. 4.4): the 2 x 2
reduction against block means computed directly, the doubling and the depth
conversion against closed forms.  CPU only."""
from __future__ import annotations

import numpy as np

import oracle


def test_reduction_of_a_constant_image_is_the_constant():
    img = np.full((6, 10, 3), (7, 200, 31), np.uint8)
    out = oracle.downscale2(img)
    assert out.shape == (3, 5, 3) and np.all(out == np.array([7, 200, 31], np.uint8))


def test_reduction_rounds_half_up_and_drops_odd_edges():
    img = np.zeros((3, 5, 3), np.uint8)
    img[0, 0] = (1, 2, 3)
    img[0, 1] = (0, 0, 0)
    img[1, 0] = (0, 1, 255)
    img[1, 1] = (1, 0, 255)
    img[0, 4] = img[2, 0] = (255, 255, 255)  # in the dropped column / row
    out = oracle.downscale2(img)
    assert out.shape == (1, 2, 3)
    # (1+0+0+1+2)>>2 = 1 (mean 0.5 rounds up), (2+0+1+0+2)>>2 = 1 (0.75),
    # (3+0+255+255+2)>>2 = 128 (128.25)
    assert out[0, 0].tolist() == [1, 1, 128]
    assert out[0, 1].tolist() == [0, 0, 0]


def test_reduction_matches_block_means():
    rng = np.random.default_rng(5)
    img = rng.integers(0, 256, (40, 66, 3), dtype=np.uint8)
    blocks = img.reshape(20, 2, 33, 2, 3).astype(np.int64).sum(axis=(1, 3))
    assert np.array_equal(oracle.downscale2(img), ((blocks + 2) // 4).astype(np.uint8))


def test_depth_closed_form():
    disp = np.array([[2.5, 0.0, 10.0, 3.0]], np.float32)
    valid = np.array([[1, 1, 1, 0]], np.uint8)
    dfull, depth = oracle.depth_half(disp, valid, 100.0)
    assert dfull.tolist() == [[5.0, 0.0, 20.0, 0.0]]
    assert depth.tolist() == [[20.0, 0.0, 5.0, 0.0]]


def test_shifted_pair_at_half_scale_recovers_half_the_shift():
    # a pair shifted by 8 pixels is shifted by 4 after the reduction; the
    # doubled disparity is 8 again wherever the match is valid and integer
    from paper_2203_02300_amd import synth
    p = synth.make_shift_pair(200, 64, 8, 3, texture="patches")
    dfull, depth, valid = oracle.match_half(p["left"], p["right"], 16, 80.0, subpixel=0)
    inner = valid[:, 12:-4] == 1
    assert inner.mean() > 0.9
    assert np.all(dfull[:, 12:-4][inner] == 8.0)
    assert np.all(depth[:, 12:-4][inner] == np.float32(10.0))
