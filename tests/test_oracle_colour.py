"""Pins of the oracle's colour transform (Sec. 4: lossless YCoCg-R, reading C1).

The pins are the textbook matrix form of YCoCg (Y = R/4 + G/2 + B/4,
Co = R - B for the reversible variant, Cg = G - (R + B)/2) within the integer
lifting's rounding, the stated value ranges, and exhaustive invertibility over
all 2^24 RGB triples.
"""
import numpy as np

import oracle


def all_rgb():
    v = np.arange(1 << 24, dtype=np.uint32)
    return np.stack([(v >> 16) & 255, (v >> 8) & 255, v & 255], axis=1).astype(np.uint8)


def test_exhaustive_round_trip_and_ranges():
    rgb = all_rgb()
    ycc = oracle.ycocg_forward(rgb)
    back = oracle.ycocg_inverse(ycc)
    assert np.array_equal(back, rgb)
    y, co, cg = ycc[:, 0].astype(np.int32), ycc[:, 1].astype(np.int32), ycc[:, 2].astype(np.int32)
    assert y.min() == 0 and y.max() == 255
    assert co.min() == -255 and co.max() == 255
    assert cg.min() == -255 and cg.max() == 255


def test_matches_textbook_matrix_within_rounding():
    rgb = all_rgb()[::97].astype(np.float64)
    ycc = oracle.ycocg_forward(rgb.astype(np.uint8)).astype(np.float64)
    r, g, b = rgb[:, 0], rgb[:, 1], rgb[:, 2]
    assert np.array_equal(ycc[:, 1], r - b)
    assert np.all(np.abs(ycc[:, 2] - (g - (r + b) / 2)) <= 0.5)
    assert np.all(np.abs(ycc[:, 0] - (r / 4 + g / 2 + b / 4)) < 1.0)


def test_inverse_clamps_out_of_gamut():
    # Y far above the gamut must clamp to 255 in every channel, far below to 0
    ycc = np.array([[400, 0, 0], [-50, 0, 0]], dtype=np.int16)
    assert np.array_equal(oracle.ycocg_inverse(ycc), np.array([[255] * 3, [0] * 3], dtype=np.uint8))
