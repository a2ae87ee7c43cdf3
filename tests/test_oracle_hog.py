"""Pins of the oracle's HOG front end (sliding windows, gradients, orientation bins, cells,
blocks) against things other than itself: exact trigonometry, floating-point angles away
from the bin boundaries, math.isqrt, a pixel-by-pixel implementation, images whose
gradients are known in closed form, and the translation property of interior windows."""
import math

import numpy as np
import pytest

from oracle import hog


def test_orientation_table_is_the_rounded_exact_directions():
    import sympy
    C, S = hog.orientation_table()
    for k in range(1, 9):
        c = sympy.N(16384 * sympy.cos(sympy.pi * k / 9), 40)
        s = sympy.N(16384 * sympy.sin(sympy.pi * k / 9), 40)
        assert C[k - 1] == int(sympy.floor(c + sympy.Rational(1, 2)))
        assert S[k - 1] == int(sympy.floor(s + sympy.Rational(1, 2)))
    assert C[2] == 8192 and C[5] == -8192  # cos 60 = 1/2, cos 120 = -1/2


def test_bins_agree_with_angles_away_from_the_boundaries():
    g = np.arange(-255, 256)
    gx, gy = np.meshgrid(g, g, indexing="ij")
    b = hog.orientation_bins(gx, gy)
    ang = np.degrees(np.arctan2(gy, gx)) % 180.0
    ang = np.where((gx == 0) & (gy == 0), 0.0, ang)
    ref = np.floor(ang / 20.0).astype(np.int64) % 9
    dist = np.abs(ang / 20.0 - np.round(ang / 20.0)) * 20.0  # degrees to the nearest boundary
    far = dist > 0.05
    assert np.array_equal(b[far], ref[far])
    # near a boundary the rule picks one of the two bins that meet there
    near = ~far
    lo = (np.round(ang / 20.0).astype(np.int64) - 1) % 9
    hi = np.round(ang / 20.0).astype(np.int64) % 9
    assert np.all((b[near] == lo[near]) | (b[near] == hi[near]))
    assert b.min() == 0 and b.max() == 8


def test_integer_square_root_is_exact():
    n = np.concatenate([np.arange(0, 200000), np.random.default_rng(0).integers(0, 2 * 255 ** 2 + 1, 100000),
                        np.random.default_rng(1).integers(0, 36 * 23040 ** 2 + 1, 100000),
                        np.array([k * k - 1 for k in range(1, 150000, 7)] + [k * k for k in range(1, 150000, 7)])])
    assert np.array_equal(hog.isqrt(n), np.array([math.isqrt(int(v)) for v in n]))


def test_closed_form_gradients_of_ramps():
    """I = 3x: gx = 6 inside (3 at the clamped borders), gy = 0: every pixel in bin 0; I = 5y: bin 4
    (90 degrees); I = x + y: 45 degrees, bin 2; magnitudes isqrt(gx^2 + gy^2)."""
    y, x = np.mgrid[0:32, 0:40]
    for img, bin_, mag in [(3 * x, 0, 6), (5 * y, 4, 10), (x + y, 2, math.isqrt(8))]:
        img = img.astype(np.uint8)
        h = hog.cell_histograms(img)
        inner = h[1:-1, 1:-1]
        assert np.all(inner[..., bin_] == 64 * mag)
        assert inner.sum() == inner[..., bin_].sum()


def test_histograms_blocks_and_windows_match_the_pixel_loop():
    rng = np.random.default_rng(1)
    for H, W, win, st in [(40, 48, 16, 8), (48, 40, 24, 16), (33, 50, 32, 8)]:
        fr = rng.integers(0, 256, (H, W)).astype(np.uint8)
        assert np.array_equal(hog.window_features(fr, win, st), hog.window_features_naive(fr, win, st))


def test_cell_totals_and_block_normalisation():
    rng = np.random.default_rng(2)
    fr = rng.integers(0, 256, (64, 72)).astype(np.uint8)
    gx, gy = hog.gradients(fr)
    mag = np.array([[math.isqrt(int(a) ** 2 + int(b) ** 2) for a, b in zip(r1, r2)] for r1, r2 in zip(gx, gy)])
    h = hog.cell_histograms(fr)
    assert np.array_equal(h.sum(axis=2), mag.reshape(8, 8, 9, 8).sum(axis=(1, 3)))
    blk = hog.block_features(h).astype(np.int64)
    # the largest of a block's values is at least a sixth of its norm: its byte is >= 212
    assert np.all(blk.max(axis=2) >= 212) and blk.max() == 255
    # a block of one non-zero value clips to 255; equal values give floor(1275 / 6) = 212
    one = np.zeros((2, 2, 9), dtype=np.int64)
    one[0, 0, 3] = 77
    assert hog.block_features(one)[0, 0, 3] == 255 and hog.block_features(one).sum() == 255
    assert np.all(hog.block_features(np.full((2, 2, 9), 5, dtype=np.int64)) == 212)


def test_interior_windows_depend_only_on_their_neighbourhood():
    """An interior window's features equal those of the same window in a crop of the frame
    that keeps one cell around it (its gradients only read neighbouring pixels)."""
    rng = np.random.default_rng(3)
    fr = rng.integers(0, 256, (96, 112)).astype(np.uint8)
    full = hog.window_features(fr, 32, 8)
    org = hog.window_origins(96, 112, 32, 8)
    for (wy, wx) in [(16, 24), (40, 64), (8, 8)]:
        crop = fr[wy - 8:wy + 32 + 8, wx - 8:wx + 32 + 8]
        sub = hog.window_features(crop, 32, 8)
        assert np.array_equal(sub[hog.window_origins(*crop.shape, 32, 8).index((8, 8))], full[org.index((wy, wx))])


def test_window_count_and_padding():
    assert hog.feature_count(64) == 1776 and hog.feature_count(16) == 48 and hog.feature_count(48) == 912
    assert len(hog.window_origins(1080, 1920, 64, 8)) == 128 * 233
    fr = np.zeros((64, 64), dtype=np.uint8)
    out = hog.window_features(fr, 64, 8)
    assert out.shape == (1, 1776) and not out[0, :1764].any() and np.all(out[0, 1764:] == 128)
