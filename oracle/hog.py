"""HOG feature maps of sliding windows (oracle; test infrastructure only).

The paper's driving example (HDC-based object detection) slides a window over an image
frame left to right, row by row, and gives each window's HOG feature map to the HDC
encoder (Our Proposed Method, applications; its HOG front end is named, not specified).
The reading used here is the usual HOG of Dalal and Triggs (CVPR 2005) in exact integer
arithmetic, so that every feature is a plain function of the pixels:

* gradient at pixel (y, x): gx = I[y][x+1] - I[y][x-1], gy = I[y+1][x] - I[y-1][x], with
  coordinates clamped to the frame (replicated border);
* magnitude floor(sqrt(gx^2 + gy^2)) (integer square root);
* unsigned orientation in 9 bins of 20 degrees: (gx, gy) is folded to the upper half plane
  ((gx, gy) -> (-gx, -gy) when gy < 0, or gy = 0 and gx < 0), and its bin is the number of
  boundaries k = 1..8 (angle 20k degrees, direction (C_k, S_k) with C_k = round(2^14 cos),
  S_k = round(2^14 sin)) it lies on or past: C_k * gy - S_k * gx >= 0;
* cells of 8 x 8 pixels; a cell's histogram adds each pixel's magnitude to its bin;
* blocks of 2 x 2 cells at a stride of one cell; a block's 36 values v (cells in row order,
  bins within) are L2-normalised with the usual clip at 0.2, scaled so that the clip is
  byte 255: min(255, floor(1275 * v / n)) with n = floor(sqrt(sum v^2)) (0 when n is 0);
* a window of w x w pixels at (wy, wx), both multiples of 8, covers (w/8 - 1)^2 blocks of
  the frame; its feature vector is their values in block row order, padded with 128 (the
  HDC encoder's zero point) to a multiple of 16 entries;
* windows at wy = 0, s, 2s, ... and wx = 0, s, 2s, ... (stride s, a multiple of 8) while
  they fit in the frame, ordered row by row.
"""
from __future__ import annotations

import math

import numpy as np

CELL = 8
BINS = 9
PAD_VALUE = 128


def orientation_table() -> tuple[np.ndarray, np.ndarray]:
    """(C_k, S_k) for k = 1..8: round(2^14 * cos(20k deg)), round(2^14 * sin(20k deg))."""
    ang = [math.pi * k / 9 for k in range(1, 9)]
    C = np.array([round(16384 * math.cos(a)) for a in ang], dtype=np.int64)
    S = np.array([round(16384 * math.sin(a)) for a in ang], dtype=np.int64)
    return C, S


def isqrt(n: np.ndarray) -> np.ndarray:
    """floor(sqrt(n)) of non-negative int64 values below 2^52, exactly."""
    n = np.asarray(n, dtype=np.int64)
    r = np.floor(np.sqrt(n.astype(np.float64))).astype(np.int64)
    r = np.where(r * r > n, r - 1, r)
    r = np.where((r + 1) * (r + 1) <= n, r + 1, r)
    return r


def gradients(frame: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """(gx, gy) int64 [H][W] by central differences with replicated borders."""
    f = np.pad(frame.astype(np.int64), 1, mode="edge")
    gx = f[1:-1, 2:] - f[1:-1, :-2]
    gy = f[2:, 1:-1] - f[:-2, 1:-1]
    return gx, gy


def orientation_bins(gx: np.ndarray, gy: np.ndarray) -> np.ndarray:
    """Unsigned orientation bin in 0..8 of every gradient (see the module docstring)."""
    flip = (gy < 0) | ((gy == 0) & (gx < 0))
    ux, uy = np.where(flip, -gx, gx), np.where(flip, -gy, gy)
    C, S = orientation_table()
    b = np.zeros(gx.shape, dtype=np.int64)
    for k in range(8):
        b += (C[k] * uy - S[k] * ux >= 0)
    return b


def cell_histograms(frame: np.ndarray) -> np.ndarray:
    """int64 [H/8][W/8][9]: per cell, the magnitudes of its pixels summed per bin."""
    H, W = frame.shape
    hc, wc = H // CELL, W // CELL
    gx, gy = gradients(frame)
    mag = isqrt(gx * gx + gy * gy)
    b = orientation_bins(gx, gy)
    hist = np.zeros((hc, wc, BINS), dtype=np.int64)
    cy = np.arange(hc * CELL) // CELL
    cx = np.arange(wc * CELL) // CELL
    Y, X = np.meshgrid(cy, cx, indexing="ij")
    np.add.at(hist, (Y, X, b[:hc * CELL, :wc * CELL]), mag[:hc * CELL, :wc * CELL])
    return hist


def block_features(hist: np.ndarray) -> np.ndarray:
    """uint8 [hc-1][wc-1][36]: 2 x 2-cell blocks, min(255, floor(1275 v / isqrt(sum v^2)))."""
    hc, wc, _ = hist.shape
    v = np.concatenate([hist[:-1, :-1], hist[:-1, 1:], hist[1:, :-1], hist[1:, 1:]], axis=2)
    n = isqrt((v * v).sum(axis=2, keepdims=True))
    out = np.where(n > 0, np.minimum(255, (1275 * v) // np.maximum(n, 1)), 0)
    return out.astype(np.uint8)


def feature_count(window: int) -> int:
    """Entries of one window's feature vector, padded to a multiple of 16."""
    nb = window // CELL - 1
    return -(-(nb * nb * 4 * BINS) // 16) * 16


def window_origins(H: int, W: int, window: int, stride: int) -> list[tuple[int, int]]:
    return [(wy, wx) for wy in range(0, H - window + 1, stride) for wx in range(0, W - window + 1, stride)]


def window_features(frame: np.ndarray, window: int, stride: int) -> np.ndarray:
    """uint8 [windows][feature_count(window)]: the HDC encoder's input for every window."""
    assert window % CELL == 0 and window >= 2 * CELL and stride % CELL == 0 and stride > 0
    H, W = frame.shape
    blocks = block_features(cell_histograms(frame))
    nb = window // CELL - 1
    F = feature_count(window)
    org = window_origins(H, W, window, stride)
    out = np.full((len(org), F), PAD_VALUE, dtype=np.uint8)
    for i, (wy, wx) in enumerate(org):
        by, bx = wy // CELL, wx // CELL
        out[i, :nb * nb * 36] = blocks[by:by + nb, bx:bx + nb].reshape(-1)
    return out


def window_features_naive(frame: np.ndarray, window: int, stride: int) -> np.ndarray:
    """The same, pixel by pixel with Python integers and math.isqrt (tiny frames only)."""
    H, W = frame.shape
    C, S = orientation_table()
    img = [[int(v) for v in row] for row in frame]

    def px(y, x):
        return img[min(max(y, 0), H - 1)][min(max(x, 0), W - 1)]

    hc, wc = H // CELL, W // CELL
    hist = [[[0] * BINS for _ in range(wc)] for _ in range(hc)]
    for y in range(hc * CELL):
        for x in range(wc * CELL):
            gx = px(y, x + 1) - px(y, x - 1)
            gy = px(y + 1, x) - px(y - 1, x)
            if gy < 0 or (gy == 0 and gx < 0):
                gx, gy = -gx, -gy
            b = sum(1 for k in range(8) if int(C[k]) * gy - int(S[k]) * gx >= 0)
            hist[y // CELL][x // CELL][b] += math.isqrt(gx * gx + gy * gy)
    nb = window // CELL - 1
    F = feature_count(window)
    rows = []
    for wy, wx in window_origins(H, W, window, stride):
        feat = []
        for by in range(wy // CELL, wy // CELL + nb):
            for bx in range(wx // CELL, wx // CELL + nb):
                v = hist[by][bx] + hist[by][bx + 1] + hist[by + 1][bx] + hist[by + 1][bx + 1]
                n = math.isqrt(sum(a * a for a in v))
                feat += [min(255, (1275 * a) // n) if n else 0 for a in v]
        rows.append(feat + [PAD_VALUE] * (F - len(feat)))
    return np.array(rows, dtype=np.uint8).reshape(-1, F)
