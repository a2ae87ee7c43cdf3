"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke check.

This module only draws data: feature vectors, base hypervectors, class
hypervectors and request traces.  It holds none of the method's arithmetic
(no encoding, no encryption, no modular reduction), so the CPU oracle and the
HIP library can both be fed from it without sharing any computation.

Every stream is SplitMix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) used in counter form:
draw n of a stream with state s0 is mix(s0 + (n + 1) * 0x9E3779B97F4A7C15).
A stream is identified by (seed, tag) and starts at s0 = seed ^ (tag << 32).

Tags used here: 1 base hypervectors, 2 class hypervectors, 3 features,
7 request traces.  Tags 4, 5 and 6 belong to key generation and encryption,
which the library and the oracle each draw with their own generator.
"""
from __future__ import annotations

import math

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

TAG_BASE = 1
TAG_CLASS = 2
TAG_FEATURES = 3
TAG_TRACE = 7


def _mix(z: np.ndarray) -> np.ndarray:
    z = z.copy()
    z ^= z >> np.uint64(30)
    z *= _M1
    z ^= z >> np.uint64(27)
    z *= _M2
    z ^= z >> np.uint64(31)
    return z


def draws(seed: int, tag: int, start: int, count: int) -> np.ndarray:
    """Draws start .. start+count-1 of stream (seed, tag), as uint64."""
    s0 = np.uint64((seed ^ (tag << 32)) & 0xFFFFFFFFFFFFFFFF)
    n = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(s0 + n * GAMMA)


def ints(seed: int, tag: int, lo: int, hi: int, shape, start: int = 0) -> np.ndarray:
    """Integers lo + (u mod (hi - lo + 1)), one draw each, in row-major order."""
    count = int(np.prod(shape))
    u = draws(seed, tag, start, count)
    span = np.uint64(hi - lo + 1)
    return (u % span).astype(np.int64).reshape(shape) + lo


def uniform01(seed: int, tag: int, count: int, start: int = 0) -> np.ndarray:
    """Doubles in [0, 1) from the top 53 bits of each draw."""
    u = draws(seed, tag, start, count)
    return (u >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


# --------------------------------------------------------------------------- HDC inputs
def base_hypervectors(seed: int, F: int, D: int) -> np.ndarray:
    """int8 [F][D], uniform in [-8, 7]: one D-dimensional random base vector per feature."""
    return ints(seed, TAG_BASE, -8, 7, (F, D)).astype(np.int8)


def class_hypervectors(seed: int, K: int, D: int) -> np.ndarray:
    """int8 [K][D], uniform in [-128, 127]: stand-in for trained, quantised class vectors."""
    return ints(seed, TAG_CLASS, -128, 127, (K, D)).astype(np.int8)


def uniform_features(seed: int, Q: int, F: int) -> np.ndarray:
    """uint8 [Q][F], uniform in [0, 255]."""
    return ints(seed, TAG_FEATURES, 0, 255, (Q, F)).astype(np.uint8)


def blob_images(seed: int, Q: int, side: int = 48) -> np.ndarray:
    """uint8 [Q][side*side]: grayscale frames with Gaussian blobs on a noisy base.

    Stand-in for 48x48 face crops (the Emotion set's frame size).  Per image:
    a base of U{0..31} noise, then 1 + (u mod 4) blobs, each with a centre
    U{0..side-1}^2, a width of 2 + (u mod 7) pixels and an amplitude U{64..255};
    the sum is clipped to [0, 255].  Image q uses draws from a fixed window of
    the stream so that any subset of images can be regenerated alone.
    """
    F = side * side
    per_image = F + 1 + 4 * 4  # noise, blob count, 4 blobs x (cx, cy, width, amplitude)
    out = np.empty((Q, F), dtype=np.uint8)
    yy, xx = np.mgrid[0:side, 0:side]
    for q in range(Q):
        u = draws(seed, TAG_FEATURES, q * per_image, per_image)
        img = (u[:F] % np.uint64(32)).astype(np.float64).reshape(side, side)
        nblob = 1 + int(u[F] % np.uint64(4))
        for b in range(nblob):
            cx, cy, w, a = (int(v) for v in u[F + 1 + 4 * b: F + 5 + 4 * b])
            cx %= side
            cy %= side
            width = 2 + (w % 7)
            amp = 64 + (a % 192)
            img += amp * np.exp(-((xx - cx) ** 2 + (yy - cy) ** 2) / (2.0 * width * width))
        out[q] = np.clip(np.floor(img), 0, 255).astype(np.uint8).reshape(F)
    return out


def frame(seed: int, H: int, W: int, n_objects: int = 24) -> np.ndarray:
    """uint8 [H][W]: one camera frame for the sliding-window detector, a stand-in for the
    face-detection frames the paper's windows are taken from.  A base of U{0..31} noise, a
    horizontal illumination ramp of up to 48 levels, and n_objects elliptical Gaussian blobs
    (centre U over the frame, widths 6 + (u mod 40) and 6 + (u mod 40) pixels, amplitude
    U{64..223}) whose sum is clipped to [0, 255]; draws from stream (seed, features tag)."""
    u = draws(seed, TAG_FEATURES, 0, H * W + 5 * n_objects)
    img = (u[:H * W] % np.uint64(32)).astype(np.float64).reshape(H, W)
    img += 48.0 * np.arange(W)[None, :] / max(1, W - 1)
    yy, xx = np.mgrid[0:H, 0:W]
    for b in range(n_objects):
        cy, cx, wy, wx, a = (int(v) for v in u[H * W + 5 * b: H * W + 5 * b + 5])
        cy %= H
        cx %= W
        sy, sx = 6 + wy % 40, 6 + wx % 40
        amp = 64 + a % 160
        y0, y1 = max(0, cy - 4 * sy), min(H, cy + 4 * sy + 1)
        x0, x1 = max(0, cx - 4 * sx), min(W, cx + 4 * sx + 1)
        dy, dx = yy[y0:y1, x0:x1] - cy, xx[y0:y1, x0:x1] - cx
        img[y0:y1, x0:x1] += amp * np.exp(-(dy * dy) / (2.0 * sy * sy) - (dx * dx) / (2.0 * sx * sx))
    return np.clip(np.floor(img), 0, 255).astype(np.uint8)


# --------------------------------------------------------------------------- request traces
def loguniform_batch_sizes(seed: int, n: int, hi: int = 4096) -> np.ndarray:
    """n batch sizes floor(exp(U[0, ln hi])), clipped to [1, hi]."""
    u = uniform01(seed, TAG_TRACE, n)
    return np.clip(np.floor(np.exp(u * math.log(hi))).astype(np.int64), 1, hi)


def batch_mix(seed: int, n: int, n_models: int, hi: int = 4096):
    """n requests of a batch: (batch sizes floor(exp(U[0, ln hi])), model index U{0..n_models-1});
    the sizes are draws 0..n-1 of the trace stream and the model choices draws n..2n-1."""
    sizes = loguniform_batch_sizes(seed, n, hi)
    models = ints(seed, TAG_TRACE, 0, n_models - 1, (n,), start=n)
    return sizes, models


def poisson_trace(seed: int, rate: float, duration: float, qmin: int, qmax: int,
                  n_tenants: int):
    """Poisson arrivals: (arrival time s, tenant, batch size) triples, sorted by time.

    Inter-arrival gaps are -ln(1-U)/rate; each request then draws its tenant
    U{0..n_tenants-1} and batch size U{qmin..qmax}.
    """
    out = []
    tnow = 0.0
    k = 0
    while True:
        u = draws(seed, TAG_TRACE, 3 * k, 3)
        gap = -math.log(1.0 - float(u[0] >> np.uint64(11)) / 9007199254740992.0) / rate
        tnow += gap
        if tnow >= duration:
            break
        tenant = int(u[1] % np.uint64(n_tenants))
        qsz = qmin + int(u[2] % np.uint64(qmax - qmin + 1))
        out.append((tnow, tenant, qsz))
        k += 1
    return out
