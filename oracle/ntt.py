"""Negacyclic transforms and polynomial products over Z_m[X]/(X^N + 1) (oracle; test infrastructure only).

Ring-LWE schemes compute over polynomials of degree N (Preliminary: HE).  The
transform used here is its plain definition: for a primitive 2N-th root of
unity w mod m, the transform of a is the vector of evaluations
A[k] = a(w^(2k+1)), k = 0..N-1, in natural order.  Because those N points are
exactly the roots of X^N + 1, the transform turns products mod X^N + 1 into
slot-wise products.  It is computed by twisting (a_j * w^j) and then a
textbook iterative radix-2 cyclic DFT with root w^2; the naive O(N^2)
evaluation and convolution below pin it in tests.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from .arith import inv, primitive_root_of_unity


@lru_cache(maxsize=None)
def root_2n(N: int, m: int) -> int:
    """The primitive 2N-th root of unity mod m used by this module (any choice gives the same products)."""
    return primitive_root_of_unity(2 * N, m)


@lru_cache(maxsize=None)
def _tables(N: int, m: int, w: int):
    twist = np.array([pow(w, j, m) for j in range(N)], dtype=np.int64)
    winv = inv(w, m)
    untwist = np.array([pow(winv, j, m) * inv(N, m) % m for j in range(N)], dtype=np.int64)
    return twist, untwist


def _cyclic_dft(b: np.ndarray, omega: int, m: int) -> np.ndarray:
    """B[k] = sum_j b[j] omega^(jk) mod m along the last axis (iterative radix-2, bit-reversed input)."""
    N = b.shape[-1]
    b = b[..., _rev(N)]
    lead = b.shape[:-1]
    length = 2
    while length <= N:
        half = length // 2
        wl = pow(omega, N // length, m)
        ws = np.array([pow(wl, i, m) for i in range(half)], dtype=np.int64)
        b = b.reshape(lead + (N // length, length))
        u = b[..., :half]
        v = b[..., half:] * ws % m
        b = np.concatenate(((u + v) % m, (u - v) % m), axis=-1)
        length *= 2
    return b.reshape(lead + (N,))


@lru_cache(maxsize=None)
def _rev(N: int) -> np.ndarray:
    bits = N.bit_length() - 1
    return np.array([int(format(i, f"0{bits}b")[::-1], 2) if bits else 0 for i in range(N)], dtype=np.int64)


def forward(a: np.ndarray, m: int, w: int | None = None) -> np.ndarray:
    """A[k] = a(w^(2k+1)) mod m for k = 0..N-1 (last axis), w a primitive 2N-th root of unity."""
    a = np.asarray(a, dtype=np.int64) % m
    N = a.shape[-1]
    w = root_2n(N, m) if w is None else w
    twist, _ = _tables(N, m, w)
    return _cyclic_dft(a * twist % m, w * w % m, m)


def inverse(A: np.ndarray, m: int, w: int | None = None) -> np.ndarray:
    """The unique a of degree < N with a(w^(2k+1)) = A[k]."""
    A = np.asarray(A, dtype=np.int64) % m
    N = A.shape[-1]
    w = root_2n(N, m) if w is None else w
    _, untwist = _tables(N, m, w)
    b = _cyclic_dft(A, inv(w * w % m, m), m)
    return b * untwist % m


def polymul(a: np.ndarray, b: np.ndarray, m: int) -> np.ndarray:
    """a * b mod (X^N + 1, m), broadcasting over leading axes."""
    return inverse(forward(a, m) * forward(b, m) % m, m)


def polymul_naive(a, b, m: int) -> np.ndarray:
    """Schoolbook negacyclic convolution with Python integers (tiny N only)."""
    a = [int(x) for x in a]
    b = [int(x) for x in b]
    N = len(a)
    out = [0] * N
    for i in range(N):
        for j in range(N):
            k = i + j
            if k < N:
                out[k] += a[i] * b[j]
            else:
                out[k - N] -= a[i] * b[j]
    return np.array([x % m for x in out], dtype=np.int64)


def evaluate_naive(a, x: int, m: int) -> int:
    """a(x) mod m by Horner's rule."""
    acc = 0
    for c in reversed([int(v) for v in a]):
        acc = (acc * x + c) % m
    return acc
