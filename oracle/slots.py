"""SIMD slots of the plaintext ring Z_t[X]/(X^N + 1) (oracle; test infrastructure only).

With t = 1 (mod 2N) the plaintext ring splits into N copies of Z_t, so one
plaintext carries a vector of N integers and ct x pt products act slot by
slot (Preliminary: HE, packing).  The paper does not fix which slot is which;
the reading used here puts slot s at an evaluation point chosen so that the
Galois automorphism X -> X^(3^k) rotates each half of the vector by k:

  zeta = g^((t-1)/(2N)) mod t   (g the smallest generator of Z_t^*, so zeta has
                                 order 2N; g = 3 for t = 65537)
  slot s < N/2      <->  point zeta^(3^s mod 2N)
  slot N/2 + s      <->  point zeta^(-3^s mod 2N)

Encode(v) is the unique mu of degree < N with mu(x_s) = v_s (mod t); Decode
is evaluation at the N points.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from . import ntt
from .arith import smallest_generator


@lru_cache(maxsize=None)
def zeta(N: int, t: int) -> int:
    return pow(smallest_generator(t), (t - 1) // (2 * N), t)


@lru_cache(maxsize=None)
def slot_exponents(N: int) -> np.ndarray:
    """Odd exponent e_s in [0, 2N) of the evaluation point of slot s."""
    e = np.empty(N, dtype=np.int64)
    g = 1
    for s in range(N // 2):
        e[s] = g
        e[N // 2 + s] = (2 * N - g) % (2 * N)
        g = g * 3 % (2 * N)
    return e


@lru_cache(maxsize=None)
def slot_to_eval_index(N: int) -> np.ndarray:
    """k_s with zeta^(2 k_s + 1) = x_s: where slot s sits in the natural-order transform."""
    return (slot_exponents(N) - 1) // 2


def decode(mu: np.ndarray, t: int) -> np.ndarray:
    """Slot vector of mu: v_s = mu(x_s) mod t (last axis)."""
    N = mu.shape[-1]
    evals = ntt.forward(mu, t, zeta(N, t))
    return evals[..., slot_to_eval_index(N)]


def encode(v: np.ndarray, t: int) -> np.ndarray:
    """mu with coefficients in [0, t) whose slot vector is v mod t (last axis)."""
    v = np.asarray(v, dtype=np.int64) % t
    N = v.shape[-1]
    evals = np.empty_like(v)
    evals[..., slot_to_eval_index(N)] = v
    return ntt.inverse(evals, t, zeta(N, t))


def decode_naive(mu, t: int) -> np.ndarray:
    """Direct evaluation at every slot point (tiny N only)."""
    N = len(mu)
    z = zeta(N, t)
    return np.array([ntt.evaluate_naive(mu, pow(z, int(e), t), t) for e in slot_exponents(N)],
                    dtype=np.int64)


def centered(x: np.ndarray, m: int) -> np.ndarray:
    """Representative of x mod m in (-m/2, m/2]."""
    x = np.asarray(x, dtype=np.int64) % m
    return np.where(x > m // 2, x - m, x)
