"""Randomness of key generation and encryption (oracle side; test infrastructure only).

The paper fixes no generator, sampler or error width; BFV needs a ternary
secret, uniform masks and small Gaussian errors (Preliminary: HE).  Readings:

* Generator: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) in counter form.
  Stream (seed, tag) starts at s0 = seed XOR (tag << 32); draw n (n >= 0) is
  mix(s0 + (n+1) * 0x9E3779B97F4A7C15 mod 2^64) with the published finaliser
  z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27; z *= 0x94D049BB133111EB;
  z ^= z >> 31.
* Uniform residue mod m: u mod m (bias below 2^-32 for m < 2^30, accepted).
* Ternary: (u mod 3) - 1.
* Discrete Gaussian, sigma = 3.2, support [-19, 19] (floor(6 sigma)): cumulative
  table T_k = round(2^53 * sum_{i<=k} rho(i) / sum_i rho(i)) for k = -19..19,
  rho(i) = exp(-i^2 / (2 sigma^2)) in IEEE double summed from i = -19 upward,
  with T_19 forced to 2^53; the sample is the least k with (u >> 11) < T_k.

Tags: 4 secret key, 5 model encryption, 6 Galois keys.
"""
from __future__ import annotations

import math

import numpy as np

TAG_SECRET = 4
TAG_ENCRYPT = 5
TAG_GALOIS = 6

SIGMA = 3.2
TAIL = 19

_G = 0x9E3779B97F4A7C15
_MASK = (1 << 64) - 1


def splitmix64_scalar(s0: int, n: int) -> int:
    """Draw n of the stream whose state is s0, in plain Python integers."""
    z = (s0 + (n + 1) * _G) & _MASK
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
    return z ^ (z >> 31)


def stream_state(seed: int, tag: int) -> int:
    return (seed ^ (tag << 32)) & _MASK


def draws(seed: int, tag: int, start: int, count: int) -> np.ndarray:
    """uint64 draws start .. start+count-1 of stream (seed, tag), vectorised."""
    s0 = np.uint64(stream_state(seed, tag))
    n = np.arange(start + 1, start + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = s0 + n * np.uint64(_G)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_mod(u: np.ndarray, m: int) -> np.ndarray:
    return (u % np.uint64(m)).astype(np.int64)


def ternary(u: np.ndarray) -> np.ndarray:
    return (u % np.uint64(3)).astype(np.int64) - 1


def gaussian_cdt() -> list[int]:
    """The 39 cumulative thresholds T_{-19} .. T_{19} (Python ints)."""
    rho = [math.exp(-(i * i) / (2.0 * SIGMA * SIGMA)) for i in range(-TAIL, TAIL + 1)]
    total = 0.0
    for v in rho:
        total += v
    table = []
    acc = 0.0
    for v in rho:
        acc += v
        table.append(int(round(acc / total * 9007199254740992.0)))
    table[-1] = 1 << 53
    return table


def gaussian(u: np.ndarray) -> np.ndarray:
    """Least k in [-19, 19] with (u >> 11) < T_k."""
    table = np.array(gaussian_cdt(), dtype=np.uint64)
    x = u >> np.uint64(11)
    idx = np.searchsorted(table, x, side="right")  # number of T_k <= x, i.e. first k with x < T_k
    return idx.astype(np.int64) - TAIL
