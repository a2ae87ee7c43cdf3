"""HDC encoding and plaintext scoring (oracle; test infrastructure only).

Random-projection encoding multiplies a flattened feature vector by random
base hypervectors (Preliminary: HDC encoding); inference scores a query
hypervector against every class hypervector and returns the best class
(Preliminary: inference).  Readings:

* Features are uint8 values read as affine-quantised with zero point 128, so
  the projection is H[q][j] = sum_f (x[q][f] - 128) * B[f][j], exact in int64.
* Binarised queries (qbits = 1): h = +1 where H >= 0, else -1.
* Q-bit queries (the paper's HE-aware quantisation, Q,C bits of the
  optimisation table): h = clamp(floor(H / 2^qshift), -2^(Q-1), 2^(Q-1) - 1).
* Similarity: class vectors are taken as already normalised and quantised, so
  the cosine score becomes the integer dot product h . C[c]; with no scaling
  operation in the configurations here, the decrypted score is that dot
  product reduced to the centred residue mod t.
"""
from __future__ import annotations

import numpy as np


def project(x: np.ndarray, base: np.ndarray) -> np.ndarray:
    """H = (x - 128) @ base, int64 [Q][D]."""
    return (x.astype(np.int64) - 128) @ base.astype(np.int64)


def quantize(H: np.ndarray, qbits: int = 1, qshift: int = 0) -> np.ndarray:
    if qbits == 1:
        return np.where(H >= 0, 1, -1).astype(np.int8)
    lo, hi = -(1 << (qbits - 1)), (1 << (qbits - 1)) - 1
    return np.clip(H >> qshift, lo, hi).astype(np.int8)


def encode(x: np.ndarray, base: np.ndarray, qbits: int = 1, qshift: int = 0) -> np.ndarray:
    """Query hypervectors h, int8 [Q][D]."""
    return quantize(project(x, base), qbits, qshift)


def scores_int(h: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Exact integer similarity h . C^T, int64 [Q][K]."""
    return h.astype(np.int64) @ C.astype(np.int64).T


def scores_mod_t(h: np.ndarray, C: np.ndarray, t: int) -> np.ndarray:
    """Centred residue of the integer similarity mod t: what decryption must return."""
    s = scores_int(h, C) % t
    return np.where(s > t // 2, s - t, s)


def argmax(scores: np.ndarray) -> np.ndarray:
    """Highest score wins; ties go to the lowest class index."""
    return np.argmax(scores, axis=1).astype(np.int32)
