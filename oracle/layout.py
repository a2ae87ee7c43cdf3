"""EP-HDC slot packing (oracle; test infrastructure only).

The proposed method encrypts the class hypervectors and leaves the queries in
plaintext.  Each query element goes to its own plaintext, replicated k times
(once per class), so floor(N/k) queries are scored at once and D model
ciphertexts hold the class vectors, each class vector element repeated for
every query position; no rotation is needed (proposed method, op-count
comparison).  Readings used here, with the fold factor r (r = 1 is the
paper's packing):

* slot index of (row rho in {0,1}, block u < r, query ql < Bq, class c < K) is
  rho*N/2 + u*W + ql*K + c, with W = N/(2r) and Bq = floor(W/K); slots with
  ql*K + c >= Bq*K stay zero;
* query index inside ciphertext group g is g*B + rho*Bq + ql, with B = 2*Bq;
* model ciphertext m holds C[c][m*r + u] at every (rho, u, ql, c);
* query plaintext (g, m) holds h[g*B + rho*Bq + ql][m*r + u];
* a missing query (index >= Q) or dimension (index >= D) contributes 0.
"""
from __future__ import annotations

import numpy as np

from .params import Params


def slot_index(P: Params, rho, u, ql, c):
    return rho * (P.N // 2) + u * P.W + ql * P.K + c


def _grid(P: Params):
    rho, u, ql, c = np.meshgrid(np.arange(2), np.arange(P.r), np.arange(P.Bq), np.arange(P.K),
                                indexing="ij")
    return rho.ravel(), u.ravel(), ql.ravel(), c.ravel()


def model_slots(P: Params, C: np.ndarray, m: int) -> np.ndarray:
    """Slot vector (int64 [N], values in [-128, 127] or 0) of model ciphertext m."""
    v = np.zeros(P.N, dtype=np.int64)
    rho, u, ql, c = _grid(P)
    j = m * P.r + u
    ok = j < P.D
    v[slot_index(P, rho, u, ql, c)[ok]] = C[c[ok], j[ok]]
    return v


def query_slots(P: Params, h: np.ndarray, g: int, m: int) -> np.ndarray:
    """Slot vector (int64 [N]) of query plaintext (g, m); h is int8 [Q][D]."""
    Qn = h.shape[0]
    v = np.zeros(P.N, dtype=np.int64)
    rho, u, ql, c = _grid(P)
    q = g * P.B + rho * P.Bq + ql
    j = m * P.r + u
    ok = (q < Qn) & (j < P.D)
    v[slot_index(P, rho, u, ql, c)[ok]] = h[q[ok], j[ok]]
    return v


def read_scores(P: Params, slots: np.ndarray, g: int, Qn: int) -> tuple[np.ndarray, np.ndarray]:
    """Query indices and their K scores from the decoded slot vector of group g (block u = 0)."""
    qi = np.arange(P.B)
    rho, ql = qi // P.Bq, qi % P.Bq
    q = g * P.B + qi
    ok = q < Qn
    idx = slot_index(P, rho[:, None], 0, ql[:, None], np.arange(P.K)[None, :])
    return q[ok], slots[idx[ok]]
