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

Subring layout (P.layout == "subring", r = 1), with K' = P.Kp and B = N/K':

* the slot exponents (odd residues e mod 2N, slots.slot_exponents) fall into the
  orbits {e * h : h = 1 (mod 2B)} = {e + 2B*c : c < K'} of the subgroup of Z_2N^*
  of order K'; query ql < B of a ciphertext takes the orbit of exponent
  e_ql = 2*brev(ql) + 1 (brev: bit reversal over log2 B bits) and class c < K' the
  slot of exponent e_ql + 2B*c mod 2N;
* query index inside group g is g*B + ql;
* model ciphertext m holds C[c][m] at class c < K and 0 at the K' - K extra classes;
* query plaintext (g, m) holds h[g*B + ql][m] at all K' slots of the orbit, so its
  slot vector is constant on every orbit and the plaintext is a polynomial in X^K'.
"""
from __future__ import annotations

from functools import lru_cache

import numpy as np

from . import slots
from .params import Params


def slot_index(P: Params, rho, u, ql, c):
    return rho * (P.N // 2) + u * P.W + ql * P.K + c


def _brev(x: np.ndarray, bits: int) -> np.ndarray:
    out = np.zeros_like(x)
    for b in range(bits):
        out |= ((x >> b) & 1) << (bits - 1 - b)
    return out


def subring_slot(P: Params, ql, c):
    """Slot of (query ql, class c) in the subring layout (module docstring)."""
    B = P.B
    e = (2 * _brev(np.asarray(ql, dtype=np.int64), B.bit_length() - 1) + 1 + 2 * B * np.asarray(c)) % (2 * P.N)
    return _exponent_to_slot(P.N)[e]


@lru_cache(maxsize=None)
def _exponent_to_slot(N: int) -> np.ndarray:
    inv = np.full(2 * N, -1, dtype=np.int64)
    inv[slots.slot_exponents(N)] = np.arange(N)
    return inv


def _subring_grid(P: Params):
    ql, c = np.meshgrid(np.arange(P.B), np.arange(P.Kp), indexing="ij")
    return ql.ravel(), c.ravel()


def _grid(P: Params):
    rho, u, ql, c = np.meshgrid(np.arange(2), np.arange(P.r), np.arange(P.Bq), np.arange(P.K),
                                indexing="ij")
    return rho.ravel(), u.ravel(), ql.ravel(), c.ravel()


def model_slots(P: Params, C: np.ndarray, m: int) -> np.ndarray:
    """Slot vector (int64 [N], values in [-128, 127] or 0) of model ciphertext m."""
    v = np.zeros(P.N, dtype=np.int64)
    if P.layout == "subring":
        ql, c = _subring_grid(P)
        ok = (c < P.K) & (m < P.D)
        v[subring_slot(P, ql[ok], c[ok])] = C[c[ok], m]
        return v
    rho, u, ql, c = _grid(P)
    j = m * P.r + u
    ok = j < P.D
    v[slot_index(P, rho, u, ql, c)[ok]] = C[c[ok], j[ok]]
    return v


def query_slots(P: Params, h: np.ndarray, g: int, m: int) -> np.ndarray:
    """Slot vector (int64 [N]) of query plaintext (g, m); h is int8 [Q][D]."""
    Qn = h.shape[0]
    v = np.zeros(P.N, dtype=np.int64)
    if P.layout == "subring":
        ql, c = _subring_grid(P)
        q = g * P.B + ql
        ok = (q < Qn) & (m < P.D)
        v[subring_slot(P, ql[ok], c[ok])] = h[q[ok], m]
        return v
    rho, u, ql, c = _grid(P)
    q = g * P.B + rho * P.Bq + ql
    j = m * P.r + u
    ok = (q < Qn) & (j < P.D)
    v[slot_index(P, rho, u, ql, c)[ok]] = h[q[ok], j[ok]]
    return v


def read_scores(P: Params, slots: np.ndarray, g: int, Qn: int) -> tuple[np.ndarray, np.ndarray]:
    """Query indices and their K scores from the decoded slot vector of group g (block u = 0)."""
    qi = np.arange(P.B)
    if P.layout == "subring":
        q = g * P.B + qi
        ok = q < Qn
        idx = subring_slot(P, qi[:, None], np.arange(P.K)[None, :])
        return q[ok], slots[idx[ok]]
    rho, ql = qi // P.Bq, qi % P.Bq
    q = g * P.B + qi
    ok = q < Qn
    idx = slot_index(P, rho[:, None], 0, ql[:, None], np.arange(P.K)[None, :])
    return q[ok], slots[idx[ok]]
