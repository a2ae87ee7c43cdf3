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

Subring layout (P.layout == "subring"), with K' = P.Kp, n = N/K' = P.n orbits and
B = n/r queries per ciphertext:

* H = {h = 1 (mod 2n)}, a subgroup of Z_2N^* of order K', acts on the slot exponents
  (odd residues e mod 2N, slots.slot_exponents); its orbits are the residue classes
  mod 2n, and orbit y < n is the class of 2*brev_n(y) + 1 (brev_n: bit reversal over
  log2 n bits).  A slot vector constant on every orbit is the evaluation of a
  polynomial in X^K', whose n-point transform has the orbit's value at position y;
* query ql < B and block v < r take orbit y = ql*r + v; the r orbits of query ql make
  up one orbit of H' = {h = 1 (mod 2n/r)} (order K' r), the one of
  e_ql = 2*brev_B(ql) + 1.  H' is cyclic with generator gamma = 1 + 2n/r (B >= 2);
* class c < K' of (ql, v) is the exponent gamma^u * (e_ql + 2n*c) mod 2N, with u < r
  the power for which gamma^u * e_ql lies in orbit ql*r + v (u = 0 at v = 0);
* rotation i of rotate-and-sum uses the Galois element gamma^(2^i) mod 2N.  Slot
  exponent e then receives the sum over k < r of the old values at e * gamma^k, which at
  e = e_ql + 2n*c are the r blocks of (ql, c): block 0 holds each class's total (the
  other blocks may mix classes and are not read);
* query index inside group g is g*B + ql;
* model ciphertext m holds C[c][m*r + v] at class c < K and 0 at the K' - K extra classes
  and at dimensions >= D;
* query plaintext (g, m) holds h[g*B + ql][m*r + v] at all K' slots of orbit ql*r + v.
For r = 1 every u is 0 and class c of query ql is exponent e_ql + 2n*c.
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


def subring_gamma(P: Params) -> int:
    """Generator 1 + 2n/r of H' = {h = 1 (mod 2n/r)} (module docstring)."""
    return 1 + 2 * P.n // P.r


@lru_cache(maxsize=None)
def _block_power(N: int, Kp: int, r: int) -> np.ndarray:
    """u[ql][v] < r with gamma^u * e_ql in orbit ql*r + v, found by trying every u."""
    n = N // Kp
    B = n // r
    gamma = 1 + 2 * n // r
    e = 2 * _brev(np.arange(B), B.bit_length() - 1) + 1
    u_of = np.full((B, r), -1, dtype=np.int64)
    for u in range(r):
        res = pow(gamma, u, 2 * n) * e % (2 * n)
        y = _brev((res - 1) // 2, n.bit_length() - 1)
        v = y - np.arange(B) * r
        assert ((v >= 0) & (v < r)).all()
        u_of[np.arange(B), v] = u
    assert (u_of >= 0).all()
    return u_of


def subring_slot(P: Params, ql, c, v=0):
    """Slot of (query ql, block v, class c) in the subring layout (module docstring)."""
    n, B, N = P.n, P.B, P.N
    ql, c, v = np.broadcast_arrays(np.asarray(ql, dtype=np.int64), np.asarray(c, dtype=np.int64),
                                   np.asarray(v, dtype=np.int64))
    e = 2 * _brev(ql, B.bit_length() - 1) + 1
    u = _block_power(N, P.Kp, P.r)[ql, v]
    gu = np.array([pow(subring_gamma(P), int(k), 2 * N) for k in range(P.r)], dtype=np.int64)
    return _exponent_to_slot(N)[gu[u] * ((e + 2 * n * c) % (2 * N)) % (2 * N)]


@lru_cache(maxsize=None)
def _exponent_to_slot(N: int) -> np.ndarray:
    inv = np.full(2 * N, -1, dtype=np.int64)
    inv[slots.slot_exponents(N)] = np.arange(N)
    return inv


def _subring_grid(P: Params):
    ql, v, c = np.meshgrid(np.arange(P.B), np.arange(P.r), np.arange(P.Kp), indexing="ij")
    return ql.ravel(), v.ravel(), c.ravel()


def _grid(P: Params):
    rho, u, ql, c = np.meshgrid(np.arange(2), np.arange(P.r), np.arange(P.Bq), np.arange(P.K),
                                indexing="ij")
    return rho.ravel(), u.ravel(), ql.ravel(), c.ravel()


def model_slots(P: Params, C: np.ndarray, m: int) -> np.ndarray:
    """Slot vector (int64 [N], values in [-128, 127] or 0) of model ciphertext m."""
    v = np.zeros(P.N, dtype=np.int64)
    if P.layout == "subring":
        ql, u, c = _subring_grid(P)
        j = m * P.r + u
        ok = (c < P.K) & (j < P.D)
        v[subring_slot(P, ql[ok], c[ok], u[ok])] = C[c[ok], j[ok]]
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
        ql, u, c = _subring_grid(P)
        q = g * P.B + ql
        j = m * P.r + u
        ok = (q < Qn) & (j < P.D)
        v[subring_slot(P, ql[ok], c[ok], u[ok])] = h[q[ok], j[ok]]
        return v
    rho, u, ql, c = _grid(P)
    q = g * P.B + rho * P.Bq + ql
    j = m * P.r + u
    ok = (q < Qn) & (j < P.D)
    v[slot_index(P, rho, u, ql, c)[ok]] = h[q[ok], j[ok]]
    return v


def read_scores(P: Params, slots: np.ndarray, g: int, Qn: int) -> tuple[np.ndarray, np.ndarray]:
    """Query indices and their K scores from the decoded slot vector of group g (block 0)."""
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
