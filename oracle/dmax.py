"""findDmax: the largest HDC dimension whose encrypted dot product still decrypts
(oracle; test infrastructure only).

The design-space exploration (Exploration Algorithm, Algorithm 1, procedure
findDmax) grows D one dimension at a time while an encrypted ciphertext x
plaintext dot product of D terms still decrypts correctly, repeats this for many
trials and returns the mean; the noise study (Effect of HE Noise) plots the
result against N and log2 t for BFV and BGV.  Readings (the paper is silent):

* One trial draws fresh inputs: a secret key, K class hypervectors and B query
  hypervectors of d_cap dimensions, the model ciphertexts of the class values
  (packed as in the scoring path, r = 1) and the query plaintexts of one group.
* evalHEcomputation(N, T, D) of a trial is the score ciphertext of the first D
  terms, sum_{m<D} ct_m * p_m; it is correct when it decrypts to the plaintext
  of the exact dot products mod t (every slot).  The while loop therefore stops
  at the first D whose D-term sum fails, and the trial's D_i is the last D that
  decrypted (0 when one term already fails; d_cap when no prefix fails).
* Trial i uses seed + i for every stream: secret key (tag 4), encryption
  (tag 5), class values (tag 8, draw m*K + c) and query values (tag 9, draw
  m*B + q).  A value of b bits is 2*(u mod 2) - 1 for b = 1, else
  -2^(b-1) + (u mod 2^b).
"""
from __future__ import annotations

import numpy as np

from . import bfv, prng, slots
from .layout import model_slots, query_slots
from .params import Params

TAG_DMAX_CLASS = 8
TAG_DMAX_QUERY = 9


def _values(u: np.ndarray, bits: int) -> np.ndarray:
    if bits == 1:
        return 2 * (u % np.uint64(2)).astype(np.int64) - 1
    return (u % np.uint64(1 << bits)).astype(np.int64) - (1 << (bits - 1))


def trial_inputs(P: Params, seed: int, d_cap: int, cbits: int):
    """(C int64 [K][d_cap], h int64 [B][d_cap]) of the trial whose seed is `seed`."""
    K, B = P.K, P.B
    uc = prng.draws(seed, TAG_DMAX_CLASS, 0, d_cap * K).reshape(d_cap, K)
    uq = prng.draws(seed, TAG_DMAX_QUERY, 0, d_cap * B).reshape(d_cap, B)
    return _values(uc, cbits).T.copy(), _values(uq, P.qbits).T.copy()


def expected_plaintext(P: Params, C: np.ndarray, h: np.ndarray, D: int) -> np.ndarray:
    """mu of the exact D-term dot products: Encode(sum_{m<D} model slots * query slots) mod t."""
    acc = np.zeros(P.N, dtype=np.int64)
    for m in range(D):
        acc = (acc + model_slots(P, C, m) * query_slots(P, h, 0, m)) % P.t
    return slots.encode(acc, P.t)


def trial(P: Params, seed: int, d_cap: int, cbits: int, from_scratch: bool = False) -> int:
    """D_i of one trial (see the module docstring); P.D must equal d_cap and P.r 1.

    With from_scratch, every evalHEcomputation(D) recomputes its D-term sum and
    expected plaintext from nothing (the literal loop); otherwise the D-term sum
    is the (D-1)-term sum plus one product, which is the same ciphertext.
    """
    assert P.D == d_cap and P.r == 1
    C, h = trial_inputs(P, seed, d_cap, cbits)
    s = bfv.secret_key(P, seed)
    model = bfv.encrypt_model(P, s, C, seed)
    L = P.L
    acc = np.zeros((2, L, P.N), dtype=np.int64)
    want = np.zeros(P.N, dtype=np.int64)
    D = 0
    while D < d_cap:
        if from_scratch:
            acc = np.zeros((2, L, P.N), dtype=np.int64)
            for m in range(D + 1):
                acc = (acc + bfv.mul_plain(P, model[m], bfv.query_plaintext(P, h, 0, m))) % \
                    np.asarray(P.q, dtype=np.int64).reshape(1, L, 1)
            mu_want = expected_plaintext(P, C, h, D + 1)
        else:
            acc = (acc + bfv.mul_plain(P, model[D], bfv.query_plaintext(P, h, 0, D))) % \
                np.asarray(P.q, dtype=np.int64).reshape(1, L, 1)
            want = (want + model_slots(P, C, D) * query_slots(P, h, 0, D)) % P.t
            mu_want = slots.encode(want, P.t)
        if not np.array_equal(bfv.decrypt(P, s, acc), mu_want):
            break
        D += 1
    return D


def find_dmax(P: Params, trials: int, d_cap: int, seed: int, cbits: int = 8):
    """(mean of D_i, [D_i]) over `trials` trials with seeds seed, seed+1, ..."""
    ds = [trial(P, seed + i, d_cap, cbits) for i in range(trials)]
    return float(np.mean(ds)), ds
