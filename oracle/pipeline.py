"""The client-side path end to end (oracle; test infrastructure only).

Client (proposed method): encode the plaintext queries into hypervectors,
batch-encode them into plaintexts, multiply them into the encrypted model and
accumulate, fold the blocks with rotations when r > 1, and send one score
ciphertext per group of B queries.  Server: decrypt and read the K scores of
each query, then take the argmax.
"""
from __future__ import annotations

import numpy as np

from . import bfv, hdc, slots
from .layout import read_scores
from .params import Params


def score_ciphertexts(P: Params, model_ct: np.ndarray, h: np.ndarray, gk=None,
                      groups=None) -> np.ndarray:
    """Score ciphertexts int64 [len(groups)][2][L][N] (coefficient domain) for query HVs h [Q][D]."""
    G = P.groups(h.shape[0])
    groups = range(G) if groups is None else groups
    out = []
    for g in groups:
        acc = bfv.mac(P, model_ct, h, g)
        if P.r > 1:
            acc = bfv.rotate_and_sum(P, acc, gk)
        out.append(acc)
    return np.stack(out)


def decrypt_scores(P: Params, s: np.ndarray, score_ct: np.ndarray, Qn: int, groups=None):
    """(scores int64 [Q][K] centred mod t, argmax int32 [Q]) from the groups' score ciphertexts."""
    groups = range(score_ct.shape[0]) if groups is None else groups
    scores = np.zeros((Qn, P.K), dtype=np.int64)
    for i, g in enumerate(groups):
        mu = bfv.decrypt(P, s, score_ct[i])
        v = slots.centered(slots.decode(mu, P.t), P.t)
        q, sc = read_scores(P, v, g, Qn)
        scores[q] = sc
    return scores, hdc.argmax(scores)


def run(P: Params, x: np.ndarray, base: np.ndarray, C: np.ndarray, seed: int, groups=None):
    """Whole protocol on the CPU: keys, model encryption, encoding, scoring, decryption."""
    s = bfv.secret_key(P, seed)
    model_ct = bfv.encrypt_model(P, s, C, seed)
    gk = bfv.galois_keys(P, s, seed) if P.r > 1 else None
    h = hdc.encode(x, base, P.qbits, P.qshift)
    cts = score_ciphertexts(P, model_ct, h, gk, groups)
    scores, am = decrypt_scores(P, s, cts, h.shape[0], groups)
    return dict(s=s, model_ct=model_ct, gk=gk, h=h, score_ct=cts, scores=scores, argmax=am)
