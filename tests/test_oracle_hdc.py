"""Pins of the oracle's HDC encoding, packing and paper-printed batch sizes."""
import os

import numpy as np

import synth
from oracle import hdc, layout
from oracle.params import Params


def test_projection_matches_loops():
    x = synth.uniform_features(1, 5, 12)
    B = synth.base_hypervectors(1, 12, 9)
    H = hdc.project(x, B)
    for q in range(5):
        for j in range(9):
            assert H[q, j] == sum((int(x[q, f]) - 128) * int(B[f, j]) for f in range(12))


def test_binarise_tie_goes_positive():
    H = np.array([[-3, 0, 5, -1]])
    assert hdc.quantize(H).tolist() == [[-1, 1, 1, -1]]


def test_qbit_quantisation():
    H = np.array([[-1000, -9, -8, 7, 8, 1000]])
    # floor division by 2^2 then clamp to 4-bit signed
    assert hdc.quantize(H, 4, 2).tolist() == [[-8, -3, -2, 1, 2, 7]]


def test_scores_mod_t_closed_form():
    t = 65537
    h = np.array([[1, -1, 1]], dtype=np.int8)
    C = np.array([[100, 20, 3], [-128, 127, -128]], dtype=np.int8)
    s = hdc.scores_mod_t(h, C, t)
    assert s.tolist() == [[83, -383]]
    big = np.full((1, 600), 127, dtype=np.int8)
    ones = np.ones((1, 600), dtype=np.int8)
    # 600 * 127 = 76200 wraps to 76200 - 65537 = 10663
    assert hdc.scores_mod_t(ones, big, t).tolist() == [[10663]]


def test_argmax_ties_lowest_class():
    assert hdc.argmax(np.array([[3, 7, 7], [-1, -1, -2]])).tolist() == [1, 0]


def test_paper_batch_sizes(golden_dir):
    """Queries per ciphertext B = 2*floor(N/(2K)) equals the batch sizes the paper prints."""
    rows = [l.split() for l in open(os.path.join(golden_dir, "paper_batch_sizes.txt"))
            if l.strip() and not l.startswith("#")]
    for N, k, batch in rows:
        P = Params(N=int(N), q=(), K=int(k), D=1024)
        assert P.B == int(batch)
        assert P.B == int(N) // int(k)


def test_paper_op_counts(golden_dir):
    """r = 1: D model ciphertexts (one MulCP + AddCC each per batch) and no rotations."""
    rows = [l.split() for l in open(os.path.join(golden_dir, "paper_op_counts.txt"))
            if l.strip() and not l.startswith("#")]
    for N, k, D, mulcp, addcc, rot in rows:
        P = Params(N=int(N), q=(), K=int(k), D=int(D))
        assert P.M == int(mulcp) == int(addcc)
        assert P.log2r == int(rot)


def test_slot_layout_is_injective_and_fills_rows():
    P = Params(N=64, q=(), K=3, D=40, r=2)
    idx = layout.slot_index(P, *np.meshgrid(np.arange(2), np.arange(P.r), np.arange(P.Bq),
                                            np.arange(P.K), indexing="ij"))
    flat = idx.ravel()
    assert len(set(flat.tolist())) == flat.size
    assert flat.max() < P.N


def test_query_and_model_slots_pair_up():
    """Slot-wise product of query (g, m) and model m summed over m = dot products at every (q, c)."""
    P = Params(N=64, q=(), K=3, D=10, r=2)
    rng = np.random.default_rng(1)
    h = rng.integers(-1, 2, (13, P.D)).astype(np.int8)
    C = rng.integers(-128, 128, (P.K, P.D)).astype(np.int8)
    for g in range(P.groups(13)):
        tot = np.zeros(P.N, dtype=np.int64)
        for m in range(P.M):
            tot += layout.query_slots(P, h, g, m) * layout.model_slots(P, C, m)
        # fold the r blocks of each row
        rows = tot.reshape(2, P.r, P.W).sum(axis=1)
        folded = np.concatenate([np.concatenate([rows[0], np.zeros(P.N // 2 - P.W, np.int64)]),
                                 np.concatenate([rows[1], np.zeros(P.N // 2 - P.W, np.int64)])])
        q, sc = layout.read_scores(P, folded, g, 13)
        assert np.array_equal(sc, hdc.scores_int(h[q], C))
