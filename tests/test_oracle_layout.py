"""Pins of the oracle's subring slot layout against the ring's structure: its slot groups
are the orbits of the subgroup {h = 1 (mod 2N/K')} of Z_2N^* (brute force over the group),
every slot is used once, query plaintexts lie in Z_t[X^K'] (a property of the ring that the
contiguous layout does not have), and whole pipelines decrypt to the exact closed form."""
import numpy as np
import pytest

import synth
from oracle import bfv, hdc, layout, ntt, pipeline, slots
from oracle.params import Params, default_primes

T = 65537


def sub(N=64, L=3, D=12, K=3, layout_="subring"):
    return Params(N=N, q=tuple(default_primes(N, L)), D=D, K=K, F=8, layout=layout_)


@pytest.mark.parametrize("N,K", [(64, 3), (64, 4), (128, 7), (128, 2), (256, 26)])
def test_query_slot_groups_are_subgroup_orbits(N, K):
    """The K' slots of each query are the orbit e * H of one exponent under the subgroup
    H = {h odd < 2N : h = 1 (mod 2N/K')}, which has K' elements; all N slots are covered once."""
    P = sub(N=N, K=K)
    P.validate()
    Kp, B = P.Kp, P.B
    assert Kp >= K and Kp & (Kp - 1) == 0 and Kp < 2 * K and B == N // Kp
    H = [h for h in range(1, 2 * N, 2) if h % (2 * B) == 1]
    assert len(H) == Kp
    exps = slots.slot_exponents(N)
    seen = set()
    for ql in range(B):
        got = {int(exps[s]) for s in layout.subring_slot(P, np.full(Kp, ql), np.arange(Kp))}
        e0 = int(exps[layout.subring_slot(P, ql, 0)])
        assert got == {e0 * h % (2 * N) for h in H}
        assert not (got & seen)
        seen |= got
    assert seen == {int(e) for e in exps}


@pytest.mark.parametrize("N,K", [(64, 3), (128, 7), (128, 2), (256, 5)])
def test_query_plaintexts_are_polynomials_in_x_to_the_kp(N, K):
    """A slot vector constant on the orbits of H is the evaluation of some p(X^K'): every
    coefficient off the multiples of K' is zero.  The contiguous layout's plaintexts are dense."""
    P = sub(N=N, K=K, D=5)
    rng = np.random.default_rng(N + K)
    h = rng.integers(-128, 128, (P.B + 3, P.D)).astype(np.int8)
    for g in range(2):
        for m in range(P.D):
            mu = slots.encode(layout.query_slots(P, h, g, m), T)
            off = np.arange(N) % P.Kp != 0
            assert not mu[off].any(), (g, m)
    Pc = sub(N=N, K=K, D=5, layout_="contiguous")
    mu = slots.encode(layout.query_slots(Pc, h, 0, 0), T)
    assert mu[np.arange(N) % 2 == 1].any()


def test_orbit_order_puts_query_ql_at_bit_reversed_exponent():
    """Query ql's orbit holds exponent 2*brev(ql) + 1 (brev over log2 B bits), the first
    exponent of its class-0 slot; class c adds 2B*c."""
    P = sub(N=64, K=4)  # B = 16
    exps = slots.slot_exponents(64)
    for ql in range(P.B):
        br = int(format(ql, "04b")[::-1], 2)
        for c in range(P.Kp):
            assert exps[layout.subring_slot(P, ql, c)] == (2 * br + 1 + 2 * P.B * c) % 128


def test_subring_batch_size_is_the_papers_for_powers_of_two():
    for N in (2048, 4096, 8192):
        for K in (2, 4, 8, 16):
            assert sub(N=N, K=K).B == N // K == Params(N=N, q=(12289,), K=K).B
        assert sub(N=N, K=7).B == N // 8 < N // 7
        assert sub(N=N, K=26).B == N // 32


@pytest.mark.parametrize("K,D,Qn,N", [(2, 16, 40, 64), (3, 9, 7, 64), (7, 33, 20, 64), (4, 10, 70, 128)])
def test_subring_pipeline_scores_equal_integer_dot_products(K, D, Qn, N):
    """Decrypted scores of the subring layout are the centred residues of h . C^T mod t,
    over ragged query groups."""
    P = sub(N=N, D=D, K=K)
    x = synth.uniform_features(7, Qn, P.F)
    base = synth.base_hypervectors(7, P.F, P.D)
    C = synth.class_hypervectors(7, P.K, P.D)
    out = pipeline.run(P, x, base, C, seed=7)
    want = hdc.scores_mod_t(out["h"], C, T)
    assert np.array_equal(out["scores"], want)
    assert np.array_equal(out["argmax"], hdc.argmax(want))


def test_subring_mac_matches_schoolbook_sum():
    """The MAC of the subring layout is the schoolbook sum of ct x pt products."""
    P = sub(N=16, D=4, K=3)
    rng = np.random.default_rng(9)
    s = bfv.secret_key(P, 9)
    C = rng.integers(-128, 128, (P.K, P.D)).astype(np.int8)
    h = rng.choice([-1, 1], (P.B + 1, P.D)).astype(np.int8)
    model = bfv.encrypt_model(P, s, C, 9)
    for g in range(P.groups(h.shape[0])):
        acc = bfv.mac(P, model, h, g)
        want = np.zeros_like(acc)
        for m in range(P.M):
            p = bfv.query_plaintext(P, h, g, m)
            for c in range(2):
                for l, q in enumerate(P.q):
                    want[c, l] = (want[c, l] + ntt.polymul_naive(model[m, c, l], p % q, q)) % q
        assert np.array_equal(acc, want)


def fold(N=64, K=3, r=2, D=12, L=4):
    primes = default_primes(N, L + 2)
    return Params(N=N, q=tuple(primes[:L]), p=tuple(primes[L:]), D=D, K=K, F=8, r=r, dnum=2,
                  layout="subring")


FOLDS = [(64, 3, 2), (64, 2, 8), (128, 2, 4), (256, 5, 4), (256, 3, 8), (128, 7, 2)]


@pytest.mark.parametrize("N,K,r", FOLDS)
def test_folded_subring_slots_are_nested_orbits(N, K, r):
    """With r > 1, block v of query ql is one orbit of H = {h = 1 (mod 2n)} (n = N/K'), the
    residue class of n-point position ql*r + v; the r blocks of a query make up one orbit of
    H' = {h = 1 (mod 2n/r)}; every slot is used once.  Brute force over both subgroups."""
    P = fold(N=N, K=K, r=r)
    P.validate()
    n, Kp, B = P.n, P.Kp, P.B
    assert n == N // Kp and B == n // r
    H = [h for h in range(1, 2 * N, 2) if h % (2 * n) == 1]
    H1 = [h for h in range(1, 2 * N, 2) if h % (2 * n // r) == 1]
    assert len(H) == Kp and len(H1) == Kp * r
    exps = slots.slot_exponents(N)
    seen = set()
    for ql in range(B):
        whole = set()
        for v in range(r):
            got = {int(exps[s]) for s in layout.subring_slot(P, ql, np.arange(Kp), v)}
            e0 = next(iter(got))
            assert got == {e0 * h % (2 * N) for h in H}
            y = ql * r + v
            br = int(format(y, f"0{n.bit_length() - 1}b")[::-1], 2)
            assert all(e % (2 * n) == 2 * br + 1 for e in got)
            assert not (got & seen)
            seen |= got
            whole |= got
        e0 = next(iter(whole))
        assert whole == {e0 * h % (2 * N) for h in H1}
    assert seen == {int(e) for e in exps}


@pytest.mark.parametrize("N,K,r", FOLDS)
def test_folded_subring_rotations_sum_blocks_into_block_zero(N, K, r):
    """Rotate-and-sum with the layout's Galois elements, applied as the ring automorphism
    X -> X^g to an encoded slot vector, leaves in slot (ql, block 0, c) the sum over the r
    blocks of (ql, c), for every query and class."""
    P = fold(N=N, K=K, r=r)
    rng = np.random.default_rng(N * r + K)
    z = rng.integers(0, 1000, N)
    mu = slots.encode(z, T)
    for g in bfv.galois_elements(P):
        mu = (mu + bfv.automorphism_int(mu, g)) % T
    out = slots.decode(mu, T)
    for ql in range(P.B):
        for c in range(P.Kp):
            blocks = [int(z[layout.subring_slot(P, ql, c, v)]) for v in range(r)]
            assert out[layout.subring_slot(P, ql, c, 0)] == sum(blocks) % T


@pytest.mark.parametrize("N,K,r", [(64, 3, 2), (128, 7, 2), (256, 5, 4)])
def test_folded_subring_plaintexts_are_polynomials_in_x_to_the_kp(N, K, r):
    P = fold(N=N, K=K, r=r, D=9)
    rng = np.random.default_rng(N + K + r)
    h = rng.integers(-128, 128, (P.B + 3, P.D)).astype(np.int8)
    off = np.arange(N) % P.Kp != 0
    for g in range(2):
        for m in range(P.M):
            mu = slots.encode(layout.query_slots(P, h, g, m), T)
            assert not mu[off].any(), (g, m)
            assert mu.any()


@pytest.mark.parametrize("N,K,r,D,Qn", [(64, 3, 2, 9, 11), (64, 2, 4, 13, 9), (128, 5, 2, 10, 70),
                                        (128, 2, 8, 17, 10)])
def test_folded_subring_pipeline_scores_equal_integer_dot_products(N, K, r, D, Qn):
    """Whole protocol with rotations in the folded subring layout (key-switched Galois
    rotations included) decrypts to the centred residues of h . C^T mod t, over ragged
    groups and a dimension count that is not a multiple of r."""
    P = fold(N=N, K=K, r=r, D=D)
    x = synth.uniform_features(21, Qn, P.F)
    base = synth.base_hypervectors(21, P.F, P.D)
    C = synth.class_hypervectors(21, P.K, P.D)
    out = pipeline.run(P, x, base, C, seed=21)
    want = hdc.scores_mod_t(out["h"], C, T)
    assert np.array_equal(out["scores"], want)
    assert np.array_equal(out["argmax"], hdc.argmax(want))


def test_folded_subring_needs_two_queries_per_ciphertext():
    with pytest.raises(AssertionError):
        fold(N=64, K=3, r=16).validate()  # n = 16, B = 1
    fold(N=64, K=3, r=8).validate()
