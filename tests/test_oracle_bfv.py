"""Pins of the oracle's BFV: definitions written out with schoolbook products, decryption
identities, the exact integer score closed form, base-conversion identities with big
integers, and rotation by Galois automorphism + key switching."""
import math

import numpy as np
import pytest

import synth
from oracle import bfv, hdc, ntt, pipeline, prng, slots
from oracle.arith import inv
from oracle.params import Params, default_primes

T = 65537


def tiny(N=32, L=3, D=12, K=3, r=1, alpha=0, dnum=0):
    primes = default_primes(N, L + alpha)
    return Params(N=N, q=tuple(primes[:L]), p=tuple(primes[L:]), D=D, K=K, r=r, F=8, dnum=dnum)


def test_encryption_definition_schoolbook():
    """c0 + c1*s = Delta*mu + e (mod q_l), with e the Gaussian draws of the ciphertext's window."""
    P = tiny(N=16)
    s = bfv.secret_key(P, 9)
    mu = np.random.default_rng(0).integers(0, T, P.N)
    ct = bfv.encrypt(P, s, mu, 9, index=2)
    e = prng.gaussian(prng.draws(9, prng.TAG_ENCRYPT, 2 * (P.L + 1) * P.N + P.L * P.N, P.N))
    for l, q in enumerate(P.q):
        lhs = (ct[0, l] + ntt.polymul_naive(ct[1, l], s % q, q)) % q
        assert np.array_equal(lhs, (P.Delta % q * mu + e) % q)
        a = prng.uniform_mod(prng.draws(9, prng.TAG_ENCRYPT, 2 * (P.L + 1) * P.N + l * P.N, P.N), q)
        assert np.array_equal(ct[1, l], a)


def test_decrypt_inverts_encrypt():
    P = tiny(N=64)
    s = bfv.secret_key(P, 1)
    mu = np.random.default_rng(1).integers(0, T, P.N)
    assert np.array_equal(bfv.decrypt(P, s, bfv.encrypt(P, s, mu, 1, 0)), mu)


def test_decrypt_of_ct_times_pt():
    """Dec(Enc(m) * p) = m * p mod (X^N + 1, t), for the centred lift of p."""
    P = tiny(N=32)
    rng = np.random.default_rng(2)
    s = bfv.secret_key(P, 2)
    mu = rng.integers(0, T, P.N)
    p = bfv.lift_centered(rng.integers(0, T, P.N), T)
    ct = bfv.mul_plain(P, bfv.encrypt(P, s, mu, 2, 0), p)
    assert np.array_equal(bfv.decrypt(P, s, ct), ntt.polymul_naive(mu, p % T, T))


def test_mac_matches_schoolbook_sum():
    P = tiny(N=16, D=5, K=2)
    rng = np.random.default_rng(3)
    s = bfv.secret_key(P, 3)
    C = rng.integers(-128, 128, (P.K, P.D)).astype(np.int8)
    h = rng.choice([-1, 1], (P.B + 3, P.D)).astype(np.int8)
    model = bfv.encrypt_model(P, s, C, 3)
    for g in range(P.groups(h.shape[0])):
        acc = bfv.mac(P, model, h, g, chunk=2)
        want = np.zeros_like(acc)
        for m in range(P.M):
            p = bfv.query_plaintext(P, h, g, m)
            for c in range(2):
                for l, q in enumerate(P.q):
                    want[c, l] = (want[c, l] + ntt.polymul_naive(model[m, c, l], p % q, q)) % q
        assert np.array_equal(acc, want)


@pytest.mark.parametrize("K,D,Qn", [(2, 16, 20), (3, 9, 7), (7, 33, 5)])
def test_pipeline_scores_equal_integer_dot_products(K, D, Qn):
    """Decrypted scores are the centred residues of h . C^T mod t (exact closed form)."""
    P = tiny(N=64, D=D, K=K)
    x = synth.uniform_features(5, Qn, P.F)
    base = synth.base_hypervectors(5, P.F, P.D)
    C = synth.class_hypervectors(5, P.K, P.D)
    out = pipeline.run(P, x, base, C, seed=5)
    want = hdc.scores_mod_t(out["h"], C, T)
    assert np.array_equal(out["scores"], want)
    assert np.array_equal(out["argmax"], hdc.argmax(want))


def test_scores_wrap_mod_t():
    """With |h . C| above t/2 the decrypted score is the centred residue, not the integer."""
    P = tiny(N=32, D=600, K=2)
    h = np.ones((3, P.D), dtype=np.int8)
    C = np.full((P.K, P.D), 127, dtype=np.int8)
    s = bfv.secret_key(P, 4)
    model = bfv.encrypt_model(P, s, C, 4)
    ct = pipeline.score_ciphertexts(P, model, h)
    scores, _ = pipeline.decrypt_scores(P, s, ct, 3)
    assert (scores == 600 * 127 - T).all()


def test_mod_up_is_exact_crt_plus_small_multiple():
    P = tiny(N=8, L=4, alpha=2, dnum=2, r=2, D=4, K=1)
    rng = np.random.default_rng(5)
    digit = P.digits()[1]
    d = np.stack([rng.integers(0, q, P.N) for q in P.q])
    y = bfv.mod_up(P, d, digit)
    Qj = 1
    for i in digit:
        Qj *= P.q[i]
    mods = list(P.q) + list(P.p)
    for k in range(P.N):
        # integer value of the digit by CRT, and the unreduced conversion sum
        dint = sum(int(d[i, k]) * (Qj // P.q[i]) * inv(Qj // P.q[i], P.q[i]) for i in digit) % Qj
        S = sum((int(d[i, k]) * inv(Qj // P.q[i], P.q[i]) % P.q[i]) * (Qj // P.q[i]) for i in digit)
        assert S % Qj == dint and 0 <= S < len(digit) * Qj
        for l, m in enumerate(mods):
            assert int(y[l, k]) == S % m


def test_mod_down_divides_by_P():
    P = tiny(N=8, L=4, alpha=2, dnum=2, r=2, D=4, K=1)
    rng = np.random.default_rng(6)
    mods = list(P.q) + list(P.p)
    PQ = P.Qmod * P.Pmod
    X = [int(rng.integers(0, 2**62)) * int(rng.integers(0, 2**62)) * 977 % PQ for _ in range(P.N)]
    x = np.array([[v % m for v in X] for m in mods], dtype=np.int64)
    out = bfv.mod_down(P, x)
    for k in range(P.N):
        SP = sum((X[k] % p * inv(P.Pmod // p, p) % p) * (P.Pmod // p) for p in P.p)
        assert (X[k] - SP) % P.Pmod == 0
        want = (X[k] - SP) // P.Pmod
        for l, q in enumerate(P.q):
            assert int(out[l, k]) == want % q


def test_automorphism_composes_polynomials():
    """sigma_g(a)(X) = a(X^g) mod X^N + 1, by substituting monomials with Python integers."""
    N, g = 16, 5
    a = np.random.default_rng(8).integers(-50, 50, N)
    want = [0] * N
    for j in range(N):
        e = j * g % (2 * N)
        if e < N:
            want[e] += int(a[j])
        else:
            want[e - N] -= int(a[j])
    assert bfv.automorphism_int(a, g).tolist() == want


def _rot_params():
    return tiny(N=64, L=4, alpha=2, dnum=2, r=4, D=16, K=2)


def test_key_switched_rotation_decrypts_to_rotated_slots():
    P = _rot_params()
    s = bfv.secret_key(P, 12)
    gk = bfv.galois_keys(P, s, 12)
    v = np.random.default_rng(12).integers(0, T, P.N)
    ct = bfv.encrypt(P, s, slots.encode(v, T), 12, 0)
    for i, g in enumerate(bfv.galois_elements(P)):
        rot = bfv.automorphism(ct, g, P.q)
        b, a = bfv.key_switch(P, rot[1], gk[i])
        ks = np.stack([(rot[0] + b) % np.array(P.q)[:, None], a])
        k = P.W << i
        h = P.N // 2
        want = np.concatenate((np.roll(v[:h], -k), np.roll(v[h:], -k)))
        assert np.array_equal(slots.decode(bfv.decrypt(P, s, ks), T), want)
        assert bfv.noise_bits(P, s, ks) < P.Delta.bit_length() - 3


def test_rotate_and_sum_scores_equal_integer_dot_products():
    P = _rot_params()
    Qn = 2 * P.B + 1
    x = synth.uniform_features(13, Qn, P.F)
    base = synth.base_hypervectors(13, P.F, P.D)
    C = synth.class_hypervectors(13, P.K, P.D)
    out = pipeline.run(P, x, base, C, seed=13)
    assert np.array_equal(out["scores"], hdc.scores_mod_t(out["h"], C, T))


def test_galois_key_definition():
    """b + a*s = e + G_j * sigma_g(s) on every modulus, with G_j = P on the digit's limbs, else 0."""
    P = _rot_params()
    s = bfv.secret_key(P, 14)
    gk = bfv.galois_keys(P, s, 14)
    mods = list(P.q) + list(P.p)
    for i, g in enumerate(bfv.galois_elements(P)):
        srot = bfv.automorphism_int(s, g)
        for j, digit in enumerate(P.digits()):
            e = prng.gaussian(prng.draws(14, prng.TAG_GALOIS,
                                         ((i * P.dnum + j) * (len(mods) + 1) + len(mods)) * P.N, P.N))
            for l, m in enumerate(mods):
                lhs = (gk[i, j, 0, l] + ntt.polymul_naive(gk[i, j, 1, l], s % m, m)) % m
                G = P.Pmod % m if l in digit else 0
                assert np.array_equal(lhs, (e + G * srot) % m)


def test_batched_model_encryption_equals_per_ciphertext():
    P = tiny(N=32, D=7, K=2)
    s = bfv.secret_key(P, 15)
    C = synth.class_hypervectors(15, P.K, P.D)
    batched = bfv.encrypt_model(P, s, C, 15, ms=[0, 3, 6], chunk=2)
    for i, m in enumerate([0, 3, 6]):
        assert np.array_equal(batched[i], bfv.encrypt(P, s, bfv.model_plaintext(P, C, m), 15, m))


def test_noise_budget_decides_correctness():
    """The invariant noise is real: with two 19-bit primes (Q about 2^38, Delta about 2^22)
    a fresh ciphertext still decrypts, but after the ct x pt products of a dot product the
    noise exceeds Delta/2 and the scores come out wrong; with the default 30-bit primes the
    same computation keeps the noise far below Delta/2 and decrypts to the exact scores. A
    dropped error term or a wrong scaling in the oracle would fail one of the two halves."""
    N, D, K = 32, 12, 3
    rng = np.random.default_rng(11)
    C = rng.integers(-128, 128, (K, D)).astype(np.int8)
    h = rng.choice([-1, 1], (5, D)).astype(np.int8)
    want = hdc.scores_mod_t(h, C, T)
    small = Params(N=N, q=tuple(default_primes(N, 2, bound=1 << 19)), D=D, K=K, F=8)
    big = tiny(N=N, L=2, D=D, K=K)
    for P, ok in ((small, False), (big, True)):
        s = bfv.secret_key(P, 5)
        mu = np.random.default_rng(5).integers(0, T, P.N)
        fresh = bfv.encrypt(P, s, mu, 5, 0)
        assert np.array_equal(bfv.decrypt(P, s, fresh), mu)  # fresh noise |e| <= 19 < Delta/2
        model = bfv.encrypt_model(P, s, C, 5)
        cts = pipeline.score_ciphertexts(P, model, h)
        scores, _ = pipeline.decrypt_scores(P, s, cts, h.shape[0])
        assert np.array_equal(scores, want) == ok, P.q
        if ok:  # the distance to the nearest codeword is the true noise when decryption is right
            noise = max(bfv.noise_bits(P, s, ct) for ct in cts)
            assert noise < math.log2(P.Delta) - 1 - 5, (noise, math.log2(P.Delta))
