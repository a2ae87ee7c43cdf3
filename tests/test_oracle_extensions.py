"""Pins of the oracle's HE-aware scaling op, general plaintext moduli t, the BGV and
rounded-scaling BFV variants, and findDmax -- each against something other than the
oracle itself: schoolbook products, exact integer division, closed-form block sums,
brute-force evaluation and the literal (recompute-from-scratch) loop of findDmax."""
import numpy as np
import pytest

from oracle import bfv, dmax, hdc, ntt, pipeline, prng, slots
from oracle.arith import is_prime
from oracle.layout import model_slots, query_slots
from oracle.params import Params, default_primes


def tiny(N=32, L=2, D=12, K=3, t=65537, **kw):
    return Params(N=N, q=tuple(default_primes(N, L)), t=t, D=D, K=K, F=8, **kw)


# ------------------------------------------------------------------ general t: slot map
@pytest.mark.parametrize("N,t", [(32, 257), (64, 7681), (16, 40961), (32, 114689), (64, 65537)])
def test_slot_map_for_other_plaintext_primes(N, t):
    """zeta has order exactly 2N; decode equals brute-force evaluation at the slot points;
    decode(encode(v)) = v; encode is multiplicative slot-wise."""
    assert is_prime(t) and t % (2 * N) == 1
    z = slots.zeta(N, t)
    assert pow(z, 2 * N, t) == 1 and pow(z, N, t) == t - 1
    rng = np.random.default_rng(N + t)
    mu = rng.integers(0, t, N)
    assert np.array_equal(slots.decode(mu, t), slots.decode_naive(mu, t))
    v, w = rng.integers(0, t, N), rng.integers(0, t, N)
    assert np.array_equal(slots.decode(slots.encode(v, t), t), v)
    prod = ntt.polymul_naive(slots.encode(v, t), slots.encode(w, t), t)
    assert np.array_equal(slots.decode(prod, t), v * w % t)


def test_slot_root_of_65537_is_unchanged():
    """The smallest generator of Z_65537^* is 3, so zeta = 3^((t-1)/2N) as before."""
    for N in (4096, 8192, 16384):
        assert slots.zeta(N, 65537) == pow(3, 65536 // (2 * N), 65537)


# ------------------------------------------------------------------ BGV and rounded BFV
def test_bgv_encryption_definition_schoolbook():
    """BGV: c0 + c1*s = t*e + centred(mu) (mod q_l), e the ciphertext's Gaussian draws."""
    P = tiny(N=16, scheme="bgv")
    s = bfv.secret_key(P, 7)
    mu = np.random.default_rng(0).integers(0, P.t, P.N)
    ct = bfv.encrypt(P, s, mu, 7, index=1)
    e = prng.gaussian(prng.draws(7, prng.TAG_ENCRYPT, (P.L + 1) * P.N + P.L * P.N, P.N))
    mc = np.where(mu > P.t // 2, mu - P.t, mu)
    for l, q in enumerate(P.q):
        lhs = (ct[0, l] + ntt.polymul_naive(ct[1, l], s % q, q)) % q
        assert np.array_equal(lhs, (P.t * e + mc) % q)


def test_rounded_bfv_encryption_definition():
    """BFV with rounded scaling: c0 + c1*s = e + round(Q*mu/t) (mod q_l), the rounding
    done on the whole product Q*mu with Python integers."""
    P = tiny(N=16, t=257, scheme="bfv-r")
    s = bfv.secret_key(P, 8)
    mu = np.random.default_rng(1).integers(0, P.t, P.N)
    ct = bfv.encrypt(P, s, mu, 8, index=0)
    e = prng.gaussian(prng.draws(8, prng.TAG_ENCRYPT, P.L * P.N, P.N))
    Qm = P.Qmod
    rnd = [(2 * Qm * int(m) + P.t) // (2 * P.t) for m in mu]
    for l, q in enumerate(P.q):
        lhs = (ct[0, l] + ntt.polymul_naive(ct[1, l], s % q, q)) % q
        want = np.array([(int(ei) + r) % q for ei, r in zip(e, rnd)], dtype=np.int64)
        assert np.array_equal(lhs, want)


@pytest.mark.parametrize("scheme,t", [("bgv", 65537), ("bgv", 257), ("bfv-r", 65537), ("bfv", 7681)])
def test_decrypt_of_ct_times_pt_other_schemes(scheme, t):
    """Dec(Enc(m)) = m and Dec(Enc(m) * p) = m * p mod (X^N + 1, t)."""
    P = tiny(N=32, L=3, t=t, scheme=scheme)
    rng = np.random.default_rng(3)
    s = bfv.secret_key(P, 3)
    mu = rng.integers(0, t, P.N)
    ct = bfv.encrypt(P, s, mu, 3, 0)
    assert np.array_equal(bfv.decrypt(P, s, ct), mu)
    p = bfv.lift_centered(rng.integers(0, t, P.N), t)
    assert np.array_equal(bfv.decrypt(P, s, bfv.mul_plain(P, ct, p)), ntt.polymul_naive(mu, p % t, t))


@pytest.mark.parametrize("scheme", ["bgv", "bfv-r"])
def test_pipeline_other_schemes_give_exact_scores(scheme):
    P = tiny(N=64, L=3, D=9, K=2, scheme=scheme)
    rng = np.random.default_rng(4)
    x = rng.integers(0, 256, (13, P.F)).astype(np.uint8)
    base = rng.integers(-8, 8, (P.F, P.D)).astype(np.int8)
    C = rng.integers(-128, 128, (P.K, P.D)).astype(np.int8)
    out = pipeline.run(P, x, base, C, seed=4)
    assert np.array_equal(out["scores"], hdc.scores_mod_t(out["h"], C, P.t))


# ------------------------------------------------------------------ HE-aware scaling op
def test_scale_constant_inverts_two_to_the_s():
    for t in (65537, 40961, 12289, 257):
        for s_ in range(0, 17):
            P = Params(N=16, q=tuple(default_primes(16, 1)), t=t, scale_shift=s_)
            c = P.scale_const
            assert (c * pow(2, s_, t)) % t == 1 and -t // 2 <= c <= t // 2
    # t = 2^16 + 1: 2^16 = -1, so the inverse of 2^s is -2^(16-s)
    assert Params(N=16, q=(97,), scale_shift=3).scale_const == -(1 << 13)


def _scaled_case(scale_every, scale_shift, mult):
    """Params, h, C, secret, model for a 3-block MAC (D = 3 * scale_every)."""
    g = scale_every
    P = tiny(N=32, L=3, D=3 * g, K=2, scale_every=g, scale_shift=scale_shift)
    rng = np.random.default_rng(5)
    C = rng.integers(-3, 4, (P.K, P.D)) * mult[None, :]
    h = rng.choice([-1, 1], (P.B, P.D)).astype(np.int8)
    s = bfv.secret_key(P, 5)
    return P, h, C, s, bfv.encrypt_model(P, s, C, 5)


def test_scaling_divides_exactly_when_divisible():
    """Block k of g accumulations is followed by n_k = 3 - k scalings; with every class value
    of block k a multiple of 2^(s*n_k), the decrypted scores are the exact integer sums of
    (C / 2^(s*n_k)) . h -- the scaling op is division by 2^s."""
    g, s_ = 2, 2
    nk = np.repeat([3, 2, 1], g)
    P, h, C, s, model = _scaled_case(g, s_, (1 << (s_ * nk)))
    ct = pipeline.score_ciphertexts(P, model, h)
    scores, _ = pipeline.decrypt_scores(P, s, ct, h.shape[0])
    want = h.astype(np.int64) @ (C // (1 << (s_ * nk))[None, :]).T
    assert np.array_equal(scores, want)


@pytest.mark.parametrize("g,s_", [(2, 14), (3, 16), (4, 15)])
def test_scaling_matches_block_sum_closed_form(g, s_):
    """Decrypted = sum_k S_k * c^(n_k) mod t, S_k the integer dot product over block k,
    n_k the scalings after it (complete blocks only), c = (2^s)^-1 mod t.  For t = 2^16 + 1,
    |c| = 2^(16-s): each scaling multiplies the noise by that, so the shifts here keep it small."""
    P = tiny(N=32, L=3, D=3 * g + 1, K=3, scale_every=g, scale_shift=s_)  # a trailing partial block
    rng = np.random.default_rng(6)
    C = rng.integers(-128, 128, (P.K, P.D)).astype(np.int8)
    h = rng.choice([-1, 1], (P.B, P.D)).astype(np.int8)
    s = bfv.secret_key(P, 6)
    ct = pipeline.score_ciphertexts(P, bfv.encrypt_model(P, s, C, 6), h)
    scores, _ = pipeline.decrypt_scores(P, s, ct, h.shape[0])
    c = pow(2, -s_, P.t)
    want = np.zeros((h.shape[0], P.K), dtype=object)
    nfull = P.M // g
    for k in range(-(-P.M // g)):
        blk = slice(k * g, min(P.M, (k + 1) * g))
        Sk = h[:, blk].astype(np.int64) @ C[:, blk].astype(np.int64).T
        n = nfull - k if k < nfull else 0
        want = want + Sk.astype(object) * pow(c, n, P.t)
    want = np.array([[int(v) % P.t for v in row] for row in want], dtype=np.int64)
    assert np.array_equal(scores, np.where(want > P.t // 2, want - P.t, want))


def test_scaling_noise_grows_by_the_scalar():
    """With s = 1 (|c| = 2^15 for t = 2^16 + 1) three scalings multiply the first block's noise
    by 2^45: the margin falls by about that much against the unscaled MAC."""
    P, h, C, s, model = _scaled_case(2, 1, np.ones(6, dtype=np.int64))
    P0 = Params(**{**P.__dict__, "scale_every": 0})
    ct, ct0 = bfv.mac(P, model, h, 0), bfv.mac(P0, model, h, 0)
    mu = bfv.decrypt(P, s, ct)
    drop = bfv.noise_margin_bits(P0, s, ct0, bfv.decrypt(P0, s, ct0)) - bfv.noise_margin_bits(P, s, ct, mu)
    assert 40 < drop < 50


# ------------------------------------------------------------------ findDmax
def _dmax_params(t, scheme, L=1, N=64, K=2, qbits=1, d_cap=24):
    return Params(N=N, q=tuple(default_primes(N, L)), t=t, D=d_cap, K=K, F=8, scheme=scheme, qbits=qbits)


@pytest.mark.parametrize("t,scheme", [(641, "bfv"), (2689, "bgv"), (3329, "bfv-r")])
def test_dmax_running_sum_equals_literal_loop(t, scheme):
    """The trial's D_i from the running sum equals the literal loop that recomputes every
    D-term dot product and its expected plaintext from scratch."""
    P = _dmax_params(t, scheme, d_cap=16)
    for seed in (1, 2):
        assert dmax.trial(P, seed, 16, 8) == dmax.trial(P, seed, 16, 8, from_scratch=True)


def test_dmax_bgv_failure_is_the_noise_bound():
    """BGV decrypts correctly exactly while the integer phase sum_m (t*e_m + centred mu_m) * p_m
    (computed over Z with schoolbook products) stays below Q/2: every prefix up to D_i does,
    the (D_i + 1)-term one does not."""
    P = _dmax_params(3457, "bgv", d_cap=24)
    t, N = P.t, P.N
    for seed in (3, 4, 5):
        D = dmax.trial(P, seed, 24, 8)
        assert 0 < D < 24
        C, h = dmax.trial_inputs(P, seed, 24, 8)
        x = np.zeros(N, dtype=object)
        for m in range(D + 1):
            mu = slots.encode(model_slots(P, C, m), t)
            e = prng.gaussian(prng.draws(seed, prng.TAG_ENCRYPT, m * (P.L + 1) * N + P.L * N, N))
            msg = [t * int(ei) + (int(v) - t if v > t // 2 else int(v)) for ei, v in zip(e, mu)]
            p = [int(v) for v in bfv.query_plaintext(P, h, 0, m)]
            for i in range(N):
                for j in range(N):
                    k = i + j
                    if k < N:
                        x[k] += msg[i] * p[j]
                    else:
                        x[k - N] -= msg[i] * p[j]
            assert (max(abs(int(v)) for v in x) < P.Qmod // 2) == (m < D)


def test_dmax_falls_as_log_t_grows():
    """The noise study's trade-off: a larger plaintext modulus leaves a smaller D_max."""
    means = [dmax.find_dmax(_dmax_params(t, "bfv-r", d_cap=40), 3, 40, seed=11)[0] for t in (1409, 2689, 4481)]
    assert means[0] > means[1] > means[2]


def test_dmax_reaches_the_cap_with_a_wide_margin():
    P = _dmax_params(257, "bfv", L=2, d_cap=12)
    assert dmax.find_dmax(P, 2, 12, seed=1) == (12.0, [12, 12])


@pytest.mark.parametrize("scheme", ["bfv", "bfv-r", "bgv"])
def test_decryption_input_is_the_sum_of_message_terms(scheme):
    """The uniform masks cancel in c0 + c1*s: the decryption input of a D-term dot product is
    sum_m (message term of ct_m) * p_m mod q_l, message term e + Delta*mu (BFV),
    e + round(Q*mu/t) (rounded BFV) or t*e + centred(mu) (BGV).  Written with schoolbook products."""
    P = _dmax_params(641, scheme, L=2, N=16, d_cap=5)
    seed = 9
    C, h = dmax.trial_inputs(P, seed, 5, 8)
    s = bfv.secret_key(P, seed)
    model = bfv.encrypt_model(P, s, C, seed)
    Qm, t = P.Qmod, P.t
    for l, q in enumerate(P.q):
        acc0 = np.zeros(P.N, dtype=np.int64)
        acc1 = np.zeros(P.N, dtype=np.int64)
        want = np.zeros(P.N, dtype=np.int64)
        for m in range(5):
            p = bfv.query_plaintext(P, h, 0, m)
            acc0 = (acc0 + ntt.polymul_naive(model[m, 0, l], p % q, q)) % q
            acc1 = (acc1 + ntt.polymul_naive(model[m, 1, l], p % q, q)) % q
            mu = slots.encode(model_slots(P, C, m), t)
            e = prng.gaussian(prng.draws(seed, prng.TAG_ENCRYPT, m * (P.L + 1) * P.N + P.L * P.N, P.N))
            if scheme == "bgv":
                msg = [t * int(ei) + (int(v) - t if v > t // 2 else int(v)) for ei, v in zip(e, mu)]
            elif scheme == "bfv-r":
                msg = [int(ei) + (2 * Qm * int(v) + t) // (2 * t) for ei, v in zip(e, mu)]
            else:
                msg = [int(ei) + (Qm // t) * int(v) for ei, v in zip(e, mu)]
            want = (want + ntt.polymul_naive(np.array([v % q for v in msg], dtype=np.int64), p % q, q)) % q
        assert np.array_equal((acc0 + ntt.polymul_naive(acc1, s % q, q)) % q, want)
