"""Pins of the SIMD slot map mod t: brute-force evaluation, bijection, multiplicativity, rotation."""
import numpy as np
import pytest
import sympy

from oracle import bfv, ntt, slots

T = 65537
RNG = np.random.default_rng(11)


@pytest.mark.parametrize("N", [8, 16, 4096, 8192, 16384])
def test_zeta_order_and_exponent_bijection(N):
    z = slots.zeta(N, T)
    assert sympy.n_order(z, T) == 2 * N
    e = slots.slot_exponents(N)
    assert sorted(e.tolist()) == list(range(1, 2 * N, 2))


def test_zeta_closed_form():
    # 3 generates Z_65537^*, so zeta = 3^(65536 / 2N)
    assert slots.zeta(4096, T) == 6561
    assert slots.zeta(8192, T) == 81
    assert slots.zeta(16384, T) == 9


@pytest.mark.parametrize("N", [16, 64])
def test_decode_is_evaluation_at_slot_points(N):
    mu = RNG.integers(0, T, N)
    assert np.array_equal(slots.decode(mu, T), slots.decode_naive(mu, T))


@pytest.mark.parametrize("N", [16, 256, 4096])
def test_decode_encode_identity(N):
    v = RNG.integers(0, T, (2, N))
    assert np.array_equal(slots.decode(slots.encode(v, T), T), v)


def test_encode_is_multiplicative():
    N = 64
    v = RNG.integers(0, T, N)
    w = RNG.integers(0, T, N)
    prod = ntt.polymul_naive(slots.encode(v, T), slots.encode(w, T), T)
    assert np.array_equal(slots.decode(prod, T), v * w % T)


@pytest.mark.parametrize("k", [1, 3, 8])
def test_automorphism_3k_rotates_each_half_left(k):
    N = 32
    v = RNG.integers(0, T, N)
    mu = slots.encode(v, T)
    rot = bfv.automorphism(mu.reshape(1, N), pow(3, k, 2 * N), [T]).reshape(N)
    h = N // 2
    want = np.concatenate((np.roll(v[:h], -k), np.roll(v[h:], -k)))
    assert np.array_equal(slots.decode(rot, T), want)


def test_conjugation_swaps_halves():
    N = 32
    v = RNG.integers(0, T, N)
    rot = bfv.automorphism(slots.encode(v, T).reshape(1, N), 2 * N - 1, [T]).reshape(N)
    assert np.array_equal(slots.decode(rot, T), np.concatenate((v[N // 2:], v[:N // 2])))


def test_centered_range():
    x = np.arange(T)
    c = slots.centered(x, T)
    assert c.min() == -32768 and c.max() == 32768
    assert np.array_equal(c % T, x)
