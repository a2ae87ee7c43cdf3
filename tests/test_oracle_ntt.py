"""Pins of the oracle's number theory and negacyclic transforms (brute force, library checks)."""
import numpy as np
import pytest
import sympy

from oracle import arith, ntt
from oracle.params import default_primes

RNG = np.random.default_rng(7)


def test_is_prime_matches_sympy():
    for n in list(range(2, 3000)) + [1073692673, 1073643521, 1073479681, 2**31 - 1, 2**31 + 1,
                                     1073479681 * 3, 4294967291, 65537]:
        assert arith.is_prime(n) == sympy.isprime(n), n


@pytest.mark.parametrize("N,count", [(4096, 3), (8192, 6), (16384, 10)])
def test_default_primes_are_the_largest_ntt_friendly_primes(N, count):
    got = default_primes(N, count)
    want = []
    q = ((1 << 30) - 1) // (2 * N) * (2 * N) + 1
    while len(want) < count:
        if q < (1 << 30) and sympy.isprime(q):
            want.append(q)
        q -= 2 * N
    assert got == want


def test_primitive_roots_have_exact_order():
    for N in (8, 64, 4096):
        for m in default_primes(N, 2) + [65537]:
            w = ntt.root_2n(N, m)
            assert sympy.n_order(w, m) == 2 * N


@pytest.mark.parametrize("N", [8, 16, 64])
def test_forward_is_evaluation_at_odd_powers(N):
    for m in default_primes(N, 2) + [65537]:
        a = RNG.integers(0, m, N)
        w = ntt.root_2n(N, m)
        got = ntt.forward(a, m)
        want = [ntt.evaluate_naive(a, pow(w, 2 * k + 1, m), m) for k in range(N)]
        assert got.tolist() == want


@pytest.mark.parametrize("N", [8, 32, 128])
def test_polymul_matches_schoolbook(N):
    for m in default_primes(N, 2) + [65537]:
        a = RNG.integers(0, m, N)
        b = RNG.integers(0, m, N)
        assert np.array_equal(ntt.polymul(a, b, m), ntt.polymul_naive(a, b, m))


def test_inverse_roundtrip_batched():
    N = 1024
    m = default_primes(N, 1)[0]
    a = RNG.integers(0, m, (3, 5, N))
    assert np.array_equal(ntt.inverse(ntt.forward(a, m), m), a)


def test_negacyclic_wrap_of_monomials():
    """X^(N-1) * X = X^N = -1 mod X^N + 1."""
    N, m = 16, 65537
    a = np.zeros(N, dtype=np.int64)
    b = np.zeros(N, dtype=np.int64)
    a[N - 1] = 1
    b[1] = 1
    want = np.zeros(N, dtype=np.int64)
    want[0] = m - 1
    assert np.array_equal(ntt.polymul(a, b, m), want)
