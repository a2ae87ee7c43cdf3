"""Number-theory helpers for the oracle (test infrastructure only).

Nothing here is specific to the paper; these are the textbook facts the BFV
parameters rest on: primes q with q = 1 (mod 2N) carry primitive 2N-th roots
of unity, which make negacyclic transforms and SIMD slots possible.
"""
from __future__ import annotations

_MR_BASES = (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37)


def is_prime(n: int) -> bool:
    """Deterministic Miller-Rabin for n < 3.3e24 (the fixed base set above)."""
    if n < 2:
        return False
    for p in _MR_BASES:
        if n % p == 0:
            return n == p
    d, s = n - 1, 0
    while d % 2 == 0:
        d //= 2
        s += 1
    for a in _MR_BASES:
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(s - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def factorize(n: int) -> list[int]:
    """Distinct prime factors by trial division (n is at most about 2^30 here)."""
    out = []
    d = 2
    while d * d <= n:
        if n % d == 0:
            out.append(d)
            while n % d == 0:
                n //= d
        d += 1
    if n > 1:
        out.append(n)
    return out


def is_generator(g: int, q: int) -> bool:
    """True when g generates the multiplicative group of the prime field Z_q."""
    return all(pow(g, (q - 1) // f, q) != 1 for f in factorize(q - 1))


def smallest_generator(q: int) -> int:
    g = 2
    while not is_generator(g, q):
        g += 1
    return g


def primitive_root_of_unity(order: int, q: int) -> int:
    """A primitive `order`-th root of unity mod prime q: g^((q-1)/order), g the smallest generator."""
    assert (q - 1) % order == 0
    return pow(smallest_generator(q), (q - 1) // order, q)


def inv(a: int, m: int) -> int:
    return pow(a % m, -1, m)
