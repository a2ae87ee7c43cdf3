"""Pins of the oracle's generator and samplers against published values and statistics."""
import math
import os
from decimal import Decimal, getcontext

import numpy as np

from oracle import prng


def _golden_ints(path):
    return [int(l) for l in open(path) if l.strip() and not l.startswith("#")]


def test_splitmix64_published_sequence(golden_dir):
    want = _golden_ints(os.path.join(golden_dir, "splitmix64_seed1234567.txt"))
    got = [prng.splitmix64_scalar(1234567, n) for n in range(len(want))]
    assert got == want


def test_vectorised_draws_match_scalar():
    seed, tag = 987654321, prng.TAG_ENCRYPT
    s0 = prng.stream_state(seed, tag)
    v = prng.draws(seed, tag, 1000, 64)
    assert [int(x) for x in v] == [prng.splitmix64_scalar(s0, 1000 + i) for i in range(64)]


def test_streams_differ_by_tag():
    a = prng.draws(0, prng.TAG_SECRET, 0, 16)
    b = prng.draws(0, prng.TAG_ENCRYPT, 0, 16)
    assert not np.array_equal(a, b)


def test_uniform_mod_range_and_mean():
    q = 1073692673
    u = prng.uniform_mod(prng.draws(1, prng.TAG_ENCRYPT, 0, 200000), q)
    assert u.min() >= 0 and u.max() < q
    assert abs(u.mean() / q - 0.5) < 0.005


def test_ternary_frequencies():
    s = prng.ternary(prng.draws(3, prng.TAG_SECRET, 0, 300000))
    assert set(np.unique(s).tolist()) == {-1, 0, 1}
    for v in (-1, 0, 1):
        assert abs((s == v).mean() - 1 / 3) < 0.005


def test_gaussian_table_against_high_precision():
    """T_k agrees within one unit with round(2^53 * CDF) computed in 50-digit decimal arithmetic."""
    getcontext().prec = 50
    two_s2 = Decimal(2) * Decimal("3.2") ** 2
    rho = [(-(Decimal(i * i) / two_s2)).exp() for i in range(-19, 20)]
    total = sum(rho)
    table = prng.gaussian_cdt()
    assert len(table) == 39 and table[-1] == 1 << 53
    assert all(a < b for a, b in zip(table, table[1:]))
    acc = Decimal(0)
    for k, r in enumerate(rho):
        acc += r
        exact = int((acc / total * Decimal(2) ** 53).to_integral_value())
        assert abs(table[k] - exact) <= 1, k


def test_gaussian_statistics():
    e = prng.gaussian(prng.draws(5, prng.TAG_ENCRYPT, 0, 400000))
    assert e.min() >= -19 and e.max() <= 19
    assert abs(e.mean()) < 0.03
    # variance of the discrete Gaussian with rho(i) = exp(-i^2 / (2 sigma^2)), sigma = 3.2
    w = np.array([math.exp(-i * i / 20.48) for i in range(-19, 20)])
    var = float((w * np.arange(-19, 20) ** 2).sum() / w.sum())
    assert abs(var - 10.24) < 0.01
    assert abs(e.var() - var) < 0.15


def test_gaussian_inverse_cdf_boundaries():
    """(u >> 11) just below T_k maps to k; at T_k it maps to k+1."""
    table = prng.gaussian_cdt()
    for k in (0, 5, 19, 25, 37):
        lo = np.array([(table[k] - 1) << 11], dtype=np.uint64)
        hi = np.array([table[k] << 11], dtype=np.uint64)
        assert prng.gaussian(lo)[0] == k - 19
        assert prng.gaussian(hi)[0] == k - 18
