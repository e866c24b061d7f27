"""Pins of the oracle's building blocks: worked examples, constants, hashing.

Each check ties the oracle to something other than itself: values the paper
prints, published generator outputs, closed forms, special cases, or a
second independent implementation of a stated reading.
"""
import math
import os

import mpmath
import numpy as np
import pytest

import oracle
from oracle.exact import Hashes, lsb_array, splitmix64_words

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append(line.split())
    return rows


def test_paper_worked_examples():
    for row in _golden("paper_worked_examples.txt"):
        name, args, want = row[0], [int(x) for x in row[1:-1]], int(row[-1])
        fn = {"lsb": oracle.lsb, "tau": oracle.tau, "sre_threshold": oracle.sre_threshold}[name]
        assert fn(*args) == want, row


def test_lsb_matches_bit_trick():
    rng = np.random.default_rng(7)
    xs = rng.integers(1, 2 ** 32, size=2000, dtype=np.uint64).tolist() + [1, 2 ** 31, 0]
    for x in xs:
        want = 32 if x == 0 else (x & -x).bit_length() - 1
        assert oracle.lsb(int(x)) == want


def test_tau_is_smallest_sampling_exponent():
    # Eq1 evaluated in high precision: ceil(log2(theta / g)), floored at 0
    for theta in [1, 2, 3, 7, 8, 9, 100, 1023, 1024, 1025, 4096, 16384, 2 ** 31]:
        for g in [1, 2, 3, 4, 7, 8, 16, 64]:
            exact = int(mpmath.ceil(mpmath.log(mpmath.mpf(theta) / g, 2)))
            assert oracle.tau(theta, g) == max(0, exact), (theta, g)


def test_rho_and_sre_threshold():
    mpmath.mp.dps = 40
    rho = 0.99 * (1 - mpmath.exp(mpmath.mpf(-1) / 3))
    assert abs(oracle.rho() - float(rho)) < 1e-15
    for g in range(1, 65):
        assert oracle.sre_threshold(g) == int(mpmath.ceil(rho * g)), g


def test_splitmix64_published_vector():
    want = [int(r[0]) for r in _golden("splitmix64_seed1234567.txt")]
    assert oracle.splitmix64(1234567, len(want)) == want
    assert splitmix64_words(1234567, len(want)) == want


def test_hash_param_expansion_order():
    a, b = oracle.hash_params(1234567, 2)
    w = [int(r[0]) for r in _golden("splitmix64_seed1234567.txt")]
    assert a == [w[0], w[2]] and b == [w[1], w[3]]


def test_multiply_add_shift_special_cases():
    rng = np.random.default_rng(3)
    for x in rng.integers(0, 2 ** 32, size=500, dtype=np.uint64).tolist():
        # a = 2^32, b = 0: (x * 2^32 mod 2^64) >> 32 is x itself
        assert oracle.mas(1 << 32, 0, x) == x
        # b = c * 2^32 adds c modulo 2^32
        assert oracle.mas(1 << 32, 12345 << 32, x) == (x + 12345) % (1 << 32)
        # a = 1, b = 0: the high half of a 32-bit x is 0
        assert oracle.mas(1, 0, x) == 0
        # a = 2^63 keeps only the low bit of x, in the top bit of the result
        assert oracle.mas(1 << 63, 0, x) == (x & 1) << 31
    # the product wraps modulo 2^64
    assert oracle.mas((1 << 64) - 1, 0, 2) == ((2 * ((1 << 64) - 1)) % (1 << 64)) >> 32


def test_range_reduction_special_cases():
    for m in [1, 2, 3, 16, 1000, 2048, 65536, 2 ** 31 + 7]:
        assert oracle.hrange(0, m) == 0
        assert oracle.hrange(2 ** 32 - 1, m) == m - 1
    for kbits in range(0, 17):
        for h in [0, 1, 12345, 2 ** 31, 2 ** 32 - 1]:
            assert oracle.hrange(h, 1 << kbits) == h >> (32 - kbits)


def test_oracle_hashes_match_independent_copy():
    """The oracle's C hashing against the numpy copy of the same reading."""
    u, v_re, g, v_le, G = 5, 131072, 8, 2048, 1024
    h = Hashes(0xABCDEF, u, v_re, g, v_le, G)
    a, b = oracle.hash_params(0xABCDEF, u + 4)
    assert a == h.a and b == h.b
    rng = np.random.default_rng(11)
    xs = rng.integers(0, 2 ** 32, size=300, dtype=np.uint64).astype(np.uint32)
    for x in xs.tolist():
        for i in range(u):
            hr = oracle.mas(a[i], b[i], x)
            assert oracle.hrange(hr, v_re) == h.col_re(i, [x])[0]
            assert oracle.hrange(hr, v_le) == h.col_le(i, [x])[0]
        assert oracle.mas(a[u], b[u], x) == h.h1([x])[0]
        assert oracle.hrange(oracle.mas(a[u + 1], b[u + 1], x), g) == h.re_idx([x])[0]
        assert oracle.hrange(oracle.mas(a[u + 2], b[u + 2], x), G) == h.le_idx([x])[0]
        assert oracle.hrange(oracle.mas(a[u + 3], b[u + 3], x), 16) == h.si_idx([x])[0]


def _chi2_p(counts, expected):
    from scipy.stats import chi2
    stat = float(((counts - expected) ** 2 / expected).sum())
    return chi2.sf(stat, len(counts) - 1)


@pytest.mark.parametrize("seed", [1, 2])
def test_hash_outputs_are_uniform(seed):
    h = Hashes(seed, 2, 257, 8, 64, 1024)
    rng = np.random.default_rng(seed)
    x = rng.integers(0, 2 ** 32, size=200_000, dtype=np.uint64).astype(np.uint32)
    for vals, m in [(h.col_re(0, x), 257), (h.col_le(1, x), 64), (h.re_idx(x), 8),
                    (h.le_idx(x), 1024), (h.si_idx(x), 16)]:
        c = np.bincount(vals, minlength=m).astype(float)
        assert c.size == m
        assert _chi2_p(c, np.full(m, x.size / m)) > 1e-4


@pytest.mark.parametrize("tau", [0, 1, 3, 7, 10])
def test_sampling_rate_is_two_to_minus_tau(tau):
    """P(LSB(H1(bip)) >= tau) = 2^-tau: the Binomial rate of Eq3."""
    h = Hashes(99 + tau, 1, 1, 8, 1, 64)
    rng = np.random.default_rng(tau)
    x = rng.integers(0, 2 ** 32, size=400_000, dtype=np.uint64).astype(np.uint32)
    frac = (lsb_array(h.h1(x)) >= tau).mean()
    p = 2.0 ** -tau
    sd = math.sqrt(p * (1 - p) / x.size)
    assert abs(frac - p) < 5 * sd + 1e-12
