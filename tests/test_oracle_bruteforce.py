"""The oracle against brute force recomputed from the stream history.

The brute force (``oracle.exact``) keeps no distance recorders: it stores the
last slice that touched each cell and derives every DR, row fill, union weight
and candidate list from window membership.  A dropped term, a wrong index or a
wrong slide in the oracle shows up as a mismatch here.
"""
import numpy as np
import pytest

import oracle
from oracle.exact import BruteForce


def _stream(rng, n, n_src, heavy=()):
    """n pairs: Zipf-like sources over n_src hosts plus heavy hitters."""
    w = 1.0 / np.arange(1, n_src + 1) ** 1.1
    src = rng.choice(n_src, size=n, p=w / w.sum()).astype(np.uint32) * np.uint32(2654435761)
    dst = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    parts = [np.stack([src, dst], 1)]
    for ip, cnt in heavy:
        parts.append(np.stack([np.full(cnt, ip, np.uint32),
                               rng.integers(0, 2 ** 32, size=cnt, dtype=np.uint64).astype(np.uint32)], 1))
    p = np.concatenate(parts)
    return p[rng.permutation(len(p))]


def _compare(r, b):
    assert r.slice == b["slice"]
    assert r.window_full == b["window_full"]
    assert np.array_equal(r.ip, b["ip"])
    assert np.array_equal(r.union_weight, b["union_weight"])
    assert np.array_equal(r.re_weight, b["re_weight"])
    assert np.array_equal(r.row_fill, b["row_fill"])
    assert np.array_equal(r.flags, b["flags"])
    assert r.up == b["up"]
    assert np.array_equal(r.est, b["est"])
    assert r.n_touched == b["n_touched"] and r.n_new == b["n_new"]


CASES = [
    # k, theta, u, v_re, g, v_le, G, pairs/slice, sources, slices
    (3, 64, 3, 64, 8, 8, 128, 3000, 200, 8),
    (1, 64, 2, 32, 8, 4, 64, 1500, 100, 5),        # discrete window
    (5, 16, 1, 16, 4, 16, 64, 800, 60, 9),         # one row, tau = 2
    (4, 4, 4, 128, 8, 32, 64, 600, 300, 7),        # tau = 0: every pair sampled
    (6, 4096, 2, 64, 16, 8, 192, 4000, 50, 8),     # tau = 8, g = 16, G not a power of 2
    (2, 256, 5, 33, 3, 7, 64, 2000, 120, 6),       # odd sizes everywhere
]


@pytest.mark.parametrize("case", CASES)
def test_reports_and_dumps_match_brute_force(case):
    k, theta, u, v_re, g, v_le, G, n, n_src, slices = case
    cfg = dict(k=k, theta=theta, u=u, v_re=v_re, g=g, v_le=v_le, G=G, hash_seed=1000 + k)
    m = oracle.Monitor(**cfg)
    bf = BruteForce(**cfg)
    rng = np.random.default_rng(k * 31 + u)
    for s in range(slices):
        pairs = _stream(rng, n if s != 2 else 0, n_src, heavy=[(7, 3 * theta // 2)] if s < 3 else ())
        m.scan(pairs)
        _compare(m.estimate(), bf.close_slice(pairs))
        for which in (oracle.LE, oracle.RE, oracle.SI):
            assert np.array_equal(m.dump(which), bf.dump(which)), which


def test_scan_in_pieces_equals_one_scan():
    cfg = dict(k=4, theta=128, u=3, v_re=64, g=8, v_le=8, G=128, hash_seed=5)
    a, b = oracle.Monitor(**cfg), oracle.Monitor(**cfg)
    rng = np.random.default_rng(0)
    for _ in range(5):
        p = _stream(rng, 3000, 150)
        a.scan(p)
        for lo in range(0, 3000, 700):
            b.scan(p[lo:lo + 700])
        ra, rb = a.estimate(), b.estimate()
        assert np.array_equal(ra.ip, rb.ip) and np.array_equal(ra.est, rb.est)
    for w in (0, 1, 2):
        assert np.array_equal(a.dump(w), b.dump(w))


@pytest.mark.parametrize("case", [CASES[0], CASES[2], CASES[5]])
def test_sequential_mode_matches_brute_force(case):
    """Algorithm 2's per-pair candidate check in stream order (the oracle's
    optional sequential mode) against a second, pure-Python implementation."""
    k, theta, u, v_re, g, v_le, G, n, n_src, slices = case
    cfg = dict(k=k, theta=theta, u=u, v_re=v_re, g=g, v_le=v_le, G=G, hash_seed=2000 + k)
    m = oracle.Monitor(**cfg, sequential=True)
    bf = BruteForce(**cfg, sequential=True)
    rng = np.random.default_rng(k * 17 + u)
    for s in range(min(slices, 6)):
        pairs = _stream(rng, min(n, 1500), n_src, heavy=[(7, 3 * theta // 2)] if s < 3 else ())
        m.scan(pairs)
        _compare(m.estimate(), bf.close_slice(pairs))
        for which in (oracle.LE, oracle.RE, oracle.SI):
            assert np.array_equal(m.dump(which), bf.dump(which)), which
