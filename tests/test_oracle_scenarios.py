"""Invariants and scenarios the paper fixes, checked on the oracle.

* k = 1 is the discrete window (Section 3.1): after every slide no DR is
  inside the window, so each slice's report equals that of a fresh monitor
  fed only that slice.
* Window semantics (Section 3.1/3.2): what is inside W(e-k+1, k) depends only
  on slices e-k+1..e.
* Under the slice-synchronous candidate reading, the order of the pairs inside
  a slice does not matter.
* Algorithm 3's carry-over (Section 4.2): a super point whose second addresses
  all arrived in earlier slices of the window is still reported.
* Accuracy against the precise method (Section 3.2) on an unsaturated stream.
"""
import numpy as np
import pytest

import oracle
from trafficgen.configs import workload, scaled


def _rand_pairs(rng, n, n_src):
    src = rng.integers(0, n_src, size=n).astype(np.uint32) * np.uint32(0x9E3779B1)
    dst = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
    return np.stack([src, dst], 1)


def _heavy(rng, ip, n):
    return np.stack([np.full(n, ip, np.uint32),
                     rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)], 1)


def _same_report(a, b, with_slice=True):
    if with_slice:
        assert a.slice == b.slice
    for f in ("ip", "est", "flags", "union_weight", "re_weight", "row_fill"):
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
    assert a.up == b.up and a.n_touched == b.n_touched and a.n_new == b.n_new


def test_discrete_window_reports_are_independent_slices():
    cfg = dict(k=1, theta=256, u=3, v_re=128, g=8, v_le=16, G=256, hash_seed=9)
    rng = np.random.default_rng(4)
    long_run = oracle.Monitor(**cfg)
    for s in range(6):
        p = np.concatenate([_rand_pairs(rng, 3000, 400), _heavy(rng, 77 + s % 2, 600)])
        long_run.scan(p)
        r = long_run.estimate()
        fresh = oracle.Monitor(**cfg)
        fresh.scan(p)
        f = fresh.estimate()
        _same_report(r, f, with_slice=False)
        assert (r.flags & oracle.KEEP).sum() == 0      # nothing survives a slide at k = 1
        assert np.all(long_run.dump(oracle.SI) == 0)


def test_window_only_depends_on_its_slices():
    k = 4
    cfg = dict(k=k, theta=128, u=3, v_re=64, g=8, v_le=16, G=128, hash_seed=21)
    rng = np.random.default_rng(8)
    slices = [np.concatenate([_rand_pairs(rng, 2000, 300), _heavy(rng, 5, 300)]) for _ in range(9)]
    full = oracle.Monitor(**cfg)
    reports = []
    for p in slices:
        full.scan(p)
        reports.append(full.estimate())
    e = len(slices) - 1
    fresh = oracle.Monitor(**cfg)
    for p in slices[e - k + 1:]:
        fresh.scan(p)
        rf = fresh.estimate()
    r = reports[-1]
    assert np.array_equal(r.row_fill, rf.row_fill) and r.up == rf.up
    common, ia, ib = np.intersect1d(r.ip, rf.ip, return_indices=True)
    assert common.size > 0
    assert np.array_equal(r.union_weight[ia], rf.union_weight[ib])
    assert np.array_equal(r.re_weight[ia], rf.re_weight[ib])
    assert np.array_equal(r.est[ia], rf.est[ib])
    # DRs inside the window (distance <= k at the open slice) agree exactly
    for which in (oracle.LE, oracle.RE):
        a, b = full.dump(which), fresh.dump(which)
        assert np.array_equal(np.minimum(a, k + 1), np.minimum(b, k + 1))


def test_pair_order_inside_a_slice_does_not_matter():
    cfg = dict(k=3, theta=64, u=4, v_re=64, g=8, v_le=8, G=128, hash_seed=33)
    rng = np.random.default_rng(12)
    a, b = oracle.Monitor(**cfg), oracle.Monitor(**cfg)
    for _ in range(6):
        p = np.concatenate([_rand_pairs(rng, 3000, 250), _heavy(rng, 9, 200)])
        a.scan(p)
        b.scan(p[rng.permutation(len(p))])
        _same_report(a.estimate(), b.estimate())
    for w in (oracle.LE, oracle.RE, oracle.SI):
        assert np.array_equal(a.dump(w), b.dump(w))


def test_carry_over_reports_a_quiet_super_point():
    k, theta = 8, 1024
    cfg = dict(k=k, theta=theta, u=4, v_re=2048, g=8, v_le=2048, G=1024, hash_seed=44)
    rng = np.random.default_rng(2)
    aip = 0x0B0B0B0B
    dsts = rng.choice(2 ** 32, size=2400, replace=False).astype(np.uint32)
    m = oracle.Monitor(**cfg)
    for s in range(k):
        bg = _rand_pairs(rng, 5000, 2000)
        if s < k - 1:     # the host is silent in the last slice of the window
            part = dsts[s * 400:(s + 1) * 400] if s < 6 else dsts[:0]
            bg = np.concatenate([bg, np.stack([np.full(part.size, aip, np.uint32), part], 1)])
        m.scan(bg)
        r = m.estimate()
    hit = np.flatnonzero(r.ip == aip)     # the carried list comes first
    assert hit.size == 1
    x = int(hit[0])
    assert not (r.flags[x] & oracle.NEW)
    assert r.flags[x] & oracle.SUPER
    assert abs(r.est[x] - 2400) < 0.15 * 2400


def test_capacity_overflow_poisons_the_monitor():
    cfg = dict(k=2, theta=8, u=2, v_re=16, g=8, v_le=4, G=64, hash_seed=1, max_candidates=3)
    m = oracle.Monitor(**cfg)
    rng = np.random.default_rng(0)
    m.scan(np.concatenate([_heavy(rng, ip, 100) for ip in range(1, 7)]))
    with pytest.raises(oracle.OracleError) as e:
        m.estimate()
    assert e.value.rc == -3
    with pytest.raises(oracle.OracleError) as e:
        m.scan(_heavy(rng, 1, 5))
    assert e.value.rc == -4


def test_empty_slices_and_fresh_state():
    cfg = dict(k=3, theta=64, u=2, v_re=32, g=8, v_le=4, G=64, hash_seed=2)
    m = oracle.Monitor(**cfg)
    assert np.all(m.dump(oracle.LE) == 65535) and np.all(m.dump(oracle.RE) == 65535)
    assert np.all(m.dump(oracle.SI) == 0)
    r = m.estimate()
    assert r.n == 0 and r.slice == 0 and not r.window_full and r.up == 0.0
    rng = np.random.default_rng(1)
    m.scan(_heavy(rng, 5, 500))
    r = m.estimate()
    assert r.n == 1 and r.flags[0] & oracle.NEW
    for s in range(2, 5):
        r = m.estimate()          # no traffic: the host ages out after k slices
        assert r.window_full
    assert r.n == 0
    assert np.all(m.dump(oracle.SI) == 0)
    le = m.dump(oracle.LE)
    assert le.min() == 4 and set(np.unique(le)) <= {4, 65535}
    with pytest.raises(ValueError):
        oracle.Monitor(k=0, theta=1, u=1, v_re=1, g=1, v_le=1, G=64, hash_seed=0)
    with pytest.raises(ValueError):
        oracle.Monitor(k=1, theta=1, u=1, v_re=1, g=1, v_le=1, G=100, hash_seed=0)


def test_accuracy_against_precise_method_on_unsaturated_stream():
    stream, mon, n_slices = workload("tiny_coupled")
    stream = scaled(stream, 40_000)
    m = oracle.Monitor(**mon)
    history = []
    for s in range(mon["k"]):
        p = stream.slice(s)
        history.append(p)
        m.scan(p)
        r = m.estimate()
    allp = np.concatenate(history)
    key = np.unique((allp[:, 0].astype(np.uint64) << np.uint64(32)) | allp[:, 1])
    ips, card = np.unique((key >> np.uint64(32)).astype(np.uint32), return_counts=True)
    truth = dict(zip(ips.tolist(), card.tolist()))
    for ip in stream.planted_ips().tolist():
        hit = np.flatnonzero(r.ip == ip)
        assert hit.size == 1 and truth[ip] == 2000
        x = int(hit[0])
        assert abs(r.est[x] - 2000) < 0.12 * 2000
    supers = [ip for ip, c in truth.items() if c >= mon["theta"]]
    detected = set(r.ip[(r.flags & oracle.SUPER) != 0].tolist())
    missed = [ip for ip in supers if ip not in detected]
    assert len(missed) <= max(1, len(supers) // 10)


def test_report_lists_the_carried_candidates_then_the_new_ones():
    """CSIP_t = NCSIP_{t-1} + N_t (Algorithms 2-3): the report lists the
    candidates carried from the previous slice (its KEEP entries), ascending,
    then the slice's new candidates (flag NEW), ascending; the two parts are
    disjoint."""
    cfg = dict(k=3, theta=64, u=2, v_re=256, g=8, v_le=32, G=128, hash_seed=31)
    rng = np.random.default_rng(12)
    m = oracle.Monitor(**cfg)
    prev_keep = np.zeros(0, np.uint32)
    seen_both = False
    for s in range(8):
        heavy = [_heavy(rng, 100 + 7 * h, 120) for h in range(s % 3, 12, 2)]
        m.scan(np.concatenate([_rand_pairs(rng, 3000, 500)] + heavy))
        r = m.estimate()
        new = (r.flags & oracle.NEW) != 0
        n_c = int((~new).sum())
        assert not new[:n_c].any() and new[n_c:].all()
        carried, news = r.ip[:n_c], r.ip[n_c:]
        assert np.array_equal(carried, prev_keep)
        assert np.all(np.diff(carried.astype(np.int64)) > 0)
        assert np.all(np.diff(news.astype(np.int64)) > 0)
        assert np.intersect1d(carried, news).size == 0
        seen_both |= n_c > 0 and news.size > 0
        prev_keep = np.sort(r.ip[(r.flags & oracle.KEEP) != 0])
    assert seen_both
