"""Host twin of the synthetic stream generator: determinism and the shape
properties the workloads rely on."""
import numpy as np

from trafficgen import StreamSpec, rank_to_ip, zipf_table
from trafficgen.configs import workload


def test_slices_are_deterministic_and_partial_ranges_agree():
    st, _, _ = workload("tiny")
    a, b = st.slice(5), st.slice(5)
    assert np.array_equal(a, b)
    assert np.array_equal(st.slice(5, 123, 4567), a[123:4567])
    assert not np.array_equal(st.slice(6), a)


def test_permutation_is_a_bijection():
    st = StreamSpec(n_pairs=10_007, n_ranks=1000, alpha=1.0, planted=[300, 50], window=4, seed=3)
    for s in range(4):
        a, b = st.perm(s)
        j = np.arange(st.n_pairs, dtype=np.uint64)
        i = (np.uint64(a) * j + np.uint64(b)) % np.uint64(st.n_pairs)
        assert np.unique(i).size == st.n_pairs


def test_planted_windows_hold_exactly_their_pool():
    st = StreamSpec(n_pairs=20_000, n_ranks=4096, alpha=1.1, planted=[1000, 333, 2048],
                    window=8, seed=11)
    ips = st.planted_ips()
    for start in (0, 3):
        allp = np.concatenate([st.slice(s) for s in range(start, start + 8)])
        for p, ip in enumerate(ips):
            d = np.unique(allp[allp[:, 0] == ip][:, 1])
            assert d.size == st.planted[p]
            assert np.array_equal(np.sort(d), np.sort(st.planted_pool(p)))


def test_zipf_frequencies():
    thr = zipf_table(1000, 1.1)
    assert thr[-1] == np.uint64(1 << 63) and np.all(np.diff(thr.astype(np.float64)) >= 0)
    st = StreamSpec(n_pairs=400_000, n_ranks=1000, alpha=1.1, seed=5)
    p = st.slice(0)
    w = np.arange(1, 1001, dtype=np.float64) ** -1.1
    w /= w.sum()
    for r in (0, 1, 9):
        frac = (p[:, 0] == rank_to_ip(np.array([r]))[0]).mean()
        sd = np.sqrt(w[r] * (1 - w[r]) / p.shape[0])
        assert abs(frac - w[r]) < 5 * sd


def test_rank_to_ip_is_injective():
    r = np.arange(1 << 20)
    assert np.unique(rank_to_ip(r)).size == r.size
