"""Seeded synthetic (aip, bip) pair streams -- host twin.

This module is input generation only: it holds none of the estimator's
arithmetic.  The same streams come out of the HIP twin in ``trafficgen.hip``
(bit-identical, checked by a GPU test), which the bench uses to fill device
memory without a host round trip.

Stream recipe (pair ``j`` of slice ``s`` is a pure function of the seed, ``s``
and ``j``):

* ``sm(base, c)`` is output ``c`` of SplitMix64 started at ``base``, i.e. the
  SplitMix64 finaliser applied to ``base + (c + 1) * 0x9E3779B97F4A7C15``;
  the counter of raw position ``i`` in slice ``s`` is ``c = (s << 32) | i``.
* First addresses (aip) follow a Zipf(alpha) law over ``N`` ranks (rank r has
  weight ``(r + 1)^-alpha``): a 63-bit uniform ``sm(SRC, c) >> 1`` is looked up
  in the cumulative table ``thr`` (uint64, scaled to 2^63) as the number of
  entries ``<= x``.  Rank r maps to the IPv4 ``(r * 0x9E3779B1 mod 2^32) ^
  0x5A5A5A5A``, a bijection.
* Second addresses (bip) are uniform 32-bit: the low half of ``sm(DST, c)``;
  with ``dst_pool = q > 0`` an ordinary source of rank r instead draws from
  its own q addresses ``perm32(key ^ DPOOL, r * q + (sm(DST, c) mod q))``
  (distinct across sources), so it has at most q distinct peers.
* Planted super points ``p < P`` use ranks ``N + p`` (outside the Zipf
  support), each with a pool of ``D_p`` distinct second addresses
  ``perm32(key, (p << 18) | x)``.  Slice ``s`` sends ``m_p = ceil(D_p / k)``
  pairs, pool entries ``(s * m_p + x) mod D_p``, so every full window of ``k``
  slices holds exactly ``D_p`` distinct second addresses for ``p``.  Planted
  pairs take the first ``sum(m_p)`` raw positions.
* The slice is then permuted: output position ``j`` holds raw position
  ``(a_s * j + b_s) mod n`` with ``gcd(a_s, n) = 1``.
"""
import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1
SRC_SALT = 0x5352435F53524C41
DST_SALT = 0x4453545F53524C41
POOL_SALT = 0x504F4F4C53524C41
DPOOL_XOR = 0x6D2B79F5
PERM_SALT = 0x5045524D53524C41
IP_MULT = 0x9E3779B1
IP_XOR = 0x5A5A5A5A
POOL_BITS = 18          # D_p < 2^18 distinct pool entries per planted host


def mix64_int(z):
    z &= M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def _mix64(z):
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def _sm_at(base, ctr):
    with np.errstate(over="ignore"):
        return _mix64(np.uint64(base) + (ctr + np.uint64(1)) * np.uint64(GAMMA))


def _perm32(key, x):
    """A 32-bit bijection (xor-shift-multiply rounds with odd constants)."""
    x = (np.asarray(x, dtype=np.uint32) ^ np.uint32(key)).astype(np.uint64)
    m32 = np.uint64(0xFFFFFFFF)
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x7FEB352D)) & m32
    x ^= x >> np.uint64(15)
    x = (x * np.uint64(0x846CA68B)) & m32
    x ^= x >> np.uint64(16)
    return x.astype(np.uint32)


def rank_to_ip(r):
    r = np.asarray(r, dtype=np.uint64)
    return (((r * np.uint64(IP_MULT)) & np.uint64(0xFFFFFFFF)) ^ np.uint64(IP_XOR)).astype(np.uint32)


def zipf_table(n_ranks, alpha):
    """Cumulative Zipf weights as uint64 thresholds on a 2^63 scale."""
    w = np.arange(1, n_ranks + 1, dtype=np.float64) ** (-float(alpha))
    c = np.cumsum(w)
    c /= c[-1]
    thr = np.floor(c * float(1 << 63))
    thr = np.minimum(thr, float(1 << 63)).astype(np.uint64)
    thr[-1] = np.uint64(1 << 63)
    return thr


@dataclass
class StreamSpec:
    """One synthetic stream: pairs per slice, Zipf sources, planted hosts."""
    n_pairs: int
    n_ranks: int
    alpha: float
    planted: list = field(default_factory=list)   # D_p of each planted host
    window: int = 1                                # k used to spread the pools
    seed: int = 0
    dst_pool: int = 0                              # 0: uniform destinations

    def __post_init__(self):
        assert all(1 <= d < (1 << POOL_BITS) for d in self.planted)
        assert len(self.planted) < (1 << 14)
        self.m = [int(math.ceil(d / self.window)) for d in self.planted]
        self.off = np.concatenate([[0], np.cumsum(self.m)]).astype(np.int64)
        self.n_planted_pairs = int(self.off[-1])
        assert self.n_planted_pairs <= self.n_pairs
        self._thr = None
        self.pool_key = mix64_int(self.seed ^ POOL_SALT) & 0xFFFFFFFF

    @property
    def thr(self):
        if self._thr is None:
            self._thr = zipf_table(self.n_ranks, self.alpha)
        return self._thr

    def planted_ips(self):
        return rank_to_ip(np.arange(self.n_ranks, self.n_ranks + len(self.planted)))

    def perm(self, s):
        """(a_s, b_s) of slice s's affine permutation of n positions."""
        n = self.n_pairs
        r1 = mix64_int(self.seed ^ PERM_SALT ^ ((s * GAMMA) & M64))
        r2 = mix64_int(r1 ^ PERM_SALT)
        a = (r1 % n) | 1 if n > 1 else 0
        while n > 1 and math.gcd(a, n) != 1:
            a = (a + 2) % n
        b = r2 % n
        return a, b

    def slice(self, s, lo=0, hi=None):
        """Pairs [lo, hi) of slice s as a (hi-lo, 2) uint32 array."""
        n = self.n_pairs
        hi = n if hi is None else hi
        a, b = self.perm(s)
        j = np.arange(lo, hi, dtype=np.uint64)
        with np.errstate(over="ignore"):
            i = (np.uint64(a) * j + np.uint64(b)) % np.uint64(max(n, 1))
        out = np.empty((hi - lo, 2), dtype=np.uint32)
        ctr = (np.uint64(s) << np.uint64(32)) | i
        x = _sm_at(self.seed ^ SRC_SALT, ctr) >> np.uint64(1)
        rank = np.searchsorted(self.thr, x, side="right")
        out[:, 0] = rank_to_ip(rank)
        dst = _sm_at(self.seed ^ DST_SALT, ctr) & np.uint64(0xFFFFFFFF)
        if self.dst_pool:
            q = np.uint64(self.dst_pool)
            idx = (rank.astype(np.uint64) * q + dst % q) & np.uint64(0xFFFFFFFF)
            dst = _perm32(self.pool_key ^ DPOOL_XOR, idx.astype(np.uint32)).astype(np.uint64)
        out[:, 1] = dst.astype(np.uint32)
        pl = i < np.uint64(self.n_planted_pairs)
        if pl.any():
            ii = i[pl].astype(np.int64)
            p = np.searchsorted(self.off, ii, side="right") - 1
            x_in = ii - self.off[p]
            m = np.asarray(self.m, dtype=np.int64)[p]
            D = np.asarray(self.planted, dtype=np.int64)[p]
            pool_idx = (s * m + x_in) % D
            out[pl, 0] = rank_to_ip(self.n_ranks + p)
            out[pl, 1] = _perm32(self.pool_key, (p.astype(np.uint64) << np.uint64(POOL_BITS))
                                 | pool_idx.astype(np.uint64))
        return out

    def planted_pool(self, p):
        """The D_p distinct second addresses of planted host p."""
        x = (np.uint64(p) << np.uint64(POOL_BITS)) | np.arange(self.planted[p], dtype=np.uint64)
        return _perm32(self.pool_key, x)


def loguniform_ints(lo, hi, n, seed):
    """n integers log-uniform on [lo, hi], from SplitMix64 outputs of seed."""
    out = []
    for c in range(n):
        uu = (mix64_int(seed + (c + 1) * GAMMA) >> 11) / float(1 << 53)
        out.append(int(round(math.exp(math.log(lo) + uu * (math.log(hi) - math.log(lo))))))
    return out
