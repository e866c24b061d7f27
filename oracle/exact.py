"""Brute-force checker for the oracle -- TEST INFRASTRUCTURE ONLY.

Everything here is recomputed from the stream history by definition, with no
distance recorders and no sliding loop:

* the DR of a cell holds the number of slices since the last pair that set
  it (Section 3.2), so at slice e it is e - last(cell), and it is inside the
  window W(e-k+1, k) iff last(cell) >= e-k+1;
* the row fills |LDR(i)|^k, the union weights |URE|^k and |ULE|^k (Algorithm
  1), the candidate lists (Algorithms 2 and 3 under the slice-synchronous
  reading) and Eq8/Eq9 follow from those window memberships;
* the exact cardinality |OP(aip, e, k)| is the number of distinct second
  addresses of aip in the window: the paper's "precise method" (Section 3.2).

The hash reading (multiply-add-shift functions drawn from SplitMix64) is
implemented here a second time in numpy/Python integers, so the oracle's C
hashing is checked against an independent copy.  Small inputs only.
"""
import math

import numpy as np

M64 = (1 << 64) - 1


def splitmix64_words(seed, n):
    s = seed & M64
    out = []
    for _ in range(n):
        s = (s + 0x9E3779B97F4A7C15) & M64
        z = s
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        out.append(z ^ (z >> 31))
    return out


class Hashes:
    """RH_0..RH_{u-1}, H1, H2, H3, H4 of one hash seed, vectorised in numpy."""

    def __init__(self, seed, u, v_re, g, v_le, G):
        w = splitmix64_words(seed, 2 * (u + 4))
        self.a = [w[2 * f] for f in range(u + 4)]
        self.b = [w[2 * f + 1] for f in range(u + 4)]
        self.u, self.v_re, self.g, self.v_le, self.G = u, v_re, g, v_le, G

    def _mas(self, f, x):
        x = np.asarray(x, dtype=np.uint64)
        with np.errstate(over="ignore"):
            v = np.uint64(self.a[f]) * x + np.uint64(self.b[f])
        return v >> np.uint64(32)

    @staticmethod
    def _rng(h, m):
        return (np.asarray(h, dtype=np.uint64) * np.uint64(m)) >> np.uint64(32)

    def row(self, i, aip):
        return self._mas(i, aip)

    def col_re(self, i, aip):
        return self._rng(self.row(i, aip), self.v_re).astype(np.int64)

    def col_le(self, i, aip):
        return self._rng(self.row(i, aip), self.v_le).astype(np.int64)

    def h1(self, bip):
        return self._mas(self.u, bip).astype(np.uint32)

    def re_idx(self, bip):
        return self._rng(self._mas(self.u + 1, bip), self.g).astype(np.int64)

    def le_idx(self, bip):
        return self._rng(self._mas(self.u + 2, bip), self.G).astype(np.int64)

    def si_idx(self, aip):
        return self._rng(self._mas(self.u + 3, aip), 16).astype(np.int64)


def lsb_array(x):
    """LSB of Definition 4 for a uint32 array, LSB(0) = 32."""
    x = np.asarray(x, dtype=np.uint64)
    out = np.full(x.shape, 32, dtype=np.int64)
    nz = x != 0
    lowbit = x[nz] & (~x[nz] + np.uint64(1))
    out[nz] = np.round(np.log2(lowbit.astype(np.float64))).astype(np.int64)
    return out


class BruteForce:
    """Last-touch bookkeeping of a whole stream, one closed slice at a time."""

    def __init__(self, k, theta, u, v_re, g, v_le, G, hash_seed, sequential=False):
        self.sequential = sequential
        self.k, self.theta = k, theta
        self.u, self.v_re, self.g, self.v_le, self.G = u, v_re, g, v_le, G
        self.h = Hashes(hash_seed, u, v_re, g, v_le, G)
        self.tau = 0
        while g * (1 << self.tau) < theta:
            self.tau += 1
        self.t_re = math.ceil(0.99 * (1.0 - math.exp(-1.0 / 3.0)) * g)
        self.last_le = np.full(u * v_le * G, -1, dtype=np.int64)
        self.last_re = np.full(u * v_re * g, -1, dtype=np.int64)
        self.history = []            # pairs of each closed slice
        self.ncsip = np.zeros(0, dtype=np.uint32)

    # --- cell addresses
    def le_cells(self, i, aip, leidx):
        return (i * self.v_le + self.h.col_le(i, aip)) * self.G + leidx

    def re_cells(self, i, aip, reidx):
        return (i * self.v_re + self.h.col_re(i, aip)) * self.g + reidx

    def _active(self, last, e, shift=0):
        """inside W(e-k+1, k) (shift=0) or after one more slide (shift=1)"""
        return (last >= 0) & (last >= e - self.k + 1 + shift)

    def union_weight(self, last, cols_fn, width, aips, e, shift=0):
        """DRs of the union estimator (max over rows) inside the window."""
        aips = np.asarray(aips, dtype=np.uint32)
        ok = np.ones((aips.size, width), dtype=bool)
        for i in range(self.u):
            base = cols_fn(i, aips)[:, None] * width + np.arange(width)[None, :]
            ok &= self._active(last[base], e, shift)
        return ok.sum(axis=1).astype(np.int64)

    def _ure(self, aips, e, shift=0):
        def cols(i, a):
            return i * self.v_re + self.h.col_re(i, a)
        return self.union_weight(self.last_re, cols, self.g, aips, e, shift)

    def _ule(self, aips, e):
        def cols(i, a):
            return i * self.v_le + self.h.col_le(i, a)
        return self.union_weight(self.last_le, cols, self.G, aips, e)

    def _si_bits(self, cands):
        """SI words set by a candidate list (Algorithm 3's marking)."""
        si = np.zeros(self.u * self.v_re, dtype=np.uint16)
        if len(cands):
            bit = (np.uint16(1) << self.h.si_idx(cands).astype(np.uint16))
            for i in range(self.u):
                idx = i * self.v_re + self.h.col_re(i, cands)
                np.bitwise_or.at(si, idx, bit)
        return si

    def close_slice(self, pairs):
        """Adds one slice and returns its report as a dict of numpy arrays."""
        pairs = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1, 2)
        e = len(self.history)
        self.history.append(pairs)
        aip, bip = pairs[:, 0], pairs[:, 1]
        leidx = self.h.le_idx(bip)
        for i in range(self.u):
            self.last_le[self.le_cells(i, aip, leidx)] = e
        sampled = lsb_array(self.h.h1(bip)) >= self.tau
        sa, sb = aip[sampled], bip[sampled]
        reidx = self.h.re_idx(sb)
        touched = np.unique(sa)
        si_start = self._si_bits(self.ncsip)
        if self.sequential:
            # Algorithm 2 literally: after each sampled pair's SRE update, the
            # host is checked against the state at that moment and, if new,
            # inserted with its SI bits set at once
            si = si_start.copy()
            new = []
            for a, r in zip(sa.tolist(), reidx.tolist()):
                a_arr = np.array([a], dtype=np.uint32)
                for i in range(self.u):
                    self.last_re[self.re_cells(i, a_arr, np.array([r]))] = e
                w = self._ure(a_arr, e)[0]
                bit = int(self.h.si_idx(a_arr)[0])
                usi = 0xFFFF
                for i in range(self.u):
                    usi &= int(si[i * self.v_re + self.h.col_re(i, a_arr)[0]])
                if w >= self.t_re and not (usi >> bit) & 1:
                    new.append(a)
                    for i in range(self.u):
                        si[i * self.v_re + self.h.col_re(i, a_arr)[0]] |= np.uint16(1 << bit)
            new = np.unique(np.array(new, dtype=np.uint32))
        else:
            for i in range(self.u):
                self.last_re[self.re_cells(i, sa, reidx)] = e
            W_t = self._ure(touched, e)
            usi = np.full(touched.size, 0xFFFF, dtype=np.uint16)
            for i in range(self.u):
                usi &= si_start[i * self.v_re + self.h.col_re(i, touched)]
            bit_clear = ((usi >> self.h.si_idx(touched).astype(np.uint16)) & 1) == 0
            new = touched[(W_t >= self.t_re) & bit_clear]
        # the carried list, then the new candidates, each ascending
        csip = np.concatenate([self.ncsip, np.sort(new)]).astype(np.uint32)

        cells = self.v_le * self.G
        act = self._active(self.last_le, e)
        L = np.array([act[i * cells:(i + 1) * cells].sum() for i in range(self.u)],
                     dtype=np.uint64)
        up = 1.0
        for i in range(self.u):
            up = up * (float(L[i]) / (float(self.G) * float(self.v_le)))
        U = self._ule(csip, e)
        W = self._ure(csip, e)
        W_after = self._ure(csip, e, shift=1)
        est = np.empty(csip.size)
        flags = np.zeros(csip.size, dtype=np.uint8)
        Gf = float(self.G)
        for x in range(csip.size):
            num = float(U[x]) - Gf * up
            den = Gf * (1.0 - up)
            if den == 0.0:
                est[x], flags[x] = math.inf, 2
            else:
                y = 1.0 - num / den
                if y <= 0.0:
                    est[x], flags[x] = math.inf, 2
                else:
                    est[x] = -Gf * math.log(y)
        flags |= np.where(est >= float(self.theta), 1, 0).astype(np.uint8)
        flags |= np.where(np.isin(csip, new), 4, 0).astype(np.uint8)
        keep = W_after >= self.t_re
        flags |= np.where(keep, 8, 0).astype(np.uint8)
        self.ncsip = np.sort(csip[keep])
        return dict(slice=e, window_full=e >= self.k - 1, ip=csip, est=est,
                    flags=flags, union_weight=U, re_weight=W, row_fill=L, up=up,
                    n_touched=touched.size, n_new=new.size)

    def dump(self, which):
        """Distances at the open slice, clamped at 32768 to 65535; SI raw."""
        now = len(self.history)
        if which == 2:
            return self._si_bits(self.ncsip)
        last = self.last_le if which == 0 else self.last_re
        d = now - last
        d = np.where((last < 0) | (d >= 32768), 65535, d)
        return d.astype(np.uint16)

    def exact_cardinality(self, e=None):
        """|OP(aip, e-k+1, k)| for every aip in the window (precise method)."""
        if e is None:
            e = len(self.history) - 1
        lo = max(0, e - self.k + 1)
        allp = np.concatenate(self.history[lo:e + 1]) if e >= lo else np.zeros((0, 2), np.uint32)
        key = (allp[:, 0].astype(np.uint64) << np.uint64(32)) | allp[:, 1].astype(np.uint64)
        key = np.unique(key)
        src = (key >> np.uint64(32)).astype(np.uint32)
        ips, counts = np.unique(src, return_counts=True)
        return dict(zip(ips.tolist(), counts.tolist()))
