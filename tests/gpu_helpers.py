"""Shared pieces of the GPU parity tests: run the HIP path and the oracle on
the same seeded pairs and compare them element by element."""
import numpy as np
import torch

import oracle

# FP64 estimates: both sides evaluate Eq8-Eq9 with the same IEEE operations in
# the same order (no contraction); only the natural logarithm differs (the
# GPU's ocml vs glibc, each within about one ulp), so the estimates agree to
# a few ulp.  1e-12 relative leaves a wide margin over that.
RTOL = 1e-12


def to_device(pairs):
    p = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1)
    return torch.from_numpy(p.view(np.int32)).cuda()


def compare_reports(rg, rc, theta, ctx=""):
    assert rg.slice == rc.slice, ctx
    assert rg.window_full == rc.window_full, ctx
    assert rg.n == rc.n, (ctx, rg.n, rc.n)
    assert np.array_equal(rg.ip, rc.ip), ctx
    assert np.array_equal(rg.union_weight, rc.union_weight), ctx
    assert np.array_equal(rg.re_weight, rc.re_weight), ctx
    assert np.array_equal(rg.row_fill, rc.row_fill), ctx
    assert rg.up == rc.up, (ctx, rg.up, rc.up)
    assert rg.n_touched == rc.n_touched and rg.n_new == rc.n_new, ctx
    fin = np.isfinite(rc.est)
    assert np.array_equal(np.isfinite(rg.est), fin), ctx
    assert np.array_equal(np.isposinf(rg.est), np.isposinf(rc.est)), ctx
    e_g, e_c = rg.est[fin], rc.est[fin]
    assert np.all(np.abs(e_g - e_c) <= RTOL * np.abs(e_c)), (ctx, np.max(np.abs(e_g - e_c)))
    # flags are integers decided by the same FP64 values: equal, except that
    # SUPER (est >= theta) may only differ for an estimate within the
    # tolerance of theta
    other = ~np.uint8(oracle.SUPER)
    assert np.array_equal(rg.flags & other, rc.flags & other), ctx
    diff = (rg.flags ^ rc.flags) & oracle.SUPER
    if diff.any():
        assert np.all(np.abs(rc.est[diff != 0] - theta) <= RTOL * theta), ctx


def compare_dumps(gm, om, ctx="", discrete=False):
    """discrete: the GPU monitor keeps one bit per DR (k = 1), so it knows a
    DR's distance only up to 1 (set in the open slice / in the slice closed
    last); larger oracle distances compare as 65535."""
    for which in (0, 1, 2):
        a, b = gm.dump(which), om.dump(which)
        if discrete and which != 2:
            b = np.where(b <= 1, b, np.uint16(65535)).astype(np.uint16)
        if not np.array_equal(a, b):
            bad = np.flatnonzero(a != b)
            raise AssertionError("%s: array %d differs at %d cells, first %d: gpu %d oracle %d"
                                 % (ctx, which, bad.size, bad[0], a[bad[0]], b[bad[0]]))


def compare_lean_reports(rg, rc, theta, ctx=""):
    """compare_reports for a report without the per-candidate weights
    (SRLA_CFG_LEAN_REPORT): ip, est, flags and the slice's counts."""
    assert rg.union_weight is None and rg.re_weight is None, ctx
    assert rg.slice == rc.slice, ctx
    assert rg.window_full == rc.window_full, ctx
    assert rg.n == rc.n, (ctx, rg.n, rc.n)
    assert np.array_equal(rg.ip, rc.ip), ctx
    assert np.array_equal(rg.row_fill, rc.row_fill), ctx
    assert rg.up == rc.up, (ctx, rg.up, rc.up)
    assert rg.n_touched == rc.n_touched and rg.n_new == rc.n_new, ctx
    fin = np.isfinite(rc.est)
    assert np.array_equal(np.isfinite(rg.est), fin), ctx
    assert np.array_equal(np.isposinf(rg.est), np.isposinf(rc.est)), ctx
    e_g, e_c = rg.est[fin], rc.est[fin]
    assert np.all(np.abs(e_g - e_c) <= RTOL * np.abs(e_c)), (ctx, np.max(np.abs(e_g - e_c)))
    other = ~np.uint8(oracle.SUPER)
    assert np.array_equal(rg.flags & other, rc.flags & other), ctx
    diff = (rg.flags ^ rc.flags) & oracle.SUPER
    if diff.any():
        assert np.all(np.abs(rc.est[diff != 0] - theta) <= RTOL * theta), ctx


class OracleThread:
    """Runs oracle monitors' scan + estimate in a worker thread (the oracle's
    C calls release the GIL), so the oracle works while the GPU side is
    driven from the test's own thread."""

    def __init__(self, workers=1):
        from concurrent.futures import ThreadPoolExecutor
        self.pool = ThreadPoolExecutor(max_workers=workers)

    def slice(self, om, pairs):
        """Future of om's report after scanning pairs (host numpy, (n, 2))."""
        def work():
            om.scan(pairs)
            return om.estimate()
        return self.pool.submit(work)

    def close(self):
        self.pool.shutdown(wait=True)


def host_pairs(dev_pairs, n):
    """The first n pairs of an int32 CUDA tensor as a host (n, 2) uint32 array."""
    return dev_pairs[:2 * n].cpu().numpy().view(np.uint32).reshape(-1, 2)
