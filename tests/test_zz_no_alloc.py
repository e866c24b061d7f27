"""srla_scan_noalloc (the scan with its scratch in the library's fixed device
array) against srla_scan, through the C ABI: the DR arrays, SI and every
report field must be identical, over two calls in a row -- the second with
fewer pairs, so stale scratch from the first call must not leak into it --
and over slices scanned by several calls.  Sizes beyond the entry point's
limits are rejected without side effects."""
import ctypes

import numpy as np
import pytest
import torch

import paper_1803_10369_amd as srla
from trafficgen.configs import scaled, workload

from gpu_helpers import to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)


def _noalloc(m, dev_pairs):
    n = dev_pairs.numel() // 2
    torch.cuda.current_stream().synchronize()
    return srla.srla_scan_noalloc(m._h, ctypes.c_void_p(dev_pairs.data_ptr()), n)


def _same(ra, rb, ctx):
    assert ra.slice == rb.slice and ra.n == rb.n, ctx
    for f in ("ip", "est", "flags", "union_weight", "re_weight", "row_fill"):
        a, b = getattr(ra, f), getattr(rb, f)
        assert np.array_equal(np.asarray(a).view(np.uint8), np.asarray(b).view(np.uint8)), (ctx, f)
    assert ra.up == rb.up and ra.n_touched == rb.n_touched and ra.n_new == rb.n_new, ctx


def _same_state(ma, mb, ctx):
    for which in (srla.SRLA_DUMP_LE, srla.SRLA_DUMP_RE, srla.SRLA_DUMP_SI):
        assert np.array_equal(ma.dump(which), mb.dump(which)), (ctx, which)


@pytest.mark.parametrize("u,v_le,sizes", [
    # u = 8: 4096 pairs per chunk, 524,288 per partition round of the fixed
    # scratch, so the first call takes two rounds
    (8, 2048, [(900_000,), (200_000,)]),
    # u = 3 (the generic row loop), 192 regions; a slice in two calls
    (3, 4096, [(700_000, 100_000), (50_000,)]),
    # 2^25 DRs, 512 regions in one band
    (4, 8192, [(1_000_000,), (300_000,)]),
    # 2^28 + 2^12 DRs (the paper's SEA geometry plus one LE per row): three
    # bands of up to 2048 regions, the last of one region; rows straddle bands
    (4, 65537, [(600_000,), (200_000,)]),
])
def test_noalloc_scan_matches_srla_scan(u, v_le, sizes):
    stream, _, _ = workload("tiny")
    mon = dict(k=3, theta=256, u=u, v_re=4096, g=8, v_le=v_le, G=1024, hash_seed=31337 + u)
    stream = scaled(stream, max(sum(s) for s in sizes))
    ref = srla.Monitor(**mon, max_candidates=1 << 20, scan_partition=True)
    new = srla.Monitor(**mon, max_candidates=1 << 20)
    for s, parts in enumerate(sizes):
        p = stream.slice(s)
        off, held = 0, []   # device pairs stay alive until the slice is estimated
        for cnt in parts:
            d = to_device(p[off:off + cnt])
            held.append(d)
            off += cnt
            print("slice", s, "u", u, "pairs", cnt, flush=True)
            ref.scan(d)
            rc = _noalloc(new, d)
            assert rc == 0, (rc, srla.srla_last_error(new._h))
        _same(ref.estimate(), new.estimate(), "slice %d" % s)
        _same_state(ref, new, "slice %d" % s)
    ref.close()
    new.close()


def test_noalloc_scan_rejects_what_it_cannot_hold():
    """Beyond the sampled-source capacity or on a discrete monitor:
    SRLA_E_INVAL and nothing scanned."""
    stream, _, _ = workload("tiny")
    p = to_device(scaled(stream, 1000).slice(0))
    disc = srla.Monitor(k=1, theta=256, u=4, v_re=1024, g=8, v_le=64, G=1024, hash_seed=2,
                        discrete=True)
    assert _noalloc(disc, p) == srla.SRLA_E_INVAL
    disc.close()
    m = srla.Monitor(k=2, theta=256, u=4, v_re=1024, g=8, v_le=64, G=1024, hash_seed=3)
    wide = torch.zeros(2 * ((1 << 20) + 1), dtype=torch.int32, device="cuda")
    assert _noalloc(m, wide) == srla.SRLA_E_INVAL
    r = m.estimate()
    assert r.n == 0 and r.n_touched == 0
    assert (m.dump(srla.SRLA_DUMP_LE) == 65535).all()
    m.close()
