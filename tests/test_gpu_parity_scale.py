"""HIP path against the oracle at the sizes the bench runs.

* the backbone workload (8M pairs per slice, SRE 8 x 2^20, SLE 2^24 DR
  cells) for 24 slices, and the paper's SEA (2^28 LE DRs) on the same stream
  for 12, in the bench's own launch configuration (streaming form, HIP
  graphs, partitioned scan, lean report, 2^25 candidate capacity),
  and with k = 16 for 40 slices so DRs leave the window at full size;
* candidate lists of more than a million entries and slices with millions
  of sampled pairs, so every end-of-slice kernel (sort, candidate check,
  compaction, merge, estimate, SI update) runs more than one pass of its
  grid;
* one member of each distinct geometry of the batched workload (16 monitors
  over one stream, both group scan forms) for 40 slices;
* an LE of more than 2^32 DRs (64-bit DR indices) with the flat and the
  partitioned scan;
* discrete slices whose sampled sources overflow the source set.

Pairs are produced by the device twin of the stream generator and copied
to the host for the oracle; the oracle runs in worker threads while the GPU
side is driven.  DR dumps, SI, candidate lists, flags and counts must match
bit for bit; FP64 estimates within 1e-12 relative.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_1803_10369_amd as srla
from trafficgen.configs import batched_monitors, scaled, workload
from trafficgen.device import DeviceStream

from gpu_helpers import (OracleThread, compare_dumps, compare_lean_reports, compare_reports,
                         host_pairs, to_device)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)


def _generate(ds, s, st):
    buf = ds.generate(s, stream=st)
    st.synchronize()
    return buf, host_pairs(buf, ds.spec.n_pairs)


@pytest.mark.parametrize("name,slices", [("backbone", 24), ("backbone_paper", 12)])
def test_full_size_in_the_bench_configuration(name, slices):
    """The backbone workload (24 slices) and the paper's SEA on the same
    stream (12 slices: a 2^28-DR LE in two bands of the partitioned scan),
    driven exactly as the bench's streaming form drives them: slice i closed
    and slice i+1's scan issued before the report of slice i-1 is collected."""
    stream, mon, _ = workload(name)
    st = torch.cuda.Stream()
    ds = DeviceStream(stream)
    g = srla.Monitor(**mon, max_candidates=1 << 25, timing=True, stream=st, graph=True,
                     lean_report=True, scan_partition=True, hold_scans=True)
    o = oracle.Monitor(**mon)
    ot = OracleThread()
    bufs, futs = {}, {}

    def feed(s):
        bufs[s], hp = _generate(ds, s, st)
        futs[s] = ot.slice(o, hp)
        print("slice", s, "scanned", flush=True)
        g.scan(bufs[s])

    feed(0)
    g.close_slice()
    feed(1)
    for i in range(1, slices + 1):
        if i < slices:
            g.close_slice()
            if i + 1 < slices:
                feed(i + 1)
        r = g.wait_report(copy=True)
        rc = futs.pop(i - 1).result()
        compare_lean_reports(r, rc, mon["theta"], "slice %d" % (i - 1))
        bufs.pop(i - 1, None)
    ot.close()
    compare_dumps(g, o, ctx="after slice %d" % (slices - 1))
    assert r.n > (30_000 if name == "backbone" else 1_000)
    g.close()
    o.close()


@pytest.mark.parametrize("scan_partition", [True, False])
def test_backbone_k16_full_size_40_slices(scan_partition):
    """Backbone stream and geometry with k = 16 for 40 slices at 8M pairs per
    slice: DRs leave the window, candidates are dropped and SI bits cleared
    at full size."""
    stream, mon, _ = workload("backbone_k16")
    st = torch.cuda.Stream()
    ds = DeviceStream(stream)
    g = srla.Monitor(**mon, max_candidates=1 << 23, stream=st, graph=True,
                     scan_partition=scan_partition)
    o = oracle.Monitor(**mon)
    ot = OracleThread()
    for s in range(40 if scan_partition else 20):
        buf, hp = _generate(ds, s, st)
        fut = ot.slice(o, hp)
        print("slice", s, flush=True)
        g.scan(buf)
        r = g.estimate()
        compare_reports(r, fut.result(), mon["theta"], "slice %d" % s)
        if s % 13 == 12:
            compare_dumps(g, o, ctx="slice %d" % s)
    ot.close()
    compare_dumps(g, o, ctx="end")
    g.close()
    o.close()


def _wide_sources(n_src, per, seed, salt=12345):
    """Slice generator: n_src sources, each with `per` fresh uniform
    destinations per slice, shuffled."""
    src0 = (np.arange(n_src, dtype=np.uint64) * np.uint64(2654435761) +
            np.uint64(salt)).astype(np.uint32)

    def gen(s):
        rng = np.random.default_rng(seed * 1000 + s)
        src = np.repeat(src0, per)
        dst = rng.integers(0, 2 ** 32, size=src.size, dtype=np.uint64).astype(np.uint32)
        p = np.stack([src, dst], 1)
        return p[rng.permutation(len(p))]
    return gen


@pytest.mark.parametrize("streaming", [False, True])
def test_candidates_beyond_one_grid_pass(streaming):
    """theta <= g (tau = 0: every pair is sampled), 1.2M sources with 5
    destinations each per slice: 6M sampled pairs per slice and about 1.2M
    candidates, so the sort, the candidate check, the compactions, the
    estimate and the SI update all take several passes of their grids."""
    mon = dict(k=3, theta=8, u=2, v_re=1 << 20, g=8, v_le=1 << 13, G=64, hash_seed=4242)
    gen = _wide_sources(1_200_000, 5, 77)
    st = torch.cuda.Stream()
    g = srla.Monitor(**mon, max_candidates=1 << 22, stream=st, graph=streaming,
                     scan_partition=streaming)
    o = oracle.Monitor(**mon)
    ot = OracleThread()
    prev = None
    for s in range(4):
        p = gen(s)
        fut = ot.slice(o, p)
        print("slice", s, flush=True)
        g.scan(to_device(p))
        if streaming:
            g.close_slice()
            if prev is not None:
                compare_reports(g.wait_report(), prev[1].result(), mon["theta"],
                                "slice %d" % prev[0])
            prev = (s, fut)
        else:
            r = g.estimate()
            rc = fut.result()
            compare_reports(r, rc, mon["theta"], "slice %d" % s)
            assert rc.n > 1_100_000 and rc.n_touched > 262_144
    if streaming:
        compare_reports(g.wait_report(), prev[1].result(), mon["theta"], "slice %d" % prev[0])
    ot.close()
    compare_dumps(g, o, ctx="end")
    g.close()
    o.close()


def test_merge_beyond_one_grid_pass():
    """4.5M sources with 5 destinations each (u = 1): about 97 % of them reach
    W >= 3 (5 draws from g = 8 DRs hit at least 3 of them), more than the
    4,194,304 candidates one pass of the merge grid writes, carried into the
    next slice."""
    mon = dict(k=2, theta=8, u=1, v_re=1 << 23, g=8, v_le=1 << 12, G=64, hash_seed=515)
    gen = _wide_sources(4_500_000, 5, 91)
    g = srla.Monitor(**mon, max_candidates=1 << 23)
    o = oracle.Monitor(**mon)
    ot = OracleThread()
    for s in range(2):
        p = gen(s)
        fut = ot.slice(o, p)
        print("slice", s, flush=True)
        g.scan(to_device(p))
        r = g.estimate()
        rc = fut.result()
        compare_reports(r, rc, mon["theta"], "slice %d" % s)
        assert rc.n > 4_194_304
    ot.close()
    compare_dumps(g, o, ctx="end")
    g.close()
    o.close()


@pytest.mark.parametrize("scan_partition", [True, False])
def test_batched_members_of_each_geometry_40_slices(scan_partition):
    """The 16 monitors of the batched workload in one group over the
    backbone stream (2M pairs per slice), 40 slices; the members of the six
    distinct geometries (SLE 2^20 .. 2^25 cells, members 0-5) are checked
    against their own oracle at every slice."""
    stream, _, _ = workload("backbone")
    stream = scaled(stream, 2_000_000)
    mons = batched_monitors(16)
    st = torch.cuda.Stream()
    ds = DeviceStream(stream)
    gms = [srla.Monitor(**m, max_candidates=1 << 22, stream=st, graph=True,
                        scan_partition=scan_partition) for m in mons]
    grp = srla.Group(gms)
    checked = list(range(6))
    oms = {i: oracle.Monitor(**mons[i]) for i in checked}
    ot = OracleThread(workers=len(checked))
    for s in range(40):
        buf, hp = _generate(ds, s, st)
        futs = {i: ot.slice(oms[i], hp) for i in checked}
        print("slice", s, flush=True)
        grp.scan(buf)
        for gm in gms:
            gm.close_slice()
        for i, gm in enumerate(gms):
            r = gm.wait_report()
            if i in futs:
                compare_reports(r, futs[i].result(), mons[i]["theta"],
                                "member %d slice %d" % (i, s))
    ot.close()
    for i in checked:
        compare_dumps(gms[i], oms[i], ctx="member %d" % i)
    grp.close()
    for gm in gms:
        gm.close()


@pytest.mark.parametrize("scan_partition", [False, True])
def test_le_beyond_2_32_drs(scan_partition):
    """u = 2 rows of (2^21 + 3) LEs of 1024 DRs: 2^32 + 6144 LE DRs, so DR
    indices, the row fills and the activity bitmap need 64 bits; the flat
    scan, and the partitioned scan in 33 bands (each row reaches into 17)."""
    mon = dict(k=2, theta=1024, u=2, v_re=4096, g=8, v_le=(1 << 21) + 3, G=1024,
               hash_seed=0x2_0000_0001)
    stream, _, _ = workload("tiny")
    stream = scaled(stream, 1_000_000)
    g = srla.Monitor(**mon, max_candidates=1 << 20, scan_partition=scan_partition)
    o = oracle.Monitor(**mon)
    ot = OracleThread()
    for s in range(3):
        p = stream.slice(s)
        fut = ot.slice(o, p)
        print("slice", s, flush=True)
        g.scan(to_device(p))
        compare_reports(g.estimate(), fut.result(), mon["theta"], "slice %d" % s)
    ot.close()
    compare_dumps(g, o, ctx="end")
    g.close()
    o.close()


def test_discrete_source_set_overflow():
    """Discrete form with a 4,096-slot source set (max_candidates 2,048) and
    400k distinct sampled sources per slice (tau = 0): most sources find
    their probes full and go straight to the list, and the candidate check
    and the drain take several passes."""
    mon = dict(k=1, theta=8, u=4, v_re=1 << 20, g=8, v_le=1024, G=64, hash_seed=606)
    wide = _wide_sources(400_000, 2, 33)
    rng = np.random.default_rng(5)
    heavy = np.stack([np.repeat(np.arange(50, dtype=np.uint32) + 7, 300),
                      rng.integers(0, 2 ** 32, size=15_000, dtype=np.uint64).astype(np.uint32)],
                     1)

    def gen(s):
        return np.concatenate([wide(s), heavy])

    g = srla.Monitor(**mon, max_candidates=2048, discrete=True)
    o = oracle.Monitor(**mon)
    for s in range(4):
        p = gen(s)
        print("slice", s, flush=True)
        g.scan(to_device(p))
        o.scan(p)
        r, rc = g.estimate(), o.estimate()
        compare_reports(r, rc, mon["theta"], "slice %d" % s)
        assert rc.n_touched > 262_144 and 50 <= rc.n <= 2048
    compare_dumps(g, o, ctx="end", discrete=True)
    g.close()
    o.close()
