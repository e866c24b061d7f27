"""HIP path against the oracle, element by element, on the same seeded pairs.

DR dumps, SI words, candidate lists, flags and integer counts must match
bit for bit; FP64 estimates within 1e-12 relative.  Sizes span many scan,
sort and compaction tiles with ragged tails.
"""
import time

import numpy as np
import pytest
import torch

import oracle
import paper_1803_10369_amd as srla
from trafficgen.configs import workload, scaled

from gpu_helpers import compare_dumps, compare_reports, to_device

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    torch.cuda.set_device(0)


def _run(stream, mon, slices, max_candidates=1 << 16, dump_every=1, split=None, host=False,
         scan_xcd=False, graph=False, discrete=False, scan_dedup=False, scan_lds_filter=False,
         scan_partition=False):
    g = srla.Monitor(**mon, max_candidates=max_candidates, scan_xcd=scan_xcd, graph=graph,
                     discrete=discrete, scan_dedup=scan_dedup, scan_lds_filter=scan_lds_filter,
                     scan_partition=scan_partition)
    o = oracle.Monitor(**mon)
    for s in slices:
        pairs = stream.slice(s) if hasattr(stream, "slice") else stream(s)
        print("slice", s, "pairs", len(pairs), flush=True)
        if split:
            for lo in range(0, len(pairs), split):
                part = pairs[lo:lo + split]
                g.scan(part if host else to_device(part))
        else:
            g.scan(pairs if host else to_device(pairs))
        o.scan(pairs)
        rg, rc = g.estimate(), o.estimate()
        compare_reports(rg, rc, mon["theta"], ctx="slice %d" % s)
        if dump_every and (s % dump_every == 0):
            compare_dumps(g, o, ctx="slice %d" % s, discrete=discrete)
    compare_dumps(g, o, ctx="end", discrete=discrete)
    g.close()
    return rg


@pytest.mark.parametrize("scan_xcd,graph", [(False, False), (True, False), (False, True)])
def test_tiny_workload_full_run(scan_xcd, graph):
    stream, mon, n = workload("tiny")
    r = _run(stream, mon, range(n), scan_xcd=scan_xcd, graph=graph)
    assert r.window_full and r.n > 0


@pytest.mark.parametrize("scan_xcd,blocks,dedup", [(False, 7, False), (True, 16, False),
                                                    (True, 5, False), (True, 24, True),
                                                    (True, 3, True)])
def test_scan_grid_cap_strides_over_all_pairs(scan_xcd, blocks, dedup):
    stream, mon, n = workload("tiny")
    g = srla.Monitor(**mon, max_candidates=1 << 16, scan_xcd=scan_xcd, scan_blocks=blocks,
                     scan_dedup=dedup)
    o = oracle.Monitor(**mon)
    for s in range(6):
        p = stream.slice(s)
        g.scan(to_device(p))
        o.scan(p)
        compare_reports(g.estimate(), o.estimate(), mon["theta"], "slice %d" % s)
    compare_dumps(g, o)
    g.close()


def test_tiny_coupled_workload_full_run():
    stream, mon, n = workload("tiny_coupled")
    r = _run(stream, mon, range(n), dump_every=4)
    assert r.n > 0 and np.isfinite(r.est).mean() > 0.5


def _rand_stream(seed, n, n_src, heavy_theta):
    def gen(s):
        rng = np.random.default_rng(seed * 1000 + s)
        w = 1.0 / np.arange(1, n_src + 1) ** 1.1
        src = rng.choice(n_src, size=n, p=w / w.sum()).astype(np.uint32) * np.uint32(2654435761)
        dst = rng.integers(0, 2 ** 32, size=n, dtype=np.uint64).astype(np.uint32)
        p = np.stack([src, dst], 1)
        if s < 3:
            h = np.stack([np.full(heavy_theta, 7, np.uint32),
                          rng.integers(0, 2 ** 32, size=heavy_theta, dtype=np.uint64).astype(np.uint32)], 1)
            p = np.concatenate([p, h])
        if s == 2:
            p = p[:0]
        return p
    return gen


SMALL = [
    # k, theta, u, v_re, g, v_le, G, pairs/slice, sources, slices
    (3, 64, 3, 64, 8, 8, 128, 30000, 2000, 8),
    (1, 64, 2, 32, 8, 4, 64, 15000, 1000, 5),
    (5, 16, 1, 16, 4, 16, 64, 8000, 600, 9),
    (4, 4, 4, 128, 8, 32, 64, 6000, 3000, 7),
    (6, 4096, 2, 64, 16, 8, 192, 40000, 500, 8),
    (2, 256, 5, 33, 3, 7, 64, 20000, 1200, 6),
    (7, 1024, 8, 4096, 8, 64, 1024, 50000, 20000, 9),
    (3, 300, 16, 97, 64, 5, 4096, 12000, 800, 5),
]


@pytest.mark.parametrize("case", SMALL)
@pytest.mark.parametrize("scan_xcd,graph", [(False, False), (True, True)])
def test_small_geometries(case, scan_xcd, graph):
    k, theta, u, v_re, g, v_le, G, n, n_src, slices = case
    mon = dict(k=k, theta=theta, u=u, v_re=v_re, g=g, v_le=v_le, G=G, hash_seed=1000 + k + u)
    _run(_rand_stream(k + u, n, n_src, 3 * theta // 2), mon, range(slices), scan_xcd=scan_xcd,
         graph=graph)


def _run_streaming(stream, mon, slices, max_candidates=1 << 16, graph=False, chunks=1,
                   discrete=False, scan_dedup=False, overlap_report=False, ahead=False,
                   scan_partition=False, hold_scans=False):
    """The next slice is scanned before the previous slice's report is taken;
    ahead: it is also closed before that report is taken (two reports pending),
    and a collected report's arrays (views, no copy) must hold until the slice
    two after it is closed."""
    g = srla.Monitor(**mon, max_candidates=max_candidates, graph=graph, discrete=discrete,
                     scan_dedup=scan_dedup, overlap_report=overlap_report,
                     scan_partition=scan_partition, hold_scans=hold_scans)
    o = oracle.Monitor(**mon)
    expected = []
    slices = list(slices)
    held = None
    for i, s in enumerate(slices):
        pairs = stream.slice(s) if hasattr(stream, "slice") else stream(s)
        step = -(-len(pairs) // chunks) if len(pairs) else 1
        for lo in range(0, max(len(pairs), 1), step):
            g.scan(to_device(pairs[lo:lo + step]))
        o.scan(pairs)
        expected.append(o.estimate())
        if ahead:
            if held is not None:
                # the report of slice s-2 (views) survived the close of s-1, its
                # pipeline and the collection of its report: they use the other
                # buffer set; the close of s below may overwrite it
                compare_reports(held, expected[i - 2], mon["theta"], "held %d" % (s - 2))
            g.close_slice()
            if i > 0:
                r = g.wait_report(copy=False)
                compare_reports(r, expected[i - 1], mon["theta"], "slice %d" % (s - 1))
                held = r
        else:
            if i > 0:
                compare_reports(g.wait_report(), expected[i - 1], mon["theta"],
                                "slice %d" % (s - 1))
            g.close_slice()
    compare_reports(g.wait_report(), expected[-1], mon["theta"], "last slice")
    compare_dumps(g, o, ctx="end", discrete=discrete)
    g.close()


@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("ahead", [False, True])
def test_streaming_form_matches_oracle(graph, ahead):
    stream, mon, n = workload("tiny")
    _run_streaming(stream, mon, range(n), graph=graph, chunks=3, ahead=ahead)


@pytest.mark.parametrize("case", SMALL[:4])
def test_streaming_small_geometries(case):
    k, theta, u, v_re, g, v_le, G, n, n_src, slices = case
    mon = dict(k=k, theta=theta, u=u, v_re=v_re, g=g, v_le=v_le, G=G, hash_seed=1000 + k + u)
    _run_streaming(_rand_stream(k + u, n, n_src, 3 * theta // 2), mon, range(slices), graph=True)


def test_streaming_call_order_errors():
    stream, mon, _ = workload("tiny")
    g = srla.Monitor(**mon, max_candidates=1 << 16)
    with pytest.raises(srla.SrlaError) as e:
        g.wait_report()
    assert e.value.rc == -4
    g.scan(to_device(stream.slice(0)))
    g.close_slice()
    g.close_slice()                  # an empty slice 1; two reports pending
    with pytest.raises(srla.SrlaError) as e:
        g.close_slice()              # a third is refused
    assert e.value.rc == -4
    with pytest.raises(srla.SrlaError) as e:
        g.estimate()                 # needs no report pending
    assert e.value.rc == -4
    r0 = g.wait_report(copy=False)
    r1 = g.wait_report(copy=False)
    assert (r0.slice, r1.slice) == (0, 1)
    assert r0.latency_ms > 0 and r1.latency_ms > 0
    with pytest.raises(srla.SrlaError) as e:
        g.wait_report()
    assert e.value.rc == -4
    g.close()


def test_host_input_chunked_and_unaligned_device_input():
    stream, mon, _ = workload("tiny")
    stream = scaled(stream, 77_777)
    # host pointers, several scans per slice
    _run(stream, mon, range(10), host=True, split=20_001, dump_every=3)
    # device pointers that are 4- but not 16-byte aligned
    g = srla.Monitor(**mon, max_candidates=1 << 16)
    o = oracle.Monitor(**mon)
    for s in range(6):
        p = stream.slice(s)
        flat = to_device(np.concatenate([np.zeros(1, np.uint32), p.reshape(-1)]))
        g.scan(flat[1:])
        o.scan(p)
        compare_reports(g.estimate(), o.estimate(), mon["theta"], "unaligned %d" % s)
    compare_dumps(g, o)
    g.close()


def test_pinned_host_input_is_copied_directly():
    """Host pairs in page-locked memory go straight to the device by DMA (no
    bounce buffer); the results equal the oracle's, and the caller may
    overwrite its buffer as soon as the scan returns."""
    stream, mon, n = workload("tiny")
    g = srla.Monitor(**mon, max_candidates=1 << 16)
    o = oracle.Monitor(**mon)
    buf = torch.empty(2 * 100_000, dtype=torch.int32, pin_memory=True)
    for s in range(n):
        p = stream.slice(s)
        for lo in range(0, len(p), 30_000):
            part = p[lo:lo + 30_000]
            view = buf[:2 * len(part)]
            view.copy_(torch.from_numpy(np.ascontiguousarray(part).reshape(-1).view(np.int32)))
            g.scan(view)
            view.fill_(-1)                  # reused at once: the scan has copied it
        o.scan(p)
        compare_reports(g.estimate(), o.estimate(), mon["theta"], "slice %d" % s)
    compare_dumps(g, o)
    g.close()


def test_large_host_scans_use_the_ring():
    """8M-pair host scans (two ring chunks each), pinned and pageable, at the
    backbone geometry."""
    stream, mon, _ = workload("backbone")
    g = srla.Monitor(**mon, max_candidates=1 << 22)
    o = oracle.Monitor(**mon)
    pinned = torch.empty(2 * stream.n_pairs, dtype=torch.int32, pin_memory=True)
    for s in range(3):
        p = stream.slice(s)
        if s == 1:
            g.scan(p)                                        # pageable numpy
        else:
            pinned.copy_(torch.from_numpy(np.ascontiguousarray(p).reshape(-1).view(np.int32)))
            g.scan(pinned)
        o.scan(p)
        compare_reports(g.estimate(), o.estimate(), mon["theta"], "slice %d" % s)
    g.close()


def test_pair_order_and_repeat_runs_are_identical():
    stream, mon, _ = workload("tiny")
    reps = []
    for variant in range(3):
        g = srla.Monitor(**mon, max_candidates=1 << 16)
        out = []
        for s in range(10):
            p = stream.slice(s)
            if variant == 2:
                p = p[np.random.default_rng(s).permutation(len(p))]
            g.scan(to_device(p))
            r = g.estimate()
            out.append((r.ip, r.est, r.flags, r.union_weight, r.re_weight, r.row_fill))
        out.append(tuple(g.dump(w) for w in (0, 1, 2)))
        reps.append(out)
        g.close()
    for other in reps[1:]:
        for x, y in zip(reps[0], other):
            for a, b in zip(x, y):
                assert np.array_equal(a, b)


def test_empty_slices_and_silence():
    stream, mon, _ = workload("tiny")
    g = srla.Monitor(**mon, max_candidates=1 << 16)
    o = oracle.Monitor(**mon)
    for s in range(12):
        if s in (0, 3, 4, 9, 10, 11):
            g.scan(to_device(np.zeros((0, 2), np.uint32)))
        else:
            p = stream.slice(s)
            g.scan(to_device(p))
            o.scan(p)
        compare_reports(g.estimate(), o.estimate(), mon["theta"], "slice %d" % s)
    compare_dumps(g, o)
    g.close()


def test_capacity_overflow_is_reported_and_poisons():
    stream, mon, _ = workload("tiny")
    g = srla.Monitor(**mon, max_candidates=5)
    g.scan(to_device(stream.slice(0)))
    with pytest.raises(srla.SrlaError) as e:
        g.estimate()
    assert e.value.rc == -3
    with pytest.raises(srla.SrlaError) as e:
        g.scan(to_device(stream.slice(1)))
    assert e.value.rc == -4
    g.close()


def test_backbone_workload_prefix_full_size():
    """The backbone-shaped workload (8M pairs per slice, SRE 8 x 2^20 cells,
    SLE 2^24 cells, k = 300) in the launch configuration the bench times: one
    device-pointer scan per slice."""
    stream, mon, _ = workload("backbone")
    _run(stream, mon, range(3), max_candidates=1 << 22)


@pytest.mark.parametrize("scan_xcd,graph", [(False, False), (True, True)])
def test_backbone_short_window_expiry(scan_xcd, graph):
    """Backbone geometry with k = 16 over 40 slices, so DRs leave the window
    and carried candidates are dropped at full column counts."""
    stream, mon, _ = workload("backbone_k16")
    stream = scaled(stream, 600_000)
    _run(stream, mon, range(40), max_candidates=1 << 22, dump_every=13, scan_xcd=scan_xcd,
         graph=graph)


def test_backbone_short_window_streaming():
    stream, mon, _ = workload("backbone_k16")
    stream = scaled(stream, 600_000)
    _run_streaming(stream, mon, range(24), max_candidates=1 << 22, graph=True)


def test_paper_geometry_prefix():
    """u = 4, v = 65,536, g' = 1,024 (the paper's chosen parameters): a 512 MB
    LE array, far beyond the last-level cache."""
    stream, mon, _ = workload("backbone_paper")
    stream = scaled(stream, 2_000_000)
    _run(stream, mon, range(3), max_candidates=1 << 22)


def test_device_generator_matches_host_twin():
    from trafficgen.device import DeviceStream
    stream, _, _ = workload("tiny")
    ds = DeviceStream(stream)
    for s in (0, 1, 7):
        d = ds.generate(s).cpu().numpy().view(np.uint32).reshape(-1, 2)
        assert np.array_equal(d, stream.slice(s))
    big, _, _ = workload("backbone")
    dsb = DeviceStream(big)
    d = dsb.generate(5).cpu().numpy().view(np.uint32).reshape(-1, 2)
    idx = np.random.default_rng(0).integers(0, big.n_pairs, size=20000)
    idx.sort()
    host = np.concatenate([big.slice(5, i, i + 1) for i in idx[:200]])
    assert np.array_equal(d[idx[:200]], host)
    lo = 3_000_000
    assert np.array_equal(d[lo:lo + 50_000], big.slice(5, lo, lo + 50_000))


def test_timings_are_recorded():
    stream, mon, _ = workload("tiny")
    g = srla.Monitor(**mon, max_candidates=1 << 16, timing=True)
    for s in range(3):
        g.scan(to_device(stream.slice(s)))
        g.estimate()
    t = g.timings(reset=True)
    assert t["scan_ms"] > 0 and t["scan_launches"] == 3 and t["scan_pairs"] == 300_000
    assert t["sweep_ms"] > 0 and t["estimate_ms"] > 0 and t["estimates"] == 3
    assert g.timings()["scan_ms"] == 0
    g.close()


@pytest.mark.parametrize("graph,overlap", [(False, False), (True, True)])
def test_timing_can_be_sampled(graph, overlap):
    """Timing switched on for slices 0 and 2 only, in the streaming call order
    (each slice closed before the previous report is collected): only their
    scans and stages are counted, and the results do not change."""
    stream, mon, _ = workload("tiny")
    g = srla.Monitor(**mon, max_candidates=1 << 16, graph=graph, overlap_report=overlap)
    o = oracle.Monitor(**mon)
    for s in range(5):
        g.set_timing(s % 2 == 0 and s < 4)
        p = stream.slice(s)
        g.scan(to_device(p[:50_000]))
        g.scan(to_device(p[50_000:]))
        g.close_slice()
        o.scan(p)
        exp = o.estimate()
        if s > 0:
            compare_reports(g.wait_report(), prev, mon["theta"], "slice %d" % (s - 1))
        prev = exp
    compare_reports(g.wait_report(), prev, mon["theta"], "last slice")
    t = g.timings(reset=True)
    assert t["scan_launches"] == 4 and t["scan_pairs"] == 2 * len(stream.slice(0))
    assert t["estimates"] == 2 and t["scan_ms"] > 0 and t["report_ms"] > 0
    g.close()


def test_timing_scans_only():
    """SRLA_TIMING_SCANS times the scans and no stage of the slices' ends;
    switched back to full timing, the stages are counted again."""
    stream, mon, _ = workload("tiny")
    g = srla.Monitor(**mon, max_candidates=1 << 16, graph=True, hold_scans=True,
                     scan_partition=True)
    o = oracle.Monitor(**mon)
    g.set_timing(srla.SRLA_TIMING_SCANS)
    for s in range(4):
        if s == 3:
            g.set_timing(True)
        p = stream.slice(s)
        g.scan(to_device(p))
        o.scan(p)
        compare_reports(g.estimate(), o.estimate(), mon["theta"], "slice %d" % s)
    t = g.timings(reset=True)
    assert t["scan_launches"] == 4 and t["scan_pairs"] == 4 * len(stream.slice(0))
    assert t["scan_ms"] > 0 and t["estimates"] == 1 and t["estimate_ms"] > 0
    g.close()


GROUP = [
    # k, theta, u, v_re, g, v_le, G
    (3, 64, 3, 64, 8, 8, 128),
    (1, 256, 4, 128, 8, 16, 1024),
    (5, 16, 1, 16, 4, 16, 64),
    (7, 4096, 8, 512, 16, 32, 192),
    (2, 300, 16, 97, 64, 5, 4096),
]


@pytest.mark.parametrize("streaming", [False, True])
def test_group_fused_scan_matches_each_members_oracle(streaming):
    """One pair stream, five monitors of different windows, geometries,
    thresholds and seeds, scanned by the fused kernel."""
    st = torch.cuda.Stream()
    mons = [dict(k=k, theta=t, u=u, v_re=vr, g=g, v_le=vl, G=G, hash_seed=77 + i)
            for i, (k, t, u, vr, g, vl, G) in enumerate(GROUP)]
    gms = [srla.Monitor(**m, max_candidates=1 << 16, stream=st, graph=bool(i % 2))
           for i, m in enumerate(mons)]
    oms = [oracle.Monitor(**m) for m in mons]
    grp = srla.Group(gms, scan_blocks=0 if streaming else 9)
    gen = _rand_stream(5, 30_000, 2500, 400)
    expected = None
    for s in range(8):
        p = gen(s)
        grp.scan(to_device(p))
        for o in oms:
            o.scan(p)
        if streaming and expected is not None:
            for gm, e, m in zip(gms, expected, mons):
                compare_reports(gm.wait_report(), e, m["theta"], "slice %d" % (s - 1))
        expected = [o.estimate() for o in oms]
        if streaming:
            for gm in gms:
                gm.close_slice()
        else:
            for gm, e, m in zip(gms, expected, mons):
                compare_reports(gm.estimate(), e, m["theta"], "slice %d" % s)
    if streaming:
        for gm, e, m in zip(gms, expected, mons):
            compare_reports(gm.wait_report(), e, m["theta"], "last slice")
    for gm, o in zip(gms, oms):
        compare_dumps(gm, o)
    grp.close()
    for gm in gms:
        gm.close()


@pytest.mark.parametrize("partitioned", [False, True])
def test_group_with_held_scans_matches_each_members_oracle(partitioned):
    """Members with SRLA_CFG_HOLD_SCANS: each member's slice end runs on the
    group's scan stream, in order, the slides on the shared pipeline stream,
    and the next group scan follows them; the host runs a slice ahead."""
    st = torch.cuda.Stream()
    mons = [dict(k=k, theta=t, u=u, v_re=vr, g=g, v_le=vl, G=G, hash_seed=91 + i)
            for i, (k, t, u, vr, g, vl, G) in enumerate(GROUP)]
    gms = [srla.Monitor(**m, max_candidates=1 << 16, stream=st, graph=bool(i % 2),
                        hold_scans=True, scan_partition=partitioned)
           for i, m in enumerate(mons)]
    oms = [oracle.Monitor(**m) for m in mons]
    grp = srla.Group(gms, scan_blocks=0)
    gen = _rand_stream(9, 30_000, 2500, 400)
    expected = None
    for s in range(7):
        p = gen(s)
        grp.scan(to_device(p))
        for o in oms:
            o.scan(p)
        if expected is not None:
            for gm, e, m in zip(gms, expected, mons):
                compare_reports(gm.wait_report(), e, m["theta"], "slice %d" % (s - 1))
        expected = [o.estimate() for o in oms]
        for gm in gms:
            gm.close_slice()
    for gm, e, m in zip(gms, expected, mons):
        compare_reports(gm.wait_report(), e, m["theta"], "last slice")
    for gm, o in zip(gms, oms):
        compare_dumps(gm, o)
    grp.close()
    for gm in gms:
        gm.close()


def test_group_rejects_mixed_streams_and_duplicates():
    stream, mon, _ = workload("tiny")
    a = srla.Monitor(**mon, max_candidates=1 << 10)
    b = srla.Monitor(**mon, max_candidates=1 << 10)
    with pytest.raises(srla.SrlaError):
        srla.Group([a, b])            # two different streams
    with pytest.raises(srla.SrlaError):
        srla.Group([a, a])
    a.close()
    b.close()


def test_stamps_survive_wraparound_of_the_slice_code():
    """70,000 slices (past 65,535, where the 16-bit slice code repeats): DRs
    set long ago must read as outside every window, never as recent."""
    mon = dict(k=3, theta=8, u=2, v_re=4, g=8, v_le=2, G=64, hash_seed=5)
    g = srla.Monitor(**mon, max_candidates=64, graph=True)
    o = oracle.Monitor(**mon)
    rng = np.random.default_rng(3)
    burst = {0, 1, 2, 40_000, 65_534, 65_535, 65_536, 65_537, 69_998}
    pairs_dev = {}
    t0 = time.time()
    for s in range(70_000):
        if s in burst:
            p = np.stack([np.full(40, 9, np.uint32),
                          rng.integers(0, 2 ** 32, size=40, dtype=np.uint64).astype(np.uint32)], 1)
            pairs_dev[s] = to_device(p)
            g.scan(pairs_dev[s])
            o.scan(p)
        rg, rc = g.estimate(copy=False), o.estimate()
        if s in burst or s % 5000 == 0 or (s - 1) in burst or (s - 3) in burst:
            compare_reports(rg, rc, mon["theta"], "slice %d" % s)
            compare_dumps(g, o, ctx="slice %d" % s)
        if s % 10000 == 0:
            print("slice", s, "%.1fs" % (time.time() - t0), flush=True)
    g.close()


def test_autotuner_picks_a_valid_shape_and_results_do_not_change(tmp_path):
    from paper_1803_10369_amd import autotune
    stream, mon, _ = workload("tiny")
    pairs = to_device(stream.slice(0))
    cache = str(tmp_path / "tune.json")
    choice = autotune.tune_scan(mon, pairs, repeats=2, cache=cache)
    assert set(choice["all"]) == {"flat/0", "flat/1024", "flat/512", "dedup/0", "partition/0",
                                  "partition/16384", "partition/65536"}
    assert choice["ms"] == min(choice["all"].values()) > 0
    assert autotune.tune_scan(mon, pairs, cache=cache) == choice      # served from the cache
    _run(stream, mon, range(6), scan_xcd=choice["scan_xcd"], scan_dedup=choice["scan_dedup"],
         scan_lds_filter=choice["scan_lds_filter"], scan_partition=choice["scan_partition"])
    # the partitioned form is tried at any LE size (here 2^26 * u DRs, bands)
    big = dict(mon, v_le=1 << 14, G=4096)
    assert "partition/0" in autotune.tune_scan(big, pairs, repeats=1, cache=None)["all"]
    # every form can still be asked for explicitly
    forms = [("xcd", 0), ("xcd_dedup", 16), ("filter", 0)]
    extra = autotune.tune_scan(mon, pairs, candidates=forms, repeats=1, cache=None)
    assert set(extra["all"]) == {"xcd/0", "xcd_dedup/16", "filter/0"}

    st = torch.cuda.Stream()
    gms = [srla.Monitor(**mon, max_candidates=1 << 16, stream=st) for _ in range(2)]
    o = oracle.Monitor(**mon)
    g_choice = autotune.tune_group(gms, pairs)
    assert g_choice["scan_blocks"] in (0, 2048, 1024, 512)
    grp = srla.Group(gms, scan_blocks=g_choice["scan_blocks"])
    grp.scan(pairs)                       # the tuning scans were of this same open slice
    o.scan(stream.slice(0))
    rc = o.estimate()
    for gm in gms:
        compare_reports(gm.estimate(), rc, mon["theta"], "tuned group")
    grp.close()
    for gm in gms:
        gm.close()


# ------------------------------------------------------------ discrete window
# k = 1 with one bit per DR (SRLA_CFG_DISCRETE): reports must equal the
# oracle's k = 1 reports bit for bit; dumps agree up to distance 1.

@pytest.mark.parametrize("case", SMALL)
@pytest.mark.parametrize("graph", [False, True])
def test_discrete_form_small_geometries(case, graph):
    _, theta, u, v_re, g, v_le, G, n, n_src, slices = case
    mon = dict(k=1, theta=theta, u=u, v_re=v_re, g=g, v_le=v_le, G=G, hash_seed=3000 + u)
    _run(_rand_stream(u + 11, n, n_src, 3 * theta // 2), mon, range(slices), graph=graph,
         discrete=True)


def test_discrete_form_tiny_workload_host_input_and_streaming():
    stream, mon, n = workload("tiny_coupled")
    mon = dict(mon, k=1)
    _run(stream, mon, range(6), discrete=True, host=True, split=30001)
    _run_streaming(stream, mon, range(6), graph=True, chunks=3, discrete=True)


def test_discrete_form_backbone_full_size():
    stream, mon, _ = workload("backbone")
    mon = dict(mon, k=1)
    r = _run(stream, mon, range(3), max_candidates=1 << 22, dump_every=0, discrete=True)
    assert r.n > 0


def test_discrete_form_rejects_longer_windows_and_groups():
    stream, mon, _ = workload("tiny")
    with pytest.raises(srla.SrlaError):
        srla.Monitor(**mon, discrete=True)                    # k = 8
    m = srla.Monitor(**dict(mon, k=1), discrete=True)
    with pytest.raises(srla.SrlaError):
        srla.Group([m])
    m.close()


def test_lean_report_carries_ip_est_flags_of_the_full_report():
    stream, mon, n = workload("tiny_coupled")
    lean = srla.Monitor(**mon, max_candidates=1 << 16, lean_report=True, graph=True)
    o = oracle.Monitor(**mon)
    for s in range(n):
        p = stream.slice(s)
        lean.scan(to_device(p))
        o.scan(p)
        rl, rc = lean.estimate(), o.estimate()
        assert rl.union_weight is None and rl.re_weight is None
        rl.union_weight, rl.re_weight = rc.union_weight, rc.re_weight
        compare_reports(rl, rc, mon["theta"], "slice %d" % s)
    lean.close()


# ------------------------------------------------------------ read-before-write scan
# SRLA_CFG_SCAN_DEDUP skips stores of stamps a DR already holds; every
# result must stay bit-identical to the oracle.

@pytest.mark.parametrize("case", SMALL)
def test_dedup_scan_small_geometries(case):
    k, theta, u, v_re, g, v_le, G, n, n_src, slices = case
    mon = dict(k=k, theta=theta, u=u, v_re=v_re, g=g, v_le=v_le, G=G, hash_seed=5000 + k + u)
    _run(_rand_stream(k + u + 3, n, n_src, 3 * theta // 2), mon, range(slices), scan_dedup=True)


def test_dedup_scan_tiny_host_input_and_streaming():
    stream, mon, n = workload("tiny")
    _run(stream, mon, range(n), scan_dedup=True, host=True, split=40001)
    _run_streaming(stream, mon, range(n), graph=True, chunks=3, scan_dedup=True)


def test_dedup_scan_backbone_expiry_and_full_size_prefix():
    stream, mon, _ = workload("backbone_k16")
    _run(scaled(stream, 600_000), mon, range(40), max_candidates=1 << 22, dump_every=13,
         scan_dedup=True)
    stream, mon, _ = workload("backbone")
    _run(stream, mon, range(3), max_candidates=1 << 22, dump_every=0, scan_dedup=True)


# SRLA_CFG_SCAN_DEDUP with SRLA_CFG_SCAN_XCD: each XCD reads and stamps only its
# own rows (u in {1, 2, 4, 8, 16}; other u and unaligned input fall back).

@pytest.mark.parametrize("case", SMALL)
def test_xcd_dedup_scan_small_geometries(case):
    k, theta, u, v_re, g, v_le, G, n, n_src, slices = case
    mon = dict(k=k, theta=theta, u=u, v_re=v_re, g=g, v_le=v_le, G=G, hash_seed=5100 + k + u)
    _run(_rand_stream(k + u + 4, n, n_src, 3 * theta // 2), mon, range(slices), scan_dedup=True,
         scan_xcd=True)


def test_xcd_dedup_scan_tiny_host_input_and_streaming():
    stream, mon, n = workload("tiny")
    _run(stream, mon, range(n), scan_dedup=True, scan_xcd=True, host=True, split=40001)
    _run(stream, mon, range(n), scan_dedup=True, scan_xcd=True, split=33333)
    g = srla.Monitor(**mon, max_candidates=1 << 16, graph=True, scan_dedup=True, scan_xcd=True)
    o = oracle.Monitor(**mon)
    for s in range(n):
        p = stream.slice(s)
        for lo in range(0, len(p), 50000):
            g.scan(to_device(p[lo:lo + 50000]))
        o.scan(p)
        compare_reports(g.estimate(), o.estimate(), mon["theta"], "slice %d" % s)
    compare_dumps(g, o)
    g.close()


def test_xcd_dedup_scan_backbone_expiry_and_full_size_prefix():
    stream, mon, _ = workload("backbone_k16")
    _run(scaled(stream, 600_000), mon, range(40), max_candidates=1 << 22, dump_every=13,
         scan_dedup=True, scan_xcd=True)
    stream, mon, _ = workload("backbone")
    _run(stream, mon, range(3), max_candidates=1 << 22, dump_every=0, scan_dedup=True,
         scan_xcd=True)


# ------------------------------------------------------------ workgroup store filter
# SRLA_CFG_SCAN_LDS_FILTER skips LE stores a workgroup already issued.

@pytest.mark.parametrize("case", SMALL)
def test_lds_filter_scan_small_geometries(case):
    k, theta, u, v_re, g, v_le, G, n, n_src, slices = case
    mon = dict(k=k, theta=theta, u=u, v_re=v_re, g=g, v_le=v_le, G=G, hash_seed=6000 + k + u)
    _run(_rand_stream(k + u + 5, n, n_src, 3 * theta // 2), mon, range(slices),
         scan_lds_filter=True)


def test_lds_filter_scan_repeats_and_full_size():
    """A stream of few flows (every workgroup repeats DRs) and the backbone
    workload at full size."""
    stream, mon, n = workload("tiny_coupled")

    def few_flows(s):
        rng = np.random.default_rng(s)
        src = rng.integers(0, 40, 60_000, dtype=np.uint64).astype(np.uint32) * np.uint32(977)
        dst = rng.integers(0, 8, 60_000, dtype=np.uint64).astype(np.uint32) * np.uint32(131)
        return np.stack([src, dst], 1)
    _run(few_flows, dict(mon, theta=4), range(6), scan_lds_filter=True)
    stream, mon, _ = workload("backbone")
    _run(stream, mon, range(3), max_candidates=1 << 22, dump_every=0, scan_lds_filter=True)


# ------------------------------------------------------------ overlapped report copy
# SRLA_CFG_OVERLAP_REPORT: candidate work before the next slice's scans, the
# report's PCIe copy alongside them; results identical in both call patterns.

@pytest.mark.parametrize("graph", [False, True])
def test_overlap_report_streaming_and_plain(graph):
    stream, mon, n = workload("tiny")
    _run_streaming(stream, mon, range(n), graph=graph, chunks=2, overlap_report=True)
    _run_streaming(stream, mon, range(n), graph=graph, chunks=2, overlap_report=True,
                   ahead=True)
    stream, mon, n = workload("tiny_coupled")
    g = srla.Monitor(**mon, max_candidates=1 << 16, graph=graph, overlap_report=True)
    o = oracle.Monitor(**mon)
    for s in range(n):
        p = stream.slice(s)
        g.scan(to_device(p))
        o.scan(p)
        compare_reports(g.estimate(), o.estimate(), mon["theta"], "slice %d" % s)
    compare_dumps(g, o)
    g.close()


@pytest.mark.parametrize("case", [SMALL[0], SMALL[5], SMALL[7]])
def test_overlap_report_small_geometries_and_discrete(case):
    k, theta, u, v_re, g, v_le, G, n, n_src, slices = case
    mon = dict(k=k, theta=theta, u=u, v_re=v_re, g=g, v_le=v_le, G=G, hash_seed=8000 + k + u)
    _run_streaming(_rand_stream(k + u + 13, n, n_src, 3 * theta // 2), mon, range(slices),
                   graph=True, overlap_report=True, ahead=True)
    _run_streaming(_rand_stream(k + u + 14, n, n_src, 3 * theta // 2), dict(mon, k=1),
                   range(slices), graph=True, discrete=True, overlap_report=True, ahead=True)


def test_overlap_report_backbone_full_size_streaming():
    stream, mon, _ = workload("backbone")
    _run_streaming(stream, mon, range(3), max_candidates=1 << 22, graph=True,
                   overlap_report=True, ahead=True)


def test_group_rejects_overlapped_report_monitors():
    stream, mon, _ = workload("tiny")
    st = torch.cuda.Stream()
    a = srla.Monitor(**mon, max_candidates=1 << 10, stream=st)
    b = srla.Monitor(**mon, max_candidates=1 << 10, stream=st, overlap_report=True)
    with pytest.raises(srla.SrlaError):
        srla.Group([a, b])
    a.close()
    b.close()


# ------------------------------------------------------------ partitioned scan
# SRLA_CFG_SCAN_PARTITION sorts each chunk's LE DR indices by region and
# stamps every region from one workgroup: same DR arrays, same reports.

@pytest.mark.parametrize("case", SMALL)
def test_partition_scan_small_geometries(case):
    k, theta, u, v_re, g, v_le, G, n, n_src, slices = case
    mon = dict(k=k, theta=theta, u=u, v_re=v_re, g=g, v_le=v_le, G=G, hash_seed=7000 + k + u)
    _run(_rand_stream(k + u + 31, n, n_src, 3 * theta // 2), mon, range(slices),
         scan_partition=True)


def test_partition_scan_tiny_host_input_split_and_streaming():
    stream, mon, n = workload("tiny")
    _run(stream, mon, range(n), scan_partition=True, host=True, split=40001)
    _run(stream, mon, range(n), scan_partition=True, split=777)
    _run_streaming(stream, mon, range(n), graph=True, chunks=3, scan_partition=True,
                   overlap_report=True, ahead=True)


def test_partition_scan_several_rounds_in_one_scan():
    """u = 16: a chunk holds 2,048 pairs, so 5M pairs in one scan take three
    partition rounds of at most 2,048 chunks."""
    mon = dict(k=4, theta=1024, u=16, v_re=4096, g=8, v_le=64, G=1024, hash_seed=77)
    _run(_rand_stream(99, 5_000_000, 200_000, 1536), mon, range(3), max_candidates=1 << 20,
         scan_partition=True)


def test_partition_scan_backbone_full_size_and_expiry():
    stream, mon, _ = workload("backbone")
    _run(stream, mon, range(3), max_candidates=1 << 22, dump_every=0, scan_partition=True)
    _run_streaming(stream, mon, range(3), max_candidates=1 << 22, graph=True,
                   overlap_report=True, ahead=True, scan_partition=True)
    stream, mon, _ = workload("backbone_k16")
    stream = scaled(stream, 600_000)
    _run(stream, mon, range(20), max_candidates=1 << 22, dump_every=7, scan_partition=True)


@pytest.mark.parametrize("unit", [8192, 131072])
def test_partition_scan_marking_unit(unit):
    """The marking unit (scan_blocks of a partitioned-scan monitor) changes
    the launch shape only: a heavy source's region gets many units at 8192,
    a whole round's indices fit one unit at 131072."""
    mon = dict(k=3, theta=1024, u=8, v_re=4096, g=8, v_le=1024, G=1024, hash_seed=77)
    g = srla.Monitor(**mon, max_candidates=1 << 20, scan_partition=True, scan_blocks=unit)
    o = oracle.Monitor(**mon)
    gen = _rand_stream(99, 400_000, 20_000, 4096)
    for s in range(4):
        p = gen(s)
        print("slice", s, "unit", unit, flush=True)
        g.scan(to_device(p))
        o.scan(p)
        compare_reports(g.estimate(), o.estimate(), mon["theta"], ctx="slice %d" % s)
    compare_dumps(g, o, ctx="end")
    g.close()


@pytest.mark.parametrize("u,v_le,G", [
    (8, 4096, 1024),           # 2^25 LE DRs: 512 regions in one band
    (2, 65536, 1024),          # 2^27: one full band of 2048 regions
    (4, 65536, 1024),          # the paper's SEA, 2^28: two bands of two rows
    (3, (1 << 17) + 1, 512),   # 3 * (2^26 + 512): a row straddles the bands,
                               # the second band has a ragged last region
])
def test_partition_scan_in_bands(u, v_le, G):
    """LEs of one band and of several (2^27 DRs each): the rows reaching into
    a band are hashed for it, the first band's pass does the SRE stores."""
    mon = dict(k=3, theta=1024, u=u, v_re=4096, g=8, v_le=v_le, G=G, hash_seed=4242 + u)
    _run(_rand_stream(4242, 300_000, 50_000, 1536), mon, range(4), max_candidates=1 << 20,
         dump_every=2, scan_partition=True)


@pytest.mark.parametrize("all_partitioned", [True, False])
def test_partition_monitors_in_a_group_mix_group_and_own_scans(all_partitioned):
    """Monitors with the partitioned scan in a group: the group scan (each
    member's partitioned scan when every member has it, else the fused flat
    kernel) and each member's own scans stamp the same arrays within one
    slice."""
    st = torch.cuda.Stream()
    mons = [dict(k=k, theta=t, u=u, v_re=vr, g=g, v_le=vl, G=G, hash_seed=300 + i)
            for i, (k, t, u, vr, g, vl, G) in enumerate(GROUP)]
    gms = [srla.Monitor(**m, max_candidates=1 << 16, stream=st,
                        scan_partition=all_partitioned or i > 0)
           for i, m in enumerate(mons)]
    oms = [oracle.Monitor(**m) for m in mons]
    grp = srla.Group(gms)
    gen = _rand_stream(8, 30_000, 2500, 400)
    for s in range(6):
        p = gen(s)
        half = len(p) // 2
        grp.scan(to_device(p[:half]))
        for gm in gms:
            gm.scan(to_device(p[half:]))
        for gm, o, m in zip(gms, oms, mons):
            o.scan(p)
            compare_reports(gm.estimate(), o.estimate(), m["theta"], "slice %d" % s)
    for gm, o in zip(gms, oms):
        compare_dumps(gm, o, ctx="end")
    grp.close()
    for gm in gms:
        gm.close()


# ------------------------------------------------------------ the sort
# The sampled sources are sorted by their top 8 bits into 256 buckets, then
# each bucket in LDS (up to 12288 keys; when one key fills at least a quarter
# of the bucket, only the other keys are sorted) or in global memory (more).
# With tau = 0 every pair is sampled: one source sending 20000 pairs fills
# one bucket past the LDS capacity, 8000 pairs leave it in LDS beside 3000
# other keys of the same bucket, below and above it; empty slices, a single
# pair and sources spread over every bucket cover the rest.

def _sort_stream(seed):
    def gen(s):
        rng = np.random.default_rng(seed * 1000 + s)
        if s == 1:
            return np.zeros((0, 2), np.uint32)
        if s == 2:
            return np.array([[0xFFFFFFFF, 5]], np.uint32)
        n_heavy = 20000 if s % 2 == 0 else 8000
        heavy = np.stack([np.full(n_heavy, 0x80800001 + s, np.uint32),
                          rng.integers(0, 2 ** 32, size=n_heavy, dtype=np.uint64).astype(np.uint32)], 1)
        same = np.stack([np.uint32(0x80000000) | rng.integers(0, 2 ** 24, size=3000).astype(np.uint32),
                         rng.integers(0, 2 ** 32, size=3000, dtype=np.uint64).astype(np.uint32)], 1)
        heavy = np.concatenate([heavy, same])
        spread = rng.integers(0, 2 ** 32, size=(15000, 2), dtype=np.uint64).astype(np.uint32)
        # duplicates of a few sources in other buckets
        dup = np.stack([rng.integers(0, 16, size=5000).astype(np.uint32) << np.uint32(28),
                        rng.integers(0, 2 ** 32, size=5000, dtype=np.uint64).astype(np.uint32)], 1)
        p = np.concatenate([heavy, spread, dup])
        return p[rng.permutation(len(p))]
    return gen


@pytest.mark.parametrize("hold", [False, True])
def test_sort_heavy_bucket_and_edges(hold):
    mon = dict(k=3, theta=4, u=4, v_re=128, g=8, v_le=32, G=64, hash_seed=8801)
    _run_streaming(_sort_stream(31), mon, range(6), graph=True, ahead=True, hold_scans=hold,
                   scan_partition=True)
    g = srla.Monitor(**mon, max_candidates=1 << 16)
    o = oracle.Monitor(**mon)
    gen = _sort_stream(32)
    for s in range(6):
        p = gen(s)
        if len(p):
            g.scan(to_device(p))
        o.scan(p)
        compare_reports(g.estimate(), o.estimate(), mon["theta"], "plain %d" % s)
    g.close()


# ------------------------------------------------------------ held scans
# SRLA_CFG_HOLD_SCANS: the next slice's scans wait until the closed slice's
# report is published; results are unchanged.

@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("ahead", [False, True])
def test_hold_scans_streaming_matches_oracle(graph, ahead):
    stream, mon, n = workload("tiny")
    _run_streaming(stream, mon, range(n), graph=graph, chunks=2, ahead=ahead, hold_scans=True)
    _run_streaming(stream, mon, range(n), graph=graph, ahead=ahead, hold_scans=True,
                   scan_partition=True)


@pytest.mark.parametrize("case", [SMALL[0], SMALL[3], SMALL[6]])
def test_hold_scans_small_geometries_and_discrete(case):
    k, theta, u, v_re, g, v_le, G, n, n_src, slices = case
    mon = dict(k=k, theta=theta, u=u, v_re=v_re, g=g, v_le=v_le, G=G, hash_seed=5100 + k + u)
    _run_streaming(_rand_stream(k + u + 71, n, n_src, 3 * theta // 2), mon, range(slices),
                   graph=True, ahead=True, hold_scans=True)
    _run_streaming(_rand_stream(k + u + 72, n, n_src, 3 * theta // 2), dict(mon, k=1),
                   range(slices), graph=True, discrete=True, ahead=True, hold_scans=True)


def test_hold_scans_plain_and_backbone_full_size():
    stream, mon, n = workload("tiny")
    g = srla.Monitor(**mon, max_candidates=1 << 16, hold_scans=True, graph=True)
    o = oracle.Monitor(**mon)
    for s in range(n):
        p = stream.slice(s)
        g.scan(to_device(p))
        o.scan(p)
        compare_reports(g.estimate(), o.estimate(), mon["theta"], "plain %d" % s)
    compare_dumps(g, o)
    g.close()
    stream, mon, _ = workload("backbone")
    _run_streaming(stream, mon, range(3), max_candidates=1 << 22, graph=True, ahead=True,
                   scan_partition=True, hold_scans=True)
