"""Throughput and slice-end latency of the SRLA hot path on one MI355X.

One step = one time slice of the backbone-shaped workload: 8M (aip, bip)
pairs scanned into the SEA (Algorithm 2), then the slice closed (candidate
check, Eq8-Eq9 estimate of every candidate, Algorithm 3 slide) and its report
delivered to host memory.  Window k = 300 slices, SRE 8 x 2^20 DR cells, SLE
2^24 DR cells, theta = 1024.  Slices 0 .. k-2 fill the window first, then
the warm-up slices run, so every warm-up and timed slice closes a full
window; the timed slices' pairs are generated into device memory before each
timed segment starts.

--mode streaming (default): the host closes slice t and issues slice t+1's
  scans before it collects the report of slice t.  With the partitioned scan
  (the autotuner's pick on the backbone workloads) slice t+1's scans wait on
  the device until slice t's report is in host memory (--hold-scans): slice
  t's sort, DR snapshot, candidate check and estimate follow its scans on the
  scan stream, and only Algorithm 3's slide of slice t (with the copy of the
  carried list into the next report) runs beside slice t+1's scans, on a
  second HIP stream.  With another scan form the candidate work runs first
  (into device memory) and only the report's copy runs beside the next scan
  (--overlap-report), its pipeline replayed as HIP graphs.  The same number
  of slices then runs in the plain form on the same monitor (`plain` in the
  output).
--mode plain: each slice is scanned, then estimated.

In both forms the latency is the device time from the start of a slice's
end-of-slice work, right after its last scan, to its report complete in host
memory.  Prints one JSON line (rank 0).  `value` is pairs (packets) scanned
per second over the timed slices; `p99_ms` is the 99th percentile of the
latency.
"""
import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "packets/s scanned + p99 slice-end estimate latency (ms), 1 MI355X"
HBM_PEAK_GBS = 8000.0


def scan_bytes_per_pair(u, tau):
    """Algorithmic bytes of Algorithm 2 per pair: the 8-byte pair, u 2-byte LE
    DR stores, and with probability 2^-tau u 2-byte SRE DR stores plus a
    4-byte sampled-source append."""
    return 8.0 + 2.0 * u + (2.0 * u + 4.0) * 2.0 ** (-tau)


def measured_traffic(kernel, workload):
    """HBM bytes per launch from the committed rocprofv3 counter runs, if they
    were taken on exactly the current scan source (else None)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    h = hashlib.sha256()
    for p in rec["sources"]:
        with open(os.path.join(ROOT, p), "rb") as f:
            h.update(f.read())
    return rec["bytes_per_launch"] if h.hexdigest() == rec["source_sha256"] else None


def calibration_copy(mib):
    """One plain device-to-device copy of `mib` MiB: a kernel of known traffic
    that scales the HBM counters of the profiled runs."""
    import torch
    src = torch.empty(mib << 20, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def oracle_baseline(stream, mon, slices):
    """Times the oracle (single-threaded C) on the first `slices` slices; each
    slice's pairs are generated outside the timed calls."""
    import oracle
    o = oracle.Monitor(**mon)
    dt, n, r = 0.0, 0, None
    for s in range(slices):
        p = stream.slice(s)
        t0 = time.perf_counter()
        o.scan(p)
        r = o.estimate()
        dt += time.perf_counter() - t0
        n += len(p)
    o.close()
    return n / dt, dt, n, (int(r.n) if r is not None else 0)


def run_batched(args):
    """The batched workload: 16 monitors of different windows, SLE sizes and
    thresholds over one 8M pairs/slice stream.  --mode plain: each monitor
    scans and estimates on its own (one monitor after another); --mode
    batched: one fused scan for all, then every member's slice closed at once
    and the reports collected; --mode streaming: batched, with the next
    slice's fused scan issued before the reports are collected."""
    import numpy as np
    import torch

    import paper_1803_10369_amd as srla
    from trafficgen.configs import batched_monitors, workload
    from trafficgen.device import DeviceStream

    torch.cuda.set_device(0)
    stream, _, _ = workload("backbone")
    n_pairs = stream.n_pairs
    mons_cfg = batched_monitors(16)
    ds = DeviceStream(stream)
    st = torch.cuda.Stream()
    torch.cuda.set_stream(st)
    fused = args.mode in ("batched", "streaming")
    # --hold-scans 1: the next slice's group scan waits on the device until
    # every member's report is published (off by default here: the sixteen
    # members' end-of-slice work is long next to the group scan, and the scan
    # beside it lost 26 % of the packets/s for no better p99)
    hold = False if args.hold_scans < 0 else bool(args.hold_scans)
    mons = [srla.Monitor(**c, max_candidates=args.max_candidates, stream=st, graph=fused,
                         scan_blocks=args.scan_blocks, lean_report=not args.full_report,
                         scan_partition=args.scan_partition, hold_scans=hold)
            for c in mons_cfg]
    grp = srla.Group(mons, scan_blocks=args.scan_blocks) if fused else None

    def scan_all(buf):
        if fused:
            grp.scan(buf)
        else:
            for m in mons:
                m.scan(buf)

    buf = torch.empty(2 * n_pairs, dtype=torch.int32, device="cuda")
    tuned = None
    t_w = time.perf_counter()
    for s in range(args.warmup):
        ds.generate(s, out=buf, stream=st)
        if s == 0 and fused and args.autotune:
            from paper_1803_10369_amd import autotune
            tuned = autotune.tune_group(mons, buf)
            grp.close()
            grp = srla.Group(mons, scan_blocks=tuned["scan_blocks"])
        scan_all(buf)
        for m in mons:
            m.estimate(copy=False)
        if s % 50 == 0:
            print("warmup slice %d (%.1fs)" % (s, time.perf_counter() - t_w), file=sys.stderr,
                  flush=True)
    lat, total_s, done, seg_bufs = [], 0.0, 0, []
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    scan_ms = []
    while done < args.steps:
        seg = min(args.segment, args.steps - done)
        while len(seg_bufs) < seg:
            seg_bufs.append(torch.empty(2 * n_pairs, dtype=torch.int32, device="cuda"))
        for i in range(seg):
            ds.generate(args.warmup + done + i, out=seg_bufs[i], stream=st)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if args.mode == "streaming":
            scan_all(seg_bufs[0])
            for m in mons:
                m.close_slice()
            t_close = time.perf_counter()
            for i in range(1, seg + 1):
                if i < seg:
                    scan_all(seg_bufs[i])
                for m in mons:
                    m.wait_report(copy=False)
                lat.append((time.perf_counter() - t_close) * 1e3)
                if i < seg:
                    for m in mons:
                        m.close_slice()
                    t_close = time.perf_counter()
        else:
            for i in range(seg):
                ev0.record(st)
                scan_all(seg_bufs[i])
                ev1.record(st)
                st.synchronize()
                scan_ms.append(ev0.elapsed_time(ev1))
                ts = time.perf_counter()
                if fused:
                    for m in mons:
                        m.close_slice()
                    for m in mons:
                        m.wait_report(copy=False)
                else:
                    for m in mons:
                        m.estimate(copy=False)
                lat.append((time.perf_counter() - ts) * 1e3)
        torch.cuda.synchronize()
        total_s += time.perf_counter() - t0
        done += seg
        print("timed %d/%d slices (%.2fs)" % (done, args.steps, total_s), file=sys.stderr,
              flush=True)
    lat = np.array(lat)
    value = args.steps * n_pairs / total_s
    stores = sum(c["u"] for c in mons_cfg)
    out = {
        "metric": METRIC, "value": value, "unit": "packets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total_s * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": ("batched16, %s form: 16 monitors over one %d pairs/slice stream "
                                "(Zipf(%g) over %d hosts), windows {10,60,300,1800}, SLE 2^20..2^25 "
                                "DR cells, thresholds 256..16384" % (args.mode, n_pairs,
                                                                    stream.alpha, stream.n_ranks)),
                   "mode": args.mode, "monitors": len(mons), "pairs_per_slice": n_pairs,
                   "scan_blocks": args.scan_blocks, "scan_partition": args.scan_partition,
                   "hold_scans": hold, "autotune": tuned},
        "monitor_pairs_per_s": value * len(mons),
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
    }
    if scan_ms:
        ms = float(np.mean(scan_ms))
        out["scan_ms_per_slice"] = ms
        out["random_stores_per_s"] = stores * n_pairs / (ms * 1e-3)
    print(json.dumps(out), flush=True)
    if grp:
        grp.close()
    for m in mons:
        m.close()


def bits_bytes_per_pair(u, tau):
    """Algorithmic bytes of the discrete-window scan per pair: the 8-byte pair,
    u 32-bit atomic ORs into the LE bit array, and with probability 2^-tau u
    atomic ORs into the SRE bit array plus a 4-byte sampled-source append."""
    return 8.0 + 4.0 * u + (4.0 * u + 4.0) * 2.0 ** (-tau)


def run_discrete(args):
    """The paper's discrete-window run: k = 1 with one-bit DRs, the paper's SEA
    (u = 4, v = 65,536, g' = 1024), one slice = one 300-second window of a
    4.5 Mpps link = 169 chunks of 8M pairs (1.352 G pairs).  Each timed
    slice's pairs are generated into HBM (10.8 GB) before its timed region;
    the region covers its 169 scans and its end-of-slice report."""
    import numpy as np
    import torch

    import paper_1803_10369_amd as srla
    import probe
    from trafficgen.configs import DISCRETE_CHUNKS, workload
    from trafficgen.device import DeviceStream

    torch.cuda.set_device(0)
    stream, mon, _ = workload(args.workload)
    C, n = DISCRETE_CHUNKS, stream.n_pairs
    ds = DeviceStream(stream)
    st = torch.cuda.Stream()
    torch.cuda.set_stream(st)
    if args.calib_copy_mb:
        calibration_copy(args.calib_copy_mb)
    m = srla.Monitor(**mon, max_candidates=args.max_candidates, timing=True, stream=st,
                     discrete=True, graph=args.graph > 0, scan_blocks=args.scan_blocks,
                     lean_report=not args.full_report)
    buf = torch.empty((C, 2 * n), dtype=torch.int32, device="cuda")

    def fill(s):
        for c in range(C):
            ds.generate(s * C + c, out=buf[c], stream=st)
        torch.cuda.synchronize()

    for s in range(args.warmup):
        fill(s)
        for c in range(C):
            m.scan(buf[c])
        m.estimate(copy=False)
        print("warmup slice %d" % s, file=sys.stderr, flush=True)
    m.timings(reset=True)
    lat, total_s = [], 0.0
    for i in range(args.steps):
        fill(args.warmup + i)
        t0 = time.perf_counter()
        for c in range(C):
            m.scan(buf[c])
        st.synchronize()
        ts = time.perf_counter()
        r = m.estimate(copy=False)
        t1 = time.perf_counter()
        lat.append((t1 - ts) * 1e3)
        total_s += t1 - t0
        print("timed slice %d: %.1f ms, %d candidates" % (i, (t1 - t0) * 1e3, r.n),
              file=sys.stderr, flush=True)
    tm = m.timings(reset=True)
    tau = 0
    while mon["g"] * (1 << tau) < mon["theta"]:
        tau += 1
    pairs = args.steps * C * n
    scan_ms = tm["scan_ms"] / max(1, tm["scan_launches"])
    bpp = bits_bytes_per_pair(mon["u"], tau)
    achieved = bpp * n / (scan_ms * 1e-3) / 1e9
    ors = mon["u"] * (1 + 2.0 ** -tau) * n / (scan_ms * 1e-3)
    footprint = (mon["u"] * (mon["v_le"] * mon["G"] + mon["v_re"] * mon["g"])) // 8
    ceiling = probe.random_or_rate(footprint)
    load_ceiling = probe.random_load_rate(footprint)
    lat = np.array(lat)
    out = {
        "metric": METRIC, "value": pairs / total_s, "unit": "packets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total_s * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u1",
        "data": "synthetic",
        "config": {
            "workload": ("%s: discrete window (k = 1, one-bit DRs), %d chunks of %d pairs per "
                         "slice, Zipf(%g) sources over %d hosts with 4 destinations each, %d "
                         "planted super points, u %d, v %d, g %d, g' %d, theta %d"
                         % (args.workload, C, n, stream.alpha, stream.n_ranks,
                            len(stream.planted), mon["u"], mon["v_le"], mon["g"], mon["G"],
                            mon["theta"])),
            "pairs_per_slice": C * n, "scan_blocks": args.scan_blocks},
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
        "stage_ms_per_slice": {k: tm[k] / args.steps for k in
                               ("scan_ms", "sweep_ms", "finalize_ms", "estimate_ms", "slide_ms")},
        "state": {"candidates": int(r.n), "up": r.up,
                  "row_fill_frac": [float(x) / (mon["v_le"] * mon["G"]) for x in r.row_fill],
                  "n_touched": int(r.n_touched), "n_new": int(r.n_new),
                  "super": int(((r.flags & 1) != 0).sum())},
        "roofline": {
            "kernel": "k_scan_bits (Algorithm 2, one-bit DRs)", "bound": "hbm",
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic("k_scan_bits", args.workload), "bytes_per_pair": bpp,
            "launch_ms": scan_ms, "dr_updates_per_s": ors,
            "random_or_ceiling_per_s": ceiling, "random_load_ceiling_per_s": load_ceiling,
            "frac_of_random_load_ceiling": ors / load_ceiling, "footprint_bytes": footprint},
    }
    if not args.no_cpu_baseline:
        import oracle
        o = oracle.Monitor(**mon)
        ps = [stream.slice(c) for c in range(args.cpu_slices)]
        t0 = time.perf_counter()
        for p in ps:
            o.scan(p)
        o.estimate()
        dt = time.perf_counter() - t0
        cnt = sum(len(p) for p in ps)
        o.close()
        out["cpu_baseline"] = {
            "value": cnt / dt, "unit": "packets/s", "cores": 1, "kind": "oracle",
            "sample": ("the first %d chunks (%d pairs) of the same workload as one k = 1 slice, "
                       "scan + end-of-slice estimate, single-threaded C oracle (16-bit DRs), "
                       "%.1f s on %s (nproc %d)" % (args.cpu_slices, cnt, dt, cpu_model(),
                                                     os.cpu_count()))}
    print(json.dumps(out), flush=True)
    m.close()


def run_serving(args):
    """The serving mix: 64 monitors of uneven sizes (LE 2^24..2^33 DR cells)
    admitted first-fit under a device-memory budget, over a bursting stream
    (2M-32M pairs per slice, per-slice Zipf exponent 0.90-1.30, 1,000
    planted super points).  --mode batched: one fused scan per slice, every
    member closed at once; --mode plain: each admitted monitor scans and
    estimates on its own, one after another."""
    import numpy as np
    import torch

    import paper_1803_10369_amd as srla
    from trafficgen.configs import ServingStream, serving_monitors
    from trafficgen.device import DeviceStream

    torch.cuda.set_device(0)
    ss = ServingStream()
    cfg_all = serving_monitors(64)
    cfgs = [srla.make_config(**c, max_candidates=args.max_candidates) for c in cfg_all]
    budget = int(args.budget_gb * 1e9)
    rc, admitted, used = srla.srla_admit(cfgs, budget)
    assert rc == 0
    chosen = [c for c, a in zip(cfg_all, admitted) if a]
    st = torch.cuda.Stream()
    torch.cuda.set_stream(st)
    fused = args.mode != "plain"
    mons = [srla.Monitor(**c, max_candidates=args.max_candidates, stream=st, graph=True,
                         lean_report=not args.full_report)
            for c in chosen]
    grp = srla.Group(mons) if fused else None
    dstreams = {a: DeviceStream(sp) for a, sp in ss.specs.items()}
    print("admitted %d of %d monitors, %.1f GB of %.1f GB" % (len(mons), len(cfg_all), used / 1e9,
                                                           budget / 1e9), file=sys.stderr,
          flush=True)

    def gen(s, out):
        n, a = ss.params(s)
        ss.spec(s)
        dstreams[a].generate(s, out=out, stream=st)
        return out[:2 * n]

    def one_slice(pairs):
        if fused:
            grp.scan(pairs)
            st.synchronize()
            ts = time.perf_counter()
            for m in mons:
                m.close_slice()
            for m in mons:
                m.wait_report(copy=False)
        else:
            for m in mons:
                m.scan(pairs)
            st.synchronize()
            ts = time.perf_counter()
            for m in mons:
                m.estimate(copy=False)
        return (time.perf_counter() - ts) * 1e3

    buf = torch.empty(2 * ss.hi, dtype=torch.int32, device="cuda")
    for s in range(args.warmup):
        one_slice(gen(s, buf))
        print("warmup slice %d" % s, file=sys.stderr, flush=True)
    bufs = [torch.empty(2 * ss.hi, dtype=torch.int32, device="cuda") for _ in range(args.steps)]
    views = [gen(args.warmup + i, bufs[i]) for i in range(args.steps)]
    torch.cuda.synchronize()
    lat, pairs = [], 0
    t0 = time.perf_counter()
    for i, v in enumerate(views):
        lat.append(one_slice(v))
        pairs += v.numel() // 2
        print("timed slice %d (%d pairs)" % (i, v.numel() // 2), file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total_s = time.perf_counter() - t0
    lat = np.array(lat)
    out = {
        "metric": METRIC, "value": pairs / total_s, "unit": "packets/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": total_s * 1e3 / args.steps,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u16",
        "data": "synthetic",
        "config": {"workload": ("serving64, %s form: %d of 64 monitors admitted under %.0f GB "
                                "(LE 2^24..2^33 DR cells, u 4/8, windows 10..1800, thresholds "
                                "256..16384); 2M-32M pairs/slice, Zipf 0.90-1.30, 1,000 planted"
                                % (args.mode, len(mons), budget / 1e9)),
                   "mode": args.mode, "admitted": len(mons),
                   "rejected": [i for i, a in enumerate(admitted) if not a],
                   "footprint_gb": used / 1e9},
        "monitor_pairs_per_s": pairs * len(mons) / total_s,
        "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
    }
    print(json.dumps(out), flush=True)
    if grp:
        grp.close()
    for m in mons:
        m.close()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--mode", choices=("plain", "streaming", "batched"), default="streaming")
    ap.add_argument("--graph", type=int, default=-1,
                    help="replay the end-of-slice pipeline as HIP graphs (default: the streaming "
                         "form without held scans only)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="pick the scan kernel's form and workgroup cap by timing them first")
    ap.add_argument("--scan-blocks", type=int, default=0,
                    help="cap on the scan kernel's workgroups (0: one per tile)")
    ap.add_argument("--block", type=int, default=20,
                    help="slices per turn when the streaming and the plain form take turns")
    ap.add_argument("--segment", type=int, default=200,
                    help="timed slices whose inputs are generated into HBM at a time")
    ap.add_argument("--steps", type=int, default=60)
    ap.add_argument("--stage-steps", type=int, default=20,
                    help="untimed slices after the timed ones with every stage timed (the "
                         "timed slices time their scans only: each timed stage costs event "
                         "records on the critical path)")
    ap.add_argument("--warmup", type=int, default=5,
                    help="untimed slices in the measured form before the timed ones (after "
                         "the k - 1 slices that fill the window)")
    ap.add_argument("--no-prefill", action="store_true",
                    help="do not fill the window before the warm-up slices")
    ap.add_argument("--compare-steps", type=int, default=-1,
                    help="slices of the plain form timed after the streaming form, on the "
                         "same monitor (default: --steps)")
    ap.add_argument("--workload", default="backbone")
    ap.add_argument("--cpu-slices", type=int, default=30,
                    help="slices of the same workload the oracle baseline scans "
                         "(about 10 s of CPU work for the backbone workload)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--max-candidates", type=int, default=1 << 25)
    ap.add_argument("--budget-gb", type=float, default=200.0,
                    help="device-memory budget for admitting the serving mix's monitors")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="also run one plain device copy of this many MiB (a known-size "
                         "reference for the HBM traffic counters)")
    ap.add_argument("--probe-mib", default="",
                    help="comma-separated extra footprints (MiB) for the random-store probe")
    ap.add_argument("--host-ingest", action="store_true",
                    help="hand the pairs over in pinned host memory (PCIe-inclusive rate; "
                         "reported as its own metric, never the headline)")
    ap.add_argument("--full-report", action="store_true",
                    help="also deliver |ULE|^k and |URE|^k per candidate (18 instead of 13 "
                         "bytes per candidate to host memory)")
    ap.add_argument("--overlap-report", type=int, default=-1,
                    help="candidate work before the next slice's scans, only the report's "
                         "PCIe copy alongside them (default: streaming form with a scan "
                         "form other than the partitioned one)")
    ap.add_argument("--scan-partition", action="store_true",
                    help="scan in partitioned form: LE stores sorted by region in LDS, "
                         "then stamped a region per workgroup (A/B of the scan kernels)")
    ap.add_argument("--hold-scans", type=int, default=-1,
                    help="the next slice's scans wait until the closed slice's report is in "
                         "host memory (default: on in the streaming form)")
    ap.add_argument("--scan-lds-filter", action="store_true",
                    help="scan with a workgroup filter of repeated DR stores (A/B)")
    ap.add_argument("--scan-dedup", action="store_true",
                    help="scan in read-before-write form (A/B of the scan kernels)")
    ap.add_argument("--scan-xcd", action="store_true",
                    help="scan with per-XCD row ownership (A/B of the scan kernels)")
    args = ap.parse_args()
    if args.compare_steps < 0:
        args.compare_steps = args.steps

    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched16":
        return run_batched(args)
    if args.workload == "serving64":
        return run_serving(args)
    if args.workload == "discrete_paper":
        return run_discrete(args)

    import numpy as np
    import torch

    import paper_1803_10369_amd as srla
    from trafficgen.configs import workload
    from trafficgen.device import DeviceStream

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    stream, mon, _ = workload(args.workload)
    n_pairs = stream.n_pairs
    ds = DeviceStream(stream)
    st = torch.cuda.Stream()
    torch.cuda.set_stream(st)     # generation, scan and estimate share one stream

    if args.calib_copy_mb:
        calibration_copy(args.calib_copy_mb)
    buf = torch.empty(2 * n_pairs, dtype=torch.int32, device="cuda")
    tuned = None
    if args.autotune:
        from paper_1803_10369_amd import autotune
        # five slices (320 MB of pairs for the backbone workload, more than the
        # last-level cache), so every tuning scan reads its pairs from HBM
        tbufs = [torch.empty(2 * n_pairs, dtype=torch.int32, device="cuda") for _ in range(5)]
        for i, tb in enumerate(tbufs):
            ds.generate(i, out=tb, stream=st)
        tuned = autotune.tune_scan(mon, tbufs, repeats=4, cache=None)
        del tbufs
        args.scan_xcd, args.scan_blocks = tuned["scan_xcd"], tuned["scan_blocks"]
        args.scan_dedup = tuned["scan_dedup"]
        args.scan_lds_filter = tuned["scan_lds_filter"]
        args.scan_partition = tuned["scan_partition"]
    # the streaming form overlaps only the report's PCIe copy with the next
    # slice's scans when the scan is the flat one; the partitioned scan leaves
    # the cache to the candidate work, which then runs beside the scans whole
    overlap = ((args.mode == "streaming" and not args.scan_partition)
               if args.overlap_report < 0 else bool(args.overlap_report))
    # the streaming form holds each slice's scans until the previous slice's
    # report is in host memory (its end-of-slice work then runs alone)
    hold = (args.mode == "streaming" and not overlap) if args.hold_scans < 0 \
        else bool(args.hold_scans)
    # HIP graphs for the overlapped-report form's pipeline; with held scans
    # the slice end runs on the scan stream, where kernels launched one by
    # one follow each other with no gap, while each graph launch leaves ~10-20
    # us (16.5 against 16.0-16.1 G packets/s on the backbone workload)
    graph = (args.mode == "streaming" and not hold) if args.graph < 0 else bool(args.graph)
    m = srla.Monitor(**mon, max_candidates=args.max_candidates, timing=True, stream=st,
                     scan_xcd=args.scan_xcd, graph=graph, scan_blocks=args.scan_blocks,
                     lean_report=not args.full_report, scan_dedup=args.scan_dedup,
                     scan_lds_filter=args.scan_lds_filter, overlap_report=overlap,
                     scan_partition=args.scan_partition, hold_scans=hold)

    # the window is filled first: slices 0 .. k-2 build the state, so that
    # every warm-up and timed slice closes a full window (Section 5.2 reports
    # the windows W(0,k), W(1,k), ...); they are neither warm-up nor timed
    prefill = 0 if args.no_prefill else mon["k"] - 1
    t_w = time.perf_counter()
    for s in range(prefill):
        ds.generate(s, out=buf, stream=st)
        m.scan(buf)
        m.estimate(copy=False)
        if s % 100 == 0:
            print("prefill slice %d (%.1fs)" % (s, time.perf_counter() - t_w), file=sys.stderr,
                  flush=True)
    del buf
    seg_bufs = []

    def segment(mode, first, count):
        """Runs slices first .. first+count-1 in `mode`, their pairs generated
        into HBM (or, for --host-ingest, pinned host memory) beforehand.
        Returns the seconds spent, each slice's slice-end latency on the device
        clock (from the start of its end-of-slice work, right after its last
        scan, to its report complete in host memory), the same on the host
        clock in the plain form (from the scan's end to the report), every
        report's candidate count and window flag, and the last report."""
        while len(seg_bufs) < count:
            seg_bufs.append(
                torch.empty(2 * n_pairs, dtype=torch.int32, pin_memory=True) if args.host_ingest
                else torch.empty(2 * n_pairs, dtype=torch.int32, device="cuda"))
        for i in range(count):
            if args.host_ingest:
                tmp = ds.generate(first + i, stream=st)
                seg_bufs[i].copy_(tmp)
            else:
                ds.generate(first + i, out=seg_bufs[i], stream=st)
        torch.cuda.synchronize()
        lat, host_lat, cands, full, news, hbytes = [], [], [], [], [], []
        r = None
        t0 = time.perf_counter()
        if mode == "plain":
            for i in range(count):
                m.scan(seg_bufs[i])
                st.synchronize()             # the slice's last pair is scanned
                ts = time.perf_counter()
                r = m.estimate(copy=False)   # returns with the report in host memory
                host_lat.append((time.perf_counter() - ts) * 1e3)
                lat.append(r.latency_ms)
                cands.append(int(r.n))
                news.append(int(r.n_new))
                hbytes.append(int(r.host_bytes))
                full.append(bool(r.window_full))
        else:
            # the host runs ahead: slice i is closed and slice i+1's scan is
            # enqueued before the report of slice i-1 is collected (two reports
            # may be pending), so the device never waits for the host
            m.scan(seg_bufs[0])
            m.close_slice()
            if count > 1:
                m.scan(seg_bufs[1])
            for i in range(1, count + 1):
                if i < count:
                    m.close_slice()
                    if i + 1 < count:
                        m.scan(seg_bufs[i + 1])   # runs while slice i is estimated
                r = m.wait_report(copy=False)
                lat.append(r.latency_ms)
                cands.append(int(r.n))
                news.append(int(r.n_new))
                hbytes.append(int(r.host_bytes))
                full.append(bool(r.window_full))
        torch.cuda.synchronize()
        return time.perf_counter() - t0, lat, host_lat, cands, full, r, (news, hbytes)

    class Timed:
        """What one form's timed slices add up to."""

        def __init__(self):
            self.total, self.lat, self.host_lat, self.cands, self.full = 0.0, [], [], [], []
            self.r, self.tm, self.done, self.slices, self.news = None, {}, 0, [], []
            self.hbytes = []

        def add(self, dt, l, hl, c, f, r, tm, first, n, nw):
            self.total += dt
            self.lat += l
            self.host_lat += hl
            self.cands += c
            self.news += nw[0]
            self.hbytes += nw[1]
            self.full += f
            self.r = r
            for k, v in tm.items():
                self.tm[k] = self.tm.get(k, 0) + v
            self.done += n
            self.slices.append([first, first + n - 1])

    first = prefill
    if args.warmup:
        segment(args.mode, first, args.warmup)
        print("warm-up: %d slices" % args.warmup, file=sys.stderr, flush=True)
        first += args.warmup
    # the streaming form and the plain form take turns in blocks of slices,
    # so that both meet the same candidate-list sizes (it grows slowly)
    compare = args.mode == "streaming" and args.compare_steps > 0
    runs = {args.mode: Timed(), "plain": Timed()}
    turns = [(args.mode, args.steps)] + ([("plain", args.compare_steps)] if compare else [])
    # the timed slices time only their scans (the roofline's launch time): a
    # timed stage costs two event records on its stream, about 8 % of the
    # throughput when every stage of every slice is timed
    m.set_timing(srla.SRLA_TIMING_SCANS)
    m.timings(reset=True)
    while any(runs[mode].done < steps for mode, steps in turns):
        for mode, steps in turns:
            t = runs[mode]
            if t.done >= steps:
                continue
            n = min(args.block, args.segment, steps - t.done)
            dt, l, hl, c, f, r, nw = segment(mode, first, n)
            t.add(dt, l, hl, c, f, r, m.timings(reset=True), first, n, nw)
            first += n
            print("%s: timed %d/%d slices (%.2fs)" % (mode, t.done, steps, t.total),
                  file=sys.stderr, flush=True)
    main_run = runs[args.mode]
    total_s, lat, host_lat = main_run.total, np.array(main_run.lat), np.array(main_run.host_lat)
    cands, full, r, tm = main_run.cands, main_run.full, main_run.r, main_run.tm
    timed_slices = main_run.slices
    # the stage breakdown: more slices of the measured form, every stage timed
    m.set_timing(True)
    m.timings(reset=True)
    stage_tm, stage_slices = {}, []
    if args.stage_steps > 0:
        segment(args.mode, first, args.stage_steps)
        stage_tm = m.timings(reset=True)
        stage_slices = [first, first + args.stage_steps - 1]
        first += args.stage_steps

    pairs = args.steps * n_pairs
    value = pairs / total_s
    g = mon
    tau = 0
    while g["g"] * (1 << tau) < g["theta"]:
        tau += 1
    scan_ms = tm["scan_ms"] / max(1, tm["scan_launches"])
    per_launch_bytes = scan_bytes_per_pair(g["u"], tau) * n_pairs
    achieved = per_launch_bytes / (scan_ms * 1e-3) / 1e9
    scan_kernel = ("k_scan_partition" if args.scan_partition else
                   "k_scan_dedup" if args.scan_dedup else
                   "k_scan_lds_filter" if args.scan_lds_filter else
                   "k_scan_xcd" if args.scan_xcd else "k_scan_flat")
    stages = {k: stage_tm.get(k, 0.0) / max(1, stage_tm.get("estimates", 0)) for k in
              ("scan_ms", "sweep_ms", "finalize_ms", "estimate_ms", "slide_ms", "report_ms")}
    # the DR arrays the scan stores into: in the 256 MB last-level cache
    # (Infinity Cache) or beyond it in HBM
    footprint = 2 * g["u"] * (g["v_le"] * g["G"] + g["v_re"] * g["g"])
    level = "mall" if footprint <= (256 << 20) else "hbm"

    out = {
        "metric": METRIC if not args.host_ingest else
        "host-ingest packets/s (pairs handed over in pinned host memory, PCIe included)",
        "value": value,
        "unit": "packets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_s * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u16",
        "data": "synthetic",
        "config": {
            "workload": ("%s, %s form: 1 monitor, window %d slices, %d pairs/slice, Zipf(%g) "
                         "sources over %d hosts, %d planted super points, SRE %d x %d DR cells, "
                         "SLE %d DR cells (uint16 slice stamps), theta %d"
                         % (args.workload, args.mode, g["k"], n_pairs, stream.alpha, stream.n_ranks,
                            len(stream.planted), g["u"], g["v_re"] * g["g"],
                            g["u"] * g["v_le"] * g["G"], g["theta"])),
            "u": g["u"], "v_re": g["v_re"], "g": g["g"], "v_le": g["v_le"], "g_le": g["G"],
            "window": g["k"], "theta": g["theta"], "pairs_per_slice": n_pairs,
            "prefill_slices": prefill,
            "slices_timed": timed_slices,
            "block": args.block,
            "mode": args.mode, "graph": graph, "scan_blocks": args.scan_blocks,
            "scan_xcd": args.scan_xcd, "scan_dedup": args.scan_dedup,
            "scan_lds_filter": args.scan_lds_filter, "overlap_report": overlap,
            "scan_partition": args.scan_partition, "hold_scans": hold, "autotune": tuned,
            "report": ("full: ip, est, flags, |ULE|^k, |URE|^k (18 B/candidate)"
                       if args.full_report else "ip, est, flags (13 B/candidate)"),
        },
        "latency_clock": "device (end of the slice's last scan to its report in host memory)",
        "p50_ms": float(np.percentile(lat, 50)),
        "p99_ms": float(np.percentile(lat, 99)),
        "stage_ms_per_slice": stages,
        "stage_timing": ("slices %s after the timed ones, every stage timed (HIP events "
                         "around each stage); the timed slices time their scans only"
                         % (stage_slices,)),
        "state": {"window_full": bool(all(full)),
                  "candidates": [min(cands), max(cands)],
                  "up": r.up,
                  "row_fill_frac": [float(x) / (g["v_le"] * g["G"]) for x in r.row_fill],
                  "n_touched": int(r.n_touched), "n_new": int(r.n_new)},
        "roofline": {
            "kernel": ("k_scan_partition (k_scan_part + k_scan_mark + k_scan_stamp, "
                       "Algorithm 2)" if args.scan_partition else
                       "%s (Algorithm 2)" % scan_kernel),
            "bound": level,
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": measured_traffic(scan_kernel, args.workload),
            "bytes_per_pair": scan_bytes_per_pair(g["u"], tau),
            "launch_ms": scan_ms, "launches_timed": tm["scan_launches"],
            "footprint_bytes": footprint,
            "random_stores_per_s": g["u"] * (1 + 2.0 ** -tau) * n_pairs / (scan_ms * 1e-3),
        },
    }
    if args.host_ingest:
        out["p50_host_ms"] = float(np.percentile(host_lat, 50)) if len(host_lat) else None

    # the report's delivery: its contents are 13 (or 18) bytes per new
    # candidate and 9 (or 14) per carried one, whose address went to the host
    # beside the slice's scans (all 13 / 18 in the overlapped-report form);
    # what crosses PCIe in the candidate work's phase is what the estimate
    # wrote: the pieces of est and flags that differ from what the host set
    # held (each report carries the count)
    per_cand = 18 if args.full_report else 13
    n_cand, n_new = float(np.mean(cands)), float(np.mean(main_run.news))
    payload = (per_cand * n_cand if overlap else
               (per_cand - 4) * (n_cand - n_new) + per_cand * n_new)
    rep_bytes = float(np.mean(main_run.hbytes)) if main_run.hbytes else payload
    est_ms = stages["estimate_ms"]
    import probe
    pcie = probe.host_write_rate()
    out["roofline_report"] = {
        "kernel": "k_estimate (Eq9, report into pinned host memory) with the candidate check "
                  "before it (one timed phase)",
        "bound": "pcie", "bytes_per_slice": rep_bytes, "phase_ms": est_ms,
        "bytes_per_slice_source": "the reports' host_bytes (what the estimate wrote over PCIe)",
        "report_payload_bytes_per_slice": payload,
        "candidates_mean": n_cand, "new_candidates_mean": n_new,
        "achieved_GBps": rep_bytes / (est_ms * 1e-3) / 1e9 if est_ms > 0 else None,
        "ceiling_GBps": pcie / 1e9,
        "ceiling_source": "measured: coalesced kernel stores into pinned host memory",
        "frac": rep_bytes / (est_ms * 1e-3) / pcie if est_ms > 0 else None}

    # the snapshot's streaming sweeps: every LE and SRE DR read once, the
    # activity bitmaps written (one bit per LE DR, two per SRE DR)
    n_le = g["u"] * g["v_le"] * g["G"]
    n_re = g["u"] * g["v_re"] * g["g"]
    sweep_bytes = 2 * n_le + n_le / 8 + 2 * n_re + n_re / 4
    sweep_ms = stages["sweep_ms"]
    read_rate = probe.stream_read_rate(2 * (n_le + n_re))
    out["roofline_sweep"] = {
        "kernel": "k_sweep (the snapshot phase: the slice's close, the LE and SRE sweeps in "
                  "one launch)",
        "bound": level, "bytes_per_slice": sweep_bytes, "phase_ms": sweep_ms,
        "achieved_GBps": sweep_bytes / (sweep_ms * 1e-3) / 1e9 if sweep_ms > 0 else None,
        "ceiling_GBps": read_rate / 1e9,
        "ceiling_source": "measured: streaming 16-byte reads over the DR arrays' footprint",
        "frac": sweep_bytes / (sweep_ms * 1e-3) / read_rate if sweep_ms > 0 else None,
        "frac_of_hbm_peak": sweep_bytes / (sweep_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
        if sweep_ms > 0 else None}

    # ceilings at the scan's own footprint: random 2-byte stores (the flat
    # scan's pattern), and a streaming copy over the partitioned scan's working
    # set (its pairs, DR-index scratch and DR arrays)
    ceiling = probe.random_store_rate(footprint)
    stores_per_s = out["roofline"]["random_stores_per_s"]
    out["roofline"]["random_store_ceiling_per_s"] = ceiling
    out["roofline"]["frac_of_random_store_ceiling"] = stores_per_s / ceiling
    if args.scan_partition:
        # the partitioned scan's pairs and DR-index blocks besides the DR arrays
        ws = footprint + 16 * n_pairs
        copy_rate = probe.stream_copy_rate(ws // 2)
        out["roofline"]["stream_copy_ceiling_GBps"] = copy_rate / 1e9
        out["roofline"]["stream_copy_footprint_bytes"] = ws
        if out["roofline"]["traffic"]:
            moved = out["roofline"]["traffic"] / (scan_ms * 1e-3)
            out["roofline"]["traffic_GBps"] = moved / 1e9
            out["roofline"]["frac_of_stream_copy_ceiling"] = moved / copy_rate
    if args.probe_mib:
        out["random_store_rates_per_s"] = {
            mib: probe.random_store_rate(int(mib) << 20) for mib in args.probe_mib.split(",")}

    if compare:
        # the plain form on the same monitor, in the blocks between the
        # streaming ones: each slice scanned, then closed and its report
        # collected before the next slice's scan
        pr = runs["plain"]
        p_total, p_lat, p_host = pr.total, np.array(pr.lat), np.array(pr.host_lat)
        p_cands, p_full, ptm = pr.cands, pr.full, pr.tm
        p_scan = ptm["scan_ms"] / max(1, ptm["scan_launches"])
        out["plain"] = {
            "value": args.compare_steps * n_pairs / p_total,
            "ms_per_step": p_total * 1e3 / args.compare_steps,
            "p50_ms": float(np.percentile(p_lat, 50)),
            "p99_ms": float(np.percentile(p_lat, 99)),
            "p99_host_ms": float(np.percentile(p_host, 99)),
            "slices_timed": pr.slices,
            "window_full": bool(all(p_full)), "candidates": [min(p_cands), max(p_cands)],
            "scan_launch_ms": p_scan}
        out["plain_p99_ms"] = out["plain"]["p99_ms"]
        alone = per_launch_bytes / (p_scan * 1e-3) / 1e9
        out["roofline"]["alone"] = {"launch_ms": p_scan, "achieved": alone,
                                    "frac": alone / HBM_PEAK_GBS,
                                    "source": "the scans of the plain-form slices, alone on "
                                              "the GPU"}
    if not args.no_cpu_baseline:
        rate, dt, n, ncand = oracle_baseline(stream, mon, args.cpu_slices)
        out["cpu_baseline"] = {
            "value": rate, "unit": "packets/s", "cores": 1, "kind": "oracle",
            "sample": ("first %d slices (%d pairs) of the same workload, scan + end-of-slice "
                       "estimate, single-threaded C oracle, %.1f s on %s (nproc %d); the window "
                       "is %d/%d slices full at the end of the sample, with %d candidates"
                       % (args.cpu_slices, n, dt, cpu_model(), os.cpu_count(),
                          args.cpu_slices, g["k"], ncand)),
        }
    print(json.dumps(out), flush=True)
    m.close()


if __name__ == "__main__":
    main()
