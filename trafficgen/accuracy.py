"""Detection accuracy against the precise method (Definition 5).

For a window with N true super points (exact |OP(aip)| >= theta, counted by
the paper's precise method: the distinct second addresses of each first
address over the window's pairs), a monitor that reports N' hosts with the
SUPER flag has N+ false positives and N- misses:
FPR = N+ / N, FNR = N- / N, TFR = FPR + FNR.

Evaluation only: nothing here is part of either implementation.
"""
import json
import sys

import numpy as np


def exact_cardinalities(slices):
    """(ips, counts): distinct second addresses per first address over the
    given slices' pairs (each an (n, 2) uint32 array)."""
    keys = [np.unique((p[:, 0].astype(np.uint64) << np.uint64(32)) | p[:, 1].astype(np.uint64))
            for p in slices if len(p)]
    if not keys:
        return np.zeros(0, np.uint32), np.zeros(0, np.int64)
    key = np.unique(np.concatenate(keys))
    return np.unique((key >> np.uint64(32)).astype(np.uint32), return_counts=True)


def rates(detected, truth):
    detected, truth = set(detected), set(truth)
    n = len(truth)
    fp = len(detected - truth)
    fn = len(truth - detected)
    fpr = fp / n if n else 0.0
    fnr = fn / n if n else 0.0
    return {"N": n, "detected": len(detected), "false_pos": fp, "false_neg": fn,
            "FPR": fpr, "FNR": fnr, "TFR": fpr + fnr}


def evaluate(monitors, stream, k, theta, n_slices, every=1, scan=None):
    """Runs each monitor (objects with scan(pairs) and estimate() returning a
    report with ip/flags) over slices 0..n_slices-1 of `stream` and returns,
    for every full window at every `every`-th slice, the rates of each."""
    history, out = [], []
    for s in range(n_slices):
        pairs = stream.slice(s)
        history.append(pairs)
        if len(history) > k:
            history.pop(0)
        reports = []
        for m in monitors:
            (scan or (lambda mm, p: mm.scan(p)))(m, pairs)
            reports.append(m.estimate())
        if s >= k - 1 and (s - k + 1) % every == 0:
            ips, cnt = exact_cardinalities(history)
            truth = ips[cnt >= theta].tolist()
            row = {"slice": s}
            for i, r in enumerate(reports):
                det = r.ip[(r.flags & 1) != 0].tolist()
                row["monitor%d" % i] = rates(det, truth)
                row["monitor%d" % i]["candidates"] = int(r.n)
            out.append(row)
    return out


SWEEP_U = (2, 4)
SWEEP_V = (16_384, 65_536)
SWEEP_G = (1024, 2048, 4096, 8192)


def sweep_monitors(mon):
    """The SEA parameter grid of the paper's accuracy comparison (Section 5.1:
    g' from 1024 to 8192, several u and v): one monitor per (u, v, g'), with
    the workload's window, threshold and hash seed."""
    out = []
    for u in SWEEP_U:
        for v in SWEEP_V:
            for G in SWEEP_G:
                out.append(dict(mon, u=u, v_re=v, v_le=v, G=G))
    return out


def main():
    """GPU accuracy run:
    python -m trafficgen.accuracy [workload] [slices] [--sweep]
    --sweep runs the (u, v, g') grid side by side on the same stream and
    windows (the precise method is evaluated once per window)."""
    import torch
    import paper_1803_10369_amd as srla
    from trafficgen.configs import workload

    argv = [a for a in sys.argv[1:] if not a.startswith("--")]
    sweep = "--sweep" in sys.argv
    name = argv[0] if argv else "accuracy"
    stream, mon, n = workload(name)
    n = int(argv[1]) if len(argv) > 1 else n
    cfgs = sweep_monitors(mon) if sweep else [mon]
    gms = [srla.Monitor(**c, max_candidates=1 << 22, lean_report=True) for c in cfgs]

    def scan(m, pairs):
        flat = np.ascontiguousarray(pairs.reshape(-1))
        m.scan(torch.from_numpy(flat.view(np.int32)).cuda())

    rows = evaluate(gms, stream, mon["k"], mon["theta"], n, every=5, scan=scan)
    results = []
    for i, c in enumerate(cfgs):
        key = "monitor%d" % i
        summary = {k: float(np.mean([r[key][k] for r in rows])) for k in ("FPR", "FNR", "TFR")}
        summary.update({"u": c["u"], "v": c["v_le"], "g_le": c["G"],
                        "worst_FNR": max(r[key]["FNR"] for r in rows),
                        "worst_FPR": max(r[key]["FPR"] for r in rows),
                        "candidates_mean": float(np.mean([r[key]["candidates"] for r in rows]))})
        results.append(summary)
    out = {"workload": name, "windows": len(rows),
           "true_super_points_mean": float(np.mean([r["monitor0"]["N"] for r in rows])),
           "summary": results if sweep else results[0]}
    if not sweep:
        out["per_window"] = rows
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
