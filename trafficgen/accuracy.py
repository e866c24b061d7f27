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


def main():
    """GPU accuracy run: python -m trafficgen.accuracy [workload] [slices]."""
    import torch
    import paper_1803_10369_amd as srla
    from trafficgen.configs import workload

    name = sys.argv[1] if len(sys.argv) > 1 else "accuracy"
    stream, mon, n = workload(name)
    n = int(sys.argv[2]) if len(sys.argv) > 2 else n
    gm = srla.Monitor(**mon, max_candidates=1 << 22)

    def scan(m, pairs):
        flat = np.ascontiguousarray(pairs.reshape(-1))
        m.scan(torch.from_numpy(flat.view(np.int32)).cuda())

    rows = evaluate([gm], stream, mon["k"], mon["theta"], n, every=5, scan=scan)
    summary = {key: float(np.mean([r["monitor0"][key] for r in rows]))
               for key in ("FPR", "FNR", "TFR")}
    summary.update({"worst_FNR": max(r["monitor0"]["FNR"] for r in rows),
                    "windows": len(rows), "workload": name,
                    "true_super_points_mean": float(np.mean([r["monitor0"]["N"] for r in rows]))})
    print(json.dumps({"summary": summary, "windows": rows}), flush=True)


if __name__ == "__main__":
    main()
