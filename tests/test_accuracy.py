"""Detection accuracy (Definition 5) of the oracle on an unsaturated stream,
under the slice-synchronous reading and under Algorithm 2's literal per-pair
check, against the precise method.  A statistical sanity check of the method
and of the reading, not a parity test."""
import numpy as np

import oracle
from trafficgen.accuracy import evaluate, exact_cardinalities, rates
from trafficgen.configs import workload


def test_rates_follow_definition_5():
    r = rates(detected=[1, 2, 3, 9], truth=[1, 2, 4, 5])
    assert r == {"N": 4, "detected": 4, "false_pos": 2, "false_neg": 2,
                 "FPR": 0.5, "FNR": 0.5, "TFR": 1.0}
    assert rates([], [])["TFR"] == 0.0


def test_precise_method_counts_distinct_peers():
    p1 = np.array([[1, 10], [1, 11], [2, 10]], np.uint32)
    p2 = np.array([[1, 10], [1, 12], [3, 7]], np.uint32)
    ips, cnt = exact_cardinalities([p1, p2])
    assert dict(zip(ips.tolist(), cnt.tolist())) == {1: 3, 2: 1, 3: 1}


def test_reading_and_literal_algorithm_are_both_accurate():
    stream, mon, n = workload("accuracy_small")
    rc = oracle.Monitor(**mon)
    seq = oracle.Monitor(**mon, sequential=True)
    rows = evaluate([rc, seq], stream, mon["k"], mon["theta"], n, every=4)
    assert len(rows) >= 4
    for row in rows:
        a, b = row["monitor0"], row["monitor1"]
        assert a["N"] >= 50                       # the planted hosts at least
        assert a["FNR"] <= 0.05 and b["FNR"] <= 0.05
        assert a["FPR"] <= 0.10 and b["FPR"] <= 0.10
        assert abs(a["TFR"] - b["TFR"]) <= 0.05
