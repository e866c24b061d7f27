"""Statistical pins of the oracle against the paper's closed forms.

* Lemma 1, Theorem 1 and Eq2-Eq5 give the exact distribution of the weight of
  one SRE after a host with |OP| distinct second addresses is scanned.
* Linear counting (Eq6, Whang et al.): a lone host with n distinct second
  addresses sets E[U] = g'(1 - (1 - 1/g')^n) DRs, and the estimate has
  Whang's standard error sqrt(g'(e^t - t - 1)) with t = n / g'.
* Eq8-Eq9 remove the DRs that other hosts set: under background traffic the
  corrected estimate stays near n while the uncorrected Eq7 drifts upward.

Seeds are fixed, so these run deterministically; bounds sit at about 4-5
standard deviations.
"""
import math
from fractions import Fraction

import numpy as np
from scipy.stats import chi2

import oracle


def surjections(alpha, g1):
    """FN(alpha, g1) of Lemma 1: ways to throw alpha balls into g1 boxes, none empty."""
    return sum((-1) ** j * math.comb(g1, j) * (g1 - j) ** alpha for j in range(g1 + 1))


def eq4_weight_distribution(n_op, g, tau, alpha_max=200):
    """Pr{|OP|, g, tau, g1} for g1 = 0..g (Eq2-Eq4)."""
    p = 2.0 ** -tau
    out = [0.0] * (g + 1)
    for alpha in range(0, min(n_op, alpha_max) + 1):
        pa = math.comb(n_op, alpha) * p ** alpha * (1 - p) ** (n_op - alpha)   # Eq3
        if pa < 1e-300:
            continue
        for g1 in range(0, min(alpha, g) + 1):
            if alpha == 0:
                pg = 1.0 if g1 == 0 else 0.0
            else:
                pg = float(Fraction(math.comb(g, g1) * surjections(alpha, g1), g ** alpha))  # Eq2
            out[g1] += pa * pg
    return np.array(out)


def test_surjection_count_closed_forms():
    # Lemma 1's recursion g^a - sum_{i<g} C(g,i) FN(a,i) against the
    # inclusion-exclusion sum, and against g! * S(a, g) for small cases
    for a in range(1, 9):
        for g in range(1, a + 1):
            rec = g ** a - sum(math.comb(g, i) * surjections(a, i) for i in range(1, g))
            assert rec == surjections(a, g)
    assert surjections(4, 2) == 14 and surjections(5, 3) == 150 and surjections(3, 3) == 6


def _lone_host_trials(n_op, trials, cfg, seed0):
    rng = np.random.default_rng(seed0)
    W, det, U, est = [], [], [], []
    aip = 0x0A000001
    for t in range(trials):
        m = oracle.Monitor(hash_seed=seed0 * 100003 + t, **cfg)
        dst = rng.choice(2 ** 32, size=n_op, replace=False).astype(np.uint32)
        m.scan(np.stack([np.full(n_op, aip, np.uint32), dst], 1))
        r = m.estimate()
        # a single slice with k = 1: the DRs set in it read 1 after the slide
        re = m.dump(oracle.RE)
        W.append(int((re == 1).sum()))
        det.append(r.n == 1)
        if r.n == 1:
            U.append(int(r.union_weight[0]))
            est.append(float(r.est[0]))
        m.close()
    return np.array(W), np.array(det), np.array(U), np.array(est)


def test_sre_weight_follows_eq4_and_detection_follows_eq5():
    g, theta, n_op, trials = 8, 1024, 1024, 3000
    tau = oracle.tau(theta, g)
    cfg = dict(k=1, theta=theta, u=1, v_re=1, g=g, v_le=1, G=64)
    W, det, _, _ = _lone_host_trials(n_op, trials, cfg, 17)
    p = eq4_weight_distribution(n_op, g, tau)
    assert abs(p.sum() - 1) < 1e-9
    counts = np.bincount(W, minlength=g + 1).astype(float)
    exp = p * trials
    # merge sparse low bins into their neighbour
    keep = exp >= 5
    cm, em = [], []
    acc_c = acc_e = 0.0
    for c, e, k in zip(counts, exp, keep):
        acc_c += c
        acc_e += e
        if k:
            cm.append(acc_c)
            em.append(acc_e)
            acc_c = acc_e = 0.0
    cm[-1] += acc_c
    em[-1] += acc_e
    stat = sum((c - e) ** 2 / e for c, e in zip(cm, em))
    assert chi2.sf(stat, len(cm) - 1) > 1e-4, (counts, exp)
    # Eq5: probability of at least ceil(rho * g) set DRs = detection probability
    t_re = oracle.sre_threshold(g)
    p_det = p[t_re:].sum()
    sd = math.sqrt(p_det * (1 - p_det) / trials)
    assert abs(det.mean() - p_det) < 5 * sd


def test_linear_counting_mean_and_whang_error():
    G, n_op, trials = 1024, 1500, 400
    cfg = dict(k=1, theta=8, u=2, v_re=1, g=8, v_le=4096, G=G)
    _, det, U, est = _lone_host_trials(n_op, trials, cfg, 23)
    assert det.all()
    q = 1 - 1 / G
    EU = G * (1 - q ** n_op)
    VarU = G * (G - 1) * (1 - 2 / G) ** n_op + G * q ** n_op - G * G * q ** (2 * n_op)
    assert abs(U.mean() - EU) < 5 * math.sqrt(VarU / trials)
    t = n_op / G
    se = math.sqrt(G * (math.exp(t) - t - 1))
    assert abs(est.mean() - n_op) < 5 * se / math.sqrt(trials)
    assert 0.8 * se < est.std() < 1.2 * se


def test_union_noise_is_removed_by_eq9():
    G, v_le, u, n_op = 1024, 16, 4, 2000
    cfg = dict(k=1, theta=64, u=u, v_re=64, g=8, v_le=v_le, G=G)
    rng = np.random.default_rng(5)
    corrected, plain = [], []
    aip = 0xC0A80001
    for t in range(40):
        m = oracle.Monitor(hash_seed=777 + t, **cfg)
        bg_src = rng.integers(0, 2 ** 32, size=20_000, dtype=np.uint64).astype(np.uint32)
        bg = np.stack([bg_src, rng.integers(0, 2 ** 32, size=bg_src.size, dtype=np.uint64).astype(np.uint32)], 1)
        dst = rng.choice(2 ** 32, size=n_op, replace=False).astype(np.uint32)
        m.scan(np.concatenate([bg, np.stack([np.full(n_op, aip, np.uint32), dst], 1)]))
        r = m.estimate()
        hit = np.flatnonzero(r.ip == aip)
        assert hit.size == 1
        x = int(hit[0])
        assert 0.15 < r.up < 0.5
        corrected.append(r.est[x])
        plain.append(-G * math.log((G - r.union_weight[x]) / G))   # Eq7 without the correction
        m.close()
    corrected, plain = np.array(corrected), np.array(plain)
    assert abs(corrected.mean() - n_op) < 0.05 * n_op
    assert plain.mean() > 1.1 * n_op


def test_degenerate_single_column_estimate_is_zero():
    """u = 1, v_le = 1: the row fill is the host's own union weight, so Eq8
    gives UP = U / g' and Eq9's numerator vanishes: the estimate is 0."""
    cfg = dict(k=2, theta=8, u=1, v_re=1, g=8, v_le=1, G=256)
    m = oracle.Monitor(hash_seed=3, **cfg)
    dst = np.random.default_rng(1).choice(2 ** 32, size=150, replace=False).astype(np.uint32)
    m.scan(np.stack([np.full(dst.size, 42, np.uint32), dst], 1))
    r = m.estimate()
    assert r.n == 1 and r.up == r.union_weight[0] / 256
    assert 0 < r.union_weight[0] < 256
    assert r.est[0] == 0.0
