"""Exact closed-form pins of Eq8-Eq9 (Section 4.2) on planted inputs.

A host a that is the only traffic of the window sets, in every row i, the DRs
H3(b) of its own LE column and nothing else.  So with U = |{H3(b)}| over the
window's second addresses b:

* the row fill is |LDR(i)|^k = U in every row,
* the union LE weight of a is |ULE(a)|^k = U (the same DRs in every row),
* Eq8 gives UP = (U / (g' v))^u,
* Eq9 gives est = -g' ln(1 - (U - g' UP) / (g' (1 - UP))).

With a second host b whose LE columns differ from a's in every row, each row
holds both hosts' DRs: the row fills become U_a + U_b, UP = ((U_a + U_b) /
(g' v))^u, while a's union weight stays U_a -- this pins the cross-host term
of Eq8 that a single host cannot distinguish from its own.

U is counted with the independent numpy copy of the hash reading; the closed
forms are evaluated in mpmath at 50 digits and the oracle's FP64 results must
agree to 1e-12 relative (Eq8 to 1e-15).  u > 1 and v > 1 throughout, so a
dropped exponent, a wrong denominator or a swapped operand fails.
"""
import mpmath
import numpy as np
import pytest

import oracle
from oracle.exact import Hashes

mpmath.mp.dps = 50


def _closed_form(U, fill, u, v_le, G):
    """(UP, est) from Eq8 and Eq9 in exact decimal arithmetic."""
    G_ = mpmath.mpf(G)
    up = (mpmath.mpf(fill) / (G_ * v_le)) ** u
    x = (U - G_ * up) / (G_ * (1 - up))
    return up, -G_ * mpmath.log(1 - x)


def _pairs(src, dsts):
    return np.stack([np.full(len(dsts), src, np.uint32), np.asarray(dsts, np.uint32)], 1)


@pytest.mark.parametrize("u,v_le,G,k,sizes", [
    (2, 3, 256, 1, [90]),
    (3, 5, 512, 2, [60, 140, 35]),
    (4, 2, 1024, 3, [400, 10, 700, 250]),
    (8, 7, 64, 2, [30, 45, 20]),
])
def test_lone_host_estimate_follows_eq8_eq9(u, v_le, G, k, sizes):
    seed = 0x5EED + 31 * u + v_le
    cfg = dict(k=k, theta=8, u=u, v_re=11, g=8, v_le=v_le, G=G, hash_seed=seed)
    h = Hashes(seed, u, cfg["v_re"], cfg["g"], v_le, G)
    rng = np.random.default_rng(seed)
    aip = 0x0A0B0C0D
    m = oracle.Monitor(**cfg)
    history = []
    for e, n in enumerate(sizes):
        dsts = rng.choice(2 ** 32, size=n, replace=False).astype(np.uint32)
        history.append(dsts)
        m.scan(_pairs(aip, dsts))
        r = m.estimate()
        window = np.concatenate(history[max(0, e - k + 1):e + 1])
        U = len(set(h.le_idx(window).tolist()))
        # theta = 8 <= g: tau = 0, every pair is sampled, so the host stays a
        # candidate while its SRE has ceil(rho g) DRs inside the window
        assert r.n == 1 and int(r.ip[0]) == aip, (e, r.n)
        assert int(r.union_weight[0]) == U
        assert [int(x) for x in r.row_fill] == [U] * u
        up, est = _closed_form(U, U, u, v_le, G)
        assert abs(r.up - float(up)) <= 1e-15 * float(up)
        assert abs(r.est[0] - float(est)) <= 1e-12 * abs(float(est)), (e, r.est[0], est)
        assert bool(r.flags[0] & oracle.SUPER) == (float(est) >= cfg["theta"])
    m.close()


def test_two_hosts_in_disjoint_columns_follow_eq8_eq9():
    u, v_le, G, v_re = 3, 4, 1024, 64
    seed = 0xE98E9
    cfg = dict(k=1, theta=8, u=u, v_re=v_re, g=8, v_le=v_le, G=G, hash_seed=seed)
    h = Hashes(seed, u, v_re, 8, v_le, G)
    a = 0x01020304
    col_a = [int(h.col_le(i, [a])[0]) for i in range(u)]
    b = next(x for x in range(a + 1, a + 100000)
             if all(int(h.col_le(i, [x])[0]) != col_a[i] for i in range(u)))
    rng = np.random.default_rng(3)
    da = rng.choice(2 ** 32, size=700, replace=False).astype(np.uint32)
    db = rng.choice(2 ** 32, size=1500, replace=False).astype(np.uint32)
    m = oracle.Monitor(**cfg)
    m.scan(np.concatenate([_pairs(a, da), _pairs(b, db)]))
    r = m.estimate()
    Ua = len(set(h.le_idx(da).tolist()))
    Ub = len(set(h.le_idx(db).tolist()))
    assert [int(x) for x in r.row_fill] == [Ua + Ub] * u
    ips = [int(x) for x in r.ip]
    assert ips == sorted([a, b])
    for ip, U in ((a, Ua), (b, Ub)):
        x = ips.index(ip)
        assert int(r.union_weight[x]) == U
        up, est = _closed_form(U, Ua + Ub, u, v_le, G)
        assert abs(r.up - float(up)) <= 1e-15 * float(up)
        assert abs(r.est[x] - float(est)) <= 1e-12 * abs(float(est)), (ip, r.est[x], est)
    m.close()
