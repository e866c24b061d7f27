"""Named synthetic workloads: a stream recipe plus a monitor geometry.

The paper measures on two one-hour CERNET backbone traces that are not
public here; these seeded streams stand in for them with the paper's known
shape (theta = 1024, 1-second slices, window k = 300, u = 4 rows, g = 8 SRE
DRs, g' = 1024 LE DRs) and the sizes of the workloads this library is
measured on.

Geometry reading: "SRE R x C" means u = R rows of C = v_re * g cells;
"SLE N cells" means N = u * v_le * g' cells in total.
"""
from . import StreamSpec, loguniform_ints

STREAM_SEED = 180310369
HASH_SEED = 0x5EED000000000000


def _monitor(k, theta, u, v_re, g, v_le, G, cfg_no):
    return dict(k=k, theta=theta, u=u, v_re=v_re, g=g, v_le=v_le, G=G,
                hash_seed=HASH_SEED + cfg_no)


def workload(name):
    """Returns (stream, monitor_kwargs, n_slices) of a named workload."""
    if name in ("tiny", "tiny_coupled"):
        # 1 monitor, window 8, 100k pairs/slice for 16 slices, Zipf(1.1) over
        # 65,536 hosts, 4 planted super points with 2,000 distinct dsts,
        # SRE 4 x 16,384 cells, SLE 65,536 cells (the coupled companion uses
        # v_le = v_re so the LE does not saturate)
        stream = StreamSpec(n_pairs=100_000, n_ranks=65_536, alpha=1.1,
                            planted=[2000] * 4, window=8, seed=STREAM_SEED + 1)
        v_le = 16 if name == "tiny" else 2048
        return stream, _monitor(8, 1024, 4, 2048, 8, v_le, 1024, 1), 16
    if name == "backbone_pool4":
        # the backbone workload with repeating flows: ordinary sources draw
        # their destinations from a pool of 4 (so most pairs of a slice repeat
        # a flow, as on a real link); same monitor as "backbone"
        planted = loguniform_ints(1000, 200_000, 200, STREAM_SEED + 2)
        stream = StreamSpec(n_pairs=8_000_000, n_ranks=1 << 24, alpha=1.05, planted=planted,
                            window=300, seed=STREAM_SEED + 9, dst_pool=4)
        return stream, _monitor(300, 1024, 8, 131_072, 8, 2048, 1024, 2), 320
    if name in ("backbone", "backbone_paper", "backbone_k16"):
        # 1 monitor, window 300 slices, 8M pairs/slice, Zipf(1.05) over 2^24
        # hosts, 200 planted super points with 1k-200k dsts,
        # SRE 8 x 2^20 cells and SLE 2^24 cells
        planted = loguniform_ints(1000, 200_000, 200, STREAM_SEED + 2)
        k = 16 if name == "backbone_k16" else 300
        stream = StreamSpec(n_pairs=8_000_000, n_ranks=1 << 24, alpha=1.05,
                            planted=planted, window=k, seed=STREAM_SEED + 2)
        if name == "backbone_paper":
            mon = _monitor(k, 1024, 4, 65_536, 8, 65_536, 1024, 2)
        else:
            mon = _monitor(k, 1024, 8, 131_072, 8, 2048, 1024, 2)
        return stream, mon, 320
    if name in ("accuracy", "accuracy_small"):
        # unsaturated backbone-shaped stream for detection accuracy: ordinary
        # sources draw from 4 destinations each, 100 planted super points of
        # 1k-50k destinations; the paper's SEA (u = 4, v = 65,536, g' = 1024)
        small = name == "accuracy_small"
        planted = loguniform_ints(1000, 50_000, 100, STREAM_SEED + 6)
        k = 8 if small else 30
        stream = StreamSpec(n_pairs=200_000 if small else 1_000_000,
                            n_ranks=1 << (18 if small else 20), alpha=1.05,
                            planted=planted, window=k, seed=STREAM_SEED + 6, dst_pool=4)
        v = 4096 if small else 65_536
        return stream, _monitor(k, 1024, 4, v, 8, v, 1024, 6), (3 * k if small else 90)
    if name == "accuracy_boundary":
        # like "accuracy", but with 400 planted hosts of 256..4096 destinations
        # (log-uniform around theta = 1024), so that detection errors near the
        # threshold show how the SEA's size matters
        planted = loguniform_ints(256, 4096, 400, STREAM_SEED + 8)
        stream = StreamSpec(n_pairs=1_000_000, n_ranks=1 << 20, alpha=1.05, planted=planted,
                            window=30, seed=STREAM_SEED + 8, dst_pool=4)
        return stream, _monitor(30, 1024, 4, 65_536, 8, 65_536, 1024, 8), 90
    if name == "discrete_paper":
        # the paper's discrete-window run (Section 5.1): k = 1, one-bit DRs,
        # u = 4, v = 65,536, g' = 1024, theta = 1024, one 300-second window of
        # a ~4.5 Mpps link per slice.  The stream is produced in chunks of 8M
        # pairs (DISCRETE_CHUNKS chunks = 1.352 G pairs per slice; chunk c of
        # slice s is stream slice s * DISCRETE_CHUNKS + c); sources draw from 4
        # destinations each, 200 planted super points with 1k-200k dsts spread
        # evenly over a slice's chunks
        planted = loguniform_ints(1000, 200_000, 200, STREAM_SEED + 7)
        stream = StreamSpec(n_pairs=8_000_000, n_ranks=1 << 24, alpha=1.05, planted=planted,
                            window=DISCRETE_CHUNKS, seed=STREAM_SEED + 7, dst_pool=4)
        return stream, _monitor(1, 1024, 4, 65_536, 8, 65_536, 1024, 7), 4
    raise KeyError(name)


# chunks of 8M pairs per slice of the discrete-window workload: 300 s x 4.5 Mpps
DISCRETE_CHUNKS = 169


def scaled(stream, n_pairs):
    """The same stream recipe with fewer pairs per slice (planted kept)."""
    return StreamSpec(n_pairs=n_pairs, n_ranks=stream.n_ranks, alpha=stream.alpha,
                      planted=list(stream.planted), window=stream.window, seed=stream.seed)


def batched_monitors(n=16, cfg_no=4):
    """Monitors of the batched workload: window [10, 60, 300, 1800][m % 4]
    slices, threshold 2^(8 + m % 7) (256 .. 16,384), SLE 2^(20 + m % 6) DR
    cells (u = 4 rows of g' = 1024, so v_le = 256 .. 8,192), SRE 4 x 2^20
    cells (v_re = 131,072, g = 8), one hash seed per monitor."""
    out = []
    for m in range(n):
        sle = 1 << (20 + m % 6)
        out.append(_monitor([10, 60, 300, 1800][m % 4], 1 << (8 + m % 7), 4, 131_072, 8,
                            sle // (4 * 1024), 1024, cfg_no * 1000 + m))
    return out


ALPHA_GRID = [0.90, 0.95, 1.00, 1.05, 1.10, 1.15, 1.20, 1.25, 1.30]


def serving_monitors(n=64, cfg_no=5):
    """Monitors of the serving mix: LE 2^e DR cells with e drawn from
    {24..33}, u in {4, 8}, window in {10, 60, 300, 1800}, threshold in
    {256 .. 16,384}, g' = 1024, g = 8, v_re = 131,072 (seeded draws)."""
    from . import mix64_int
    out = []
    for m in range(n):
        r = [mix64_int(STREAM_SEED * 31 + cfg_no * 7919 + 97 * m + j) for j in range(4)]
        e = 24 + r[0] % 10
        u = 4 if r[1] % 2 == 0 else 8
        k = [10, 60, 300, 1800][r[2] % 4]
        theta = 1 << (8 + r[3] % 7)
        out.append(_monitor(k, theta, u, 131_072, 8, (1 << e) // (u * 1024), 1024,
                            cfg_no * 1000 + m))
    return out


class ServingStream:
    """The serving mix's stream: slice s has n_s pairs (log-uniform on
    [lo, hi]) and a Zipf exponent alpha_s drawn from ALPHA_GRID, over 2^24
    hosts, with 1,000 planted super points of 1k-200k destinations spread
    over a 300-slice window.  slice(s) / device generation delegate to one
    StreamSpec per alpha, resized to n_s."""

    def __init__(self, lo=2_000_000, hi=32_000_000, n_ranks=1 << 24, planted=1000, seed=None):
        from . import StreamSpec, mix64_int
        self.seed = STREAM_SEED + 5 if seed is None else seed
        self.lo, self.hi = lo, hi
        self.planted = loguniform_ints(1000, 200_000, planted, self.seed)
        self.specs = {a: StreamSpec(n_pairs=hi, n_ranks=n_ranks, alpha=a, planted=self.planted,
                                    window=300, seed=self.seed) for a in ALPHA_GRID}
        self._mix = mix64_int

    def params(self, s):
        """(n_s, alpha_s) of slice s."""
        import math
        r1 = self._mix(self.seed ^ (0xA5A5 + 2 * s))
        r2 = self._mix(self.seed ^ (0xA5A5 + 2 * s + 1))
        uu = (r1 >> 11) / float(1 << 53)
        n = int(round(math.exp(math.log(self.lo) + uu * (math.log(self.hi) - math.log(self.lo)))))
        return n, ALPHA_GRID[r2 % len(ALPHA_GRID)]

    def spec(self, s):
        """The StreamSpec that generates slice s (its n_pairs set to n_s)."""
        n, a = self.params(s)
        sp = self.specs[a]
        sp.n_pairs = n
        return sp
