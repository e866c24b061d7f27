"""The C-ABI library loads and exports what include/srla.h declares; host-side
validation needs no GPU.  No test here launches device work."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "srla.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(srla_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def P():
    import paper_1803_10369_amd as P
    P.srla.lib()
    return P


def test_every_declared_symbol_is_exported(P):
    names = _declared_functions()
    assert set(names) == {"srla_footprint_bytes", "srla_create", "srla_scan", "srla_scan_noalloc",
                          "srla_estimate",
                          "srla_close_slice", "srla_wait_report", "srla_dump_state",
                          "srla_timings", "srla_set_timing", "srla_destroy", "srla_last_error",
                          "srla_group_create", "srla_group_scan", "srla_group_destroy",
                          "srla_group_last_error", "srla_admit"}
    L = ctypes.CDLL(P.srla.LIB_PATH)
    for n in names:
        assert hasattr(L, n), n
    assert set(P.EXPORTS) == set(names)


def test_binding_struct_layouts_match_header(P, tmp_path):
    """ctypes layouts against what a C compiler makes of include/srla.h."""
    import subprocess
    src = tmp_path / "layout.c"
    src.write_text('''
#include <stddef.h>
#include <stdio.h>
#include "srla.h"
int main(void) {
  printf("%zu %zu %zu %zu\\n", sizeof(srla_geometry_t), sizeof(srla_config_t),
         sizeof(srla_report_t), sizeof(srla_timings_t));
  printf("%zu %zu %zu %zu %zu\\n", offsetof(srla_config_t, max_candidates),
         offsetof(srla_config_t, scan_blocks),
         offsetof(srla_report_t, row_fill), offsetof(srla_report_t, up),
         offsetof(srla_timings_t, estimates));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    S = P.srla
    want = [ctypes.sizeof(S.srla_geometry_t), ctypes.sizeof(S.srla_config_t),
            ctypes.sizeof(S.srla_report_t), ctypes.sizeof(S.srla_timings_t),
            S.srla_config_t.max_candidates.offset, S.srla_config_t.scan_blocks.offset,
            S.srla_report_t.row_fill.offset,
            S.srla_report_t.up.offset, S.srla_timings_t.estimates.offset]
    assert [int(x) for x in out] == want


def test_binding_constants_match_header(P, tmp_path):
    """The binding's config flags, dump selectors, report flags and timing
    mode against what a C compiler makes of include/srla.h."""
    import subprocess
    names = ["SRLA_CFG_TIMING", "SRLA_CFG_SCAN_XCD", "SRLA_CFG_GRAPH", "SRLA_CFG_DISCRETE",
             "SRLA_CFG_LEAN_REPORT", "SRLA_CFG_SCAN_DEDUP", "SRLA_CFG_SCAN_LDS_FILTER",
             "SRLA_CFG_OVERLAP_REPORT", "SRLA_CFG_SCAN_PARTITION", "SRLA_CFG_HOLD_SCANS",
             "SRLA_DUMP_LE", "SRLA_DUMP_RE", "SRLA_DUMP_SI", "SRLA_FLAG_SUPER", "SRLA_FLAG_SAT",
             "SRLA_FLAG_NEW", "SRLA_FLAG_KEEP", "SRLA_TIMING_SCANS"]
    names = [n for n in names if hasattr(P.srla, n)]
    assert "SRLA_TIMING_SCANS" in names and "SRLA_CFG_HOLD_SCANS" in names
    src = tmp_path / "consts.c"
    src.write_text('#include <stdio.h>\n#include "srla.h"\nint main(void) {\n' +
                   "".join('  printf("%%ld\\n", (long)(%s));\n' % n for n in names) +
                   "  return 0;\n}\n")
    exe = tmp_path / "consts"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    assert [int(x) for x in out] == [getattr(P.srla, n) for n in names]


BAD = [
    dict(k=0), dict(k=32768), dict(theta=0), dict(u=0), dict(u=17), dict(g=0), dict(g=65),
    dict(G=0), dict(G=100), dict(G=32), dict(v_re=0), dict(v_le=0),
]


@pytest.mark.parametrize("bad", BAD)
def test_invalid_configs_are_rejected_without_a_device(P, bad):
    base = dict(k=8, theta=1024, u=4, v_re=2048, g=8, v_le=16, G=1024, hash_seed=1)
    base.update(bad)
    cfg = P.make_config(**base)
    assert P.srla_footprint_bytes(cfg) == 0
    rc, h = P.srla_create(cfg)
    assert rc == -1 and not h.value


def test_bad_flags_and_capacity_rejected(P):
    cfg = P.make_config(8, 1024, 4, 2048, 8, 16, 1024, 1, max_candidates=0)
    assert P.srla_create(cfg)[0] == -1
    cfg = P.make_config(8, 1024, 4, 2048, 8, 16, 1024, 1, flags=4096)
    assert P.srla_create(cfg)[0] == -1
    lean = P.make_config(8, 1024, 4, 2048, 8, 16, 1024, 1, flags=P.srla.SRLA_CFG_LEAN_REPORT)
    assert P.srla_footprint_bytes(lean) > 0
    # the discrete (one-bit DR) form exists only for k = 1
    cfg = P.make_config(8, 1024, 4, 2048, 8, 16, 1024, 1, flags=P.srla.SRLA_CFG_DISCRETE)
    assert P.srla_footprint_bytes(cfg) == 0 and P.srla_create(cfg)[0] == -1


def test_footprint_counts_dr_arrays(P):
    # backbone-shaped monitor: SRE 8 x 2^20 cells, SLE 2^24 cells
    cfg = P.make_config(300, 1024, 8, 131072, 8, 2048, 1024, 1, max_candidates=1)
    fp = P.srla_footprint_bytes(cfg)
    le_cells, re_cells, ses = 1 << 24, 1 << 23, 8 * 131072
    # uint16 stamps, one activity bit per LE DR and two per SRE DR for each
    # slice parity, 16 x uint32 SI counters per SE
    want = 2 * le_cells + 2 * le_cells // 8 + 2 * re_cells + 4 * re_cells // 8 + 64 * ses
    # plus counters, row fills and the LE sweep's partial row sums (a few KiB)
    assert want <= fp < want + 8192
    big = P.make_config(300, 1024, 8, 131072, 8, 2048, 1024, 1, max_candidates=1 << 20)
    assert P.srla_footprint_bytes(big) - fp >= (13 + 27) * ((1 << 20) - 1)


def test_overlap_report_staging_is_counted(P):
    # two staging sets (by slice parity) of 13 (lean) or 18 bytes per candidate
    # and the two staged counts; the direct report instead keeps device copies
    # of its three host sets' est and flags arrays (9 bytes per candidate each)
    n = 1 << 20
    for lean, per in ((P.srla.SRLA_CFG_LEAN_REPORT, 13), (0, 18)):
        base = P.make_config(300, 1024, 8, 131072, 8, 2048, 1024, 1, max_candidates=n, flags=lean)
        ov = P.make_config(300, 1024, 8, 131072, 8, 2048, 1024, 1, max_candidates=n,
                           flags=lean | P.srla.SRLA_CFG_OVERLAP_REPORT)
        assert P.srla_footprint_bytes(ov) - P.srla_footprint_bytes(base) == \
            2 * per * n + 8 - 3 * 9 * n


def test_discrete_footprint_is_bits(P):
    cfg = P.make_config(1, 1024, 8, 131072, 8, 2048, 1024, 1, max_candidates=1,
                        flags=P.srla.SRLA_CFG_DISCRETE)
    fp = P.srla_footprint_bytes(cfg)
    le_cells, re_cells, ses = 1 << 24, 1 << 23, 8 * 131072
    # two LE bit arrays (slice parities), two interleaved SRE maps (their
    # "after the slide" halves stay clear), the SI counters, two
    # sampled-source sets of 2^12 64-bit slots
    want = 2 * le_cells // 8 + 4 * re_cells // 8 + 64 * ses + 2 * 8 * 4096
    assert want <= fp < want + 4096
    stamps = P.make_config(1, 1024, 8, 131072, 8, 2048, 1024, 1, max_candidates=1)
    assert P.srla_footprint_bytes(stamps) - fp > 2 * le_cells


def test_null_handles(P):
    L = P.srla.lib()
    assert L.srla_destroy(None) == 0
    assert L.srla_last_error(None) == b"no monitor"
    assert L.srla_scan(None, None, 0, 0) == -1
    assert L.srla_estimate(None, None) == -1
    assert L.srla_close_slice(None) == -1
    assert L.srla_wait_report(None, None) == -1
    assert L.srla_group_scan(None, None, 0, 1) == -1
    assert L.srla_group_destroy(None) == 0
    assert L.srla_group_last_error(None) == b"no group"


def test_product_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_1803_10369_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "import oracle" not in text and "from oracle" not in text, f
                assert "srla_oracle" not in text, f


def test_admission_is_first_fit_under_the_budget(P):
    from trafficgen.configs import serving_monitors
    cfgs = [P.make_config(**m, max_candidates=1 << 22) for m in serving_monitors(64)]
    fps = [P.srla_footprint_bytes(c) for c in cfgs]
    budget = 200 * 10 ** 9
    rc, adm, used = P.srla_admit(cfgs, budget)
    assert rc == 0
    # first fit, in order, recomputed here
    left, want = budget, []
    for fp in fps:
        want.append(fp <= left)
        if fp <= left:
            left -= fp
    assert adm == want and used == budget - left <= budget
    assert 0 < sum(adm) < len(cfgs)          # the mix does not fit whole
    rc, adm, used = P.srla_admit(cfgs, 0)
    assert rc == 0 and not any(adm) and used == 0
    rc, adm, used = P.srla_admit(cfgs[:3], 1 << 62)
    assert all(adm) and used == sum(fps[:3])
    bad = P.make_config(0, 1, 1, 1, 1, 1, 64, 0)
    assert P.srla_admit([cfgs[0], bad], budget)[0] == -1


def test_partition_scan_scratch_in_the_footprint(P):
    """The partitioned scan takes any LE, in bands of at most 2048 regions of
    2^16 DRs, and counts its scratch in the footprint: 128 MiB of DR indices,
    (R + 1) * 2048 16-bit region offsets for the R regions of the largest
    band, the marking plan (2 * 2048 + 2 words, rounded up to 256 bytes) and
    R + 2048 unit bitmaps of 8 KiB (a round of 2048 chunks makes at most
    R + 2048 units)."""
    part = P.srla.SRLA_CFG_SCAN_PARTITION

    def extra(*geo):
        plain = P.make_config(*geo, max_candidates=1)
        cfg = P.make_config(*geo, max_candidates=1, flags=part)
        return P.srla_footprint_bytes(cfg) - P.srla_footprint_bytes(plain)

    def scratch(regions):
        return (2 * 2048 * 32768 + 2 * (regions + 1) * 2048 +
                4 * (4160 + (regions + 2048) * 2048))

    # backbone: 2^24 LE DRs, 256 regions in one band
    assert extra(300, 1024, 8, 131072, 8, 2048, 1024, 1) == scratch(256)
    # the paper's SEA: 2^28 LE DRs, two bands of 2048 regions
    assert extra(300, 1024, 4, 65536, 8, 65536, 1024, 1) == scratch(2048)
    # a ragged last region: 2^25 + 2^10 DRs in 513 regions
    assert extra(3, 1024, 1, 64, 8, 32769, 1024, 1) == scratch(513)
    # scan_blocks sets the marking unit: 2^26 / unit units beyond R
    geo = (300, 1024, 8, 131072, 8, 2048, 1024, 1)
    plain = P.srla_footprint_bytes(P.make_config(*geo, max_candidates=1))
    for unit in (8192, 131072):
        cfg = P.make_config(*geo, max_candidates=1, flags=part, scan_blocks=unit)
        assert P.srla_footprint_bytes(cfg) - plain == \
            scratch(256) + 4 * 2048 * ((1 << 26) // unit - 2048)
    for bad in (4096, 12288, 262144):
        assert P.srla_footprint_bytes(P.make_config(*geo, max_candidates=1, flags=part,
                                                    scan_blocks=bad)) == 0
    # beyond 2^32 LE DRs
    big = P.make_config(2, 1024, 2, 4096, 8, (1 << 21) + 3, 1024, 1, max_candidates=1, flags=part)
    assert P.srla_footprint_bytes(big) > 2 * ((1 << 32) + 6144)
    # the discrete form has no LE stamps: the flag has no effect there
    disc = P.make_config(1, 1024, 4, 65536, 8, 65536, 1024, 1, max_candidates=1,
                         flags=part | P.srla.SRLA_CFG_DISCRETE)
    assert P.srla_footprint_bytes(disc) > 0
