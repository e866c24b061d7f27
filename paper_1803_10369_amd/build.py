"""Builds libsrla.so (the C-ABI library of include/srla.h) for gfx950 with hipcc.

Every call compiles; the library is written in-tree next to this file.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsrla.so")
SOURCES = ["srla_runtime.hip", "srla_scan.hip", "srla_kernels.hip", "srla_sort.hip",
           "srla_discrete.hip", "srla_scan_dedup.hip", "srla_scan_filter.hip",
           "srla_scan_part.hip", "srla_noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# -ffp-contract=off keeps Eq8/Eq9 operation by operation (no fused
# multiply-add), so the FP64 estimate follows the same rounding steps as a
# plain IEEE evaluation; packed FP32 instructions are disabled.
FLAGS = ["-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wall", "-Wno-unused-result"]


def build(verbose=False, extra_flags=()):
    objs = []
    os.makedirs(os.path.join(HERE, "_build"), exist_ok=True)
    for s in SOURCES:
        src = os.path.join(CSRC, s)
        obj = os.path.join(HERE, "_build", s.replace(".hip", ".o"))
        cmd = [HIPCC, *FLAGS, *extra_flags, "-I", os.path.join(ROOT, "include"),
               "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs.append(obj)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
