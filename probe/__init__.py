"""Memory-system probes that calibrate the SRLA kernels' ceilings.

``random_store_rate(bytes)`` measures random 2-byte stores per second over a
footprint of ``bytes`` (the flat scan's access pattern without its pair loads
and hashing); ``random_or_rate(bytes)`` the same for one-bit atomic ORs into
32-bit words (the discrete-window scan's pattern), ``random_load_rate(bytes)``
for random 2-byte loads.  ``stream_read_rate(bytes)`` and
``stream_copy_rate(bytes)`` measure streaming 16-byte reads (and copies) over
``bytes`` (the sweeps' and the partitioned scan's pattern), and
``host_write_rate`` coalesced kernel stores into pinned host memory (the
report's path over PCIe).  Measurement infrastructure only; the SRLA library
does not use it.
"""
import ctypes
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libprobe.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
_lib = None


def build():
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           os.path.join(HERE, "random_store.hip"), "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("probe build failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


def _load():
    global _lib
    if _lib is None:
        import torch  # noqa: F401  (shares torch's HIP runtime)
        if not os.path.exists(LIB):
            raise RuntimeError("libprobe.so is not built")
        L = ctypes.CDLL(LIB)
        L.probe_random_store.restype = ctypes.c_double
        L.probe_random_store.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                         ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p]
        L.probe_random_or.restype = ctypes.c_double
        L.probe_random_or.argtypes = L.probe_random_store.argtypes
        L.probe_host_write.restype = ctypes.c_double
        L.probe_host_write.argtypes = [ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                                       ctypes.c_void_p]
        L.probe_stream.restype = ctypes.c_double
        L.probe_stream.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                                   ctypes.c_uint32, ctypes.c_void_p, ctypes.c_void_p]
        L.probe_random_load.restype = ctypes.c_double
        L.probe_random_load.argtypes = L.probe_random_store.argtypes
        _lib = L
    return _lib


def random_store_rate(nbytes, stores=1 << 27, repeats=3):
    """Best-of-`repeats` random 2-byte stores per second over `nbytes`."""
    return _rate("probe_random_store", nbytes, stores, repeats)


def random_or_rate(nbytes, ops=1 << 27, repeats=3):
    """Best-of-`repeats` random one-bit atomic ORs per second over `nbytes`."""
    return _rate("probe_random_or", nbytes, ops, repeats)


def host_write_rate(nbytes=64 << 20, blocks=2048, repeats=3):
    """Best-of-`repeats` bytes/s of a kernel's coalesced stores into pinned host
    memory (through its device-visible address)."""
    import torch
    L = _load()
    host = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    st = torch.cuda.current_stream()
    best = None
    for r in range(repeats + 1):
        ms = L.probe_host_write(ctypes.c_void_p(host.data_ptr()), nbytes, blocks,
                                ctypes.c_void_p(st.cuda_stream))
        if ms <= 0:
            raise RuntimeError("probe failed (%g)" % ms)
        if r > 0:
            best = ms if best is None else min(best, ms)
    return nbytes / (best * 1e-3)


def random_load_rate(nbytes, loads=1 << 27, repeats=3):
    """Best-of-`repeats` random 2-byte loads per second over `nbytes`."""
    return _rate("probe_random_load", nbytes, loads, repeats)


def _rate(fn, nbytes, stores, repeats):
    import torch
    L = _load()
    buf = torch.zeros(max(nbytes, 4) // 4, dtype=torch.int32, device="cuda")
    per_lane = 64
    blocks = max(1, stores // (256 * per_lane))
    st = torch.cuda.current_stream()
    best = None
    for r in range(repeats + 1):
        ms = getattr(L, fn)(ctypes.c_void_p(buf.data_ptr()), buf.numel() * 4, blocks,
                            per_lane, 1234 + r, ctypes.c_void_p(st.cuda_stream))
        if ms <= 0:
            raise RuntimeError("probe failed (%g)" % ms)
        if r > 0:   # the first launch warms the footprint
            best = ms if best is None else min(best, ms)
    del buf
    return blocks * 256 * per_lane / (best * 1e-3)


def _stream(nbytes, copy, repeats, blocks):
    import torch
    L = _load()
    n = max(16, nbytes // 16 * 16)
    src = torch.zeros(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty(n, dtype=torch.uint8, device="cuda") if copy else None
    sink = torch.zeros(4, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream()
    best = None
    for r in range(repeats + 1):
        ms = L.probe_stream(ctypes.c_void_p(src.data_ptr()),
                            ctypes.c_void_p(dst.data_ptr()) if copy else None, n, blocks,
                            ctypes.c_void_p(sink.data_ptr()), ctypes.c_void_p(st.cuda_stream))
        if ms <= 0:
            raise RuntimeError("probe failed (%g)" % ms)
        if r > 0:   # the first launch warms the footprint
            best = ms if best is None else min(best, ms)
    del src, dst, sink
    return n * (2 if copy else 1) / (best * 1e-3)


def stream_read_rate(nbytes, repeats=5, blocks=4096):
    """Best-of-`repeats` bytes/s of streaming 16-byte reads over `nbytes`
    (a footprint up to the 256 MB last-level cache stays resident in it
    between repeats)."""
    return _stream(nbytes, False, repeats, blocks)


def stream_copy_rate(nbytes, repeats=5, blocks=4096):
    """Best-of-`repeats` bytes/s (read + written) of a streaming copy of
    `nbytes` into a second buffer of the same size."""
    return _stream(nbytes, True, repeats, blocks)
