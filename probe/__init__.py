"""Memory-system probes that calibrate the SRLA kernels' ceilings.

``random_store_rate(bytes)`` measures random 2-byte stores per second over a
footprint of ``bytes`` (the scan's access pattern without its pair loads and
hashing); ``random_or_rate(bytes)`` the same for one-bit atomic ORs into
32-bit words (the discrete-window scan's pattern), ``random_load_rate(bytes)``
for random 2-byte loads.  Measurement
infrastructure only; the SRLA library does not use it.
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
        L.probe_two_streams.restype = ctypes.c_double
        L.probe_two_streams.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_double)]
        L.probe_event_order.restype = ctypes.c_double
        L.probe_event_order.argtypes = L.probe_two_streams.argtypes + [ctypes.c_uint32,
                                                                        ctypes.c_uint32]
        L.probe_xcc_of_blocks.restype = ctypes.c_int
        L.probe_xcc_of_blocks.argtypes = [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_void_p]
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


def dma_d2h_rate(nbytes=64 << 20, repeats=3):
    """Best-of-`repeats` bytes/s of a device-to-host copy into pinned memory."""
    import torch
    dev = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    host = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    best = None
    for r in range(repeats + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        host.copy_(dev, non_blocking=True)
        b.record()
        b.synchronize()
        if r > 0:
            ms = a.elapsed_time(b)
            best = ms if best is None else min(best, ms)
    return nbytes / (best * 1e-3)


def two_streams(blocks=512, iters=200_000):
    """(ms of one spin kernel of `blocks` workgroups alone, ms of two such
    kernels on two streams released together): equal when they overlap."""
    import torch
    buf = torch.empty(2 * blocks * 256, dtype=torch.int32, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    both = ctypes.c_double(0.0)
    one = _load().probe_two_streams(ctypes.c_void_p(buf.data_ptr()), blocks, iters,
                                    ctypes.c_void_p(s1.cuda_stream),
                                    ctypes.c_void_p(s2.cuda_stream), ctypes.byref(both))
    if one < 0:
        raise RuntimeError("probe failed (%g)" % one)
    return one, both.value


def event_order(blocks=64, iters=200_000, blocks3=1, iters3=1):
    """(ms from stream 1's first spin to stream 2's kernel that waits for an
    event recorded after that spin, ms of stream 1's two spins)."""
    import torch
    buf = torch.empty((blocks + (blocks3 & 0x7FFFFFFF)) * 256, dtype=torch.int32, device="cuda")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    both = ctypes.c_double(0.0)
    t3 = _load().probe_event_order(ctypes.c_void_p(buf.data_ptr()), blocks, iters,
                                   ctypes.c_void_p(s1.cuda_stream),
                                   ctypes.c_void_p(s2.cuda_stream), ctypes.byref(both),
                                   blocks3, iters3)
    if t3 < 0:
        raise RuntimeError("probe failed (%g)" % t3)
    return t3, both.value


def xcc_of_blocks(blocks=64):
    """The XCD each of `blocks` workgroups of one launch ran on (a list)."""
    import torch
    out = torch.full((blocks,), 0xFF, dtype=torch.int32, device="cuda")
    st = torch.cuda.current_stream()
    if _load().probe_xcc_of_blocks(ctypes.c_void_p(out.data_ptr()), blocks,
                                   ctypes.c_void_p(st.cuda_stream)) != 0:
        raise RuntimeError("probe failed")
    return out.cpu().tolist()


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
