"""ctypes binding of libsrla.so (include/srla.h), argument marshalling only.

Every step of the SRLA path runs in the library's HIP kernels; this module
only converts arguments.  PyTorch is imported first so that the library and
torch share one HIP runtime (device tensors and streams cross the boundary as
raw pointers).  If the library has not been built, loading fails loudly:
there is no CPU fallback.
"""
import ctypes
import os

import numpy as np
import torch  # noqa: F401  (loads the HIP runtime this library links against)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsrla.so")

SRLA_OK, SRLA_E_INVAL, SRLA_E_NOMEM, SRLA_E_CAPACITY, SRLA_E_STATE, SRLA_E_DEVICE = 0, -1, -2, -3, -4, -5
SRLA_DUMP_LE, SRLA_DUMP_RE, SRLA_DUMP_SI = 0, 1, 2
SRLA_FLAG_SUPER, SRLA_FLAG_SAT, SRLA_FLAG_NEW, SRLA_FLAG_KEEP = 1, 2, 4, 8
SRLA_CFG_TIMING = 1
SRLA_TIMING_SCANS = 2   # srla_set_timing: time the scans only
SRLA_CFG_SCAN_XCD = 2
SRLA_CFG_GRAPH = 4
SRLA_CFG_DISCRETE = 8
SRLA_CFG_LEAN_REPORT = 16
SRLA_CFG_SCAN_DEDUP = 32
SRLA_CFG_SCAN_LDS_FILTER = 64
SRLA_CFG_OVERLAP_REPORT = 128
SRLA_CFG_SCAN_PARTITION = 256
SRLA_CFG_HOLD_SCANS = 1024


class srla_geometry_t(ctypes.Structure):
    _fields_ = [("u", ctypes.c_uint32), ("v_re", ctypes.c_uint32), ("g", ctypes.c_uint32),
                ("v_le", ctypes.c_uint32), ("g_le", ctypes.c_uint32),
                ("hash_seed", ctypes.c_uint64)]


class srla_config_t(ctypes.Structure):
    _fields_ = [("window_slices", ctypes.c_uint32), ("threshold", ctypes.c_uint32),
                ("geom", srla_geometry_t), ("max_candidates", ctypes.c_uint64),
                ("flags", ctypes.c_uint32), ("scan_blocks", ctypes.c_uint32)]


class srla_report_t(ctypes.Structure):
    _fields_ = [("slice", ctypes.c_uint64), ("window_full", ctypes.c_uint32),
                ("n", ctypes.c_uint64),
                ("ip", ctypes.POINTER(ctypes.c_uint32)),
                ("est", ctypes.POINTER(ctypes.c_double)),
                ("flags", ctypes.POINTER(ctypes.c_uint8)),
                ("union_weight", ctypes.POINTER(ctypes.c_uint32)),
                ("re_weight", ctypes.POINTER(ctypes.c_uint8)),
                ("row_fill", ctypes.POINTER(ctypes.c_uint64)),
                ("up", ctypes.c_double), ("n_touched", ctypes.c_uint64),
                ("n_new", ctypes.c_uint64), ("latency_ms", ctypes.c_double),
                ("host_bytes", ctypes.c_uint64)]


class srla_timings_t(ctypes.Structure):
    _fields_ = [("scan_ms", ctypes.c_double), ("scan_launches", ctypes.c_uint64),
                ("scan_pairs", ctypes.c_uint64), ("sweep_ms", ctypes.c_double),
                ("finalize_ms", ctypes.c_double), ("estimate_ms", ctypes.c_double),
                ("slide_ms", ctypes.c_double), ("report_ms", ctypes.c_double),
                ("estimates", ctypes.c_uint64)]


EXPORTS = ["srla_footprint_bytes", "srla_create", "srla_scan", "srla_scan_noalloc", "srla_estimate",
           "srla_close_slice", "srla_wait_report", "srla_dump_state", "srla_timings",
           "srla_set_timing", "srla_destroy", "srla_last_error", "srla_group_create", "srla_group_scan",
           "srla_group_destroy", "srla_group_last_error", "srla_admit"]

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libsrla.so is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        vp = ctypes.c_void_p
        L.srla_footprint_bytes.restype = ctypes.c_uint64
        L.srla_footprint_bytes.argtypes = [ctypes.POINTER(srla_config_t)]
        L.srla_create.restype = ctypes.c_int
        L.srla_create.argtypes = [ctypes.POINTER(srla_config_t), vp, ctypes.POINTER(vp)]
        L.srla_scan.restype = ctypes.c_int
        L.srla_scan.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_int]
        L.srla_scan_noalloc.restype = ctypes.c_int
        L.srla_scan_noalloc.argtypes = [vp, vp, ctypes.c_uint64]
        L.srla_estimate.restype = ctypes.c_int
        L.srla_estimate.argtypes = [vp, ctypes.POINTER(srla_report_t)]
        L.srla_close_slice.restype = ctypes.c_int
        L.srla_close_slice.argtypes = [vp]
        L.srla_wait_report.restype = ctypes.c_int
        L.srla_wait_report.argtypes = [vp, ctypes.POINTER(srla_report_t)]
        L.srla_dump_state.restype = ctypes.c_int
        L.srla_dump_state.argtypes = [vp, ctypes.c_int, vp, ctypes.c_uint64]
        L.srla_timings.restype = ctypes.c_int
        L.srla_timings.argtypes = [vp, ctypes.POINTER(srla_timings_t), ctypes.c_int]
        L.srla_set_timing.restype = ctypes.c_int
        L.srla_set_timing.argtypes = [vp, ctypes.c_int]
        L.srla_destroy.restype = ctypes.c_int
        L.srla_destroy.argtypes = [vp]
        L.srla_last_error.restype = ctypes.c_char_p
        L.srla_last_error.argtypes = [vp]
        L.srla_group_create.restype = ctypes.c_int
        L.srla_group_create.argtypes = [ctypes.POINTER(vp), ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.POINTER(vp)]
        L.srla_group_scan.restype = ctypes.c_int
        L.srla_group_scan.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_int]
        L.srla_group_destroy.restype = ctypes.c_int
        L.srla_group_destroy.argtypes = [vp]
        L.srla_group_last_error.restype = ctypes.c_char_p
        L.srla_group_last_error.argtypes = [vp]
        L.srla_admit.restype = ctypes.c_int
        L.srla_admit.argtypes = [ctypes.POINTER(srla_config_t), ctypes.c_uint32, ctypes.c_uint64,
                                 ctypes.POINTER(ctypes.c_uint8), ctypes.POINTER(ctypes.c_uint64)]
        _lib = L
    return _lib


# ---------------------------------------------------------------- C names

def make_config(k, theta, u, v_re, g, v_le, G, hash_seed, max_candidates=1 << 22, flags=0,
                scan_blocks=0):
    return srla_config_t(k, theta, srla_geometry_t(u, v_re, g, v_le, G, hash_seed),
                         max_candidates, flags, scan_blocks)


def srla_footprint_bytes(cfg):
    return lib().srla_footprint_bytes(ctypes.byref(cfg))


def srla_create(cfg, hip_stream=None):
    """Returns (status, handle)."""
    h = ctypes.c_void_p()
    rc = lib().srla_create(ctypes.byref(cfg), hip_stream, ctypes.byref(h))
    return rc, h


def srla_scan(handle, pairs_ptr, n, on_device):
    return lib().srla_scan(handle, pairs_ptr, n, int(on_device))


def srla_scan_noalloc(handle, pairs_ptr, n):
    return lib().srla_scan_noalloc(handle, pairs_ptr, n)


def srla_estimate(handle, report):
    return lib().srla_estimate(handle, ctypes.byref(report))


def srla_close_slice(handle):
    return lib().srla_close_slice(handle)


def srla_wait_report(handle, report):
    return lib().srla_wait_report(handle, ctypes.byref(report))


def srla_dump_state(handle, which, out_ptr, cells):
    return lib().srla_dump_state(handle, which, out_ptr, cells)


def srla_set_timing(handle, enabled):
    return lib().srla_set_timing(handle, int(enabled))


def srla_timings(handle, out, reset):
    return lib().srla_timings(handle, ctypes.byref(out), int(reset))


def srla_destroy(handle):
    return lib().srla_destroy(handle)


def srla_last_error(handle):
    s = lib().srla_last_error(handle)
    return s.decode() if s else ""


def srla_group_create(handles, scan_blocks=0):
    """Returns (status, group handle)."""
    arr = (ctypes.c_void_p * len(handles))(*[h.value for h in handles])
    g = ctypes.c_void_p()
    rc = lib().srla_group_create(arr, len(handles), scan_blocks, ctypes.byref(g))
    return rc, g


def srla_group_scan(group, pairs_ptr, n, on_device):
    return lib().srla_group_scan(group, pairs_ptr, n, int(on_device))


def srla_group_destroy(group):
    return lib().srla_group_destroy(group)


def srla_group_last_error(group):
    s = lib().srla_group_last_error(group)
    return s.decode() if s else ""


def srla_admit(cfgs, budget_bytes):
    """Returns (status, admitted flags, used bytes) for a list of srla_config_t."""
    arr = (srla_config_t * len(cfgs))(*cfgs)
    flags = (ctypes.c_uint8 * len(cfgs))()
    used = ctypes.c_uint64()
    rc = lib().srla_admit(arr, len(cfgs), budget_bytes, flags, ctypes.byref(used))
    return rc, [bool(x) for x in flags], used.value


# ---------------------------------------------------------------- convenience

class SrlaError(RuntimeError):
    def __init__(self, rc, msg):
        super().__init__("srla status %d: %s" % (rc, msg))
        self.rc = rc


class Report:
    """One slice's report as numpy arrays: copies, or (copy=False) views of the
    library's report buffers, which stay valid until the slice two after this
    one is closed."""

    def __init__(self, r, u, copy=True):
        n = r.n

        def arr(p, dt):
            if not p:
                return None          # left out of a lean report
            if not n:
                return np.zeros(0, dt)
            a = np.ctypeslib.as_array(p, (n,))
            return a.copy() if copy else a

        self.slice = r.slice
        self.window_full = bool(r.window_full)
        self.n = n
        self.ip = arr(r.ip, np.uint32)
        self.est = arr(r.est, np.float64)
        self.flags = arr(r.flags, np.uint8)
        self.union_weight = arr(r.union_weight, np.uint32)
        self.re_weight = arr(r.re_weight, np.uint8)
        self.row_fill = np.ctypeslib.as_array(r.row_fill, (u,)).copy()
        self.up = r.up
        self.n_touched = r.n_touched
        self.n_new = r.n_new
        self.latency_ms = r.latency_ms
        self.host_bytes = r.host_bytes


class Monitor:
    """One SRLA monitor on the current HIP device.

    stream: the torch.cuda.Stream the monitor's work is issued on (a new
    stream when None).  Device tensors handed to scan() are ordered after the
    caller's current stream and kept alive for the monitor's stream."""

    def __init__(self, k, theta, u, v_re, g, v_le, G, hash_seed, max_candidates=1 << 22,
                 timing=False, stream=None, scan_xcd=False, graph=False, scan_blocks=0,
                 discrete=False, lean_report=False, scan_dedup=False, scan_lds_filter=False,
                 overlap_report=False, scan_partition=False, hold_scans=False):
        flags = ((SRLA_CFG_TIMING if timing else 0) | (SRLA_CFG_SCAN_XCD if scan_xcd else 0) |
                 (SRLA_CFG_GRAPH if graph else 0) | (SRLA_CFG_DISCRETE if discrete else 0) |
                 (SRLA_CFG_LEAN_REPORT if lean_report else 0) |
                 (SRLA_CFG_SCAN_DEDUP if scan_dedup else 0) |
                 (SRLA_CFG_SCAN_LDS_FILTER if scan_lds_filter else 0) |
                 (SRLA_CFG_OVERLAP_REPORT if overlap_report else 0) |
                 (SRLA_CFG_SCAN_PARTITION if scan_partition else 0) |
                 (SRLA_CFG_HOLD_SCANS if hold_scans else 0))
        self.cfg = make_config(k, theta, u, v_re, g, v_le, G, hash_seed, max_candidates, flags,
                               scan_blocks)
        self._h = None
        self.stream = stream if stream is not None else torch.cuda.Stream()
        rc, h = srla_create(self.cfg, ctypes.c_void_p(self.stream.cuda_stream))
        if rc != SRLA_OK:
            raise SrlaError(rc, "srla_create failed")
        self._h = h

    def _check(self, rc):
        if rc != SRLA_OK:
            raise SrlaError(rc, srla_last_error(self._h))

    def close(self):
        if getattr(self, "_h", None):
            srla_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def scan(self, pairs):
        """pairs: torch uint32/int32 CUDA tensor or numpy uint32 array, 2n values
        (aip, bip interleaved) or shape (n, 2)."""
        if isinstance(pairs, torch.Tensor):
            if not pairs.is_cuda:
                pairs = pairs.numpy()
            else:
                assert pairs.is_contiguous() and pairs.element_size() == 4
                n = pairs.numel() // 2
                cur = torch.cuda.current_stream()
                if cur != self.stream:
                    self.stream.wait_stream(cur)
                    pairs.record_stream(self.stream)
                self._check(srla_scan(self._h, ctypes.c_void_p(pairs.data_ptr()), n, True))
                return
        p = np.asarray(pairs)
        if p.dtype == np.int32:
            p = p.view(np.uint32)          # no copy: pinned buffers stay pinned
        p = np.ascontiguousarray(p, dtype=np.uint32).reshape(-1)
        self._check(srla_scan(self._h, ctypes.c_void_p(p.ctypes.data), p.size // 2, False))

    def estimate(self, copy=True):
        r = srla_report_t()
        self._check(srla_estimate(self._h, r))
        return Report(r, self.cfg.geom.u, copy)

    def close_slice(self):
        """Closes the open slice without waiting (see srla_close_slice)."""
        self._check(srla_close_slice(self._h))

    def wait_report(self, copy=True):
        """The report of the slice closed by close_slice()."""
        r = srla_report_t()
        self._check(srla_wait_report(self._h, r))
        return Report(r, self.cfg.geom.u, copy)

    def cells(self, which):
        g = self.cfg.geom
        return {SRLA_DUMP_LE: g.u * g.v_le * g.g_le, SRLA_DUMP_RE: g.u * g.v_re * g.g,
                SRLA_DUMP_SI: g.u * g.v_re}[which]

    def dump(self, which):
        n = self.cells(which)
        out = np.empty(n, dtype=np.uint16)
        self._check(srla_dump_state(self._h, which, ctypes.c_void_p(out.ctypes.data), n))
        return out

    def set_timing(self, enabled):
        """Times the following scans and closed slices (True), the scans only
        (SRLA_TIMING_SCANS), or nothing (False)."""
        self._check(srla_set_timing(self._h, int(enabled)))

    def timings(self, reset=False):
        t = srla_timings_t()
        self._check(srla_timings(self._h, t, reset))
        return {f: getattr(t, f) for f, _ in srla_timings_t._fields_}

    @property
    def footprint_bytes(self):
        return srla_footprint_bytes(self.cfg)


class Group:
    """Monitors fed one pair stream through the fused scan kernel.  All
    members must share one stream; pass it to every Monitor."""

    def __init__(self, monitors, scan_blocks=0):
        self.monitors = list(monitors)
        self.stream = self.monitors[0].stream
        rc, g = srla_group_create([m._h for m in self.monitors], scan_blocks)
        if rc != SRLA_OK:
            raise SrlaError(rc, "srla_group_create failed")
        self._g = g

    def scan(self, pairs):
        """pairs: a contiguous 32-bit CUDA tensor of 2n values (aip, bip)."""
        assert isinstance(pairs, torch.Tensor) and pairs.is_cuda and pairs.is_contiguous()
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            self.stream.wait_stream(cur)
            pairs.record_stream(self.stream)
        rc = srla_group_scan(self._g, ctypes.c_void_p(pairs.data_ptr()), pairs.numel() // 2, True)
        if rc != SRLA_OK:
            raise SrlaError(rc, srla_group_last_error(self._g))

    def close(self):
        if getattr(self, "_g", None):
            srla_group_destroy(self._g)
            self._g = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
