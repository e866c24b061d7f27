"""SRLA oracle (arXiv 1803.10369, Sections 3-4) -- TEST INFRASTRUCTURE ONLY.

A plain single-threaded C statement of the method (``srla_oracle.c``) behind
ctypes, plus a brute-force checker (``exact``) that pins it.  Only the tests,
the smoke check and the CPU-baseline leg of the bench may import this package;
the GPU library never does, and the two share no code.
"""
import ctypes
import os

import numpy as np

from . import build as _build

_HERE = os.path.dirname(os.path.abspath(__file__))
_lib = None

SUPER, SAT, NEW, KEEP = 1, 2, 4, 8
LE, RE, SI = 0, 1, 2
MAX_U = 16


class _Config(ctypes.Structure):
    _fields_ = [("k", ctypes.c_uint32), ("theta", ctypes.c_uint32),
                ("u", ctypes.c_uint32), ("v_re", ctypes.c_uint32),
                ("g", ctypes.c_uint32), ("v_le", ctypes.c_uint32),
                ("G", ctypes.c_uint32), ("hash_seed", ctypes.c_uint64),
                ("max_candidates", ctypes.c_uint64), ("sequential", ctypes.c_uint32)]


class _Report(ctypes.Structure):
    _fields_ = [("slice", ctypes.c_uint64), ("window_full", ctypes.c_uint32),
                ("n", ctypes.c_uint64),
                ("ip", ctypes.POINTER(ctypes.c_uint32)),
                ("est", ctypes.POINTER(ctypes.c_double)),
                ("flags", ctypes.POINTER(ctypes.c_uint8)),
                ("union_weight", ctypes.POINTER(ctypes.c_uint32)),
                ("re_weight", ctypes.POINTER(ctypes.c_uint8)),
                ("row_fill", ctypes.POINTER(ctypes.c_uint64)),
                ("up", ctypes.c_double), ("n_touched", ctypes.c_uint64),
                ("n_new", ctypes.c_uint64)]


def lib():
    """Loads the oracle library, building it first if it is not there."""
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        u32, u64, p64 = ctypes.c_uint32, ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint64)
        L.orc_splitmix64_next.restype = u64
        L.orc_splitmix64_next.argtypes = [p64]
        L.orc_lsb.restype = u32
        L.orc_lsb.argtypes = [u32]
        L.orc_tau.restype = u32
        L.orc_tau.argtypes = [u32, u32]
        L.orc_sre_threshold.restype = u32
        L.orc_sre_threshold.argtypes = [u32]
        L.orc_rho.restype = ctypes.c_double
        L.orc_rho.argtypes = []
        L.orc_mas.restype = u32
        L.orc_mas.argtypes = [u64, u64, u32]
        L.orc_range.restype = u32
        L.orc_range.argtypes = [u32, u32]
        L.orc_hash_params.restype = None
        L.orc_hash_params.argtypes = [u64, u32, p64, p64]
        L.orc_create.restype = ctypes.c_void_p
        L.orc_create.argtypes = [ctypes.POINTER(_Config)]
        L.orc_scan.restype = ctypes.c_int
        L.orc_scan.argtypes = [ctypes.c_void_p, ctypes.c_void_p, u64]
        L.orc_estimate.restype = ctypes.c_int
        L.orc_estimate.argtypes = [ctypes.c_void_p, ctypes.POINTER(_Report)]
        L.orc_dump.restype = ctypes.c_int
        L.orc_dump.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, u64]
        L.orc_slice.restype = u64
        L.orc_slice.argtypes = [ctypes.c_void_p]
        L.orc_destroy.restype = None
        L.orc_destroy.argtypes = [ctypes.c_void_p]
        _lib = L
    return _lib


# ---------------------------------------------------------------- building blocks

def splitmix64(seed, n):
    st = ctypes.c_uint64(seed)
    return [lib().orc_splitmix64_next(ctypes.byref(st)) for _ in range(n)]


def lsb(x):
    return lib().orc_lsb(x)


def tau(theta, g):
    return lib().orc_tau(theta, g)


def sre_threshold(g):
    return lib().orc_sre_threshold(g)


def rho():
    return lib().orc_rho()


def mas(a, b, x):
    return lib().orc_mas(a, b, x)


def hrange(h, m):
    return lib().orc_range(h, m)


def hash_params(seed, nfun):
    a = (ctypes.c_uint64 * nfun)()
    b = (ctypes.c_uint64 * nfun)()
    lib().orc_hash_params(seed, nfun, a, b)
    return list(a), list(b)


# ---------------------------------------------------------------- monitor

class Report:
    """A copy of one slice's report (numpy arrays)."""

    def __init__(self, r, u):
        n = r.n
        self.slice = r.slice
        self.window_full = bool(r.window_full)
        self.n = n
        self.ip = np.ctypeslib.as_array(r.ip, (n,)).copy() if n else np.zeros(0, np.uint32)
        self.est = np.ctypeslib.as_array(r.est, (n,)).copy() if n else np.zeros(0, np.float64)
        self.flags = np.ctypeslib.as_array(r.flags, (n,)).copy() if n else np.zeros(0, np.uint8)
        self.union_weight = (np.ctypeslib.as_array(r.union_weight, (n,)).copy()
                             if n else np.zeros(0, np.uint32))
        self.re_weight = (np.ctypeslib.as_array(r.re_weight, (n,)).copy()
                          if n else np.zeros(0, np.uint8))
        self.row_fill = np.ctypeslib.as_array(r.row_fill, (u,)).copy()
        self.up = r.up
        self.n_touched = r.n_touched
        self.n_new = r.n_new


class OracleError(RuntimeError):
    def __init__(self, rc):
        super().__init__("oracle call failed with status %d" % rc)
        self.rc = rc


class Monitor:
    """One SRLA monitor: a SEA of u rows, fed slice by slice."""

    def __init__(self, k, theta, u, v_re, g, v_le, G, hash_seed, max_candidates=1 << 26,
                 sequential=False):
        self.cfg = _Config(k, theta, u, v_re, g, v_le, G, hash_seed, max_candidates,
                           int(bool(sequential)))
        self._h = lib().orc_create(ctypes.byref(self.cfg))
        if not self._h:
            raise ValueError("invalid oracle configuration")

    def close(self):
        if self._h:
            lib().orc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def scan(self, pairs):
        """pairs: uint32 array of shape (n, 2) or (2n,), (aip, bip) interleaved."""
        p = np.ascontiguousarray(pairs, dtype=np.uint32).reshape(-1)
        rc = lib().orc_scan(self._h, p.ctypes.data, p.size // 2)
        if rc:
            raise OracleError(rc)

    def estimate(self):
        r = _Report()
        rc = lib().orc_estimate(self._h, ctypes.byref(r))
        if rc:
            raise OracleError(rc)
        return Report(r, self.cfg.u)

    def cells(self, which):
        c = self.cfg
        return {LE: c.u * c.v_le * c.G, RE: c.u * c.v_re * c.g, SI: c.u * c.v_re}[which]

    def dump(self, which):
        n = self.cells(which)
        out = np.empty(n, dtype=np.uint16)
        rc = lib().orc_dump(self._h, which, out.ctypes.data, n)
        if rc:
            raise OracleError(rc)
        return out

    @property
    def slice(self):
        return lib().orc_slice(self._h)
