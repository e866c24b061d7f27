"""Device twin of the stream generator: fills torch CUDA tensors with the same
pairs ``StreamSpec.slice`` returns on the host."""
import ctypes
import os

import numpy as np
import torch

from .build import LIB

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError("libtrafficgen.so is not built")
        L = ctypes.CDLL(LIB)
        u64, u32, vp = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p
        L.tg_generate.restype = ctypes.c_int
        L.tg_generate.argtypes = [vp, u64, u64, u64, u64, u64, vp, u32, vp, vp, vp, u32, u32, u32,
                                  vp]
        _lib = L
    return _lib


class DeviceStream:
    """Holds a StreamSpec's tables on the device and generates slices there."""

    def __init__(self, spec, device="cuda"):
        self.spec = spec
        self.device = device
        self.thr = torch.from_numpy(spec.thr.view(np.int64)).to(device)
        P = len(spec.planted)
        self.P = P
        if P:
            self.off = torch.from_numpy(spec.off.astype(np.uint32).view(np.int32)).to(device)
            self.mp = torch.from_numpy(np.asarray(spec.m, np.uint32).view(np.int32)).to(device)
            self.dp = torch.from_numpy(np.asarray(spec.planted, np.uint32).view(np.int32)).to(device)
        else:
            self.off = self.mp = self.dp = None

    def generate(self, s, out=None, stream=None):
        """Pairs of slice s as an int32 CUDA tensor of 2n values (aip, bip)."""
        n = self.spec.n_pairs
        if out is None:
            out = torch.empty(2 * n, dtype=torch.int32, device=self.device)
        assert out.numel() >= 2 * n and out.is_contiguous()
        a, b = self.spec.perm(s)
        st = stream if stream is not None else torch.cuda.current_stream()
        rc = _load().tg_generate(
            ctypes.c_void_p(out.data_ptr()), n, s, self.spec.seed, a, b,
            ctypes.c_void_p(self.thr.data_ptr()), self.spec.n_ranks,
            ctypes.c_void_p(self.off.data_ptr()) if self.P else None,
            ctypes.c_void_p(self.mp.data_ptr()) if self.P else None,
            ctypes.c_void_p(self.dp.data_ptr()) if self.P else None,
            self.P, self.spec.pool_key, self.spec.dst_pool, ctypes.c_void_p(st.cuda_stream))
        if rc != 0:
            raise RuntimeError("tg_generate failed with %d" % rc)
        return out
