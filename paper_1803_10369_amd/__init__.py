"""SRLA sliding super-point cardinality estimation on MI355X (gfx950).

The hot path -- Algorithm 2's scan of (aip, bip) pairs into the SEA's
distance recorders and the end-of-slice candidate check, Eq8-Eq9 estimate and
Algorithm 3 slide of arXiv 1803.10369 -- runs in the HIP kernels of
``libsrla.so`` behind the C ABI of ``include/srla.h``; ``srla`` is its
ctypes binding.
"""
from .srla import (Monitor, Report, SrlaError, Group, srla_group_create, srla_group_scan,
                   srla_group_destroy, srla_group_last_error, srla_admit, make_config, srla_create, srla_destroy,  # noqa: F401
                   srla_close_slice, srla_wait_report,
                   srla_dump_state, srla_estimate, srla_footprint_bytes, srla_last_error,
                   srla_scan, srla_scan_noalloc, srla_timings, SRLA_DUMP_LE, SRLA_DUMP_RE, SRLA_DUMP_SI,
                   SRLA_FLAG_SUPER, SRLA_FLAG_SAT, SRLA_FLAG_NEW, SRLA_FLAG_KEEP, EXPORTS,
                   SRLA_OK, SRLA_E_INVAL, SRLA_E_CAPACITY, SRLA_E_STATE, SRLA_TIMING_SCANS)
