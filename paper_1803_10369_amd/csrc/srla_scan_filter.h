// Launcher of the scan with a workgroup filter of repeated DR stores; see
// srla_scan_filter.hip.
#pragma once
#include "srla_internal.h"

namespace srla {

// Algorithm 2 for n pairs of the open slice (stamp code `code`); a workgroup
// skips LE stores it has already issued in this launch.  Same arguments and
// results as launch_scan (which it falls back to when the LE has 2^32 DRs or
// more).
hipError_t launch_scan_lds_filter(const uint32_t* pairs, uint64_t n, const Geo& geo,
                                  uint16_t code, uint16_t* le, uint16_t* re, uint32_t* touched,
                                  uint32_t* tcount, uint32_t* claim, uint32_t* slot,
                                  uint32_t max_blocks, hipStream_t st);

}  // namespace srla
