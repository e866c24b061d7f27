// Launcher of the read-before-write form of the scan; see srla_scan_dedup.hip.
#pragma once
#include "srla_internal.h"

namespace srla {

// Algorithm 2 for n pairs of the open slice (stamp code `code`), storing a
// stamp only where the DR does not hold it yet; same arguments and results
// as launch_scan.  xcd_aware: each XCD reads and stamps only its own rows
// (u in {1, 2, 4, 8, 16} and 16-byte aligned pairs; otherwise ignored).
hipError_t launch_scan_dedup(const uint32_t* pairs, uint64_t n, const Geo& geo, uint16_t code,
                             uint16_t* le, uint16_t* re, uint32_t* touched, uint32_t* tcount,
                             bool xcd_aware, uint32_t max_blocks, hipStream_t st);

}  // namespace srla
