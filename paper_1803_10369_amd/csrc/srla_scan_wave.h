// Launcher of the wave-deduplicating form of the scan; see srla_scan_wave.hip.
#pragma once
#include "srla_internal.h"

namespace srla {

// Algorithm 2 for n pairs of the open slice (stamp code `code`); within each
// wavefront, of several lanes that would store the same LE DR only one
// stores.  Same arguments and results as launch_scan.
hipError_t launch_scan_wave_dedup(const uint32_t* pairs, uint64_t n, const Geo& geo,
                                  uint16_t code, uint16_t* le, uint16_t* re, uint32_t* touched,
                                  uint32_t* tcount, uint32_t max_blocks, hipStream_t st);

}  // namespace srla
