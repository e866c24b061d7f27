// The fixed device scratch of the allocation-free scan; see srla_noalloc.hip.
#pragma once
#include "srla_scan_part.h"

namespace srla {

// Partition rounds of kNoAllocChunks chunks and kNoAllocSplit marking
// workgroups per region: DR indices kNoAllocChunks * kPartEntries uint16
// (8 MiB), region offsets (regions + 1) * kNoAllocChunks uint16 (at most
// 257 KiB), marking bitmaps regions * kNoAllocSplit * 4 KiB (at most 16 MiB
// for the 1024 regions of a 2^25-DR LE).
constexpr uint32_t kNoAllocChunks = 128;
constexpr uint32_t kNoAllocSplit = 4;
constexpr uint64_t kNoAllocEntryBytes = (uint64_t)kNoAllocChunks * kPartEntries * 2;
constexpr uint64_t kNoAllocMarkBytes = (uint64_t)kPartMaxRegions * kNoAllocSplit * 4096;
constexpr uint64_t kNoAllocOffsBytes = ((uint64_t)(kPartMaxRegions + 1) * kNoAllocChunks * 2 +
                                        255) / 256 * 256;
constexpr uint64_t kNoAllocScratchBytes = kNoAllocEntryBytes + kNoAllocMarkBytes +
                                          kNoAllocOffsBytes;

// Looks up the scratch array's address on `device` (which must be current)
// and keeps it; later calls for the same device do nothing.
hipError_t noalloc_setup(int device);
// The scratch's device address on `device`, or nullptr before noalloc_setup.
void* noalloc_scratch(int device);

}  // namespace srla
