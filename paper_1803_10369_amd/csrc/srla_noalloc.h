// The fixed device scratch of the allocation-free scan; see srla_noalloc.hip.
#pragma once
#include "srla_scan_part.h"

namespace srla {

// Partition rounds of kNoAllocChunks chunks: DR indices kNoAllocChunks *
// kPartEntries uint16 (8 MiB), region offsets (band regions + 1) *
// kNoAllocChunks uint16 (at most 512.3 KiB), the marking plan and unit
// bitmaps (at most 2048 + 128 units of 8 KiB: 17 MiB); 25.5 MiB in all, for
// an LE of any size.
constexpr uint32_t kNoAllocChunks = 128;
constexpr uint64_t kNoAllocLe = (uint64_t)kPartBandRegions << kPartLog;   // a full band
constexpr uint64_t kNoAllocEntryBytes = part_entry_words(kNoAllocChunks) * 2;
constexpr uint64_t kNoAllocMarkBytes = part_mark_words(kNoAllocLe, kNoAllocChunks) * 4;
constexpr uint64_t kNoAllocOffsBytes =
    (part_offset_words(kNoAllocLe, kNoAllocChunks) * 2 + 255) / 256 * 256;
constexpr uint64_t kNoAllocScratchBytes = kNoAllocEntryBytes + kNoAllocMarkBytes +
                                          kNoAllocOffsBytes;

// Looks up the scratch array's address on `device` (which must be current)
// and keeps it; later calls for the same device do nothing.
hipError_t noalloc_setup(int device);
// The scratch's device address on `device`, or nullptr before noalloc_setup.
void* noalloc_scratch(int device);

}  // namespace srla
