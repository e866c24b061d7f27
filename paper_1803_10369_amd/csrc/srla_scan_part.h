// Launcher of the partitioned scan; see srla_scan_part.hip.
#pragma once
#include "srla_internal.h"

namespace srla {

// LE regions of the partitioned scan: 2^15 DRs each, at most 1024 of them
constexpr uint32_t kPartLog = 15;
constexpr uint32_t kPartMaxRegions = 1024;
// DR indices one chunk of pairs produces, and chunks per partition round
constexpr uint32_t kPartEntries = 32768;
constexpr uint32_t kPartChunks = 2048;
// workgroups that share one region's marking
constexpr uint32_t kPartSplit = 16;

// whether a monitor with n_le LE DRs can use the partitioned scan
inline bool part_scan_fits(uint64_t n_le) {
  return n_le <= (uint64_t)kPartMaxRegions << kPartLog;
}
// device scratch of the partitioned scan: DR indices (uint16) and region offsets (uint16)
inline uint64_t part_entry_words(void) { return (uint64_t)kPartChunks * kPartEntries; }
inline uint64_t part_regions(uint64_t n_le) { return (n_le + (1ull << kPartLog) - 1) >> kPartLog; }
inline uint64_t part_offset_words(uint64_t n_le) {
  return part_regions(n_le) * kPartChunks + kPartChunks;
}
// and the marking bitmaps (uint32)
inline uint64_t part_mark_words(uint64_t n_le) {
  return part_regions(n_le) * kPartSplit * ((1ull << kPartLog) / 32);
}

// Algorithm 2 for n pairs of the open slice (stamp code `code`), the LE
// stores sorted by region before they are issued.  Same results as
// launch_scan.  entries / offs: part_entry_words() and
// part_offset_words(n_le) uint16 words, marks: part_mark_words(n_le) uint32
// words of device scratch, reused by every launch on the stream.  A smaller
// scratch serves fewer chunks per partition round (round_chunks <=
// kPartChunks: round_chunks * kPartEntries entry words and (regions + 1) *
// round_chunks offset words) and fewer marking workgroups per region (split
// <= kPartSplit: regions * split * 1024 mark words).  With ps, the last
// workgroup of the scan's last kernel records the end of the scan (the
// device clock) in ps->t_scan[parity].
hipError_t launch_scan_partition(const uint32_t* pairs, uint64_t n, const Geo& geo,
                                 uint16_t code, uint16_t* le, uint16_t* re, uint32_t* touched,
                                 uint32_t* tcount, uint16_t* entries, uint16_t* offs,
                                 uint32_t* marks, hipStream_t st,
                                 uint32_t round_chunks = kPartChunks,
                                 uint32_t split = kPartSplit, PipeState* ps = nullptr,
                                 uint32_t parity = 0);

}  // namespace srla
