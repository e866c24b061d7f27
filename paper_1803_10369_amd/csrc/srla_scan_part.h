// Launcher of the partitioned scan; see srla_scan_part.hip.
#pragma once
#include "srla_internal.h"

namespace srla {

// LE regions of the partitioned scan: 2^16 DRs each, so that a DR's offset
// in its region is one uint16.  The LE is taken in bands of at most
// kPartBandRegions regions (2^27 DRs), one partition pass per band.
constexpr uint32_t kPartLog = 16;
constexpr uint32_t kPartBandRegions = 2048;
constexpr uint32_t kPartBandLog = 27;
static_assert((1ull << kPartBandLog) == ((uint64_t)kPartBandRegions << kPartLog), "band size");
// DR indices one chunk of pairs produces, and chunks per partition round
constexpr uint32_t kPartEntries = 32768;
constexpr uint32_t kPartChunks = 2048;
// DR indices per marking unit: a region's marking is cut into
// ceil(indices / unit) units (workgroups), each with its own bitmap; unit is
// a power of two in [kPartUnitMin, kPartUnitMax], kPartUnit by default
constexpr uint32_t kPartUnit = 32768;
constexpr uint32_t kPartUnitMin = 8192;
constexpr uint32_t kPartUnitMax = 131072;
constexpr bool part_unit_ok(uint32_t unit) {
  return unit >= kPartUnitMin && unit <= kPartUnitMax && (unit & (unit - 1)) == 0;
}
// uint32 words of one region's bitmap
constexpr uint32_t kPartRegionWords = (1u << kPartLog) / 32;

// any LE: bands of 2^27 DRs
constexpr uint64_t part_bands(uint64_t n_le) {
  return (n_le + (1ull << kPartBandLog) - 1) >> kPartBandLog;
}
// regions of the largest band
constexpr uint64_t part_band_regions(uint64_t n_le) {
  const uint64_t r = (n_le + (1ull << kPartLog) - 1) >> kPartLog;
  return r < kPartBandRegions ? r : kPartBandRegions;
}
// marking units of one partition round of round_chunks chunks, at most
constexpr uint64_t part_mark_units(uint64_t n_le, uint32_t round_chunks,
                                   uint32_t unit = kPartUnit) {
  return part_band_regions(n_le) + (uint64_t)round_chunks * kPartEntries / unit;
}
// device scratch of the partitioned scan: DR indices (uint16) and region offsets (uint16)
constexpr uint64_t part_entry_words(uint32_t round_chunks = kPartChunks) {
  return (uint64_t)round_chunks * kPartEntries;
}
constexpr uint64_t part_offset_words(uint64_t n_le, uint32_t round_chunks = kPartChunks) {
  return (part_band_regions(n_le) + 1) * round_chunks;
}
// and the marking units' bitmaps after the marking plan (uint32): units per
// region and the regions' first units (rounded to 256 bytes, so that the
// bitmaps start aligned)
constexpr uint64_t part_plan_words(void) { return (2ull * kPartBandRegions + 2 + 63) / 64 * 64; }
constexpr uint64_t part_mark_words(uint64_t n_le, uint32_t round_chunks = kPartChunks,
                                   uint32_t unit = kPartUnit) {
  return part_plan_words() + part_mark_units(n_le, round_chunks, unit) * kPartRegionWords;
}

// Algorithm 2 for n pairs of the open slice (stamp code `code`), the LE
// stores sorted by region before they are issued.  Same results as
// launch_scan.  Device scratch, reused by every launch on the stream:
// entries part_entry_words(round_chunks) and offs
// part_offset_words(n_le, round_chunks) uint16 words, marks
// part_mark_words(n_le, round_chunks, unit) uint32 words, where round_chunks
// (<= kPartChunks) is the number of chunks per partition round (a smaller
// scratch takes the pairs in more rounds) and unit the DR indices per
// marking unit (part_unit_ok).  With ps, the scan's last kernel
// records the end of the scan (the device clock) in ps->t_end[parity].  With sampled, the
// event is recorded on st as soon as every sampled source of the pairs is
// appended (after the first band's last partition kernel), before the
// marking and stamping.
hipError_t launch_scan_partition(const uint32_t* pairs, uint64_t n, const Geo& geo,
                                 uint16_t code, uint16_t* le, uint16_t* re, uint32_t* touched,
                                 uint32_t* tcount, uint16_t* entries, uint16_t* offs,
                                 uint32_t* marks, hipStream_t st,
                                 uint32_t round_chunks = kPartChunks, PipeState* ps = nullptr,
                                 uint32_t parity = 0, uint32_t unit = kPartUnit,
                                 hipEvent_t sampled = nullptr);

}  // namespace srla
