// Launchers of the discrete-window form (k = 1, one-bit DRs); see
// srla_discrete.hip.  The LE bit array is flat over [u][v_le][G], 64 bits per
// word (the stamp form's `bitmap` layout); the SRE bits, flat over
// [u][v_re][g], fill the even words of an array twice that size (the stamp
// form's interleaved `act` layout).
#pragma once
#include "srla_internal.h"

namespace srla {

// Algorithm 2 for n pairs: sets bits of the open slice's LE and SRE bit
// arrays and records sampled sources in the slice's source set (`set_slots`
// 64-bit slots, a power of two), or appends them to `touched` (count in
// *tcount) when the set has no room near their hash
hipError_t launch_scan_bits(const uint32_t* pairs, uint64_t n, const Geo& geo, uint64_t* lebits,
                            uint64_t* rebits, uint64_t* set, uint32_t set_slots,
                            uint32_t* touched, uint32_t* tcount, uint32_t max_blocks,
                            hipStream_t st);

// appends the set's sources to `touched` (count in *tcount) and empties it
hipError_t launch_drain_set(uint64_t* set, uint32_t set_slots, uint32_t* touched,
                            uint32_t* tcount, hipStream_t st);

// |LDR(i)|^k of every row of a LE bit array (rows of v_le*G bits), added
// into row_fill[u]
hipError_t launch_row_popcount(const uint64_t* bits, unsigned long long* row_fill,
                               const Geo& geo, hipStream_t st);

}  // namespace srla
