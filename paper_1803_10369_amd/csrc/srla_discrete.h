// Launchers of the discrete-window form (k = 1, one-bit DRs); see
// srla_discrete.hip.  The bit arrays are flat over [u][v_le][G] (LE) and
// [u][v_re][g] (SRE), 64 bits per word -- the layouts of the stamp form's
// `bitmap` and `act_now`.
#pragma once
#include "srla_internal.h"

namespace srla {

// Algorithm 2 for n pairs: sets bits of the open slice's LE and SRE bit
// arrays and appends sampled sources to `touched` (count in *tcount)
hipError_t launch_scan_bits(const uint32_t* pairs, uint64_t n, const Geo& geo, uint64_t* lebits,
                            uint64_t* rebits, uint32_t* touched, uint32_t* tcount,
                            uint32_t max_blocks, hipStream_t st);

// |LDR(i)|^k of every row of a LE bit array (rows of v_le*G bits), added
// into row_fill[u]
hipError_t launch_row_popcount(const uint64_t* bits, unsigned long long* row_fill,
                               const Geo& geo, hipStream_t st);

}  // namespace srla
