// gfx950 scan of the SRLA hot path (Algorithm 2 of arXiv 1803.10369) with a
// workgroup filter of repeated DR stores.  Pairs that repeat a flow, or share
// a source and an LE index, store the same stamp into the same LE DR; on a
// real link (few destinations per source, a heavy-tailed source mix) a large
// share of a slice's stores repeat a DR that the same workgroup stored a
// moment before, and such stores pile onto the same cache lines.  Each
// workgroup keeps in LDS a direct-mapped table of the LE DRs it stored last
// (their flat indices); a lane whose DR is in the table skips the store, any
// other lane stores and records its DR.  The table lives for one launch, and
// every store of a launch writes the same stamp, so a hit always means the
// very same store was issued before: races between lanes (two lanes missing
// together, a slot overwritten) only cost a redundant store, never a lost
// one.  A wavefront-level variant (lanes of one wavefront claiming LDS slots
// for identical addresses) removed only 0.1 % of the writes and was dropped:
// repeats come from different wavefronts of the workgroup, seldom from the
// same round of one wavefront.  Results are identical to the plain form.
#include "srla_scan_filter.h"

namespace srla {

constexpr int kLfSteps = 4;
constexpr uint64_t kLfTile = (uint64_t)kBlock * 2 * kLfSteps;  // pairs per block
constexpr uint32_t kLfBits = 12;
constexpr uint32_t kLfSlots = 1u << kLfBits;                   // 16 KiB of LDS per workgroup
constexpr uint32_t kLfEmpty = 0xFFFFFFFFu;                     // no LE DR has this index

__device__ __forceinline__ uint32_t lf_slot(uint32_t cell) {
  return (cell * 0x9E3779B1u) >> (32 - kLfBits);
}

__device__ __forceinline__ uint32_t le_cell32(const Geo& geo, uint32_t row, uint32_t a,
                                              uint32_t lei) {
  return (row * geo.v_le + hrange(mas(geo.rh[row], a), geo.v_le)) * geo.G + lei;
}

template <int U, bool VEC>
__global__ __launch_bounds__(kBlock) void k_scan_lds_filter(const uint32_t* __restrict__ pairs,
                                                           uint64_t n, Geo geo, uint16_t code,
                                                           uint16_t* __restrict__ le,
                                                           uint16_t* __restrict__ re,
                                                           uint32_t* __restrict__ touched,
                                                           uint32_t* __restrict__ tcount) {
  __shared__ uint32_t tbl[kLfSlots];
  for (uint32_t i = threadIdx.x; i < kLfSlots; i += kBlock) tbl[i] = kLfEmpty;
  __syncthreads();
  const uint32_t nu = U > 0 ? (uint32_t)U : geo.u;
  for (uint64_t base = (uint64_t)blockIdx.x * kLfTile; base < n;
       base += (uint64_t)gridDim.x * kLfTile) {
    uint32_t a[kLfSteps][2], b[kLfSteps][2];
    bool v[kLfSteps][2];
#pragma unroll
    for (int s = 0; s < kLfSteps; ++s) {
      const uint64_t p = base + (uint64_t)s * (2 * kBlock) + 2u * threadIdx.x;
      v[s][0] = p < n;
      v[s][1] = p + 1 < n;
      if (VEC && v[s][1]) {
        const uint4 q = *reinterpret_cast<const uint4*>(pairs + 2 * p);
        a[s][0] = q.x; b[s][0] = q.y; a[s][1] = q.z; b[s][1] = q.w;
      } else {
        a[s][0] = v[s][0] ? pairs[2 * p] : 0u;
        b[s][0] = v[s][0] ? pairs[2 * p + 1] : 0u;
        a[s][1] = v[s][1] ? pairs[2 * p + 2] : 0u;
        b[s][1] = v[s][1] ? pairs[2 * p + 3] : 0u;
      }
    }
#pragma unroll
    for (int s = 0; s < kLfSteps; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t aa = a[s][h], bb = b[s][h];
        const bool valid = v[s][h];
        if (valid) {
          const uint32_t lei = hrange(mas(geo.h3, bb), geo.G);
          if constexpr (U > 0) {
            uint32_t cell[U], seen[U];
#pragma unroll
            for (int i = 0; i < U; ++i) {
              cell[i] = le_cell32(geo, (uint32_t)i, aa, lei);
              seen[i] = tbl[lf_slot(cell[i])];
            }
#pragma unroll
            for (int i = 0; i < U; ++i)
              if (seen[i] != cell[i]) {
                le[cell[i]] = code;
                tbl[lf_slot(cell[i])] = cell[i];
              }
          } else {
            for (uint32_t i = 0; i < nu; ++i) {
              const uint32_t c = le_cell32(geo, i, aa, lei);
              if (tbl[lf_slot(c)] != c) {
                le[c] = code;
                tbl[lf_slot(c)] = c;
              }
            }
          }
        }
        // the SRE half (2^-tau of the pairs) and the wave-aggregated append
        const bool sampled = valid && (mas(geo.h1, bb) & geo.tau_mask) == 0u;
        if (sampled) {
          const uint32_t rei = hrange(mas(geo.h2, bb), geo.g);
          for (uint32_t i = 0; i < nu; ++i)
            re[((uint64_t)i * geo.v_re + hrange(mas(geo.rh[i], aa), geo.v_re)) * geo.g + rei] =
                code;
        }
        const uint64_t mask = __ballot(sampled);
        if (mask != 0ull) {
          const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1u;
          uint32_t at = 0;
          if (__lane_id() == leader) at = atomicAdd(tcount, (uint32_t)__popcll(mask));
          at = __shfl(at, (int)leader);
          if (sampled) touched[at + lane_rank(mask)] = aa;
        }
      }
  }
}

template <int U>
static hipError_t launch_lf_u(const uint32_t* pairs, uint64_t n, const Geo& geo, uint16_t code,
                              uint16_t* le, uint16_t* re, uint32_t* touched, uint32_t* tcount,
                              uint32_t max_blocks, hipStream_t st) {
  uint64_t blocks = (n + kLfTile - 1) / kLfTile;
  if (max_blocks && blocks > max_blocks) blocks = max_blocks;
  if (((uintptr_t)pairs & 15u) == 0)
    hipLaunchKernelGGL((k_scan_lds_filter<U, true>), dim3((uint32_t)blocks), dim3(kBlock), 0, st,
                       pairs, n, geo, code, le, re, touched, tcount);
  else
    hipLaunchKernelGGL((k_scan_lds_filter<U, false>), dim3((uint32_t)blocks), dim3(kBlock), 0,
                       st, pairs, n, geo, code, le, re, touched, tcount);
  return hipGetLastError();
}

hipError_t launch_scan_lds_filter(const uint32_t* pairs, uint64_t n, const Geo& geo,
                                  uint16_t code, uint16_t* le, uint16_t* re, uint32_t* touched,
                                  uint32_t* tcount, uint32_t* claim, uint32_t* slot,
                                  uint32_t max_blocks, hipStream_t st) {
  if (n == 0) return hipSuccess;
  // 32-bit DR indices (and one spare value for an empty slot)
  if ((uint64_t)geo.u * geo.v_le * geo.G >= (uint64_t)kLfEmpty)
    return launch_scan(pairs, n, geo, code, le, re, touched, tcount, claim, slot, false,
                       max_blocks, st);
  switch (geo.u) {
    case 4: return launch_lf_u<4>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
    case 8: return launch_lf_u<8>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
    default: return launch_lf_u<0>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
  }
}

}  // namespace srla
