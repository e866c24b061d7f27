// gfx950 scan of the SRLA hot path (Algorithm 2 of arXiv 1803.10369), in the
// read-before-write form.  Within a slice most LE DRs are set many times (a
// slice of the backbone-shaped workload sets each LE DR of a row about four
// times; every repeat of a flow sets the same DRs again).  DRset of the stamp
// form is idempotent, so a DR that already holds the open slice's stamp needs
// no store.  This form first loads every DR a thread's pairs touch, then
// stores only the stamps that differ: it trades one random 2-byte load per
// (pair, row) for the stores of all repeats.  Which form is faster depends on
// the repeat rate and on the footprint (the loads miss the L2 as the stores
// do); the autotuner times both.  Results are identical to the plain form.
#include "srla_scan_dedup.h"

namespace srla {

constexpr int kDedupSteps = 4;
constexpr uint64_t kDedupTile = (uint64_t)kBlock * 2 * kDedupSteps;  // pairs per block

__device__ __forceinline__ uint32_t peek16(const uint16_t* __restrict__ p, uint64_t i) {
  return __hip_atomic_load(p + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

__device__ __forceinline__ uint64_t le_cell(const Geo& geo, uint32_t row, uint32_t a,
                                            uint32_t lei) {
  return ((uint64_t)row * geo.v_le + hrange(mas(geo.rh[row], a), geo.v_le)) * geo.G + lei;
}

// the SRE half (2^-tau of the pairs) and the wave-aggregated append
__device__ __forceinline__ void sample_stamp(uint32_t a, uint32_t b, bool valid, const Geo& geo,
                                             uint16_t code, uint16_t* __restrict__ re,
                                             uint32_t* __restrict__ touched,
                                             uint32_t* __restrict__ tcount) {
  const bool sampled = valid && (mas(geo.h1, b) & geo.tau_mask) == 0u;
  if (sampled) {
    const uint32_t rei = hrange(mas(geo.h2, b), geo.g);
    for (uint32_t i = 0; i < geo.u; ++i)
      re[((uint64_t)i * geo.v_re + hrange(mas(geo.rh[i], a), geo.v_re)) * geo.g + rei] = code;
  }
  const uint64_t mask = __ballot(sampled);
  if (mask != 0ull) {
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1u;
    uint32_t base = 0;
    if (__lane_id() == leader) base = atomicAdd(tcount, (uint32_t)__popcll(mask));
    base = __shfl(base, (int)leader);
    if (sampled) touched[base + lane_rank(mask)] = a;
  }
}

template <int U, bool VEC>
__global__ __launch_bounds__(kBlock) void k_scan_dedup(const uint32_t* __restrict__ pairs,
                                                      uint64_t n, Geo geo, uint16_t code,
                                                      uint16_t* __restrict__ le,
                                                      uint16_t* __restrict__ re,
                                                      uint32_t* __restrict__ touched,
                                                      uint32_t* __restrict__ tcount) {
  for (uint64_t base = (uint64_t)blockIdx.x * kDedupTile; base < n;
       base += (uint64_t)gridDim.x * kDedupTile) {
    uint32_t a[kDedupSteps][2], b[kDedupSteps][2];
    bool v[kDedupSteps][2];
#pragma unroll
    for (int s = 0; s < kDedupSteps; ++s) {
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
    if constexpr (U > 0) {
      // every load first, then the stores of the stamps that differ
      uint32_t seen[kDedupSteps][2][U];
#pragma unroll
      for (int s = 0; s < kDedupSteps; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint32_t lei = hrange(mas(geo.h3, b[s][h]), geo.G);
#pragma unroll
          for (int i = 0; i < U; ++i)
            seen[s][h][i] = v[s][h] ? peek16(le, le_cell(geo, i, a[s][h], lei)) : code;
        }
#pragma unroll
      for (int s = 0; s < kDedupSteps; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (!v[s][h]) continue;
          const uint32_t lei = hrange(mas(geo.h3, b[s][h]), geo.G);
#pragma unroll
          for (int i = 0; i < U; ++i)
            if (seen[s][h][i] != code) le[le_cell(geo, i, a[s][h], lei)] = code;
        }
    } else {
#pragma unroll
      for (int s = 0; s < kDedupSteps; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (!v[s][h]) continue;
          const uint32_t lei = hrange(mas(geo.h3, b[s][h]), geo.G);
          for (uint32_t i = 0; i < geo.u; ++i) {
            const uint64_t c = le_cell(geo, i, a[s][h], lei);
            if (peek16(le, c) != code) le[c] = code;
          }
        }
    }
#pragma unroll
    for (int s = 0; s < kDedupSteps; ++s) {
      sample_stamp(a[s][0], b[s][0], v[s][0], geo, code, re, touched, tcount);
      sample_stamp(a[s][1], b[s][1], v[s][1], geo, code, re, touched, tcount);
    }
  }
}

template <int U>
static hipError_t launch_dedup_u(const uint32_t* pairs, uint64_t n, const Geo& geo, uint16_t code,
                                 uint16_t* le, uint16_t* re, uint32_t* touched, uint32_t* tcount,
                                 uint32_t max_blocks, hipStream_t st) {
  uint64_t blocks = (n + kDedupTile - 1) / kDedupTile;
  if (max_blocks && blocks > max_blocks) blocks = max_blocks;
  if (((uintptr_t)pairs & 15u) == 0)
    hipLaunchKernelGGL((k_scan_dedup<U, true>), dim3((uint32_t)blocks), dim3(kBlock), 0, st,
                       pairs, n, geo, code, le, re, touched, tcount);
  else
    hipLaunchKernelGGL((k_scan_dedup<U, false>), dim3((uint32_t)blocks), dim3(kBlock), 0, st,
                       pairs, n, geo, code, le, re, touched, tcount);
  return hipGetLastError();
}

hipError_t launch_scan_dedup(const uint32_t* pairs, uint64_t n, const Geo& geo, uint16_t code,
                             uint16_t* le, uint16_t* re, uint32_t* touched, uint32_t* tcount,
                             uint32_t max_blocks, hipStream_t st) {
  if (n == 0) return hipSuccess;
  switch (geo.u) {
    case 4: return launch_dedup_u<4>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
    case 8: return launch_dedup_u<8>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
    default: return launch_dedup_u<0>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
  }
}

}  // namespace srla
