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
      // every load first (unconditionally: a missing pair reads as (0, 0),
      // whose cells are in range, so no branch separates the loads), then the
      // stores of the stamps that differ
      uint32_t seen[kDedupSteps][2][U];
#pragma unroll
      for (int s = 0; s < kDedupSteps; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint32_t lei = hrange(mas(geo.h3, b[s][h]), geo.G);
#pragma unroll
          for (int i = 0; i < U; ++i)
            seen[s][h][i] = peek16(le, le_cell(geo, i, a[s][h], lei));
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

// Per-XCD read-before-write form.  Workgroups are dispatched to the eight
// XCDs round-robin by index, so with block b stamping only the rows of XCD
// (b mod 8) every row is read and written by one XCD, and the row (4 MiB of
// LE DRs for the backbone geometry) stays in that XCD's L2, where the DR
// loads hit (91 % for that geometry).  The stores are not absorbed there: a
// store that hits the L2 still goes out as its own write request, so only the
// skipped repeats save write traffic.  Every XCD reads all pairs (non-
// temporally, so they do not push the row out); the reads after the first
// come from the last-level cache.  Sampled sources are appended by the blocks
// of the XCDs that own row 0, once per pair.
constexpr uint32_t kXcdCount = 8;
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

template <int U>
__global__ __launch_bounds__(kBlock) void k_scan_xcd_dedup(const uint32_t* __restrict__ pairs,
                                                          uint64_t n, Geo geo, uint16_t code,
                                                          uint16_t* __restrict__ le,
                                                          uint16_t* __restrict__ re,
                                                          uint32_t* __restrict__ touched,
                                                          uint32_t* __restrict__ tcount) {
  constexpr uint32_t kParts = U >= (int)kXcdCount ? 1 : kXcdCount / U;  // tiles per block group
  constexpr int kRows = U >= (int)kXcdCount ? U / (int)kXcdCount : 1;   // rows per XCD
  const uint32_t xcd = blockIdx.x % kXcdCount;
  const uint32_t row0 = U >= (int)kXcdCount ? xcd : xcd % U;
  const uint32_t part = U >= (int)kXcdCount ? 0u : xcd / U;
  const bool appender = row0 == 0;
  const uint64_t groups = gridDim.x / kXcdCount;
  for (uint64_t group = blockIdx.x / kXcdCount;; group += groups) {
    const uint64_t base = (group * kParts + part) * kDedupTile;
    if (base >= n) break;
    uint32_t a[kDedupSteps][2], b[kDedupSteps][2];
    bool v[kDedupSteps][2];
    if (base + kDedupTile <= n) {
      // a whole tile: every pair load issued before the first use.  Non-
      // temporal: the pairs stream past, the row stays in the L2.
      u32x4 q[kDedupSteps];
#pragma unroll
      for (int s = 0; s < kDedupSteps; ++s)
        q[s] = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(
            pairs + 2 * (base + (uint64_t)s * (2 * kBlock) + 2u * threadIdx.x)));
#pragma unroll
      for (int s = 0; s < kDedupSteps; ++s) {
        a[s][0] = q[s].x; b[s][0] = q[s].y; a[s][1] = q[s].z; b[s][1] = q[s].w;
        v[s][0] = v[s][1] = true;
      }
    } else {
#pragma unroll
      for (int s = 0; s < kDedupSteps; ++s) {
        const uint64_t p = base + (uint64_t)s * (2 * kBlock) + 2u * threadIdx.x;
        v[s][0] = p < n;
        v[s][1] = p + 1 < n;
        a[s][0] = v[s][0] ? pairs[2 * p] : 0u;
        b[s][0] = v[s][0] ? pairs[2 * p + 1] : 0u;
        a[s][1] = v[s][1] ? pairs[2 * p + 2] : 0u;
        b[s][1] = v[s][1] ? pairs[2 * p + 3] : 0u;
      }
    }
    // every load first, unconditionally (a missing pair reads as (0, 0)),
    // then the stores of the stamps that differ
    uint32_t seen[kDedupSteps][2][kRows];
#pragma unroll
    for (int s = 0; s < kDedupSteps; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t lei = hrange(mas(geo.h3, b[s][h]), geo.G);
#pragma unroll
        for (int j = 0; j < kRows; ++j)
          seen[s][h][j] = peek16(le, le_cell(geo, row0 + j * kXcdCount, a[s][h], lei));
      }
#pragma unroll
    for (int s = 0; s < kDedupSteps; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        if (!v[s][h]) continue;
        const uint32_t lei = hrange(mas(geo.h3, b[s][h]), geo.G);
#pragma unroll
        for (int j = 0; j < kRows; ++j)
          if (seen[s][h][j] != code) le[le_cell(geo, row0 + j * kXcdCount, a[s][h], lei)] = code;
      }
#pragma unroll
    for (int s = 0; s < kDedupSteps; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const bool sampled = v[s][h] && (mas(geo.h1, b[s][h]) & geo.tau_mask) == 0u;
        if (sampled) {
          const uint32_t rei = hrange(mas(geo.h2, b[s][h]), geo.g);
#pragma unroll
          for (int j = 0; j < kRows; ++j) {
            const uint32_t r = row0 + j * kXcdCount;
            re[((uint64_t)r * geo.v_re + hrange(mas(geo.rh[r], a[s][h]), geo.v_re)) * geo.g +
               rei] = code;
          }
        }
        if (appender) {
          const uint64_t mask = __ballot(sampled);
          if (mask != 0ull) {
            const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1u;
            uint32_t slot = 0;
            if (__lane_id() == leader) slot = atomicAdd(tcount, (uint32_t)__popcll(mask));
            slot = __shfl(slot, (int)leader);
            if (sampled) touched[slot + lane_rank(mask)] = a[s][h];
          }
        }
      }
  }
}

template <int U>
static hipError_t launch_xcd_dedup_u(const uint32_t* pairs, uint64_t n, const Geo& geo,
                                     uint16_t code, uint16_t* le, uint16_t* re,
                                     uint32_t* touched, uint32_t* tcount, uint32_t max_blocks,
                                     hipStream_t st) {
  constexpr uint64_t kParts = U >= (int)kXcdCount ? 1 : kXcdCount / U;
  const uint64_t tiles = (n + kDedupTile - 1) / kDedupTile;
  uint64_t blocks = kXcdCount * ((tiles + kParts - 1) / kParts);
  if (max_blocks && blocks > max_blocks)
    blocks = max_blocks >= kXcdCount ? max_blocks / kXcdCount * kXcdCount : kXcdCount;
  hipLaunchKernelGGL((k_scan_xcd_dedup<U>), dim3((uint32_t)blocks), dim3(kBlock), 0, st, pairs,
                     n, geo, code, le, re, touched, tcount);
  return hipGetLastError();
}

hipError_t launch_scan_dedup(const uint32_t* pairs, uint64_t n, const Geo& geo, uint16_t code,
                             uint16_t* le, uint16_t* re, uint32_t* touched, uint32_t* tcount,
                             bool xcd_aware, uint32_t max_blocks, hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (xcd_aware && ((uintptr_t)pairs & 15u) == 0) {
    switch (geo.u) {
      case 1: return launch_xcd_dedup_u<1>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
      case 2: return launch_xcd_dedup_u<2>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
      case 4: return launch_xcd_dedup_u<4>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
      case 8: return launch_xcd_dedup_u<8>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
      case 16: return launch_xcd_dedup_u<16>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
      default: break;   // other row counts: the plain read-before-write form
    }
  }
  switch (geo.u) {
    case 4: return launch_dedup_u<4>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
    case 8: return launch_dedup_u<8>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
    default: return launch_dedup_u<0>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
  }
}

}  // namespace srla
