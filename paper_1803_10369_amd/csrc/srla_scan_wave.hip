// gfx950 scan of the SRLA hot path (Algorithm 2 of arXiv 1803.10369) with
// wavefront deduplication of same-DR stores.  Pairs that repeat a flow, or
// share a source and an LE index, store the same stamp into the same LE DR;
// inside a wavefront such stores are merged before they reach the memory
// system.  gfx950 has no match-any instruction, so lanes claim an LDS slot
// chosen by a hash of their DR address (each lane writes its lane id, the
// last writer wins), read the winner back, and fetch the winner's address
// with a cross-lane permute: a lane whose winner is another lane with the
// same address drops its store (the winner stores the identical stamp); a
// hash collision with a different address keeps both stores.  Per store this
// costs an LDS write, an LDS read and two permutes, in wavefront order (no
// barriers).  Results are identical to the plain form; whether it is faster
// depends on how often a wavefront repeats a DR, which the autotuner
// measures.
#include "srla_scan_wave.h"

namespace srla {

constexpr int kWdSteps = 4;
constexpr uint64_t kWdTile = (uint64_t)kBlock * 2 * kWdSteps;  // pairs per block
constexpr uint32_t kWdSlots = 256;                             // LDS slots per wavefront

// true if this lane's store of `cell` is taken over by another lane
__device__ __forceinline__ bool wave_duplicate(uint64_t cell, bool valid,
                                               uint32_t* __restrict__ slots, uint32_t lane) {
  const uint32_t key = (uint32_t)cell ^ (uint32_t)(cell >> 32);
  const uint32_t slot = (key * 0x9E3779B1u) >> 24;   // 8 bits: kWdSlots
  if (valid) slots[slot] = lane;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
  const uint32_t winner = valid ? slots[slot] : lane;
  const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)cell, (int)winner);
  const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(cell >> 32), (int)winner);
  __builtin_amdgcn_wave_barrier();   // every read of this round before the next round's writes
  return valid && winner != lane && ((((uint64_t)hi) << 32) | lo) == cell;
}

__device__ __forceinline__ uint64_t le_cell_of(const Geo& geo, uint32_t row, uint32_t a,
                                               uint32_t lei) {
  return ((uint64_t)row * geo.v_le + hrange(mas(geo.rh[row], a), geo.v_le)) * geo.G + lei;
}

template <int U, bool VEC>
__global__ __launch_bounds__(kBlock) void k_scan_wave_dedup(const uint32_t* __restrict__ pairs,
                                                           uint64_t n, Geo geo, uint16_t code,
                                                           uint16_t* __restrict__ le,
                                                           uint16_t* __restrict__ re,
                                                           uint32_t* __restrict__ touched,
                                                           uint32_t* __restrict__ tcount) {
  __shared__ uint32_t s_slots[kBlock / kWave][kWdSlots];
  const uint32_t lane = __lane_id();
  uint32_t* slots = s_slots[threadIdx.x / kWave];
  const uint32_t nu = U > 0 ? (uint32_t)U : geo.u;
  for (uint64_t base = (uint64_t)blockIdx.x * kWdTile; base < n;
       base += (uint64_t)gridDim.x * kWdTile) {
    uint32_t a[kWdSteps][2], b[kWdSteps][2];
    bool v[kWdSteps][2];
#pragma unroll
    for (int s = 0; s < kWdSteps; ++s) {
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
    for (int s = 0; s < kWdSteps; ++s)
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const uint32_t aa = a[s][h], bb = b[s][h];
        const bool valid = v[s][h];
        const uint32_t lei = hrange(mas(geo.h3, bb), geo.G);
#pragma unroll
        for (uint32_t i = 0; i < nu; ++i) {
          const uint64_t cell = le_cell_of(geo, i, aa, lei);
          if (!wave_duplicate(cell, valid, slots, lane) && valid) le[cell] = code;
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
          if (lane == leader) at = atomicAdd(tcount, (uint32_t)__popcll(mask));
          at = __shfl(at, (int)leader);
          if (sampled) touched[at + lane_rank(mask)] = aa;
        }
      }
  }
}

template <int U>
static hipError_t launch_wd_u(const uint32_t* pairs, uint64_t n, const Geo& geo, uint16_t code,
                              uint16_t* le, uint16_t* re, uint32_t* touched, uint32_t* tcount,
                              uint32_t max_blocks, hipStream_t st) {
  uint64_t blocks = (n + kWdTile - 1) / kWdTile;
  if (max_blocks && blocks > max_blocks) blocks = max_blocks;
  if (((uintptr_t)pairs & 15u) == 0)
    hipLaunchKernelGGL((k_scan_wave_dedup<U, true>), dim3((uint32_t)blocks), dim3(kBlock), 0, st,
                       pairs, n, geo, code, le, re, touched, tcount);
  else
    hipLaunchKernelGGL((k_scan_wave_dedup<U, false>), dim3((uint32_t)blocks), dim3(kBlock), 0,
                       st, pairs, n, geo, code, le, re, touched, tcount);
  return hipGetLastError();
}

hipError_t launch_scan_wave_dedup(const uint32_t* pairs, uint64_t n, const Geo& geo,
                                  uint16_t code, uint16_t* le, uint16_t* re, uint32_t* touched,
                                  uint32_t* tcount, uint32_t max_blocks, hipStream_t st) {
  if (n == 0) return hipSuccess;
  switch (geo.u) {
    case 4: return launch_wd_u<4>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
    case 8: return launch_wd_u<8>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
    default: return launch_wd_u<0>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
  }
}

}  // namespace srla
