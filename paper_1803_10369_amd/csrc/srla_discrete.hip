// gfx950 kernels of the discrete-window form of the SRLA hot path (arXiv
// 1803.10369): k = 1 with one-bit DRs.  Section 3.2 notes that one bit per DR
// is enough when the window is a single slice, and Section 5.1 runs the
// discrete-window experiments so (z = 1); the SE array then holds bit arrays,
// the slide clears them, and the LE becomes the classic linear counter of
// Eq6.  Only the scan and the row fills differ from the 16-bit stamp form:
// the bit arrays have exactly the layout of the activity bitmaps that the
// end-of-slice kernels (finalize, estimate) read, so those run unchanged.
#include "srla_discrete.h"

namespace srla {

constexpr int kBitSteps = 4;
constexpr uint64_t kBitTile = (uint64_t)kBlock * 2 * kBitSteps;  // pairs per block

// ------------------------------------------------------------------ scan
// Algorithm 2 with one-bit DRs.  A DR is set by an atomic OR into a 32-bit
// word of a flat bit array over [u][v_le][G] (LE), or over [u][v_re][g]
// (SRE) spread over the even 64-bit words of an array twice that size --
// the layouts of the LE activity bitmap and of the interleaved SRE activity
// map (whose odd words, "inside after the slide", stay clear at k = 1) that
// the end-of-slice kernels read, so those kernels read these arrays directly.  Bits of different pairs share
// words, hence atomics; device-scope atomics run at the memory side and cost
// several plain stores each, while most DRs of a slice are set many times
// (every repeat of a flow, every pair of a hot source).  So each DR is first
// tested with a plain cached load and the atomic is issued only if the bit
// is still clear.  A stale clear bit only costs a redundant OR (idempotent);
// a stale set bit cannot occur, since bits are only set within the kernel and
// caches are invalidated at its start.  The loads of a thread's 8 pairs are
// all issued before any of its atomics.

__device__ __forceinline__ uint32_t peek_word(const uint64_t* __restrict__ bits, uint64_t i) {
  const uint32_t* w = reinterpret_cast<const uint32_t*>(bits) + (i >> 5);
  return __hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
}

__device__ __forceinline__ void set_bit_if_clear(uint64_t* __restrict__ bits, uint64_t i,
                                                 uint32_t seen) {
  const uint32_t m = 1u << (uint32_t)(i & 31u);
  if ((seen & m) == 0u)
    __hip_atomic_fetch_or(reinterpret_cast<uint32_t*>(bits) + (i >> 5), m, __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
}

// 32-bit word of SRE DR i in the interleaved layout (bit i & 31 of it)
__device__ __forceinline__ uint64_t re_word32(uint64_t i) {
  return 4 * (i >> 6) + ((i >> 5) & 1u);
}

__device__ __forceinline__ uint64_t le_bit(const Geo& geo, uint32_t row, uint32_t a,
                                           uint32_t lei) {
  return ((uint64_t)row * geo.v_le + hrange(mas(geo.rh[row], a), geo.v_le)) * geo.G + lei;
}

// Sampled sources.  A discrete slice is long (the paper's is 300 s), so
// most sampled pairs repeat a source already sampled in the slice.  Each
// source is first inserted into the slice's source set -- open addressing
// over 64-bit slots holding aip + 1 (0 = empty), probed linearly from a
// MurmurHash3-finalizer hash, each slot tested with a plain load before any
// compare-and-swap -- and only appended to the sampled-source list when
// kSetProbes slots are all taken by other sources.  The slice end drains the
// set into the list, so the list holds every sampled source at least once
// (what the candidate check needs) and the sort sees few duplicates.
constexpr uint32_t kSetProbes = 16;

__device__ __forceinline__ uint32_t fmix32(uint32_t h) {
  h ^= h >> 16;
  h *= 0x85EBCA6Bu;
  h ^= h >> 13;
  h *= 0xC2B2AE35u;
  h ^= h >> 16;
  return h;
}

// true if aip is in the set (now or already), false if its probes are full
__device__ __forceinline__ bool set_insert(unsigned long long* __restrict__ set,
                                           uint32_t set_mask, uint32_t a) {
  const unsigned long long key = (unsigned long long)a + 1ull;
  uint32_t slot = fmix32(a) & set_mask;
  for (uint32_t j = 0; j < kSetProbes; ++j, slot = (slot + 1u) & set_mask) {
    unsigned long long cur =
        __hip_atomic_load(set + slot, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    if (cur == 0ull) cur = atomicCAS(set + slot, 0ull, key);
    if (cur == 0ull || cur == key) return true;
  }
  return false;
}

// the SRE half of Algorithm 2 for one pair (2^-tau of the pairs), and the
// recording of its source (set, else a wave-aggregated append)
__device__ __forceinline__ void sample_bits(uint32_t a, uint32_t b, bool valid, const Geo& geo,
                                            uint64_t* __restrict__ rebits,
                                            unsigned long long* __restrict__ set,
                                            uint32_t set_mask,
                                            uint32_t* __restrict__ touched,
                                            uint32_t* __restrict__ tcount) {
  const bool sampled = valid && (mas(geo.h1, b) & geo.tau_mask) == 0u;
  bool append = false;
  if (sampled) {
    const uint32_t rei = hrange(mas(geo.h2, b), geo.g);
    for (uint32_t i = 0; i < geo.u; ++i) {
      const uint64_t bit =
          ((uint64_t)i * geo.v_re + hrange(mas(geo.rh[i], a), geo.v_re)) * geo.g + rei;
      uint32_t* w = reinterpret_cast<uint32_t*>(rebits) + re_word32(bit);
      const uint32_t m = 1u << (uint32_t)(bit & 31u);
      if ((__hip_atomic_load(w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT) & m) == 0u)
        __hip_atomic_fetch_or(w, m, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    append = !set_insert(set, set_mask, a);
  }
  const uint64_t mask = __ballot(append);
  if (mask != 0ull) {
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1u;
    uint32_t base = 0;
    if (__lane_id() == leader) base = atomicAdd(tcount, (uint32_t)__popcll(mask));
    base = __shfl(base, (int)leader);
    if (append) touched[base + lane_rank(mask)] = a;
  }
}

template <int U, bool VEC>
__global__ __launch_bounds__(kBlock) void k_scan_bits(const uint32_t* __restrict__ pairs,
                                                     uint64_t n, Geo geo,
                                                     uint64_t* __restrict__ lebits,
                                                     uint64_t* __restrict__ rebits,
                                                     unsigned long long* __restrict__ set,
                                                     uint32_t set_mask,
                                                     uint32_t* __restrict__ touched,
                                                     uint32_t* __restrict__ tcount) {
  for (uint64_t base = (uint64_t)blockIdx.x * kBitTile; base < n;
       base += (uint64_t)gridDim.x * kBitTile) {
    uint32_t a[kBitSteps][2], b[kBitSteps][2];
    bool v[kBitSteps][2];
#pragma unroll
    for (int s = 0; s < kBitSteps; ++s) {
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
      // LE: every test load first, then the ORs of the bits still clear
      uint32_t seen[kBitSteps][2][U];
#pragma unroll
      for (int s = 0; s < kBitSteps; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const uint32_t lei = hrange(mas(geo.h3, b[s][h]), geo.G);
#pragma unroll
          for (int i = 0; i < U; ++i)
            seen[s][h][i] = v[s][h] ? peek_word(lebits, le_bit(geo, i, a[s][h], lei)) : ~0u;
        }
#pragma unroll
      for (int s = 0; s < kBitSteps; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (!v[s][h]) continue;
          const uint32_t lei = hrange(mas(geo.h3, b[s][h]), geo.G);
#pragma unroll
          for (int i = 0; i < U; ++i)
            set_bit_if_clear(lebits, le_bit(geo, i, a[s][h], lei), seen[s][h][i]);
        }
    } else {
#pragma unroll
      for (int s = 0; s < kBitSteps; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (!v[s][h]) continue;
          const uint32_t lei = hrange(mas(geo.h3, b[s][h]), geo.G);
          for (uint32_t i = 0; i < geo.u; ++i) {
            const uint64_t bit = le_bit(geo, i, a[s][h], lei);
            set_bit_if_clear(lebits, bit, peek_word(lebits, bit));
          }
        }
    }
#pragma unroll
    for (int s = 0; s < kBitSteps; ++s) {
      sample_bits(a[s][0], b[s][0], v[s][0], geo, rebits, set, set_mask, touched, tcount);
      sample_bits(a[s][1], b[s][1], v[s][1], geo, rebits, set, set_mask, touched, tcount);
    }
  }
}

template <int U>
static hipError_t launch_scan_bits_u(const uint32_t* pairs, uint64_t n, const Geo& geo,
                                     uint64_t* lebits, uint64_t* rebits, uint64_t* set,
                                     uint32_t set_slots, uint32_t* touched, uint32_t* tcount,
                                     uint32_t max_blocks, hipStream_t st) {
  uint64_t blocks = (n + kBitTile - 1) / kBitTile;
  if (max_blocks && blocks > max_blocks) blocks = max_blocks;
  unsigned long long* s = reinterpret_cast<unsigned long long*>(set);
  if (((uintptr_t)pairs & 15u) == 0)
    hipLaunchKernelGGL((k_scan_bits<U, true>), dim3((uint32_t)blocks), dim3(kBlock), 0, st,
                       pairs, n, geo, lebits, rebits, s, set_slots - 1u, touched, tcount);
  else
    hipLaunchKernelGGL((k_scan_bits<U, false>), dim3((uint32_t)blocks), dim3(kBlock), 0, st,
                       pairs, n, geo, lebits, rebits, s, set_slots - 1u, touched, tcount);
  return hipGetLastError();
}

hipError_t launch_scan_bits(const uint32_t* pairs, uint64_t n, const Geo& geo, uint64_t* lebits,
                            uint64_t* rebits, uint64_t* set, uint32_t set_slots,
                            uint32_t* touched, uint32_t* tcount, uint32_t max_blocks,
                            hipStream_t st) {
  if (n == 0) return hipSuccess;
  if (set_slots == 0 || (set_slots & (set_slots - 1u)) != 0) return hipErrorInvalidValue;
  switch (geo.u) {
    case 4:
      return launch_scan_bits_u<4>(pairs, n, geo, lebits, rebits, set, set_slots, touched,
                                   tcount, max_blocks, st);
    case 8:
      return launch_scan_bits_u<8>(pairs, n, geo, lebits, rebits, set, set_slots, touched,
                                   tcount, max_blocks, st);
    default:
      return launch_scan_bits_u<0>(pairs, n, geo, lebits, rebits, set, set_slots, touched,
                                   tcount, max_blocks, st);
  }
}

// ------------------------------------------------------------------ set drain
// Appends every source of the slice's source set to the sampled-source list
// (after the entries the scans appended on overflow) and empties the set for
// the slice that will use it next.  Each block owns a contiguous chunk of
// slots: it counts the chunk's sources, reserves their places with a single
// atomic, then writes them in slot order (wave ballots + an LDS prefix over
// the block's waves) and clears the slots.  One atomic per block, not per
// wave: the list's counter would otherwise serialize the drain.
constexpr uint32_t kDrainBlocks = 2048;

__device__ __forceinline__ uint32_t block_prefix(bool flag, uint32_t* s_wave, uint32_t* total) {
  const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint64_t mask = __ballot(flag);
  if (lane == 0) s_wave[wave] = (uint32_t)__popcll(mask);
  __syncthreads();
  uint32_t before = 0, all = 0;
  for (uint32_t w = 0; w < kBlock / kWave; ++w) {
    if (w < wave) before += s_wave[w];
    all += s_wave[w];
  }
  __syncthreads();
  *total = all;
  return before + lane_rank(mask);
}

__global__ __launch_bounds__(kBlock) void k_drain_set(unsigned long long* __restrict__ set,
                                                     uint32_t slots,
                                                     uint32_t* __restrict__ touched,
                                                     uint32_t* __restrict__ tcount) {
  __shared__ uint32_t s_wave[kBlock / kWave];
  __shared__ uint32_t s_base;
  const uint64_t chunk = ((uint64_t)slots + gridDim.x - 1) / gridDim.x;
  const uint64_t lo = (uint64_t)blockIdx.x * chunk;
  const uint64_t hi = lo + chunk < slots ? lo + chunk : slots;
  uint32_t mine = 0;
  for (uint64_t i = lo + threadIdx.x; i < hi; i += kBlock) mine += set[i] != 0ull;
  for (int off = kWave / 2; off > 0; off >>= 1) mine += __shfl_xor(mine, off);
  if ((threadIdx.x & (kWave - 1)) == 0) s_wave[threadIdx.x / kWave] = mine;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (uint32_t w = 0; w < kBlock / kWave; ++w) t += s_wave[w];
    s_base = t ? atomicAdd(tcount, t) : 0u;
  }
  __syncthreads();
  uint32_t at = s_base;
  // the loop bound is uniform per block, so every thread reaches the barriers
  for (uint64_t base = lo; base < hi; base += kBlock) {
    const uint64_t i = base + threadIdx.x;
    const unsigned long long key = i < hi ? set[i] : 0ull;
    uint32_t step;
    const uint32_t pos = block_prefix(key != 0ull, s_wave, &step);
    if (key) {
      touched[at + pos] = (uint32_t)(key - 1ull);
      set[i] = 0ull;
    }
    at += step;
  }
}

hipError_t launch_drain_set(uint64_t* set, uint32_t set_slots, uint32_t* touched,
                            uint32_t* tcount, hipStream_t st) {
  const uint32_t blocks = set_slots / kBlock < kDrainBlocks ? (set_slots + kBlock - 1) / kBlock
                                                             : kDrainBlocks;
  hipLaunchKernelGGL(k_drain_set, dim3(blocks), dim3(kBlock), 0, st,
                     reinterpret_cast<unsigned long long*>(set), set_slots, touched, tcount);
  return hipGetLastError();
}

// ------------------------------------------------------------------ row fills
// |LDR(i)|^k: the LE is already a bit array
// (one bit per DR, rows of v_le*G bits = whole 64-bit words), so the row
// fill is a popcount.  Grid: x = chunks of a row, y = row.
constexpr int kPopSteps = 4;

__global__ __launch_bounds__(kBlock) void k_row_popcount(const uint64_t* __restrict__ bits,
                                                        uint64_t row_words,
                                                        unsigned long long* __restrict__ row_fill) {
  const uint32_t row = blockIdx.y;
  const uint64_t* rowp = bits + (uint64_t)row * row_words;
  uint32_t count = 0;
#pragma unroll
  for (int s = 0; s < kPopSteps; ++s) {
    const uint64_t w = (uint64_t)blockIdx.x * (kBlock * kPopSteps) + (uint64_t)s * kBlock + threadIdx.x;
    if (w < row_words) count += (uint32_t)__popcll(rowp[w]);
  }
  for (int off = kWave / 2; off > 0; off >>= 1) count += __shfl_xor(count, off);
  __shared__ uint32_t part[kBlock / kWave];
  const uint32_t lane = threadIdx.x & (kWave - 1);
  if (lane == 0) part[threadIdx.x / kWave] = count;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += part[w];
    if (t) atomicAdd(&row_fill[row], t);
  }
}

hipError_t launch_row_popcount(const uint64_t* bits, unsigned long long* row_fill,
                               const Geo& geo, hipStream_t st) {
  const uint64_t row_words = (uint64_t)geo.v_le * geo.G / 64;
  const uint64_t bx = (row_words + kBlock * kPopSteps - 1) / (kBlock * kPopSteps);
  hipLaunchKernelGGL(k_row_popcount, dim3((uint32_t)bx, geo.u), dim3(kBlock), 0, st, bits,
                     row_words, row_fill);
  return hipGetLastError();
}

}  // namespace srla
