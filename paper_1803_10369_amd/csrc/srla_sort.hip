// Sorting and stream compaction for the end-of-slice candidate pipeline:
// a keys-only LSD radix sort of uint32 sources (8-bit digits, 4 passes) and
// a stable compaction of flagged elements.
//
// Element counts are read from device memory, so no host round trip sizes
// these kernels and the whole pipeline can be replayed as a graph.  Work is
// cut into tiles of kBlock * kItems elements; a fixed grid walks the tiles
// (tile = block, block + grid, ...).  Inside a tile, round `it` gives thread
// t element tile + it*kBlock + t, so loads are coalesced and the order
// (round, thread) is the index order that stability needs.
#include "srla_internal.h"

namespace srla {

constexpr int kItems = 4;   // small tiles: the slice's few 10^4 keys spread over many blocks
constexpr uint64_t kTile = (uint64_t)kBlock * kItems;
constexpr int kWaves = kBlock / kWave;
constexpr int kScanThreads = 1024;
constexpr uint32_t kMaxTileBlocks = 1024;

__device__ __forceinline__ uint32_t tiles_of(uint64_t n) {
  return (uint32_t)((n + kTile - 1) / kTile);
}

// Exclusive scan of one value per thread over a block of kScanThreads.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* lds16, uint32_t* total) {
  const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t x = v;
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(x, off);
    if (lane >= (uint32_t)off) x += y;
  }
  if (lane == kWave - 1) lds16[wave] = x;
  __syncthreads();
  if (wave == 0) {
    uint32_t t = lane < kScanThreads / kWave ? lds16[lane] : 0u;
    for (int off = 1; off < kScanThreads / kWave; off <<= 1) {
      const uint32_t y = __shfl_up(t, off);
      if (lane >= (uint32_t)off) t += y;
    }
    if (lane < kScanThreads / kWave) lds16[lane] = t;
  }
  __syncthreads();
  const uint32_t before = wave ? lds16[wave - 1] : 0u;
  *total = lds16[kScanThreads / kWave - 1];
  __syncthreads();
  return before + x - v;
}

// In-place exclusive scan, by one block, of the first mult * tiles_of(*n_dev)
// words of v; the grand total goes to *total_out when it is not null.  The
// words go through LDS in chunks of kScanChunk: loaded and stored coalesced
// (thread t takes words t, t + kScanThreads, ...), scanned as kScanPer
// consecutive words per thread, with a running carry between chunks.
constexpr int kScanPer = 16;
constexpr uint64_t kScanChunk = (uint64_t)kScanThreads * kScanPer;   // 64 KiB of LDS

__global__ __launch_bounds__(kScanThreads) void k_scan_words(uint32_t* __restrict__ v,
                                                            const uint32_t* __restrict__ n_dev,
                                                            uint32_t mult,
                                                            uint32_t* __restrict__ total_out) {
  __shared__ uint32_t lds16[kScanThreads / kWave];
  __shared__ uint32_t chunk[kScanChunk];
  const uint64_t n = (uint64_t)mult * tiles_of(*n_dev);
  uint32_t carry = 0;
  for (uint64_t base = 0; base < n; base += kScanChunk) {
    const uint64_t len = n - base < kScanChunk ? n - base : kScanChunk;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      const uint64_t i = (uint64_t)j * kScanThreads + threadIdx.x;
      chunk[i] = i < len ? v[base + i] : 0u;
    }
    __syncthreads();
    uint32_t x[kScanPer];
    uint32_t sum = 0;
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      x[j] = chunk[threadIdx.x * kScanPer + j];
      sum += x[j];
    }
    uint32_t total;
    uint32_t run = carry + block_exclusive_scan(sum, lds16, &total);
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      chunk[threadIdx.x * kScanPer + j] = run;
      run += x[j];
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < kScanPer; ++j) {
      const uint64_t i = (uint64_t)j * kScanThreads + threadIdx.x;
      if (i < len) v[base + i] = chunk[i];
    }
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0 && total_out) *total_out = carry;
}

// ------------------------------------------------------------------ radix sort

// per-tile digit counts, layout [digit][tile]
__global__ __launch_bounds__(kBlock) void k_rs_hist(const uint32_t* __restrict__ keys,
                                                   const uint32_t* __restrict__ n_dev,
                                                   uint32_t shift, uint32_t* __restrict__ hist) {
  __shared__ uint32_t h[256];
  const uint64_t n = *n_dev;
  const uint32_t nt = tiles_of(n);
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)tile * kTile;
#pragma unroll 4
    for (int it = 0; it < kItems; ++it) {
      const uint64_t i = base + (uint64_t)it * kBlock + threadIdx.x;
      if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(uint64_t)threadIdx.x * nt + tile] = h[threadIdx.x];
    __syncthreads();
  }
}

// Stable scatter: lanes holding the same digit find each other with 8
// wavefront ballots (one per digit bit); the lowest such lane publishes the
// wave's count for that digit, and waves are ordered through LDS.
__global__ __launch_bounds__(kBlock) void k_rs_scatter(const uint32_t* __restrict__ in,
                                                      uint32_t* __restrict__ out,
                                                      const uint32_t* __restrict__ n_dev,
                                                      uint32_t shift,
                                                      const uint32_t* __restrict__ hist) {
  __shared__ uint32_t base[256];
  __shared__ uint32_t wcnt[kWaves][256];
  const uint32_t wave = threadIdx.x / kWave;
  const uint64_t n = *n_dev;
  const uint32_t nt = tiles_of(n);
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    base[threadIdx.x] = hist[(uint64_t)threadIdx.x * nt + tile];
    for (int w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)tile * kTile;
    for (int it = 0; it < kItems; ++it) {
      const uint64_t i = t0 + (uint64_t)it * kBlock + threadIdx.x;
      const bool valid = i < n;
      const uint32_t key = valid ? in[i] : 0u;
      const uint32_t d = (key >> shift) & 255u;
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < 8; ++b) {
        const uint64_t bal = __ballot((d >> b) & 1u);
        peers &= ((d >> b) & 1u) ? bal : ~bal;
      }
      const uint32_t rank = lane_rank(peers);
      if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(peers);
      __syncthreads();
      if (valid) {
        uint32_t off = base[d];
        for (uint32_t w = 0; w < wave; ++w) off += wcnt[w][d];
        out[off + rank] = key;
      }
      __syncthreads();
      uint32_t add = 0;
      for (int w = 0; w < kWaves; ++w) {
        add += wcnt[w][threadIdx.x];
        wcnt[w][threadIdx.x] = 0;
      }
      base[threadIdx.x] += add;
      __syncthreads();
    }
  }
}

uint64_t radix_hist_words(uint64_t n) { return 256 * ((n + kTile - 1) / kTile) + 256; }

static uint32_t tile_grid(uint64_t n_max) {
  uint64_t t = (n_max + kTile - 1) / kTile;
  if (t < 1) t = 1;
  return (uint32_t)(t < kMaxTileBlocks ? t : kMaxTileBlocks);
}

hipError_t radix_sort_u32(uint32_t* keys, uint32_t* tmp, const uint32_t* n_dev, uint64_t n_max,
                          uint32_t* block_hist, hipStream_t st) {
  const uint32_t grid = tile_grid(n_max);
  uint32_t* src = keys;
  uint32_t* dst = tmp;
  for (uint32_t shift = 0; shift < 32; shift += 8) {
    hipLaunchKernelGGL(k_rs_hist, dim3(grid), dim3(kBlock), 0, st, src, n_dev, shift, block_hist);
    hipLaunchKernelGGL(k_scan_words, dim3(1), dim3(kScanThreads), 0, st, block_hist, n_dev, 256u,
                       (uint32_t*)nullptr);
    hipLaunchKernelGGL(k_rs_scatter, dim3(grid), dim3(kBlock), 0, st, src, dst, n_dev, shift,
                       block_hist);
    uint32_t* t = src;
    src = dst;
    dst = t;
  }
  return hipGetLastError();   // four passes: the sorted keys are back in `keys`
}

// ------------------------------------------------------------------ compaction

__global__ __launch_bounds__(kBlock) void k_compact_count(const uint8_t* __restrict__ flags,
                                                         uint8_t mask,
                                                         const uint32_t* __restrict__ n_dev,
                                                         uint32_t* __restrict__ counts) {
  __shared__ uint32_t part[kWaves];
  const uint64_t n = *n_dev;
  const uint32_t nt = tiles_of(n);
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const uint64_t base = (uint64_t)tile * kTile;
    uint32_t c = 0;
    for (int it = 0; it < kItems; ++it) {
      const uint64_t i = base + (uint64_t)it * kBlock + threadIdx.x;
      if (i < n && (flags[i] & mask)) ++c;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off);
    if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t = 0;
      for (int w = 0; w < kWaves; ++w) t += part[w];
      counts[tile] = t;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kBlock) void k_compact_scatter(const uint8_t* __restrict__ flags,
                                                           uint8_t mask,
                                                           const uint32_t* __restrict__ vals,
                                                           const uint32_t* __restrict__ n_dev,
                                                           const uint32_t* __restrict__ offsets,
                                                           uint32_t* __restrict__ out) {
  __shared__ uint32_t wsum[kWaves];
  const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const uint64_t n = *n_dev;
  const uint32_t nt = tiles_of(n);
  for (uint32_t tile = blockIdx.x; tile < nt; tile += gridDim.x) {
    const uint64_t base = (uint64_t)tile * kTile;
    uint32_t run = offsets[tile];
    for (int it = 0; it < kItems; ++it) {
      const uint64_t i = base + (uint64_t)it * kBlock + threadIdx.x;
      const bool take = i < n && (flags[i] & mask);
      const uint64_t bal = __ballot(take);
      if (lane == 0) wsum[wave] = (uint32_t)__popcll(bal);
      __syncthreads();
      uint32_t before = run;
      uint32_t round = 0;
      for (int w = 0; w < kWaves; ++w) {
        if ((uint32_t)w < wave) before += wsum[w];
        round += wsum[w];
      }
      if (take) out[before + lane_rank(bal)] = vals[i];
      run += round;
      __syncthreads();
    }
  }
}

uint64_t compact_block_words(uint64_t n) { return (n + kTile - 1) / kTile + 1; }

hipError_t compact_u32(const uint8_t* flags, uint8_t mask, const uint32_t* vals,
                       const uint32_t* n_dev, uint64_t n_max, uint32_t* out,
                       uint32_t* out_count, uint32_t* block_words, hipStream_t st) {
  const uint32_t grid = tile_grid(n_max);
  hipLaunchKernelGGL(k_compact_count, dim3(grid), dim3(kBlock), 0, st, flags, mask, n_dev,
                     block_words);
  hipLaunchKernelGGL(k_scan_words, dim3(1), dim3(kScanThreads), 0, st, block_words, n_dev, 1u,
                     out_count);
  hipLaunchKernelGGL(k_compact_scatter, dim3(grid), dim3(kBlock), 0, st, flags, mask, vals,
                     n_dev, block_words, out);
  return hipGetLastError();
}

}  // namespace srla
