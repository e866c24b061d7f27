// Sorting and stream compaction for the end-of-slice candidate pipeline:
// a keys-only sort of uint32 sources (by the top 8 bits into 256 buckets,
// then each bucket by three stable 8-bit counting passes) and a stable
// compaction of flagged elements.
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

// ------------------------------------------------------------------ sort
// Keys-only ascending sort in three launches, whatever the count (read on
// the device): the slice's few 10^4 sampled sources take about 30 us instead
// of the 70 us of a four-pass LSD radix sort's twelve small launches.
//   k_bucket_count: how many keys have each value of the top 8 bits (256
//     buckets), added into cnt[];
//   k_bucket_scatter: every workgroup reserves a range of each bucket (an
//     atomic add on cur[]) and scatters its keys there, in no particular
//     order; block 0 writes the buckets' starts;
//   k_bucket_sort: one workgroup per bucket sorts it by the low 24 bits in
//     three stable 8-bit counting passes, in LDS when it fits (the copies of
//     a key that fills a quarter of the bucket set aside first) and in place
//     in global memory when it does not (a heavy source can fill one bucket),
//     then clears its bucket's counters for the next sort.
// The 768-word scratch `aux` holds cnt[256], cur[256] and start[256]; cnt and
// cur are zero between sorts (cleared when the scratch is allocated).

constexpr uint32_t kBuckets = 256;
constexpr uint32_t kBucketGrid = 256;      // counting / scattering workgroups
constexpr int kSortThreads = 1024;
constexpr int kSortWaves = kSortThreads / kWave;
constexpr uint32_t kSortLds = 12288;      // keys per LDS buffer (two of them)
static_assert(kBlock == (int)kBuckets, "one thread per bucket");

// Exclusive scan of one value per thread over 256 threads (four waves).
__device__ __forceinline__ uint32_t scan256(uint32_t v, uint32_t* w4) {
  const uint32_t lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  uint32_t x = v;
  for (int off = 1; off < kWave; off <<= 1) {
    const uint32_t y = __shfl_up(x, off);
    if (lane >= (uint32_t)off) x += y;
  }
  if (lane == kWave - 1) w4[wave] = x;
  __syncthreads();
  uint32_t before = 0;
  for (uint32_t w = 0; w < wave; ++w) before += w4[w];
  __syncthreads();
  return before + x - v;
}

__global__ __launch_bounds__(kBlock) void k_bucket_count(const uint32_t* __restrict__ keys,
                                                        const uint32_t* __restrict__ n_dev,
                                                        uint32_t* __restrict__ aux) {
  __shared__ uint32_t h[kBuckets];
  h[threadIdx.x] = 0;
  __syncthreads();
  const uint64_t n = *n_dev;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += stride)
    atomicAdd(&h[keys[i] >> 24], 1u);
  __syncthreads();
  if (h[threadIdx.x]) atomicAdd(&aux[threadIdx.x], h[threadIdx.x]);
}

// Visits the same keys as k_bucket_count's workgroup of the same index.
__global__ __launch_bounds__(kBlock) void k_bucket_scatter(const uint32_t* __restrict__ keys,
                                                          uint32_t* __restrict__ out,
                                                          const uint32_t* __restrict__ n_dev,
                                                          uint32_t* __restrict__ aux) {
  __shared__ uint32_t h[kBuckets];
  __shared__ uint32_t pos[kBuckets];
  __shared__ uint32_t w4[kBlock / kWave];
  const uint32_t t = threadIdx.x;
  h[t] = 0;
  __syncthreads();
  const uint64_t n = *n_dev;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + t; i < n; i += stride)
    atomicAdd(&h[keys[i] >> 24], 1u);
  const uint32_t start = scan256(aux[t], w4);   // its barriers also complete h
  if (blockIdx.x == 0) aux[2 * kBuckets + t] = start;
  pos[t] = start + (h[t] ? atomicAdd(&aux[kBuckets + t], h[t]) : 0u);
  __syncthreads();
  for (uint64_t i = (uint64_t)blockIdx.x * kBlock + t; i < n; i += stride) {
    const uint32_t k = keys[i];
    out[atomicAdd(&pos[k >> 24], 1u)] = k;
  }
}

// One stable counting pass of s keys from src to dst by the digit at bit
// `shift`: a round of kSortThreads keys at a time, in index order; lanes of a
// wave holding the same digit find each other with 8 ballots, and the waves
// of a round are ordered through wcnt.
__device__ __forceinline__ void sort_pass(const uint32_t* src, uint32_t* dst, uint32_t s,
                                          uint32_t shift, uint32_t* hc, uint32_t* base,
                                          uint32_t (*wcnt)[kBuckets], uint32_t* w16) {
  const uint32_t t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
  if (t < kBuckets) hc[t] = 0;
  __syncthreads();
  // the digit counts, one LDS add per digit and wave: a heavy source's
  // thousands of equal keys would otherwise queue on one counter
  for (uint32_t r = 0; r < s; r += kSortThreads) {
    const uint32_t i = r + t;
    const bool valid = i < s;
    const uint32_t d = valid ? (src[i] >> shift) & 255u : 0u;
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((d >> b) & 1u);
      peers &= ((d >> b) & 1u) ? bal : ~bal;
    }
    if (valid && lane_rank(peers) == 0) atomicAdd(&hc[d], (uint32_t)__popcll(peers));
  }
  __syncthreads();
  // exclusive scan of hc over the first four waves
  uint32_t v = 0, x = 0;
  if (t < kBuckets) {
    v = hc[t];
    x = v;
    for (int off = 1; off < kWave; off <<= 1) {
      const uint32_t y = __shfl_up(x, off);
      if (lane >= (uint32_t)off) x += y;
    }
    if (lane == kWave - 1) w16[wave] = x;
  }
  __syncthreads();
  if (t < kBuckets) {
    uint32_t before = 0;
    for (uint32_t w = 0; w < wave; ++w) before += w16[w];
    base[t] = before + x - v;
  }
  __syncthreads();
  for (uint32_t r = 0; r < s; r += kSortThreads) {
    const uint32_t i = r + t;
    const bool valid = i < s;
    const uint32_t key = valid ? src[i] : 0u;
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
      dst[off + rank] = key;
    }
    __syncthreads();
    if (t < kBuckets) {
      uint32_t add = 0;
      for (int w = 0; w < kSortWaves; ++w) {
        add += wcnt[w][t];
        wcnt[w][t] = 0;
      }
      base[t] += add;
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(kSortThreads) void k_bucket_sort(uint32_t* __restrict__ keys,
                                                             uint32_t* __restrict__ tmp,
                                                             uint32_t* __restrict__ aux) {
  __shared__ uint32_t la[kSortLds], lb[kSortLds];
  __shared__ uint32_t hc[kBuckets], base[kBuckets], w16[kSortWaves];
  __shared__ uint32_t wcnt[kSortWaves][kBuckets];
  __shared__ uint32_t n_eq, n_oth;
  const uint32_t b = blockIdx.x, t = threadIdx.x;
  const uint32_t s = aux[b];
  const uint32_t start = aux[2 * kBuckets + b];
  if (t < kBuckets)
    for (int w = 0; w < kSortWaves; ++w) wcnt[w][t] = 0;
  __syncthreads();
  if (t == 0) {   // every thread has read this bucket's count and start
    aux[b] = 0u;
    aux[kBuckets + b] = 0u;
  }
  if (s == 0) return;
  if (s == 1) {
    if (t == 0) keys[start] = tmp[start];
    return;
  }
  if (s <= kSortLds) {
    for (uint32_t i = t; i < s; i += kSortThreads) la[i] = tmp[start + i];
    if (t == 0) {
      n_eq = 0u;
      n_oth = 0u;
    }
    __syncthreads();
    // A heavy source fills its bucket with one key: the keys equal to a
    // pivot (the bucket's middle entry, in no particular order after the
    // scatter) are set aside and only the others sorted, when the pivot
    // holds at least a quarter of the bucket.  Correct for any pivot.
    const uint32_t pivot = la[s / 2];
    const uint32_t lane = t & (kWave - 1);
    for (uint32_t r = 0; r < s; r += kSortThreads) {   // uniform trip count
      const uint32_t i = r + t;
      const bool valid = i < s;
      const uint32_t key = valid ? la[i] : 0u;
      const uint64_t eq = __ballot(valid && key == pivot);
      const uint64_t oth = __ballot(valid && key != pivot);
      uint32_t at = 0;
      if (lane == 0) {
        if (eq) atomicAdd(&n_eq, (uint32_t)__popcll(eq));
        if (oth) at = atomicAdd(&n_oth, (uint32_t)__popcll(oth));
      }
      at = __shfl(at, 0);
      if (valid && key != pivot) lb[at + lane_rank(oth)] = key;
    }
    __syncthreads();
    const uint32_t c_eq = n_eq, c_oth = n_oth;
    if (4u * c_eq >= s) {
      // the others: lb -> la -> lb -> la, then the pivot's run where it
      // belongs among them
      sort_pass(lb, la, c_oth, 0, hc, base, wcnt, w16);
      sort_pass(la, lb, c_oth, 8, hc, base, wcnt, w16);
      sort_pass(lb, la, c_oth, 16, hc, base, wcnt, w16);
      if (t == 0) {
        uint32_t lo = 0, hi = c_oth;   // first index whose key is not below the pivot
        while (lo < hi) {
          const uint32_t mid = (lo + hi) / 2;
          if (la[mid] < pivot) lo = mid + 1; else hi = mid;
        }
        n_eq = lo;   // reused: the count of others below the pivot
      }
      __syncthreads();
      const uint32_t below = n_eq;
      for (uint32_t i = t; i < s; i += kSortThreads)
        keys[start + i] = i < below ? la[i] : i < below + c_eq ? pivot : la[i - c_eq];
    } else {
      sort_pass(la, lb, s, 0, hc, base, wcnt, w16);
      sort_pass(lb, la, s, 8, hc, base, wcnt, w16);
      sort_pass(la, lb, s, 16, hc, base, wcnt, w16);
      for (uint32_t i = t; i < s; i += kSortThreads) keys[start + i] = lb[i];
    }
  } else {
    // in place: tmp -> keys -> tmp -> keys over the bucket's own ranges
    sort_pass(tmp + start, keys + start, s, 0, hc, base, wcnt, w16);
    sort_pass(keys + start, tmp + start, s, 8, hc, base, wcnt, w16);
    sort_pass(tmp + start, keys + start, s, 16, hc, base, wcnt, w16);
  }
}

uint64_t sort_aux_words() { return 3 * kBuckets; }

hipError_t sort_u32(uint32_t* keys, uint32_t* tmp, const uint32_t* n_dev, uint32_t* aux,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_bucket_count, dim3(kBucketGrid), dim3(kBlock), 0, st, keys, n_dev, aux);
  hipLaunchKernelGGL(k_bucket_scatter, dim3(kBucketGrid), dim3(kBlock), 0, st, keys, tmp, n_dev,
                     aux);
  hipLaunchKernelGGL(k_bucket_sort, dim3(kBuckets), dim3(kSortThreads), 0, st, keys, tmp, aux);
  return hipGetLastError();   // the sorted keys are back in `keys`
}

// ------------------------------------------------------------------ compaction

static uint32_t tile_grid(uint64_t n_max) {
  uint64_t t = (n_max + kTile - 1) / kTile;
  if (t < 1) t = 1;
  return (uint32_t)(t < kMaxTileBlocks ? t : kMaxTileBlocks);
}

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
