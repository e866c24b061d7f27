// Partitioned scan of the SRLA hot path for gfx950: Algorithm 2 of
// arXiv 1803.10369 (Section 4.1) with the LE stamp stores grouped by address
// before they are issued.
//
// The flat scan issues one random 2-byte store per (pair, row), and every
// such store is a write request of its own to the last-level cache, so the
// scan runs at the chip's random-store rate.  Here the LE is cut into
// regions of 2^15 DRs.  The partition kernel takes a chunk of pairs per
// workgroup, hashes them as the flat scan does (the SRE stores are
// unchanged, they concern 2^-tau of the pairs; the chunk's sampled sources
// are gathered in LDS and appended to the slice's list at once),
// counting-sorts the chunk's LE DR indices by region in LDS and writes them
// out as one contiguous block, with the chunk's region offsets.  The marking
// kernel has kPartSplit workgroups per region, each marking the DRs that its
// share of the chunks names in an LDS bitmap; the stamping kernel ORs a
// region's bitmaps and stores the stamp into the marked DRs with consecutive
// lanes on consecutive DRs, so a wavefront's stores fill whole cache lines.
// DRset is an idempotent plain store, so the order of the stores does not
// matter and the DR arrays end up exactly as the flat scan leaves them.
#include "srla_scan_part.h"

namespace srla {

namespace {

constexpr uint32_t kPartThreads = 1024;
constexpr uint32_t kPartWaves = kPartThreads / kWave;
constexpr uint32_t kPartRegion = 1u << kPartLog;
constexpr uint32_t kPartMask = kPartRegion - 1u;
static_assert(kPartMaxRegions <= kPartThreads, "one region counter per partition thread");
static_assert(kPartEntries <= 65535, "chunk offsets are 16-bit");

// LE DR index of row i for source hash column col and DR lei
__device__ __forceinline__ uint32_t le_cell(const Geo& geo, uint32_t i, uint32_t a, uint32_t lei) {
  const uint32_t col = hrange(mas(geo.rh[i], a), geo.v_le);
  return (i * geo.v_le + col) * geo.G + lei;   // < 2^25: fits part_scan_fits
}

// SRE stores and the sampled-source append of one pair (as the flat scan);
// the append goes to an LDS list (count in LDS) when `stage` is given, else
// straight to the slice's list
template <int U>
__device__ __forceinline__ void sre_pair(uint32_t a, uint32_t b, bool valid, const Geo& geo,
                                         uint16_t code, uint16_t* __restrict__ re,
                                         uint32_t* __restrict__ touched,
                                         uint32_t* __restrict__ tcount, uint32_t* stage,
                                         uint32_t* stage_n) {
  const uint32_t nu = U > 0 ? (uint32_t)U : geo.u;
  const bool sampled = valid && (mas(geo.h1, b) & geo.tau_mask) == 0u;
  if (sampled) {
    const uint32_t rei = hrange(mas(geo.h2, b), geo.g);
#pragma unroll
    for (uint32_t i = 0; i < nu; ++i) {
      const uint32_t col = hrange(mas(geo.rh[i], a), geo.v_re);
      re[((uint64_t)i * geo.v_re + col) * geo.g + rei] = code;
    }
  }
  const uint64_t mask = __ballot(sampled);
  if (mask != 0ull) {
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1u;
    uint32_t base = 0;
    if (__lane_id() == leader)
      base = atomicAdd(stage ? stage_n : tcount, (uint32_t)__popcll(mask));
    base = __shfl(base, (int)leader);
    if (sampled) (stage ? stage : touched)[base + lane_rank(mask)] = a;
  }
}

// Chunk c of the round holds pairs [c * ppc, c * ppc + cnt); its LE DR
// indices (cnt * u <= kPartEntries of them) go to entries[c * kPartEntries
// ...], region r's at offsets [offs[r][c], offs[r + 1][c]) (offs is region-
// major with `stride` >= chunks-per-round columns, regions + 1 rows).  U > 0: u is U and each
// thread keeps its DR indices in registers between the counting and the
// placing pass (then ppc * U == kPartEntries); U == 0: any u, recomputed.
template <int U>
__global__ __launch_bounds__(kPartThreads) void k_scan_part(
    const uint32_t* __restrict__ pairs, uint64_t n, uint32_t ppc, Geo geo, uint16_t code,
    uint16_t* __restrict__ re, uint32_t* __restrict__ touched, uint32_t* __restrict__ tcount,
    uint32_t regions, uint16_t* __restrict__ entries, uint16_t* __restrict__ offs,
    uint32_t stride) {
  __shared__ __align__(16) uint16_t ent[kPartEntries];
  __shared__ uint32_t hist[kPartMaxRegions + 1];
  __shared__ uint32_t cur[kPartMaxRegions];
  __shared__ uint32_t wsum[kPartWaves];
  __shared__ uint32_t n_samp, samp_base;
  constexpr uint32_t kPer = U > 0 ? kPartEntries / U / kPartThreads : 1;
  const uint32_t nu = U > 0 ? (uint32_t)U : geo.u;
  const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid / kWave;
  const uint64_t p0 = (uint64_t)blockIdx.x * ppc;
  const uint32_t cnt = (uint32_t)(n - p0 < ppc ? n - p0 : ppc);
  hist[tid] = 0u;
  if (tid == 0) n_samp = 0u;
  __syncthreads();
  // with U >= 2 a chunk has at most kPartEntries / 2 pairs, so its sampled
  // sources (4 bytes each) fit the entry array, which is free until the
  // placing pass: one append to the slice's list per chunk instead of one per
  // wavefront
  static_assert(U == 0 || U >= 2, "the staged sampled sources must fit the entry array");
  uint32_t* stage = U > 0 ? reinterpret_cast<uint32_t*>(ent) : nullptr;

  // counting pass: region histogram of the LE DR indices, SRE stores and
  // sampled sources
  uint32_t cell[U > 0 ? kPer : 1][U > 0 ? U : 1];
  for (uint32_t it = 0, j0 = 0; j0 < cnt; ++it, j0 += kPartThreads) {   // uniform trip count
    const uint32_t j = j0 + tid;
    const bool valid = j < cnt;
    const uint32_t a = valid ? pairs[2 * (p0 + j)] : 0u;
    const uint32_t b = valid ? pairs[2 * (p0 + j) + 1] : 0u;
    if (valid) {
      const uint32_t lei = hrange(mas(geo.h3, b), geo.G);
      if constexpr (U > 0) {
#pragma unroll
        for (uint32_t s = 0; s < kPer; ++s) {
          if (s == it) {
#pragma unroll
            for (uint32_t i = 0; i < (uint32_t)U; ++i) {
              cell[s][i] = le_cell(geo, i, a, lei);
              atomicAdd(&hist[cell[s][i] >> kPartLog], 1u);
            }
          }
        }
      } else {
        for (uint32_t i = 0; i < nu; ++i) atomicAdd(&hist[le_cell(geo, i, a, lei) >> kPartLog], 1u);
      }
    }
    sre_pair<U>(a, b, valid, geo, code, re, touched, tcount, stage, &n_samp);
  }
  __syncthreads();
  if constexpr (U > 0) {
    if (tid == 0) samp_base = n_samp ? atomicAdd(tcount, n_samp) : 0u;
    __syncthreads();
    for (uint32_t k = tid; k < n_samp; k += kPartThreads) touched[samp_base + k] = stage[k];
    __syncthreads();
  }

  // exclusive scan of the histogram: region starts in hist and cur, the
  // chunk's entry count in hist[regions]
  const uint32_t v = tid < regions ? hist[tid] : 0u;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= (uint32_t)d) x += y;
  }
  if (lane == kWave - 1) wsum[wave] = x;
  __syncthreads();
  if (tid == 0) {
    uint32_t s = 0;
    for (uint32_t w = 0; w < kPartWaves; ++w) {
      const uint32_t t = wsum[w];
      wsum[w] = s;
      s += t;
    }
    hist[regions] = s;
  }
  __syncthreads();
  if (tid < regions) {
    hist[tid] = x - v + wsum[wave];
    cur[tid] = x - v + wsum[wave];
  }
  __syncthreads();

  // placing pass
  for (uint32_t it = 0, j0 = 0; j0 < cnt; ++it, j0 += kPartThreads) {
    const uint32_t j = j0 + tid;
    if (j >= cnt) continue;
    if constexpr (U > 0) {
#pragma unroll
      for (uint32_t s = 0; s < kPer; ++s) {
        if (s == it) {
#pragma unroll
          for (uint32_t i = 0; i < (uint32_t)U; ++i) {
            const uint32_t pos = atomicAdd(&cur[cell[s][i] >> kPartLog], 1u);
            ent[pos] = (uint16_t)(cell[s][i] & kPartMask);
          }
        }
      }
    } else {
      const uint32_t a = pairs[2 * (p0 + j)], b = pairs[2 * (p0 + j) + 1];
      const uint32_t lei = hrange(mas(geo.h3, b), geo.G);
      for (uint32_t i = 0; i < nu; ++i) {
        const uint32_t c = le_cell(geo, i, a, lei);
        const uint32_t pos = atomicAdd(&cur[c >> kPartLog], 1u);
        ent[pos] = (uint16_t)(c & kPartMask);
      }
    }
  }
  __syncthreads();

  // the sorted block (16-byte pieces; the tail of the last piece is unused)
  // and the region offsets
  const uint32_t total = hist[regions];
  uint4* dst = reinterpret_cast<uint4*>(entries + (uint64_t)blockIdx.x * kPartEntries);
  const uint4* srcv = reinterpret_cast<const uint4*>(ent);
  for (uint32_t q = tid; q * 8u < total; q += kPartThreads) dst[q] = srcv[q];
  for (uint32_t r = tid; r <= regions; r += kPartThreads)
    offs[(uint64_t)r * stride + blockIdx.x] = (uint16_t)hist[r];
}

// Marking: workgroup (r, q) takes region r's segments of the q-th of
// gridDim.y (at most kPartSplit) equal shares of the chunks, marks the DRs
// they name in an LDS bitmap and writes the bitmap to its slot of `marks`.  Each wavefront works
// on 8 chunks' segments at a time, consecutive lanes on consecutive entries.
// A region that holds a heavy source gets many times the average number of
// entries; splitting its chunks over kPartSplit workgroups keeps it from
// setting the pace of the whole launch.
constexpr uint32_t kApplyThreads = 256;
constexpr uint32_t kApplyWaves = kApplyThreads / kWave;
constexpr uint32_t kApplySegs = 8;
constexpr uint32_t kWords = kPartRegion / 32;

__global__ __launch_bounds__(kApplyThreads) void k_scan_mark(
    const uint16_t* __restrict__ entries, const uint16_t* __restrict__ offs, uint32_t chunks,
    uint32_t stride, uint32_t* __restrict__ marks) {
  __shared__ uint32_t bm[kWords];
  const uint32_t tid = threadIdx.x, lane = __lane_id();
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  const uint32_t r = blockIdx.x, q = blockIdx.y;
  for (uint32_t w = tid; w < kWords; w += kApplyThreads) bm[w] = 0u;
  __syncthreads();
  const uint32_t share = (chunks + gridDim.y - 1) / gridDim.y;
  const uint32_t c_lo = q * share < chunks ? q * share : chunks;
  const uint32_t c_hi = c_lo + share < chunks ? c_lo + share : chunks;
  // this wavefront's chunks: [w_lo, w_hi), their offsets loaded 64 at a time
  // (one chunk per lane) and read back lane by lane
  const uint32_t per_w = (c_hi - c_lo + kApplyWaves - 1) / kApplyWaves;
  const uint32_t w_lo = c_lo + wave * per_w < c_hi ? c_lo + wave * per_w : c_hi;
  const uint32_t w_hi = w_lo + per_w < c_hi ? w_lo + per_w : c_hi;
  const uint16_t* lo_row = offs + (uint64_t)r * stride;
  const uint16_t* hi_row = lo_row + stride;
  for (uint32_t g0 = w_lo; g0 < w_hi; g0 += kWave) {   // uniform per wave
    const uint32_t c = g0 + lane;
    uint32_t lo = 0u, len = 0u;
    if (c < w_hi) {
      lo = lo_row[c];
      len = (uint32_t)hi_row[c] - lo;
    }
    const uint32_t in_group = w_hi - g0 < kWave ? w_hi - g0 : kWave;
    for (uint32_t b0 = 0; b0 < in_group; b0 += kApplySegs) {   // uniform per wave
      // segment t covers entries [al[t] + off[t], al[t] + end[t]) of the
      // chunk, al[t] rounded down to 64 entries, so that one load instruction
      // reads one aligned 128-byte line of a segment
      uint32_t al[kApplySegs], off[kApplySegs], end[kApplySegs], most = 0;
#pragma unroll
      for (uint32_t t = 0; t < kApplySegs; ++t) {   // b0 + t < 64; lanes past w_hi have len 0
        const uint32_t slo = (uint32_t)__builtin_amdgcn_readlane((int)lo, (int)(b0 + t));
        const uint32_t slen = (uint32_t)__builtin_amdgcn_readlane((int)len, (int)(b0 + t));
        al[t] = slo & ~(kWave - 1u);
        off[t] = slo - al[t];
        end[t] = slen ? off[t] + slen : 0u;
        most = end[t] > most ? end[t] : most;
      }
      for (uint32_t k = lane; k - lane < most; k += kWave) {   // uniform per wave
        uint32_t e[kApplySegs];
#pragma unroll
        for (uint32_t t = 0; t < kApplySegs; ++t)
          e[t] = (k >= off[t] && k < end[t])
                     ? (uint32_t)entries[(uint64_t)(g0 + b0 + t) * kPartEntries + al[t] + k]
                     : 0xFFFFFFFFu;
#pragma unroll
        for (uint32_t t = 0; t < kApplySegs; ++t) {
          if (e[t] != 0xFFFFFFFFu) {
            const uint32_t bit = 1u << (e[t] & 31u);
            if (!(bm[e[t] >> 5] & bit)) atomicOr(&bm[e[t] >> 5], bit);
          }
        }
      }
    }
  }
  __syncthreads();
  uint32_t* out = marks + ((uint64_t)q * gridDim.x + r) * kWords;
  for (uint32_t w = tid; w < kWords; w += kApplyThreads) out[w] = bm[w];
}

// Stamping: workgroup r ORs region r's `split` bitmaps and stores the stamp
// into every marked DR, consecutive lanes on consecutive DRs.
__global__ __launch_bounds__(kApplyThreads) void k_scan_stamp(const uint32_t* __restrict__ marks,
                                                             uint32_t regions, uint32_t split,
                                                             uint16_t code,
                                                             uint16_t* __restrict__ le,
                                                             PipeState* ps, uint32_t parity) {
  __shared__ uint32_t bm[kWords];
  const uint32_t tid = threadIdx.x, r = blockIdx.x;
  for (uint32_t w = tid; w < kWords; w += kApplyThreads) {
    uint32_t x = 0u;
    for (uint32_t q = 0; q < split; ++q) x |= marks[((uint64_t)q * regions + r) * kWords + w];
    bm[w] = x;
  }
  __syncthreads();
  const uint64_t base = (uint64_t)r << kPartLog;
  for (uint32_t c = tid; c < kPartRegion; c += kApplyThreads)
    if ((bm[c >> 5] >> (c & 31u)) & 1u) le[base + c] = code;
  if (ps) {
    // the workgroup that finishes last reads the clock: the end of the scan
    __syncthreads();
    if (tid == 0) {
      __threadfence();
      if (atomicAdd(&ps->scan_done[parity], 1u) == gridDim.x - 1u) {
        ps->t_scan[parity] = wall_clock64();
        ps->scanned[parity] = 1u;
        ps->scan_done[parity] = 0u;
      }
    }
  }
}

template <int U>
hipError_t launch_part_u(const uint32_t* pairs, uint64_t n, const Geo& geo, uint16_t code,
                         uint16_t* le, uint16_t* re, uint32_t* touched, uint32_t* tcount,
                         uint16_t* entries, uint16_t* offs, uint32_t* marks,
                         uint32_t round_chunks, uint32_t split, PipeState* ps, uint32_t parity,
                         hipStream_t st) {
  const uint64_t n_le = (uint64_t)geo.u * geo.v_le * geo.G;
  const uint32_t regions = (uint32_t)((n_le + kPartRegion - 1) >> kPartLog);
  const uint32_t ppc = kPartEntries / geo.u;
  const uint64_t per_round = (uint64_t)ppc * round_chunks;
  for (uint64_t p = 0; p < n; p += per_round) {
    const uint64_t np = n - p < per_round ? n - p : per_round;
    const uint32_t chunks = (uint32_t)((np + ppc - 1) / ppc);
    hipLaunchKernelGGL((k_scan_part<U>), dim3(chunks), dim3(kPartThreads), 0, st, pairs + 2 * p,
                       np, ppc, geo, code, re, touched, tcount, regions, entries, offs,
                       round_chunks);
    hipLaunchKernelGGL(k_scan_mark, dim3(regions, split), dim3(kApplyThreads), 0, st,
                       entries, offs, chunks, round_chunks, marks);
    hipLaunchKernelGGL(k_scan_stamp, dim3(regions), dim3(kApplyThreads), 0, st, marks, regions,
                       split, code, le, p + per_round < n ? nullptr : ps, parity);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace

hipError_t launch_scan_partition(const uint32_t* pairs, uint64_t n, const Geo& geo,
                                 uint16_t code, uint16_t* le, uint16_t* re, uint32_t* touched,
                                 uint32_t* tcount, uint16_t* entries, uint16_t* offs,
                                 uint32_t* marks, hipStream_t st, uint32_t round_chunks,
                                 uint32_t split, PipeState* ps, uint32_t parity) {
  if (n == 0) return hipSuccess;
  if (!part_scan_fits((uint64_t)geo.u * geo.v_le * geo.G)) return hipErrorInvalidValue;
  if (round_chunks == 0 || round_chunks > kPartChunks || split == 0 || split > kPartSplit)
    return hipErrorInvalidValue;
  switch (geo.u) {
    case 4:
      return launch_part_u<4>(pairs, n, geo, code, le, re, touched, tcount, entries, offs, marks,
                              round_chunks, split, ps, parity, st);
    case 8:
      return launch_part_u<8>(pairs, n, geo, code, le, re, touched, tcount, entries, offs, marks,
                              round_chunks, split, ps, parity, st);
    case 16:
      return launch_part_u<16>(pairs, n, geo, code, le, re, touched, tcount, entries, offs, marks,
                               round_chunks, split, ps, parity, st);
    default:
      return launch_part_u<0>(pairs, n, geo, code, le, re, touched, tcount, entries, offs, marks,
                              round_chunks, split, ps, parity, st);
  }
}

}  // namespace srla
