// Partitioned scan of the SRLA hot path for gfx950: Algorithm 2 of
// arXiv 1803.10369 (Section 4.1) with the LE stamp stores grouped by address
// before they are issued.
//
// The flat scan issues one random 2-byte store per (pair, row), and every
// such store is a write request of its own to the last-level cache or HBM,
// so the scan runs at the chip's random-store rate.  Here the LE is cut into
// regions of 2^16 DRs, taken in bands of up to 2048 regions (2^27 DRs).  For
// each band, the partition kernel takes a chunk of pairs per workgroup,
// hashes them for the rows that reach into the band (the first band also
// issues the SRE stores, which concern 2^-tau of the pairs, and gathers the
// chunk's sampled sources in LDS to append them at once), counting-sorts the
// chunk's LE DR indices that fall in the band by region in LDS and writes
// them out as one contiguous block of 16-bit offsets, with the chunk's region
// offsets.  A small plan counts each region's indices and cuts its marking
// into units of up to `unit` indices (32768 by default, a launch-shape knob
// that leaves results unchanged); the marking kernel has one workgroup
// per unit, which marks the DRs its share of the chunks names in an LDS
// bitmap of the region, reading the segments in aligned 16-byte pieces.  The
// stamping kernel ORs a region's unit bitmaps and stores the stamp into the
// marked DRs with consecutive lanes on consecutive DRs, so a wavefront's
// stores fill whole cache lines.  DRset is an idempotent plain store, so the
// order of the stores does not matter and the DR arrays end up exactly as
// the flat scan leaves them.  An LE beyond one band costs one more read of
// the pairs per band; a row's hash is computed once per band it reaches
// into.
#include "srla_scan_part.h"

namespace srla {

namespace {

constexpr uint32_t kPartThreads = 1024;
constexpr uint32_t kPartWaves = kPartThreads / kWave;
constexpr uint32_t kPartRegion = 1u << kPartLog;
constexpr uint32_t kPartMask = kPartRegion - 1u;
static_assert(kPartBandRegions == 2 * kPartThreads, "two region counters per partition thread");
static_assert(kPartEntries <= 65535, "chunk offsets are 16-bit");

// the band one partition pass covers: DRs [lo, lo + span) of the LE, in
// `regions` regions, reached by rows [row_lo, row_hi); the first band's pass
// also does the SRE stores and the sampled-source appends (sre != 0)
struct Band {
  uint64_t lo, span;
  uint32_t regions, row_lo, row_hi, sre;
};

// LE DR index of row i for source a and DR lei: 32-bit when the whole LE is
// one band (at most 2^27 DRs), else 64-bit
__device__ __forceinline__ uint32_t le_cell(const Geo& geo, uint32_t i, uint32_t a, uint32_t lei) {
  const uint32_t col = hrange(mas(geo.rh[i], a), geo.v_le);
  return (i * geo.v_le + col) * geo.G + lei;
}
__device__ __forceinline__ uint64_t le_cell64(const Geo& geo, uint32_t i, uint32_t a,
                                              uint32_t lei) {
  const uint32_t col = hrange(mas(geo.rh[i], a), geo.v_le);
  return ((uint64_t)i * geo.v_le + col) * geo.G + lei;
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
// indices inside the band (at most kPartEntries of them) go to
// entries[c * kPartEntries ...] as offsets within their region, region r's at
// [offs[r][c], offs[r + 1][c]) (offs is region-major with `stride` >=
// chunks-per-round columns, band.regions + 1 rows).  U > 0: the band is the
// whole LE, u is U and each thread keeps its DR indices in registers between
// the counting and the placing pass (then ppc * U == kPartEntries); U == 0:
// any u and band, the rows [band.row_lo, band.row_hi) hashed again in the
// placing pass and indices outside the band skipped.
template <int U>
__global__ __launch_bounds__(kPartThreads) void k_scan_part(
    const uint32_t* __restrict__ pairs, uint64_t n, uint32_t ppc, Geo geo, uint16_t code,
    uint16_t* __restrict__ re, uint32_t* __restrict__ touched, uint32_t* __restrict__ tcount,
    Band band, uint16_t* __restrict__ entries, uint16_t* __restrict__ offs, uint32_t stride) {
  __shared__ __align__(16) uint16_t ent[kPartEntries];
  __shared__ uint32_t hist[kPartBandRegions];
  __shared__ uint32_t wsum[kPartWaves];
  __shared__ uint32_t n_samp, samp_base;
  constexpr uint32_t kPer = U > 0 ? kPartEntries / U / kPartThreads : 1;
  const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid / kWave;
  const uint32_t regions = band.regions;
  const uint64_t p0 = (uint64_t)blockIdx.x * ppc;
  const uint32_t cnt = (uint32_t)(n - p0 < ppc ? n - p0 : ppc);
  for (uint32_t r = tid; r < kPartBandRegions; r += kPartThreads) hist[r] = 0u;
  if (tid == 0) n_samp = 0u;
  __syncthreads();
  // a pass that samples (band.sre) has at most kPartEntries / 2 pairs per
  // chunk, so the chunk's sampled sources (4 bytes each) fit the entry array,
  // which is free until the placing pass: one append to the slice's list per
  // chunk instead of one per wavefront (appends to one counter from every
  // wavefront queue up behind each other)
  static_assert(U == 0 || U >= 2, "the staged sampled sources must fit the entry array");
  uint32_t* stage = reinterpret_cast<uint32_t*>(ent);

  // counting pass: region histogram of the LE DR indices, SRE stores and
  // sampled sources
  uint32_t cell[U > 0 ? kPer : 1][U > 0 ? U : 1];
  if constexpr (U > 0) {
    // all of the thread's pairs are loaded before any is hashed
    uint32_t pa[kPer], pb[kPer];
#pragma unroll
    for (uint32_t s = 0; s < kPer; ++s) {
      const uint32_t j = s * kPartThreads + tid;
      pa[s] = j < cnt ? pairs[2 * (p0 + j)] : 0u;
      pb[s] = j < cnt ? pairs[2 * (p0 + j) + 1] : 0u;
    }
#pragma unroll
    for (uint32_t s = 0; s < kPer; ++s) {
      const bool valid = s * kPartThreads + tid < cnt;
      if (valid) {
        const uint32_t lei = hrange(mas(geo.h3, pb[s]), geo.G);
#pragma unroll
        for (uint32_t i = 0; i < (uint32_t)U; ++i) {
          cell[s][i] = le_cell(geo, i, pa[s], lei);
          atomicAdd(&hist[cell[s][i] >> kPartLog], 1u);
        }
      }
      sre_pair<U>(pa[s], pb[s], valid, geo, code, re, touched, tcount, stage, &n_samp);
    }
  } else {
    for (uint32_t j0 = 0; j0 < cnt; j0 += kPartThreads) {   // uniform trip count
      const uint32_t j = j0 + tid;
      const bool valid = j < cnt;
      const uint32_t a = valid ? pairs[2 * (p0 + j)] : 0u;
      const uint32_t b = valid ? pairs[2 * (p0 + j) + 1] : 0u;
      if (valid) {
        const uint32_t lei = hrange(mas(geo.h3, b), geo.G);
        for (uint32_t i = band.row_lo; i < band.row_hi; ++i) {
          const uint64_t off = le_cell64(geo, i, a, lei) - band.lo;
          if (off < band.span) atomicAdd(&hist[(uint32_t)(off >> kPartLog)], 1u);
        }
      }
      if (band.sre) sre_pair<U>(a, b, valid, geo, code, re, touched, tcount, stage, &n_samp);
    }
  }
  __syncthreads();
  if (band.sre) {
    if (tid == 0) samp_base = n_samp ? atomicAdd(tcount, n_samp) : 0u;
    __syncthreads();
    for (uint32_t k = tid; k < n_samp; k += kPartThreads) touched[samp_base + k] = stage[k];
    __syncthreads();
  }

  // exclusive scan of the histogram, two regions per thread: region starts in
  // hist, which the placing pass advances to the region ends
  const uint32_t r0 = 2u * tid;
  const uint32_t v0 = r0 < regions ? hist[r0] : 0u;
  const uint32_t v1 = r0 + 1u < regions ? hist[r0 + 1u] : 0u;
  const uint32_t v = v0 + v1;
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
  }
  __syncthreads();
  const uint32_t start = x - v + wsum[wave];
  if (r0 < regions) hist[r0] = start;
  if (r0 + 1u < regions) hist[r0 + 1u] = start + v0;
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
            const uint32_t pos = atomicAdd(&hist[cell[s][i] >> kPartLog], 1u);
            ent[pos] = (uint16_t)(cell[s][i] & kPartMask);
          }
        }
      }
    } else {
      const uint32_t a = pairs[2 * (p0 + j)], b = pairs[2 * (p0 + j) + 1];
      const uint32_t lei = hrange(mas(geo.h3, b), geo.G);
      for (uint32_t i = band.row_lo; i < band.row_hi; ++i) {
        const uint64_t off = le_cell64(geo, i, a, lei) - band.lo;
        if (off < band.span) {
          const uint32_t pos = atomicAdd(&hist[(uint32_t)(off >> kPartLog)], 1u);
          ent[pos] = (uint16_t)(off & kPartMask);
        }
      }
    }
  }
  __syncthreads();

  // the sorted block (16-byte pieces; the tail of the last piece is unused)
  // and the region offsets: region r starts where region r - 1 ends
  const uint32_t total = hist[regions - 1u];
  uint4* dst = reinterpret_cast<uint4*>(entries + (uint64_t)blockIdx.x * kPartEntries);
  const uint4* srcv = reinterpret_cast<const uint4*>(ent);
  for (uint32_t q = tid; q * 8u < total; q += kPartThreads) dst[q] = srcv[q];
  for (uint32_t r = tid; r <= regions; r += kPartThreads)
    offs[(uint64_t)r * stride + blockIdx.x] = r ? (uint16_t)hist[r - 1u] : (uint16_t)0u;
}

// Marking plan: region r's DR indices in the round (the sum over chunks of
// its segment lengths) and the number of marking units they make, then the
// regions' first units (exclusive prefix, total in ustart[regions]).  plan
// holds ucount[kPartBandRegions + 1] then ustart[kPartBandRegions + 1].
constexpr uint32_t kPlanThreads = 256;

__global__ __launch_bounds__(kPlanThreads) void k_mark_count(const uint16_t* __restrict__ offs,
                                                             uint32_t chunks, uint32_t stride,
                                                             uint32_t unit,
                                                             uint32_t* __restrict__ plan) {
  __shared__ uint32_t wsum[kPlanThreads / kWave];
  const uint32_t r = blockIdx.x, tid = threadIdx.x;
  const uint16_t* lo = offs + (uint64_t)r * stride;
  const uint16_t* hi = lo + stride;
  uint32_t e = 0;
  for (uint32_t c = tid; c < chunks; c += kPlanThreads) e += (uint32_t)hi[c] - lo[c];
  for (int d = kWave / 2; d >= 1; d >>= 1) e += (uint32_t)__shfl_xor((int)e, d);
  if (__lane_id() == 0) wsum[tid / kWave] = e;
  __syncthreads();
  if (tid == 0) {
    uint32_t t = 0;
    for (uint32_t w = 0; w < kPlanThreads / kWave; ++w) t += wsum[w];
    plan[r] = (t + unit - 1) / unit;
  }
}

constexpr uint32_t kPrefixThreads = 1024;
static_assert(2 * kPrefixThreads == kPartBandRegions, "two regions per prefix thread");

__global__ __launch_bounds__(kPrefixThreads) void k_mark_prefix(uint32_t regions,
                                                                uint32_t* __restrict__ plan) {
  __shared__ uint32_t wsum[kPrefixThreads / kWave];
  const uint32_t tid = threadIdx.x, lane = __lane_id(), wave = tid / kWave;
  const uint32_t* ucount = plan;
  uint32_t* ustart = plan + kPartBandRegions + 1;
  const uint32_t r0 = 2u * tid;
  const uint32_t v0 = r0 < regions ? ucount[r0] : 0u;
  const uint32_t v1 = r0 + 1u < regions ? ucount[r0 + 1u] : 0u;
  const uint32_t v = v0 + v1;
  uint32_t x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t y = __shfl_up(x, d);
    if (lane >= (uint32_t)d) x += y;
  }
  if (lane == kWave - 1) wsum[wave] = x;
  __syncthreads();
  if (tid == 0) {
    uint32_t t = 0;
    for (uint32_t w = 0; w < kPrefixThreads / kWave; ++w) {
      const uint32_t y = wsum[w];
      wsum[w] = t;
      t += y;
    }
    ustart[regions] = t;
  }
  __syncthreads();
  const uint32_t start = x - v + wsum[wave];
  if (r0 < regions) ustart[r0] = start;
  if (r0 + 1u < regions) ustart[r0 + 1u] = start + v0;
}

// Marking: one workgroup per unit (the grid is an upper bound; workgroups
// past the last unit return at once).  Unit j of region r, which has n_r
// units, takes the chunks [j * chunks / n_r, (j + 1) * chunks / n_r): it
// copies their segment bounds to LDS, marks the DRs their indices name in an
// LDS bitmap of the region and writes the bitmap to its slot of `marks`.
// Lanes work in slots of W (a power of two <= 64, about a segment's length
// in 16-byte pieces): slot s of a wavefront takes one chunk, each of its
// lanes one aligned piece of 8 indices of that chunk's segment, and further
// pieces W apart while any segment has some left, so that a region holding a
// heavy source (many times the average number of indices) makes longer
// segments but more units, not a slower one.
constexpr uint32_t kMarkThreads = 256;
constexpr uint32_t kMarkWaves = kMarkThreads / kWave;
constexpr uint32_t kMarkDepth = 2;

__global__ __launch_bounds__(kMarkThreads) void k_scan_mark(
    const uint16_t* __restrict__ entries, const uint16_t* __restrict__ offs, uint32_t chunks,
    uint32_t stride, uint32_t regions, uint32_t w_log, const uint32_t* __restrict__ plan,
    uint32_t* __restrict__ marks) {
  __shared__ uint32_t bm[kPartRegionWords];
  __shared__ uint16_t s_lo[kPartChunks], s_hi[kPartChunks];
  __shared__ uint32_t s_r;
  const uint32_t* ustart = plan + kPartBandRegions + 1;
  const uint32_t b = blockIdx.x, tid = threadIdx.x, lane = __lane_id();
  const uint32_t wave = __builtin_amdgcn_readfirstlane(tid / kWave);
  if (b >= ustart[regions]) return;   // past the last unit (uniform)
  // the region of unit b: the r with ustart[r] <= b < ustart[r + 1]
  for (uint32_t r = tid; r < regions; r += kMarkThreads)
    if (ustart[r] <= b && b < ustart[r + 1]) s_r = r;
  for (uint32_t w = tid; w < kPartRegionWords; w += kMarkThreads) bm[w] = 0u;
  __syncthreads();
  const uint32_t r = s_r;
  const uint32_t n_r = ustart[r + 1] - ustart[r], j = b - ustart[r];
  const uint32_t c0 = (uint32_t)((uint64_t)j * chunks / n_r);
  const uint32_t c1 = (uint32_t)((uint64_t)(j + 1) * chunks / n_r);
  const uint32_t nc = c1 - c0;
  const uint16_t* lo_row = offs + (uint64_t)r * stride + c0;
  const uint16_t* hi_row = lo_row + stride;
  for (uint32_t c = tid; c < nc; c += kMarkThreads) {
    s_lo[c] = lo_row[c];
    s_hi[c] = hi_row[c];
  }
  __syncthreads();
  // each lane keeps kMarkDepth chunks' pieces in flight: its slot's chunk in
  // kMarkDepth consecutive steps of the wavefront
  const uint32_t W = 1u << w_log, per_wave = kWave >> w_log;   // chunks per wavefront step
  const uint32_t slot = lane >> w_log, k0 = lane & (W - 1u);
  for (uint32_t base = wave * per_wave * kMarkDepth; base < nc;
       base += kMarkWaves * per_wave * kMarkDepth) {   // uniform
    uint32_t lo[kMarkDepth], hi[kMarkDepth], al[kMarkDepth], np[kMarkDepth];
    const uint16_t* seg[kMarkDepth];
#pragma unroll
    for (uint32_t d = 0; d < kMarkDepth; ++d) {
      const uint32_t c = base + d * per_wave + slot;
      lo[d] = c < nc ? (uint32_t)s_lo[c] : 0u;
      hi[d] = c < nc ? (uint32_t)s_hi[c] : 0u;
      al[d] = lo[d] & ~7u;
      np[d] = hi[d] > lo[d] ? (hi[d] - al[d] + 7u) >> 3 : 0u;
      seg[d] = entries + (uint64_t)(c0 + (c < nc ? c : 0u)) * kPartEntries + al[d];
    }
    uint32_t most = 0;
#pragma unroll
    for (uint32_t d = 0; d < kMarkDepth; ++d) most = np[d] > most ? np[d] : most;
    for (uint32_t k = k0; __ballot(k < most) != 0ull; k += W) {   // uniform per wave
      uint4 piece[kMarkDepth];
#pragma unroll
      for (uint32_t d = 0; d < kMarkDepth; ++d)
        piece[d] = k < np[d] ? *reinterpret_cast<const uint4*>(seg[d] + 8u * k)
                             : make_uint4(0u, 0u, 0u, 0u);
#pragma unroll
      for (uint32_t d = 0; d < kMarkDepth; ++d) {
        if (k >= np[d]) continue;
        const uint32_t w4[4] = {piece[d].x, piece[d].y, piece[d].z, piece[d].w};
        const uint32_t p0 = al[d] + 8u * k;
#pragma unroll
        for (uint32_t q = 0; q < 8; ++q) {
          if (p0 + q < lo[d] || p0 + q >= hi[d]) continue;
          const uint32_t e = (w4[q >> 1] >> (16u * (q & 1u))) & 0xFFFFu;
          // an OR whose result is not read: the LDS takes it without a wait
          atomicOr(&bm[e >> 5], 1u << (e & 31u));
        }
      }
    }
  }
  __syncthreads();
  uint32_t* out = marks + (uint64_t)b * kPartRegionWords;
  for (uint32_t w = tid; w < kPartRegionWords; w += kMarkThreads) out[w] = bm[w];
}

// Stamping: workgroup 2r + h ORs half h of region r's unit bitmaps and stores
// the stamp into every marked DR of that half (2^15 DRs), consecutive lanes on
// consecutive DRs.  With ps, every workgroup raises its slot of ps->t_end to
// the clock once all its stores are issued; the end of the scan is the
// largest slot.
constexpr uint32_t kStampThreads = 256;
constexpr uint32_t kHalf = (1u << kPartLog) / 2;
constexpr uint32_t kHalfWords = kPartRegionWords / 2;

__global__ __launch_bounds__(kStampThreads) void k_scan_stamp(const uint32_t* __restrict__ marks,
                                                             const uint32_t* __restrict__ plan,
                                                             uint16_t code,
                                                             uint16_t* __restrict__ le,
                                                             PipeState* ps, uint32_t parity) {
  __shared__ __align__(16) uint32_t bm[kHalfWords];
  const uint32_t tid = threadIdx.x, r = blockIdx.x >> 1, h = blockIdx.x & 1u;
  const uint32_t* ustart = plan + kPartBandRegions + 1;
  const uint32_t u0 = ustart[r], u1 = ustart[r + 1];
  if (u1 > u0) {   // uniform: a region without indices has no unit
    // four words per lane, four units' loads in flight
    static_assert(kHalfWords == 4 * kStampThreads, "one 16-byte piece per lane");
    const uint4* src = reinterpret_cast<const uint4*>(marks + h * kHalfWords) + tid;
    constexpr uint32_t kStride = kPartRegionWords / 4;   // uint4 per unit bitmap
    uint4 x = make_uint4(0u, 0u, 0u, 0u);
    uint32_t u = u0;
    for (; u + 4 <= u1; u += 4) {
      uint4 y[4];
#pragma unroll
      for (uint32_t i = 0; i < 4; ++i) y[i] = src[(uint64_t)(u + i) * kStride];
#pragma unroll
      for (uint32_t i = 0; i < 4; ++i) {
        x.x |= y[i].x; x.y |= y[i].y; x.z |= y[i].z; x.w |= y[i].w;
      }
    }
    for (; u < u1; ++u) {
      const uint4 y = src[(uint64_t)u * kStride];
      x.x |= y.x; x.y |= y.y; x.z |= y.z; x.w |= y.w;
    }
    reinterpret_cast<uint4*>(bm)[tid] = x;
    __syncthreads();
    const uint64_t base = ((uint64_t)r << kPartLog) + (uint64_t)h * kHalf;
    for (uint32_t c = tid; c < kHalf; c += kStampThreads)
      if ((bm[c >> 5] >> (c & 31u)) & 1u) le[base + c] = code;
  }
  if (ps) {
    __syncthreads();
    if (tid == 0) {
      atomicMax(&ps->t_end[parity][blockIdx.x % kEndSlots], (unsigned long long)wall_clock64());
      if (blockIdx.x == 0) ps->scanned[parity] = 1u;
    }
  }
}

// One band: partition rounds of round_chunks chunks, each followed by its
// marking plan, marking and stamping; with ps, the last stamping launch of
// the last band records the end of the scan.
template <int U>
hipError_t launch_band(const uint32_t* pairs, uint64_t n, const Geo& geo, const Band& band,
                       uint16_t code, uint16_t* le, uint16_t* re, uint32_t* touched,
                       uint32_t* tcount, uint16_t* entries, uint16_t* offs, uint32_t* marks,
                       uint32_t round_chunks, PipeState* ps, uint32_t parity, uint32_t unit,
                       hipEvent_t sampled, hipStream_t st) {
  // pairs per chunk: at most kPartEntries / 2 in the pass that samples, so
  // that the chunk's sampled sources fit its LDS entry array
  const uint32_t rows = band.row_hi - band.row_lo;
  const uint32_t ppc = U > 0 ? kPartEntries / (uint32_t)U
                             : kPartEntries / (band.sre && rows < 2 ? 2u : rows);
  const uint64_t per_round = (uint64_t)ppc * round_chunks;
  uint32_t* plan = marks;
  uint32_t* bitmaps = marks + part_plan_words();
  for (uint64_t p = 0; p < n; p += per_round) {
    const uint64_t np = n - p < per_round ? n - p : per_round;
    const uint32_t chunks = (uint32_t)((np + ppc - 1) / ppc);
    // the segment width in 16-byte pieces, about: indices per chunk and region
    const uint64_t per_seg = (np * rows) / ((uint64_t)chunks * band.regions) + 1;
    uint32_t w_log = 0;
    while (w_log < 6 && (8ull << w_log) < per_seg) ++w_log;
    const uint32_t units = band.regions + (uint32_t)((uint64_t)chunks * kPartEntries / unit);
    hipLaunchKernelGGL((k_scan_part<U>), dim3(chunks), dim3(kPartThreads), 0, st, pairs + 2 * p,
                       np, ppc, geo, code, re, touched, tcount, band, entries, offs,
                       round_chunks);
    if (sampled && band.sre && p + per_round >= n) {
      const hipError_t er = hipEventRecord(sampled, st);
      if (er != hipSuccess) return er;
    }
    hipLaunchKernelGGL(k_mark_count, dim3(band.regions), dim3(kPlanThreads), 0, st, offs,
                       chunks, round_chunks, unit, plan);
    hipLaunchKernelGGL(k_mark_prefix, dim3(1), dim3(kPrefixThreads), 0, st, band.regions, plan);
    hipLaunchKernelGGL(k_scan_mark, dim3(units), dim3(kMarkThreads), 0, st, entries, offs,
                       chunks, round_chunks, band.regions, w_log, plan, bitmaps);
    hipLaunchKernelGGL(k_scan_stamp, dim3(2 * band.regions), dim3(kStampThreads), 0, st,
                       bitmaps, plan, code, le + band.lo, p + per_round < n ? nullptr : ps,
                       parity);
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
                                 PipeState* ps, uint32_t parity, uint32_t unit,
                                 hipEvent_t sampled) {
  if (n == 0) return hipSuccess;
  const uint64_t n_le = (uint64_t)geo.u * geo.v_le * geo.G;
  if (round_chunks == 0 || round_chunks > kPartChunks || n_le == 0 || !part_unit_ok(unit))
    return hipErrorInvalidValue;
  const uint64_t row = (uint64_t)geo.v_le * geo.G, band_span = 1ull << kPartBandLog;
  for (uint64_t lo = 0; lo < n_le; lo += band_span) {
    Band b;
    b.lo = lo;
    b.span = n_le - lo < band_span ? n_le - lo : band_span;
    b.regions = (uint32_t)((b.span + kPartRegion - 1) >> kPartLog);
    b.row_lo = (uint32_t)(lo / row);
    b.row_hi = (uint32_t)((lo + b.span - 1) / row + 1);
    b.sre = lo == 0 ? 1u : 0u;
    const bool last = lo + b.span == n_le;
    PipeState* bps = last ? ps : nullptr;
    hipError_t e;
    if (lo == 0 && last && (geo.u == 4 || geo.u == 8 || geo.u == 16)) {
      e = geo.u == 4 ? launch_band<4>(pairs, n, geo, b, code, le, re, touched, tcount, entries,
                                      offs, marks, round_chunks, bps, parity, unit, sampled, st)
        : geo.u == 8 ? launch_band<8>(pairs, n, geo, b, code, le, re, touched, tcount, entries,
                                      offs, marks, round_chunks, bps, parity, unit, sampled, st)
                     : launch_band<16>(pairs, n, geo, b, code, le, re, touched, tcount, entries,
                                       offs, marks, round_chunks, bps, parity, unit, sampled, st);
    } else {
      e = launch_band<0>(pairs, n, geo, b, code, le, re, touched, tcount, entries, offs, marks,
                         round_chunks, bps, parity, unit, sampled, st);
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace srla
