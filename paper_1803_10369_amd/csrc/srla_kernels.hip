// gfx950 end-of-slice kernels of the SRLA hot path (arXiv 1803.10369,
// Section 4.2 and Algorithm 3): the LE and SRE sweeps, the candidate check,
// the merge, Eq8-Eq9 and the SI update.  (The scan is in srla_scan.hip, the
// sort and compaction primitives in srla_sort.hip.)
//
// Memory layout (all device-resident for the monitor's lifetime):
//   LE      uint16 stamps [u][v_le][G]     one LE of G DRs per (row, column)
//   RE      uint16 stamps [u][v_re][g]     one SRE of g DRs per (row, column)
//   SI      uint32 counters [u][v_re][16]  SI bit = counter > 0
//   bitmap  uint64 [u][v_le][G/64]         LE DRs inside the window
//   act     uint64 pairs, 1 bit per SRE DR: word 2w holds bits 64w..64w+63
//           "inside now", word 2w+1 the same DRs "inside after the slide"
// A DR is a 16-bit slice stamp (see srla_internal.h), so Algorithm 3's slide
// of every DR costs nothing.  No kernel here contains a dense contraction, so
// nothing uses MFMA; the sweeps stream HBM, the estimate gathers from the
// L2-resident bitmaps.
#include "srla_internal.h"

namespace srla {

// ------------------------------------------------------------------ fill

__global__ __launch_bounds__(kBlock) void k_fill_u32(uint32_t* __restrict__ p, uint32_t v,
                                                    uint64_t n) {
  uint64_t i = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  for (; i < n; i += stride) p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, uint32_t value, uint64_t n, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint64_t blocks = (n + kBlock - 1) / kBlock;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(kBlock), 0, st, p, value, n);
  return hipGetLastError();
}

// ------------------------------------------------------------------ sweep
// |LDR(i)|^k of Section 4.2 for every row, the LE activity bitmap that the
// estimate kernel ANDs across rows, and the scrub of stamps about to alias.
// One thread reads 8 DRs (16 bytes) per step, all steps' loads first; 8
// neighbouring lanes OR their 8-bit masks into one 64-bit bitmap word.  A
// block's count goes to one of kFillSlots partial sums of its row (by block
// index), so no more than a few blocks add to one address; the RE sweep
// folds the partial sums into the row fills.  Grid: x = chunks of a row,
// y = row.

constexpr int kSweepSteps = 8;
constexpr uint64_t kSweepTile = (uint64_t)kBlock * 8 * kSweepSteps;  // DRs per block

// The slice's close, by one wavefront: the end of its scans is the latest of
// the marker's clock and the partitioned scan's slots, which start over at
// zero (a slice without scans: now); the snapshot's stamp code is recorded
// for the other parity's next snapshot.
__device__ __forceinline__ void close_slice_clock(PipeState* __restrict__ ps, uint32_t p,
                                                  uint32_t lane, uint32_t now) {
  unsigned long long t = ps->t_end[p][lane];
  ps->t_end[p][lane] = 0ull;
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)t, d);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(t >> 32), d);
    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
    t = o > t ? o : t;
  }
  if (lane == 0) {
    const unsigned long long ts = ps->t_scan[p] > t ? ps->t_scan[p] : t;
    ps->t_close[p] = ps->scanned[p] ? ts : wall_clock64();
    ps->t_scan[p] = 0ull;
    ps->scanned[p] = 0u;
    ps->snap_code[p] = now;
  }
}

// LE tile bx of row `row`
__device__ __forceinline__ void sweep_le_tile(uint16_t* __restrict__ le,
                                              uint64_t* __restrict__ bitmap,
                                              unsigned long long* __restrict__ fill_part,
                                              uint64_t row_cells, uint32_t now, uint32_t k,
                                              uint32_t bx, uint32_t row, uint32_t* part) {
  // The window's stamp codes form one interval on the circle of codes: a
  // nonzero cell c is inside iff (c - lo) mod 2^16 <= w, with lo the code of
  // slice e-k+1 (the interval may pass over the unused code 0, which widens w
  // by one); the same test with k = kScrubAge tells the cells to keep.
  const uint32_t lo_w = now > k - 1u ? now - (k - 1u) : now + kStampPeriod - (k - 1u);
  const uint32_t w_w = (now - lo_w) & 0xFFFFu;
  const uint32_t lo_s =
      now > kScrubAge - 1u ? now - (kScrubAge - 1u) : now + kStampPeriod - (kScrubAge - 1u);
  const uint32_t w_s = (now - lo_s) & 0xFFFFu;
  uint16_t* rowp = le + (uint64_t)row * row_cells;
  uint64_t* bmp = bitmap + (uint64_t)row * (row_cells / 64);
  const uint32_t lane = threadIdx.x & (kWave - 1);
  uint32_t count = 0;
  // every step's load first (a lane past the row's end reads the row's first
  // 8 DRs and ignores them), so the block has all its loads in flight at once
  uint4 qs[kSweepSteps];
#pragma unroll
  for (int s = 0; s < kSweepSteps; ++s) {
    const uint64_t c8 = ((uint64_t)bx * kSweepTile) + ((uint64_t)s * kBlock + threadIdx.x) * 8;
    qs[s] = *reinterpret_cast<const uint4*>(rowp + (c8 < row_cells ? c8 : 0));
  }
#pragma unroll
  for (int s = 0; s < kSweepSteps; ++s) {
    const uint64_t c8 = ((uint64_t)bx * kSweepTile) + ((uint64_t)s * kBlock + threadIdx.x) * 8;
    const bool valid = c8 < row_cells;
    uint32_t m8 = 0;
    if (valid) {
      const uint4 q = qs[s];
      uint32_t w[4] = {q.x, q.y, q.z, q.w};
      bool dirty = false;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const uint32_t lo = w[j] & 0xFFFFu, hi = w[j] >> 16;
        const bool in_lo = lo != 0u && ((lo - lo_w) & 0xFFFFu) <= w_w;
        const bool in_hi = hi != 0u && ((hi - lo_w) & 0xFFFFu) <= w_w;
        const bool old_lo = lo != 0u && ((lo - lo_s) & 0xFFFFu) > w_s;
        const bool old_hi = hi != 0u && ((hi - lo_s) & 0xFFFFu) > w_s;
        m8 |= ((uint32_t)in_lo << (2 * j)) | ((uint32_t)in_hi << (2 * j + 1));
        dirty |= old_lo | old_hi;
        w[j] = (old_lo ? 0u : lo) | ((old_hi ? 0u : hi) << 16);
      }
      if (dirty) *reinterpret_cast<uint4*>(rowp + c8) = make_uint4(w[0], w[1], w[2], w[3]);
      count += __popc(m8);
    }
    // lanes 8q..8q+7 cover 64 consecutive DRs: bit 8*(lane%8)+x is DR c8+x
    uint32_t lo32 = (lane & 4) ? 0u : m8 << (8 * (lane & 3));
    uint32_t hi32 = (lane & 4) ? m8 << (8 * (lane & 3)) : 0u;
    lo32 |= __shfl_xor(lo32, 1); hi32 |= __shfl_xor(hi32, 1);
    lo32 |= __shfl_xor(lo32, 2); hi32 |= __shfl_xor(hi32, 2);
    lo32 |= __shfl_xor(lo32, 4); hi32 |= __shfl_xor(hi32, 4);
    if (valid && (lane & 7) == 0) bmp[c8 / 64] = ((uint64_t)hi32 << 32) | lo32;
  }
  // block total -> one 64-bit atomic per block
  for (int off = kWave / 2; off > 0; off >>= 1) count += __shfl_xor(count, off);
  if (lane == 0) part[threadIdx.x / kWave] = count;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += part[w];
    if (t) atomicAdd(&fill_part[(uint64_t)row * kFillSlots + (bx % kFillSlots)], t);
  }
}


// RE activity: every SRE DR of the array (flat index i over [u][v_re][g]) as
// two interleaved bitmaps -- bit i of `now` = DR inside the window ending at
// this slice, bit i of `next` = still inside after Algorithm 3's slide
// (distance + 1 < k); the now and next words of the same DRs sit side by
// side, so a candidate's SRE costs one 16-byte load per row.  The finalize
// and estimate kernels read g bits per (row, column) from these (L2-resident)
// maps instead of g scattered stamps.  Old stamps are scrubbed here as in the
// LE sweep.  Handles any cell count (ragged last word).

// Eq8: UP = prod_i |LDR(i)|^k / (g' * v), in this order, in FP64.
__device__ __forceinline__ double eq8(const unsigned long long* __restrict__ row_fill, uint32_t u,
                                     uint32_t G, uint32_t v_le) {
  double p = 1.0;
  for (uint32_t i = 0; i < u; ++i) p = p * ((double)row_fill[i] / ((double)G * (double)v_le));
  return p;
}

// One thread takes kReSteps groups of 8 DRs of RE tile bx, their loads
// issued first.
constexpr int kReSteps = 4;

__device__ __forceinline__ void sweep_re_tile(uint16_t* __restrict__ re, uint64_t n,
                                              uint64_t* __restrict__ act, uint32_t now,
                                              uint32_t k, uint32_t bx) {
  const uint32_t lane = threadIdx.x & (kWave - 1);
  uint4 qs[kReSteps];
#pragma unroll
  for (int st8 = 0; st8 < kReSteps; ++st8) {
    const uint64_t c8 = (((uint64_t)bx * kReSteps + st8) * kBlock + threadIdx.x) * 8;
    qs[st8] = c8 + 8 <= n ? *reinterpret_cast<const uint4*>(re + c8) : make_uint4(0u, 0u, 0u, 0u);
  }
#pragma unroll
  for (int st8 = 0; st8 < kReSteps; ++st8) {
  const uint64_t c8 = (((uint64_t)bx * kReSteps + st8) * kBlock + threadIdx.x) * 8;
  uint32_t m_now = 0, m_next = 0;
  if (c8 < n) {
    uint32_t cell[8];
    const bool full = c8 + 8 <= n;
    if (full) {
      const uint4 q = qs[st8];
      const uint32_t w[4] = {q.x, q.y, q.z, q.w};
#pragma unroll
      for (int j = 0; j < 4; ++j) { cell[2 * j] = w[j] & 0xFFFFu; cell[2 * j + 1] = w[j] >> 16; }
    } else {
#pragma unroll
      for (int j = 0; j < 8; ++j) cell[j] = c8 + j < n ? re[c8 + j] : 0u;
    }
    bool dirty = false;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
      if (cell[j]) {
        const uint32_t age = stamp_age(now, cell[j]);
        if (age < k) m_now |= 1u << j;
        if (age + 1u < k) m_next |= 1u << j;
        if (age >= kScrubAge) { cell[j] = 0; dirty = true; }
      }
    }
    if (dirty) {
      if (full) {
        *reinterpret_cast<uint4*>(re + c8) =
            make_uint4(cell[0] | (cell[1] << 16), cell[2] | (cell[3] << 16),
                       cell[4] | (cell[5] << 16), cell[6] | (cell[7] << 16));
      } else {
        for (int j = 0; j < 8; ++j)
          if (c8 + j < n) re[c8 + j] = (uint16_t)cell[j];
      }
    }
  }
  const uint32_t sh = 8 * (lane & 3);
  uint32_t a_lo = (lane & 4) ? 0u : m_now << sh, a_hi = (lane & 4) ? m_now << sh : 0u;
  uint32_t b_lo = (lane & 4) ? 0u : m_next << sh, b_hi = (lane & 4) ? m_next << sh : 0u;
#pragma unroll
  for (int off = 1; off < 8; off <<= 1) {
    a_lo |= __shfl_xor(a_lo, off); a_hi |= __shfl_xor(a_hi, off);
    b_lo |= __shfl_xor(b_lo, off); b_hi |= __shfl_xor(b_hi, off);
  }
  if (c8 < n && (lane & 7) == 0) {
    act[2 * (c8 / 64)] = ((uint64_t)a_hi << 32) | a_lo;
    act[2 * (c8 / 64) + 1] = ((uint64_t)b_hi << 32) | b_lo;
  }
  }
}

// The snapshot's sweeps in one launch: blocks [0, u * le_tiles) take the LE
// tiles (row by row), the rest the RE tiles, side by side.
__global__ __launch_bounds__(kBlock) void k_sweep(uint16_t* __restrict__ le,
                                                 uint64_t* __restrict__ bitmap,
                                                 unsigned long long* __restrict__ fill_part,
                                                 uint64_t row_cells, uint32_t le_tiles,
                                                 uint32_t u, uint16_t* __restrict__ re,
                                                 uint64_t n_re, uint64_t* __restrict__ act,
                                                 PipeState* __restrict__ ps, uint32_t p,
                                                 uint32_t k) {
  __shared__ uint32_t part[kBlock / kWave];
  // the slice being snapshotted: the code after the other parity's
  const uint32_t now = ps->snap_code[p ^ 1u] % kStampPeriod + 1u;
  const uint32_t b = blockIdx.x, n_le_blocks = le_tiles * u;
  if (b == 0 && threadIdx.x < kWave) close_slice_clock(ps, p, threadIdx.x, now);
  if (b < n_le_blocks)
    sweep_le_tile(le, bitmap, fill_part, row_cells, now, k, b % le_tiles, b / le_tiles, part);
  else
    sweep_re_tile(re, n_re, act, now, k, b - n_le_blocks);
}

hipError_t launch_sweep(uint16_t* le, uint64_t* bitmap, unsigned long long* fill_part,
                        uint16_t* re, uint64_t n_re, uint64_t* act, const Geo& geo,
                        PipeState* ps, uint32_t p, hipStream_t st) {
  const uint64_t row_cells = (uint64_t)geo.v_le * geo.G;
  const uint64_t le_tiles = (row_cells + kSweepTile - 1) / kSweepTile;
  const uint64_t per = (uint64_t)8 * kBlock * kReSteps;
  const uint64_t re_tiles = n_re ? (n_re + per - 1) / per : 1;
  const uint64_t blocks = le_tiles * geo.u + re_tiles;
  if (blocks > 0x7FFFFFFFull) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sweep, dim3((uint32_t)blocks), dim3(kBlock), 0, st, le, bitmap, fill_part,
                     row_cells, (uint32_t)le_tiles, geo.u, re, n_re, act, ps, p, geo.k);
  return hipGetLastError();
}

// |LDR(i)|^k from the LE sweep's partial sums and Eq8, by one block
__device__ __forceinline__ void fold_row_fills(const unsigned long long* __restrict__ fill_part,
                                               unsigned long long* __restrict__ row_fill,
                                               uint32_t u, uint32_t G, uint32_t v_le,
                                               double* __restrict__ up) {
  // one wave per row: lane l adds slot l and clears it for the parity's
  // next snapshot
  const uint32_t lane0 = threadIdx.x & (kWave - 1);
  for (uint32_t r = threadIdx.x / kWave; r < u; r += kBlock / kWave) {
    unsigned long long v = 0ull;
    if (lane0 < kFillSlots) {
      v = fill_part[(uint64_t)r * kFillSlots + lane0];
      const_cast<unsigned long long*>(fill_part)[(uint64_t)r * kFillSlots + lane0] = 0ull;
    }
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off);
    if (lane0 == 0) row_fill[r] = v;
  }
  __syncthreads();
  if (threadIdx.x == 0) *up = eq8(row_fill, u, G, v_le);
}

// The g "now" and g "next" activity bits of the SRE in row r, column col
// (g <= 64) from the interleaved map, in two steps so that callers can issue
// the loads early: sre_fetch reads the 16-byte word that holds the SRE's first
// bit and, unless g divides 64 (then no SRE straddles two words), the one
// after it (the map is allocated with a spare word, so this stays in bounds);
// sre_combine extracts the bits, taking the second word only when the SRE
// straddles a 64-bit boundary.
struct SreWords {
  uint4 q0, q1;
  uint32_t sh;
};

__device__ __forceinline__ SreWords sre_fetch(const uint64_t* __restrict__ act, const Geo& geo,
                                              uint32_t r, uint32_t col) {
  const uint64_t off = ((uint64_t)r * geo.v_re + col) * geo.g;
  const uint64_t w = off >> 6;
  SreWords s;
  s.q0 = reinterpret_cast<const uint4*>(act)[w];
  s.q1 = (64u % geo.g) != 0u ? reinterpret_cast<const uint4*>(act)[w + 1]
                             : make_uint4(0u, 0u, 0u, 0u);
  s.sh = (uint32_t)(off & 63u);
  return s;
}

__device__ __forceinline__ void sre_combine(const SreWords& s, uint32_t g, uint64_t* now,
                                            uint64_t* next) {
  uint64_t a = ((((uint64_t)s.q0.y) << 32) | s.q0.x) >> s.sh;
  uint64_t b = ((((uint64_t)s.q0.w) << 32) | s.q0.z) >> s.sh;
  if (s.sh + g > 64u) {
    a |= ((((uint64_t)s.q1.y) << 32) | s.q1.x) << (64u - s.sh);
    b |= ((((uint64_t)s.q1.w) << 32) | s.q1.z) << (64u - s.sh);
  }
  const uint64_t mask = g == 64u ? ~0ull : ((1ull << g) - 1ull);
  *now = a & mask;
  *next = b & mask;
}

__device__ __forceinline__ void sre_bits(const uint64_t* __restrict__ act, const Geo& geo,
                                         uint32_t r, uint32_t col, uint64_t* now,
                                         uint64_t* next) {
  sre_combine(sre_fetch(act, geo, r, col), geo.g, now, next);
}

// SI as per-bit counters: counter (r, col, b) = number of carried candidates
// whose row-r column is col and whose own SI bit H4(aip) is b, so SI bit
// (r, col, b) of the paper is "counter > 0" (Section 4.1: the bit is set for
// every carried candidate, Algorithm 3).
__device__ __forceinline__ uint64_t si_slot(const Geo& geo, uint32_t r, uint32_t col,
                                            uint32_t bit) {
  return ((uint64_t)r * geo.v_re + col) * 16u + bit;
}

// ------------------------------------------------------------------ finalize
// Algorithm 2's candidate check under the slice-synchronous reading: every
// distinct source sampled in the slice (sorted[] is sorted, so the first of
// each run stands for the source) is a new candidate iff its union SRE has
// at least ceil(rho*g) DRs inside the window (Algorithm 1 with DRjoin = max:
// a union DR is inside iff it is inside in every row) and its own bit of the
// union SI (AND over rows) is still clear.  SI is as the previous slide left it.

// kU >= geo.u: the rows are unrolled so that every row's SRE and SI loads are
// in flight before the first is used.
template <int kU>
__global__ __launch_bounds__(kBlock) void k_finalize(const uint32_t* __restrict__ sorted,
                                                    const uint32_t* __restrict__ n_dev,
                                                    const uint64_t* __restrict__ act,
                                                    const uint32_t* __restrict__ si_cnt,
                                                    Geo geo, uint8_t* __restrict__ mark,
                                                    Counters* __restrict__ cnt,
                                                    const unsigned long long* __restrict__ fill_part,
                                                    unsigned long long* __restrict__ row_fill,
                                                    double* __restrict__ up) {
  // the snapshot's LE sweep left partial row sums: block 0 folds them and
  // evaluates Eq8 for the estimate that follows
  if (fill_part && blockIdx.x == 0) fold_row_fills(fill_part, row_fill, geo.u, geo.G, geo.v_le, up);
  const uint32_t n = *n_dev;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  uint32_t firsts = 0;
  // the loop bound is uniform per wavefront, so the ballot below sees all lanes
  for (uint64_t base = (uint64_t)blockIdx.x * kBlock; base < n; base += stride) {
    const uint64_t i = base + threadIdx.x;
    bool first = false;
    if (i < n) {
      const uint32_t a = sorted[i];
      first = (i == 0) || (sorted[i - 1] != a);
      uint8_t f = 0;
      if (first) {
        const uint32_t bit = hrange(mas(geo.h4, a), 16u);
        SreWords sw[kU];
        uint32_t si[kU];
#pragma unroll
        for (int r = 0; r < kU; ++r) {
          if (r < (int)geo.u) {
            const uint32_t col = hrange(mas(geo.rh[r], a), geo.v_re);
            sw[r] = sre_fetch(act, geo, r, col);
            si[r] = si_cnt[si_slot(geo, r, col, bit)];
          }
        }
        uint64_t ure = ~0ull;
        bool usi = true;
#pragma unroll
        for (int r = 0; r < kU; ++r) {
          if (r < (int)geo.u) {
            uint64_t now, next;
            sre_combine(sw[r], geo.g, &now, &next);
            ure &= now;
            usi = usi && si[r] != 0u;
          }
        }
        f = ((uint32_t)__popcll(ure) >= geo.t_re && !usi) ? 1 : 0;
      }
      mark[i] = f;
    }
    firsts += (uint32_t)__popcll(__ballot(first));
  }
  // one add per workgroup to the shared counter
  __shared__ uint32_t part[kBlock / kWave];
  if (__lane_id() == 0) part[threadIdx.x / kWave] = firsts;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += part[w];
    if (t) atomicAdd(&cnt->n_unique, t);
  }
}

hipError_t launch_finalize(const uint32_t* sorted, const uint32_t* n_dev, const uint64_t* act,
                           const uint32_t* si_cnt, const Geo& geo, uint8_t* mark, Counters* cnt,
                           const unsigned long long* fill_part, unsigned long long* row_fill,
                           double* up, hipStream_t st) {
  if (geo.u <= 4)
    hipLaunchKernelGGL(k_finalize<4>, dim3(kPipeBlocks), dim3(kBlock), 0, st, sorted, n_dev, act,
                       si_cnt, geo, mark, cnt, fill_part, row_fill, up);
  else if (geo.u <= 8)
    hipLaunchKernelGGL(k_finalize<8>, dim3(kPipeBlocks), dim3(kBlock), 0, st, sorted, n_dev, act,
                       si_cnt, geo, mark, cnt, fill_part, row_fill, up);
  else
    hipLaunchKernelGGL(k_finalize<16>, dim3(kPipeBlocks), dim3(kBlock), 0, st, sorted, n_dev,
                       act, si_cnt, geo, mark, cnt, fill_part, row_fill, up);
  return hipGetLastError();
}

// ------------------------------------------------------------------ join
// CSIP_t = NCSIP_{t-1} + N_t (Algorithms 2-3), listed as the carried list
// (ascending, already in `cand`) followed by the new candidates (ascending):
// N_t is appended behind the carried list.  The two sets are disjoint (a
// carried candidate's own SI bit is set, so it never passes the check).

__global__ __launch_bounds__(kBlock) void k_join(const PipeState* __restrict__ ps,
                                                const uint32_t* __restrict__ news,
                                                Counters* __restrict__ cnt, uint64_t cap,
                                                uint32_t* __restrict__ cand) {
  const uint64_t n_old = ps->n_ncsip;
  const uint64_t n_new = cnt->n_new;
  const uint64_t total = n_old + n_new;
  const uint64_t m = total < cap ? total : cap;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    cnt->n_cand = (uint32_t)m;
    cnt->overflow = total > cap ? 1u : 0u;
  }
  for (uint64_t k = n_old + (uint64_t)blockIdx.x * kBlock + threadIdx.x; k < m;
       k += (uint64_t)gridDim.x * kBlock)
    cand[k] = news[k - n_old];
}

hipError_t launch_join(const PipeState* ps, const uint32_t* news, Counters* cnt, uint64_t cap,
                       uint32_t* cand, hipStream_t st) {
  hipLaunchKernelGGL(k_join, dim3(kPipeBlocks), dim3(kBlock), 0, st, ps, news, cnt, cap, cand);
  return hipGetLastError();
}

// ------------------------------------------------------------------ carried list
// NCSIP_t, ascending, from the candidates CSIP_t kept by Algorithm 3: their
// compaction lists the kept carried candidates (ascending) and then the kept
// new ones (ascending); k_count_keep counts the first run, and k_merge_runs
// merges the two by merge path (each thread writes kMergePer outputs after
// one binary search along its diagonal).

// A few workgroups, 16 flags per load: every workgroup adds its count to
// one counter, and such adds queue up behind each other.
constexpr uint32_t kCountKeepBlocks = 64;

__global__ __launch_bounds__(kBlock) void k_count_keep(const uint8_t* __restrict__ cflags,
                                                      const PipeState* __restrict__ ps,
                                                      Counters* __restrict__ cnt) {
  const uint64_t n_c = ps->n_ncsip < cnt->n_cand ? ps->n_ncsip : cnt->n_cand;
  const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  uint32_t c = 0;
  const uint4* f4 = reinterpret_cast<const uint4*>(cflags);
  for (uint64_t q = t; q < n_c / 16; q += stride) {
    const uint4 v = f4[q];
    c += __popc(v.x & 0x08080808u) + __popc(v.y & 0x08080808u) + __popc(v.z & 0x08080808u) +
         __popc(v.w & 0x08080808u);
  }
  for (uint64_t k = n_c / 16 * 16 + t; k < n_c; k += stride) c += (cflags[k] & 8u) ? 1u : 0u;
  for (int off = kWave / 2; off > 0; off >>= 1) c += __shfl_xor(c, off);
  __shared__ uint32_t part[kBlock / kWave];
  if ((threadIdx.x & (kWave - 1)) == 0) part[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int w = 0; w < kBlock / kWave; ++w) t += part[w];
    if (t) atomicAdd(&cnt->n_keep_a, t);
  }
}

hipError_t launch_count_keep(const uint8_t* cflags, const PipeState* ps, Counters* cnt,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_count_keep, dim3(kCountKeepBlocks), dim3(kBlock), 0, st, cflags, ps, cnt);
  return hipGetLastError();
}

constexpr uint32_t kMergePer = 8;

// runs [0, *na) and [*na, *n) of `in`, each ascending, merged into out
__global__ __launch_bounds__(kBlock) void k_merge_runs(const uint32_t* __restrict__ in,
                                                      const uint32_t* __restrict__ na_p,
                                                      const uint32_t* __restrict__ n_p,
                                                      uint32_t* __restrict__ out) {
  const uint64_t m = *n_p;
  const uint64_t na = *na_p < m ? *na_p : m;
  const uint64_t nb = m - na;
  const uint32_t* a = in;
  const uint32_t* b = in + na;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock * kMergePer;
  for (uint64_t k0 = ((uint64_t)blockIdx.x * kBlock + threadIdx.x) * kMergePer; k0 < m;
       k0 += stride) {
    uint64_t lo = k0 > nb ? k0 - nb : 0, hi = k0 < na ? k0 : na;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (a[mid] < b[k0 - mid - 1]) lo = mid + 1; else hi = mid;
    }
    uint64_t i = lo, j = k0 - lo;
    const uint64_t kend = k0 + kMergePer < m ? k0 + kMergePer : m;
    for (uint64_t k = k0; k < kend; ++k) {
      // i + j = k < na + nb, so with run b used up run a has one left
      if (j >= nb || (i < na && a[i] < b[j])) out[k] = a[i++];
      else out[k] = b[j++];
    }
  }
}

hipError_t launch_merge_runs(const uint32_t* in, const uint32_t* na, const uint32_t* n,
                             uint32_t* out, hipStream_t st) {
  // twice the pipeline grid: every CU full, so more of the binary searches'
  // dependent loads are in flight at once
  hipLaunchKernelGGL(k_merge_runs, dim3(2 * kPipeBlocks), dim3(kBlock), 0, st, in, na, n, out);
  return hipGetLastError();
}

// The carried list NCSIP_t is the head of the next slice's report: its *n
// addresses go into that report's ip array (pinned host memory) now, beside
// the next slice's scans, instead of after its candidate check.
//
// Stores into host memory go out over PCIe, far slower than HBM, and they
// hold up the other traffic of the caches they pass: from workgroups spread
// over the XCDs, with ordinary stores, the next slice's partition kernel ran
// 262 instead of 133 us beside the copy.  So the copy runs on one XCD only
// (workgroups are dispatched to the XCDs round-robin: only the blocks with
// blockIdx % kPrecopyXcds == 0 work, the others return at once) and with
// non-temporal stores, which still fill the link (9 MB in about 170 us) but
// leave that kernel almost untouched (a standalone copy of 9 MB beside the
// partition kernel: 139 us alone, 139 us beside 8 such workgroups, 188 us
// beside 16 ordinary spread ones).
constexpr uint32_t kPrecopyXcds = 8;
constexpr uint32_t kPrecopyBlocks = 8;   // working workgroups, all on one XCD

__global__ __launch_bounds__(kBlock) void k_ip_precopy(const uint32_t* __restrict__ src,
                                                      const uint32_t* __restrict__ n_p,
                                                      uint32_t* __restrict__ dst) {
  if (blockIdx.x % kPrecopyXcds) return;
  const uint64_t n = *n_p;
  const uint64_t n4 = n / 4;
  const uint64_t stride = (uint64_t)(gridDim.x / kPrecopyXcds) * kBlock;
  const uint64_t t = (uint64_t)(blockIdx.x / kPrecopyXcds) * kBlock + threadIdx.x;
  for (uint64_t i = t; i < n4; i += stride) {
    const uint4 v = reinterpret_cast<const uint4*>(src)[i];
    uint32_t* d = dst + 4 * i;   // one 16-byte non-temporal store
    __builtin_nontemporal_store(v.x, d);
    __builtin_nontemporal_store(v.y, d + 1);
    __builtin_nontemporal_store(v.z, d + 2);
    __builtin_nontemporal_store(v.w, d + 3);
  }
  if (t < n - n4 * 4) __builtin_nontemporal_store(src[n4 * 4 + t], dst + n4 * 4 + t);
}

hipError_t launch_ip_precopy(const uint32_t* src, const uint32_t* n, uint32_t* dst,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_ip_precopy, dim3(kPrecopyXcds * kPrecopyBlocks), dim3(kBlock), 0, st, src,
                     n, dst);
  return hipGetLastError();
}

// ------------------------------------------------------------------ Eq8
// UP = prod_i |LDR(i)|^k / (g' * v), in this order, in FP64.

__global__ void k_union_prob(const unsigned long long* __restrict__ row_fill, Geo geo,
                             double* __restrict__ up) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *up = eq8(row_fill, geo.u, geo.G, geo.v_le);
}

hipError_t launch_union_prob(const unsigned long long* row_fill, const Geo& geo, double* up,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_union_prob, dim3(1), dim3(1), 0, st, row_fill, geo, up);
  return hipGetLastError();
}


// ------------------------------------------------------------------ estimate
// For every candidate: |ULE|^k from the LE activity bitmap (AND over the u
// rows, popcount), |URE|^k now and after the slide from the RE activity
// bitmaps, Eq9 in FP64, and the flags.
//
// A block takes 256 candidates at a time.  Their addresses are staged in LDS
// first; then a group of 2^lg_log2 lanes owns one candidate: every lane hashes
// the address for all u rows in registers and issues its u bitmap loads of
// kWpl words each (with G = 1024, eight lanes read one 128-byte line per row
// in 16-byte pieces) and, for the lane whose index is a row number, that
// row's SRE load, all before the first wait, so a candidate costs one cache
// round trip rather than one per row.
// Cross-lane shuffles reduce the group; the counts go to LDS.  Eq9 then runs
// with one thread per candidate, and the report entries leave with one
// coalesced store per array (into pinned host memory mapped into the GPU's
// address space, or into device staging).  The block barriers order LDS
// only, so a block's report stores stay in flight while it gathers its next
// candidates; U and W are written only when their buffers are given (the lean
// report leaves them out).

constexpr uint32_t kEstPerBlock = kBlock;
// workgroups that work when no LE row needs gathering (every row full): four
// per CU keep the report's PCIe writes near their ceiling (measured on the
// backbone workload, 2M candidates: 0.53 ms with 1024 workgroups, 0.56 ms
// with 512, 0.61 ms with 256) and leave room on every CU for a scan running
// beside the estimate
constexpr uint32_t kEstBlocksNoGather = 1024;

// a workgroup barrier that orders LDS accesses only (global stores issued
// before it may still be in flight)
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// kU >= geo.u is the unrolled row count; kWpl (1 or 2) bitmap words per lane
// and load, 2 only when G / 64 is even; the launch guarantees 2^lg_log2 >= u
// (each lane handles at most one SRE row).
template <int kU, int kWpl>
__global__ __launch_bounds__(kBlock) void k_estimate(
    const uint32_t* __restrict__ csip, const Counters* __restrict__ cnt,
    const PipeState* __restrict__ ps, uint32_t skip_carried_ip,
    const uint64_t* __restrict__ bitmap, const uint64_t* __restrict__ act,
    const double* __restrict__ up_p, const unsigned long long* __restrict__ row_fill, Geo geo,
    uint32_t lg_log2, uint8_t* __restrict__ cflags, uint32_t* __restrict__ out_ip,
    double* __restrict__ out_est, uint8_t* __restrict__ out_flags, uint32_t* __restrict__ out_U,
    uint8_t* __restrict__ out_W, double* __restrict__ mir_est,
    uint8_t* __restrict__ mir_flags, unsigned long long* __restrict__ rep_bytes) {
  __shared__ uint32_t s_ip[kEstPerBlock], s_U[kEstPerBlock];
  __shared__ uint8_t s_W[kEstPerBlock], s_Wn[kEstPerBlock];
  __shared__ __align__(16) double s_e[kEstPerBlock];
  __shared__ __align__(16) uint8_t s_f[kEstPerBlock];
  const uint32_t lg = 1u << lg_log2;
  const uint32_t per_round = kBlock >> lg_log2;          // candidates per round
  const uint32_t sub = threadIdx.x & (lg - 1u);
  const uint32_t n = cnt->n_cand;
  // CSIP is the carried list (its first n_c entries) and then the new
  // candidates; with skip_carried_ip the carried addresses are in the
  // report's ip array already
  const uint64_t n_c = ps->n_ncsip;
  const uint64_t ip_from = skip_carried_ip ? n_c : 0;
  const uint64_t gmask = geo.g == 64u ? ~0ull : ((1ull << geo.g) - 1ull);
  // rows whose every LE DR is inside the window (|LDR(i)|^k = g' * v): their
  // bitmap words are all ones, the identity of the AND, so they are not read
  uint32_t gather = 0;
  const unsigned long long row_cells = (unsigned long long)geo.G * geo.v_le;
#pragma unroll
  for (int r = 0; r < kU; ++r)
    if (r < (int)geo.u && row_fill[r] != row_cells) gather |= 1u << r;
  // with nothing to gather from the LE the kernel is bound by its report
  // stores into host memory, which a few workgroups saturate: the rest exit
  // at once and leave their CUs to a scan running beside it
  const uint32_t active =
      gather == 0u && gridDim.x > kEstBlocksNoGather ? kEstBlocksNoGather : gridDim.x;
  if (blockIdx.x >= active) return;
  uint32_t wrote = 0;   // bytes this thread stores into the report arrays
  for (uint64_t base = (uint64_t)blockIdx.x * kEstPerBlock; base < n;
       base += (uint64_t)active * kEstPerBlock) {
    const uint32_t in_batch =
        (uint32_t)(n - base < (uint64_t)kEstPerBlock ? n - base : (uint64_t)kEstPerBlock);
    if (threadIdx.x < in_batch) s_ip[threadIdx.x] = csip[base + threadIdx.x];
    lds_barrier();
    for (uint32_t first = 0; first < in_batch; first += per_round) {
      const uint32_t local = first + (threadIdx.x >> lg_log2);
      const bool valid = local < in_batch;
      const uint32_t a = s_ip[valid ? local : 0u];
      uint32_t my_h = 0;
#pragma unroll
      for (int r = 0; r < kU; ++r)
        if (r < (int)geo.u && (uint32_t)r == sub) my_h = mas(geo.rh[r], a);
      uint32_t ucount = 0;
      uint64_t m_now = ~0ull, m_next = ~0ull;
      const bool sre_lane = valid && sub < geo.u;
      SreWords sw;
      if (sre_lane) sw = sre_fetch(act, geo, sub, hrange(my_h, geo.v_re));
      if (valid && gather == 0u) {
        // every row full: the union LE is full as well
        if (sub == 0) ucount = geo.G;
      } else if (valid) {
        for (uint32_t x = kWpl * sub; x < geo.words; x += kWpl * lg) {
          if constexpr (kWpl == 2) {
            uint4 w[kU];
#pragma unroll
            for (int r = 0; r < kU; ++r)
              w[r] = (gather >> r) & 1u
                         ? *reinterpret_cast<const uint4*>(
                               bitmap + ((uint64_t)r * geo.v_le +
                                         hrange(mas(geo.rh[r], a), geo.v_le)) * geo.words + x)
                         : make_uint4(~0u, ~0u, ~0u, ~0u);
            uint32_t acc[4] = {~0u, ~0u, ~0u, ~0u};
#pragma unroll
            for (int r = 0; r < kU; ++r) {
              acc[0] &= w[r].x; acc[1] &= w[r].y; acc[2] &= w[r].z; acc[3] &= w[r].w;
            }
            ucount += (uint32_t)(__popc(acc[0]) + __popc(acc[1]) + __popc(acc[2]) +
                                 __popc(acc[3]));
          } else {
            uint64_t w[kU];
#pragma unroll
            for (int r = 0; r < kU; ++r)
              w[r] = (gather >> r) & 1u
                         ? bitmap[((uint64_t)r * geo.v_le + hrange(mas(geo.rh[r], a), geo.v_le)) *
                                      geo.words + x]
                         : ~0ull;
            uint64_t acc = ~0ull;
#pragma unroll
            for (int r = 0; r < kU; ++r) acc &= w[r];
            ucount += (uint32_t)__popcll(acc);
          }
        }
      }
      if (sre_lane) sre_combine(sw, geo.g, &m_now, &m_next);
      uint32_t now_lo = (uint32_t)m_now, now_hi = (uint32_t)(m_now >> 32);
      uint32_t nx_lo = (uint32_t)m_next, nx_hi = (uint32_t)(m_next >> 32);
      for (uint32_t off = lg >> 1; off > 0; off >>= 1) {
        ucount += __shfl_xor(ucount, (int)off);
        now_lo &= __shfl_xor(now_lo, (int)off);
        now_hi &= __shfl_xor(now_hi, (int)off);
        nx_lo &= __shfl_xor(nx_lo, (int)off);
        nx_hi &= __shfl_xor(nx_hi, (int)off);
      }
      if (valid && sub == 0) {
        s_U[local] = ucount;
        s_W[local] = (uint8_t)__popcll((((uint64_t)now_hi << 32) | now_lo) & gmask);
        s_Wn[local] = (uint8_t)__popcll((((uint64_t)nx_hi << 32) | nx_lo) & gmask);
      }
    }
    lds_barrier();
    if (threadIdx.x < in_batch) {
      const uint64_t gid = base + threadIdx.x;
      const uint32_t ucount = s_U[threadIdx.x];
      const double up = *up_p;
      const double G = (double)geo.G;
      // Eq9, operation by operation, no contraction (built with -ffp-contract=off)
      const double num = (double)ucount - G * up;
      const double den = G * (1.0 - up);
      double e;
      uint8_t fl = gid >= n_c ? 4u : 0u;   // NEW: listed behind the carried list
      if (den == 0.0) {
        e = __builtin_inf();
        fl |= 2u;
      } else {
        const double y = 1.0 - num / den;
        if (y <= 0.0) {
          e = __builtin_inf();
          fl |= 2u;
        } else {
          e = -G * log(y);
        }
      }
      if (e >= (double)geo.theta) fl |= 1u;
      if (s_Wn[threadIdx.x] >= geo.t_re) fl |= 8u;   // carried by Algorithm 3
      cflags[gid] = fl;
      s_e[threadIdx.x] = e;
      s_f[threadIdx.x] = fl;
      if (out_U) out_U[gid] = ucount;
      if (out_W) out_W[gid] = s_W[threadIdx.x];
      wrote += (out_U ? 4u : 0u) + (out_W ? 1u : 0u);
    }
    lds_barrier();
    // the batch's report entries leave in 16-byte pieces (ip: 64 lanes, est:
    // 128 lanes, flags: 16 lanes), so the writes into host memory go out in
    // whole lines; a partial batch at the end of the list is written entry
    // by entry
    if (in_batch == kEstPerBlock) {
      const uint32_t t = threadIdx.x;
      if (base >= ip_from) {
        if (t < kEstPerBlock / 4) {
          reinterpret_cast<uint4*>(out_ip + base)[t] = reinterpret_cast<const uint4*>(s_ip)[t];
          wrote += 16u;
        }
      } else if (base + t >= ip_from) {
        out_ip[base + t] = s_ip[t];
        wrote += 4u;
      }
      // with the mirrors, a piece goes to host memory only if it differs
      // from what the host array holds there (the mirror), and the mirror
      // follows
      if (t < kEstPerBlock / 2) {
        const uint4 v = reinterpret_cast<const uint4*>(s_e)[t];
        if (mir_est) {
          uint4* mp = reinterpret_cast<uint4*>(mir_est + base) + t;
          const uint4 o = *mp;
          if (o.x != v.x || o.y != v.y || o.z != v.z || o.w != v.w) {
            reinterpret_cast<uint4*>(out_est + base)[t] = v;
            *mp = v;
            wrote += 16u;
          }
        } else {
          reinterpret_cast<uint4*>(out_est + base)[t] = v;
          wrote += 16u;
        }
      }
      if (t < kEstPerBlock / 16) {
        const uint4 v = reinterpret_cast<const uint4*>(s_f)[t];
        if (mir_flags) {
          uint4* mp = reinterpret_cast<uint4*>(mir_flags + base) + t;
          const uint4 o = *mp;
          if (o.x != v.x || o.y != v.y || o.z != v.z || o.w != v.w) {
            reinterpret_cast<uint4*>(out_flags + base)[t] = v;
            *mp = v;
            wrote += 16u;
          }
        } else {
          reinterpret_cast<uint4*>(out_flags + base)[t] = v;
          wrote += 16u;
        }
      }
    } else if (threadIdx.x < in_batch) {
      const uint64_t gid = base + threadIdx.x;
      if (gid >= ip_from) {
        out_ip[gid] = s_ip[threadIdx.x];
        wrote += 4u;
      }
      const double e = s_e[threadIdx.x];
      const uint8_t f = s_f[threadIdx.x];
      if (!mir_est || __double_as_longlong(mir_est[gid]) != __double_as_longlong(e)) {
        out_est[gid] = e;
        if (mir_est) mir_est[gid] = e;
        wrote += 8u;
      }
      if (!mir_flags || mir_flags[gid] != f) {
        out_flags[gid] = f;
        if (mir_flags) mir_flags[gid] = f;
        wrote += 1u;
      }
    }
    lds_barrier();
  }
  // the workgroup's byte count into one of the slots
  for (int off = kWave / 2; off > 0; off >>= 1) wrote += __shfl_xor(wrote, off);
  if ((threadIdx.x & (kWave - 1)) == 0) s_U[threadIdx.x / kWave] = wrote;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long b = 0;
    for (uint32_t w = 0; w < kBlock / kWave; ++w) b += s_U[w];
    if (b) atomicAdd(&rep_bytes[blockIdx.x % kEndSlots], b);
  }
}

static uint32_t est_wpl(const Geo& geo) { return geo.words % 2 == 0 ? 2u : 1u; }

static uint32_t est_lg_log2(const Geo& geo) {
  const uint32_t pieces = geo.words / est_wpl(geo);
  const uint32_t need = pieces > geo.u ? pieces : geo.u;
  uint32_t l = 2;  // at least 4 lanes per candidate
  while ((1u << l) < need && l < 6) ++l;
  return l;   // 2^l >= u, since u <= kMaxU <= 64
}

// One resident wave of blocks: every block then runs the same number of
// grid-stride batches, instead of a second partial wave of blocks starting
// after the first has finished (the kernel's register use allows fewer
// blocks per CU than the pipeline's default grid).
template <int kU, int kWpl>
static uint32_t est_grid() {
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_estimate<kU, kWpl>, (int)kBlock,
                                                   0) != hipSuccess ||
      cus <= 0 || per_cu <= 0)
    return 2 * kPipeBlocks;
  return (uint32_t)cus * (uint32_t)per_cu;
}

template <int kU, int kWpl>
static hipError_t launch_estimate_u(const uint32_t* csip, const Counters* cnt,
                                    const PipeState* ps, uint32_t skip,
                                    const uint64_t* bitmap, const uint64_t* act, const double* up,
                                    const unsigned long long* row_fill, const Geo& geo,
                                    uint32_t l, uint8_t* cflags, const ReportPtrs& out,
                                    hipStream_t st) {
  static const uint32_t grid = est_grid<kU, kWpl>();
  hipLaunchKernelGGL((k_estimate<kU, kWpl>), dim3(grid), dim3(kBlock), 0, st, csip, cnt, ps,
                     skip, bitmap,
                     act, up, row_fill, geo, l, cflags, out.ip, out.est, out.flags,
                     out.U, out.W, out.mir_est, out.mir_flags,
                     const_cast<PipeState*>(ps)->rep_bytes);
  return hipGetLastError();
}

template <int kU>
static hipError_t launch_estimate_w(const uint32_t* csip, const Counters* cnt,
                                    const PipeState* ps, uint32_t skip,
                                    const uint64_t* bitmap, const uint64_t* act, const double* up,
                                    const unsigned long long* row_fill, const Geo& geo,
                                    uint32_t l, uint8_t* cflags, const ReportPtrs& out,
                                    hipStream_t st) {
  if (est_wpl(geo) == 2)
    return launch_estimate_u<kU, 2>(csip, cnt, ps, skip, bitmap, act, up, row_fill, geo, l,
                                    cflags, out, st);
  return launch_estimate_u<kU, 1>(csip, cnt, ps, skip, bitmap, act, up, row_fill, geo, l, cflags,
                                  out, st);
}

hipError_t launch_estimate(const uint32_t* csip, const Counters* cnt, const PipeState* ps,
                           bool skip_carried_ip, const uint64_t* bitmap,
                           const uint64_t* act, const double* up,
                           const unsigned long long* row_fill, const Geo& geo, uint8_t* cflags,
                           const ReportPtrs& out, hipStream_t st) {
  static_assert(kMaxU <= 16, "k_estimate is unrolled for at most 16 rows");
  const uint32_t l = est_lg_log2(geo);
  if (geo.u > (1u << l)) return hipErrorInvalidValue;
  if (geo.u <= 4)
    return launch_estimate_w<4>(csip, cnt, ps, skip_carried_ip, bitmap, act, up, row_fill, geo, l,
                                cflags, out, st);
  if (geo.u <= 8)
    return launch_estimate_w<8>(csip, cnt, ps, skip_carried_ip, bitmap, act, up, row_fill, geo, l,
                                cflags, out, st);
  return launch_estimate_w<16>(csip, cnt, ps, skip_carried_ip, bitmap, act, up, row_fill, geo, l,
                               cflags, out, st);
}

// ------------------------------------------------------------------ SI
// Algorithm 3's SI step as counter updates: a new candidate that is carried
// adds 1 to its u counters, a carried candidate of the previous slice that is
// dropped subtracts 1.  Afterwards every counter equals its count over
// NCSIP_t, so "counter > 0" is exactly the SI bit that clearing SI and
// marking every carried candidate would produce, at a cost proportional to
// the candidates that entered or left.

__global__ __launch_bounds__(kBlock) void k_si_update(const uint32_t* __restrict__ csip,
                                                     const uint8_t* __restrict__ cflags,
                                                     const Counters* __restrict__ cnt,
                                                     uint32_t* __restrict__ si_cnt, Geo geo) {
  const uint32_t n = cnt->n_cand;
  for (uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x; t < n;
       t += (uint64_t)gridDim.x * kBlock) {
    const uint32_t f = cflags[t];
    const bool is_new = f & 4u, keep = f & 8u;
    uint32_t delta;
    if (is_new && keep) delta = 1u;                 // enters NCSIP_t
    else if (!is_new && !keep) delta = 0xFFFFFFFFu;  // leaves: -1
    else continue;                                   // stays, or never counted
    const uint32_t a = csip[t];
    const uint32_t bit = hrange(mas(geo.h4, a), 16u);
    for (uint32_t r = 0; r < geo.u; ++r)
      atomicAdd(&si_cnt[si_slot(geo, r, hrange(mas(geo.rh[r], a), geo.v_re), bit)], delta);
  }
}

hipError_t launch_si_update(const uint32_t* csip, const uint8_t* cflags, const Counters* cnt,
                            uint32_t* si_cnt, const Geo& geo, hipStream_t st) {
  hipLaunchKernelGGL(k_si_update, dim3(kPipeBlocks), dim3(kBlock), 0, st, csip, cflags, cnt,
                     si_cnt, geo);
  return hipGetLastError();
}

// ------------------------------------------------------------------ status
// The slice's counters, Eq8 and the row fills go into the pinned host status
// block, so the host reads everything after one wait.  Then the state moves
// to the next slice: |NCSIP_t| is carried, the stamp code advances, and the
// slice's counters (and the sampled-source count of its parity, which the
// scans of the slice after next reuse) are cleared.

// the estimate's byte count: slot t per lane, summed over the wavefront, the
// slots cleared for the next slice
__device__ __forceinline__ unsigned long long take_rep_bytes(PipeState* ps, uint32_t t) {
  unsigned long long b = t < kEndSlots ? ps->rep_bytes[t] : 0ull;
  if (t < kEndSlots) ps->rep_bytes[t] = 0ull;
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)b, d);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(b >> 32), d);
    b += ((unsigned long long)hi << 32) | lo;
  }
  return b;
}

__global__ void k_status(Counters* __restrict__ cnt, uint32_t* __restrict__ tcount,
                         const double* __restrict__ up,
                         const unsigned long long* __restrict__ row_fill, uint32_t u,
                         PipeState* __restrict__ ps, uint32_t p, HostStatus* __restrict__ out,
                         uint32_t* __restrict__ report_n) {
  if (blockIdx.x != 0) return;
  const uint32_t t = threadIdx.x;
  const unsigned long long host_bytes = take_rep_bytes(ps, t);
  Counters c = *cnt;
  c.touched = *tcount;
  if (t < sizeof(Counters) / 4) ((uint32_t*)&out->cnt)[t] = ((const uint32_t*)&c)[t];
  if (t < u) out->row_fill[t] = row_fill[t];
  if (t == 0) {
    out->up = *up;
    out->slice = ps->slice;
    out->t_close = ps->t_close[p];
    out->host_bytes = host_bytes;   // the staged report's bytes (its copy follows)
    out->t_done = wall_clock64();   // every earlier kernel of the report has finished
    if (report_n) *report_n = c.n_cand;
  }
  __syncthreads();
  if (t == 0) {
    ps->n_ncsip = c.n_keep;
    ps->slice = ps->slice + 1;
    ps->now = (uint32_t)(ps->slice % kStampPeriod) + 1u;
    *tcount = 0u;
  }
  if (t < sizeof(Counters) / 4) ((uint32_t*)cnt)[t] = 0u;
}

// ------------------------------------------------------------------ report copy
// Copies the slice's report from the device staging arrays (written by
// k_estimate) into the pinned host arrays: 16-byte loads and stores, grid
// stride, the count read from device memory.  Used when the report's PCIe
// transfer is to overlap the next slice's scan: this kernel needs little
// besides PCIe bandwidth, while the gathers of k_estimate have already run.

__device__ __forceinline__ void copy_bytes_16(const uint8_t* __restrict__ src,
                                              uint8_t* __restrict__ dst, uint64_t bytes) {
  const uint64_t n16 = bytes / 16;
  const uint64_t stride = (uint64_t)gridDim.x * kBlock;
  const uint64_t t = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
  for (uint64_t i = t; i < n16; i += stride)
    reinterpret_cast<uint4*>(dst)[i] = reinterpret_cast<const uint4*>(src)[i];
  const uint64_t tail = n16 * 16 + t;
  if (tail < bytes && t < 16) dst[tail] = src[tail];
}

// expect != 0: the copy waits until *started == expect, i.e. until the next
// slice's first scan is about to start on the other stream (its streams of
// host writes would otherwise hold up that scan's dispatch).  The wait is
// bounded: after kCopyWaitSpins polls the copy proceeds anyway.
constexpr uint32_t kCopyWaitSpins = 1u << 20;

__global__ __launch_bounds__(kBlock) void k_report_copy(const uint32_t* __restrict__ n_p,
                                                       ReportPtrs from, ReportPtrs to,
                                                       const uint32_t* started, uint32_t expect) {
  if (expect != 0u) {
    if (threadIdx.x == 0) {
      for (uint32_t i = 0; i < kCopyWaitSpins; ++i) {
        if (__hip_atomic_load(started, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == expect)
          break;
        __builtin_amdgcn_s_sleep(2);
      }
    }
    __syncthreads();
  }
  const uint64_t n = *n_p;
  copy_bytes_16((const uint8_t*)from.ip, (uint8_t*)to.ip, 4 * n);
  copy_bytes_16((const uint8_t*)from.est, (uint8_t*)to.est, 8 * n);
  copy_bytes_16(from.flags, to.flags, n);
  if (to.U) copy_bytes_16((const uint8_t*)from.U, (uint8_t*)to.U, 4 * n);
  if (to.W) copy_bytes_16(from.W, to.W, n);
}

// A small grid: 64 workgroups already saturate PCIe writes, and the copy
// runs beside the next slice's scan, which needs the rest of the GPU's wave
// slots (a kernel whose workgroups fill every slot keeps a kernel of another
// stream from starting until its own workgroups retire).
constexpr uint32_t kCopyBlocks = 128;

hipError_t launch_report_copy(const uint32_t* n, const ReportPtrs& from, const ReportPtrs& to,
                              const uint32_t* started, uint32_t expect, hipStream_t st) {
  hipLaunchKernelGGL(k_report_copy, dim3(kCopyBlocks), dim3(kBlock), 0, st, n, from, to, started,
                     expect);
  return hipGetLastError();
}

__global__ void k_mark_scan(uint32_t* started, uint32_t value) {
  if (blockIdx.x == 0 && threadIdx.x == 0)
    __hip_atomic_store(started, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

hipError_t launch_mark_scan(uint32_t* started, uint32_t value, hipStream_t st) {
  hipLaunchKernelGGL(k_mark_scan, dim3(1), dim3(64), 0, st, started, value);
  return hipGetLastError();
}

// one wavefront: the end of the closed slice's scans is the latest of the
// marker's clock and the partitioned scan's slots, which start over at zero
__global__ void k_begin_close(PipeState* __restrict__ ps, unsigned long long* __restrict__ row_fill,
                              uint32_t n_clear, uint32_t p) {
  static_assert(kEndSlots == kWave, "one slot per lane");
  if (blockIdx.x != 0) return;
  const uint32_t lane = threadIdx.x;
  unsigned long long t = ps->t_end[p][lane];
  ps->t_end[p][lane] = 0ull;
  for (int d = kWave / 2; d >= 1; d >>= 1) {
    const uint32_t lo = (uint32_t)__shfl_xor((int)(uint32_t)t, d);
    const uint32_t hi = (uint32_t)__shfl_xor((int)(uint32_t)(t >> 32), d);
    const unsigned long long o = ((unsigned long long)hi << 32) | lo;
    t = o > t ? o : t;
  }
  if (lane == 0) {
    const unsigned long long ts = ps->t_scan[p] > t ? ps->t_scan[p] : t;
    ps->t_close[p] = ps->scanned[p] ? ts : wall_clock64();
    ps->t_scan[p] = 0ull;
    ps->scanned[p] = 0u;
    ps->snap = ps->snap % kStampPeriod + 1u;
  }
  for (uint32_t i = threadIdx.x; i < n_clear; i += blockDim.x) row_fill[i] = 0ull;
}

hipError_t launch_begin_close(PipeState* ps, unsigned long long* row_fill, uint32_t n_clear,
                              uint32_t p, hipStream_t st) {
  hipLaunchKernelGGL(k_begin_close, dim3(1), dim3(kWave), 0, st, ps, row_fill, n_clear, p);
  return hipGetLastError();
}

__global__ void k_scan_end(PipeState* __restrict__ ps, uint32_t p) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ps->t_scan[p] = wall_clock64();   // every earlier kernel of the stream has finished
    ps->scanned[p] = 1u;
  }
}

hipError_t launch_scan_end(PipeState* ps, uint32_t p, hipStream_t st) {
  hipLaunchKernelGGL(k_scan_end, dim3(1), dim3(64), 0, st, ps, p);
  return hipGetLastError();
}

__global__ void k_mark_done(HostStatus* __restrict__ out) {
  if (blockIdx.x == 0 && threadIdx.x == 0) out->t_done = wall_clock64();
}

hipError_t launch_mark_done(HostStatus* out, hipStream_t st) {
  hipLaunchKernelGGL(k_mark_done, dim3(1), dim3(64), 0, st, out);
  return hipGetLastError();
}

__global__ void k_publish(const Counters* __restrict__ cnt, const uint32_t* __restrict__ tcount,
                          const double* __restrict__ up,
                          const unsigned long long* __restrict__ row_fill, uint32_t u,
                          PipeState* __restrict__ ps, uint32_t p,
                          HostStatus* __restrict__ out) {
  if (blockIdx.x != 0) return;
  const uint32_t t = threadIdx.x;
  const unsigned long long host_bytes = take_rep_bytes(ps, t);
  Counters c = *cnt;
  c.touched = *tcount;
  if (t < sizeof(Counters) / 4) ((uint32_t*)&out->cnt)[t] = ((const uint32_t*)&c)[t];
  if (t < u) out->row_fill[t] = row_fill[t];
  if (t == 0) {
    out->up = *up;
    out->slice = ps->slice;
    out->t_close = ps->t_close[p];
    out->host_bytes = host_bytes;
    out->t_done = wall_clock64();   // every earlier kernel of the report has finished
  }
}

__global__ void k_advance(Counters* __restrict__ cnt, uint32_t* __restrict__ tcount,
                          PipeState* __restrict__ ps) {
  if (blockIdx.x != 0) return;
  const uint32_t t = threadIdx.x;
  if (t == 0) {
    ps->n_ncsip = cnt->n_keep;
    ps->slice = ps->slice + 1;
    ps->now = (uint32_t)(ps->slice % kStampPeriod) + 1u;
    *tcount = 0u;
  }
  __syncthreads();
  if (t < sizeof(Counters) / 4) ((uint32_t*)cnt)[t] = 0u;
}

hipError_t launch_publish(const Counters* cnt, const uint32_t* tcount, const double* up,
                          const unsigned long long* row_fill, uint32_t u, PipeState* ps,
                          uint32_t p, HostStatus* out, hipStream_t st) {
  hipLaunchKernelGGL(k_publish, dim3(1), dim3(64), 0, st, cnt, tcount, up, row_fill, u, ps, p,
                     out);
  return hipGetLastError();
}

hipError_t launch_advance(Counters* cnt, uint32_t* tcount, PipeState* ps, hipStream_t st) {
  hipLaunchKernelGGL(k_advance, dim3(1), dim3(64), 0, st, cnt, tcount, ps);
  return hipGetLastError();
}

hipError_t launch_status(Counters* cnt, uint32_t* tcount, const double* up,
                         const unsigned long long* row_fill, uint32_t u, PipeState* ps,
                         uint32_t p, HostStatus* out, uint32_t* report_n, hipStream_t st) {
  hipLaunchKernelGGL(k_status, dim3(1), dim3(64), 0, st, cnt, tcount, up, row_fill, u, ps, p,
                     out, report_n);
  return hipGetLastError();
}

}  // namespace srla
