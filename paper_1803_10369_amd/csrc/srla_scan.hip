// gfx950 scan kernel of the SRLA hot path: Algorithm 2 of arXiv 1803.10369
// (Section 4.1) for every (aip, bip) pair of a slice.
//
// Per pair: u + 3 multiply-add-shift hashes in registers, u 2-byte LE stamp
// stores, and -- for the 2^-tau of pairs whose H1(bip) has LSB >= tau -- u
// 2-byte SRE stamp stores and one append of aip to the slice's sampled-source
// list.  A stamp store is DRset: plain and idempotent, so concurrent pairs
// need no atomics.  The kernel is bound by the rate of random 2-byte stores;
// there is no dense contraction, hence no MFMA.
#include "srla_internal.h"

namespace srla {

// ------------------------------------------------------------------ scan
// Algorithm 2 for every pair.  One thread owns two adjacent pairs per step
// (a 16-byte load), kScanSteps steps per block; all loads of a thread are
// issued before its stores.  Sampled sources are appended to `touched` with
// one atomic per wavefront (ballot + lane rank).

constexpr int kScanSteps = 4;
constexpr uint64_t kScanTile = (uint64_t)kBlock * 2 * kScanSteps;  // pairs per block

template <int U>
__device__ __forceinline__ void scan_one(uint32_t a, uint32_t b, bool valid, const Geo& geo,
                                         uint16_t code, uint16_t* __restrict__ le,
                                         uint16_t* __restrict__ re,
                                         uint32_t* __restrict__ touched,
                                         uint32_t* __restrict__ tcount) {
  const uint32_t nu = U > 0 ? (uint32_t)U : geo.u;
  bool sampled = false;
  if (valid) {
    // every pair sets one LE DR per row: H3(bip) picks the DR, RH_i(aip) the LE
    const uint32_t lei = hrange(mas(geo.h3, b), geo.G);
#pragma unroll
    for (uint32_t i = 0; i < nu; ++i) {
      const uint32_t col = hrange(mas(geo.rh[i], a), geo.v_le);
      le[((uint64_t)i * geo.v_le + col) * geo.G + lei] = code;
    }
    // only pairs with LSB(H1(bip)) >= tau reach the SRE
    sampled = (mas(geo.h1, b) & geo.tau_mask) == 0u;
    if (sampled) {
      const uint32_t rei = hrange(mas(geo.h2, b), geo.g);
#pragma unroll
      for (uint32_t i = 0; i < nu; ++i) {
        const uint32_t col = hrange(mas(geo.rh[i], a), geo.v_re);
        re[((uint64_t)i * geo.v_re + col) * geo.g + rei] = code;
      }
    }
  }
  // the candidate check of sampled sources happens at the end of the slice
  const uint64_t mask = __ballot(sampled);
  if (mask != 0ull) {
    const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1u;
    uint32_t base = 0;
    if (__lane_id() == leader) base = atomicAdd(tcount, (uint32_t)__popcll(mask));
    base = __shfl(base, (int)leader);
    if (sampled) touched[base + lane_rank(mask)] = a;
  }
}

// Waves claim tiles of kWaveTile pairs from a launch-wide counter, so a wave
// slowed by other work on its CU (the report copy of the previous slice runs
// beside the scan) takes fewer tiles instead of holding up the whole launch,
// as a fixed share of the tiles would.  claim[slot] counts this launch's
// claims and is zero when it starts; the grid's first thread clears
// claim[slot ^ 1] for the next launch on the stream.  Each wave asks for its
// next tile while it works on the current one.  mark != 0: the same thread
// also sets *started = mark, the scan-start mark a report copy on another
// stream may be waiting for.
constexpr uint64_t kWaveTile = (uint64_t)kWave * 2 * kScanSteps;   // 512 pairs

template <int U, bool VEC>
__global__ __launch_bounds__(kBlock) void k_scan_flat(const uint32_t* __restrict__ pairs, uint64_t n,
                                                Geo geo, uint16_t code,
                                                uint16_t* __restrict__ le,
                                                uint16_t* __restrict__ re,
                                                uint32_t* __restrict__ touched,
                                                uint32_t* __restrict__ tcount,
                                                uint32_t* __restrict__ claim, uint32_t slot,
                                                uint32_t* started, uint32_t mark) {
  const uint32_t lane = __lane_id();
  const uint64_t tiles = (n + kWaveTile - 1) / kWaveTile;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    claim[slot ^ 1u] = 0u;
    if (mark != 0u) __hip_atomic_store(started, mark, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  uint32_t t = 0;
  if (lane == 0) t = atomicAdd(claim + slot, 1u);
  t = __shfl(t, 0);
  while (t < tiles) {   // uniform per wave: the ballots below see every lane
    uint32_t next = 0;
    if (lane == 0) next = atomicAdd(claim + slot, 1u);
    const uint64_t base = (uint64_t)t * kWaveTile;
    uint32_t a[kScanSteps][2], b[kScanSteps][2];
    bool v[kScanSteps][2];
#pragma unroll
    for (int s = 0; s < kScanSteps; ++s) {
      const uint64_t p = base + (uint64_t)s * (2 * kWave) + 2u * lane;
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
    for (int s = 0; s < kScanSteps; ++s) {
      scan_one<U>(a[s][0], b[s][0], v[s][0], geo, code, le, re, touched, tcount);
      scan_one<U>(a[s][1], b[s][1], v[s][1], geo, code, le, re, touched, tcount);
    }
    t = __shfl(next, 0);
  }
}

// XCD-aware form.  Workgroups are dispatched to the 8 XCDs round-robin, so
// block b runs on XCD b % 8 and only ever touches the SEA rows that XCD owns:
// with u >= 8, XCD x owns rows x, x+8, ...; with u in {1, 2, 4}, XCD x owns
// row x % u and every u-th XCD takes the next tile.  Each XCD's L2 then sees
// one LE row (4 MiB for 2048 x 1024 DRs) instead of all of them.  Each
// (pair, row) is still stored exactly once, and the sampled-source append is
// done by the owner of row 0; results do not depend on the actual placement.
constexpr int kXcds = 8;

template <int U>
__global__ __launch_bounds__(kBlock) void k_scan_xcd(const uint32_t* __restrict__ pairs,
                                                    uint64_t n, Geo geo, uint16_t code,
                                                    uint16_t* __restrict__ le,
                                                    uint16_t* __restrict__ re,
                                                    uint32_t* __restrict__ touched,
                                                    uint32_t* __restrict__ tcount) {
  constexpr int kParts = U >= kXcds ? 1 : kXcds / U;      // tiles per XCD group
  constexpr int kRowsPerXcd = U >= kXcds ? U / kXcds : 1;
  const uint32_t xcd = blockIdx.x % kXcds;
  const uint32_t row0 = U >= kXcds ? xcd : xcd % U;
  const bool appender = row0 == 0;
  for (uint64_t group = blockIdx.x / kXcds;; group += gridDim.x / kXcds) {
  const uint64_t tile = group * kParts + (U >= kXcds ? 0u : xcd / U);
  const uint64_t base = tile * kScanTile;
  if (base >= n) break;
  uint32_t a[kScanSteps][2], b[kScanSteps][2];
  bool v[kScanSteps][2];
#pragma unroll
  for (int s = 0; s < kScanSteps; ++s) {
    const uint64_t p = base + (uint64_t)s * (2 * kBlock) + 2u * threadIdx.x;
    v[s][0] = p < n;
    v[s][1] = p + 1 < n;
    if (v[s][1]) {
      const uint4 q = *reinterpret_cast<const uint4*>(pairs + 2 * p);
      a[s][0] = q.x; b[s][0] = q.y; a[s][1] = q.z; b[s][1] = q.w;
    } else {
      a[s][0] = v[s][0] ? pairs[2 * p] : 0u;
      b[s][0] = v[s][0] ? pairs[2 * p + 1] : 0u;
      a[s][1] = 0u; b[s][1] = 0u;
    }
  }
#pragma unroll
  for (int s = 0; s < kScanSteps; ++s) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const uint32_t aa = a[s][h], bb = b[s][h];
      bool sampled = false;
      if (v[s][h]) {
        const uint32_t lei = hrange(mas(geo.h3, bb), geo.G);
        sampled = (mas(geo.h1, bb) & geo.tau_mask) == 0u;
        const uint32_t rei = sampled ? hrange(mas(geo.h2, bb), geo.g) : 0u;
#pragma unroll
        for (int j = 0; j < kRowsPerXcd; ++j) {
          const uint32_t r = row0 + (uint32_t)j * kXcds;
          const uint32_t hr = mas(geo.rh[r], aa);
          le[((uint64_t)r * geo.v_le + hrange(hr, geo.v_le)) * geo.G + lei] = code;
          if (sampled) re[((uint64_t)r * geo.v_re + hrange(hr, geo.v_re)) * geo.g + rei] = code;
        }
      }
      if (appender) {
        const uint64_t mask = __ballot(sampled);
        if (mask != 0ull) {
          const uint32_t leader = (uint32_t)__ffsll((unsigned long long)mask) - 1u;
          uint32_t slot = 0;
          if (__lane_id() == leader) slot = atomicAdd(tcount, (uint32_t)__popcll(mask));
          slot = __shfl(slot, (int)leader);
          if (sampled) touched[slot + lane_rank(mask)] = aa;
        }
      }
    }
  }
  }
}

template <int U>
static hipError_t launch_scan_xcd(const uint32_t* pairs, uint64_t n, const Geo& geo,
                                  uint16_t code, uint16_t* le, uint16_t* re, uint32_t* touched,
                                  uint32_t* tcount, uint32_t max_blocks, hipStream_t st) {
  constexpr uint64_t kParts = U >= kXcds ? 1 : kXcds / U;
  const uint64_t tiles = (n + kScanTile - 1) / kScanTile;
  uint64_t blocks = kXcds * ((tiles + kParts - 1) / kParts);
  if (max_blocks && blocks > max_blocks) blocks = max_blocks >= kXcds ? max_blocks / kXcds * kXcds : kXcds;
  hipLaunchKernelGGL((k_scan_xcd<U>), dim3((uint32_t)blocks), dim3(kBlock), 0, st, pairs, n, geo,
                     code, le, re, touched, tcount);
  return hipGetLastError();
}

template <int U>
static hipError_t launch_scan_u(const uint32_t* pairs, uint64_t n, const Geo& geo, uint16_t code,
                                uint16_t* le, uint16_t* re, uint32_t* touched, uint32_t* tcount,
                                uint32_t* claim, uint32_t* slot, uint32_t* started, uint32_t mark,
                                uint32_t max_blocks, hipStream_t st) {
  uint64_t blocks = (n + kScanTile - 1) / kScanTile;
  if (max_blocks && blocks > max_blocks) blocks = max_blocks;
  const bool vec = ((uintptr_t)pairs & 15u) == 0;
  if (vec)
    hipLaunchKernelGGL((k_scan_flat<U, true>), dim3((uint32_t)blocks), dim3(kBlock), 0, st, pairs, n,
                       geo, code, le, re, touched, tcount, claim, *slot, started, mark);
  else
    hipLaunchKernelGGL((k_scan_flat<U, false>), dim3((uint32_t)blocks), dim3(kBlock), 0, st, pairs, n,
                       geo, code, le, re, touched, tcount, claim, *slot, started, mark);
  const hipError_t e = hipGetLastError();
  if (e == hipSuccess) *slot ^= 1u;
  return e;
}

hipError_t launch_scan(const uint32_t* pairs, uint64_t n, const Geo& geo, uint16_t code,
                       uint16_t* le, uint16_t* re, uint32_t* touched, uint32_t* tcount,
                       uint32_t* claim, uint32_t* slot, bool xcd_aware, uint32_t max_blocks,
                       hipStream_t st, uint32_t* started, uint32_t mark) {
  if (n == 0) return hipSuccess;
  if (xcd_aware && ((uintptr_t)pairs & 15u) == 0) {
    if (mark != 0u) {
      const hipError_t e = launch_mark_scan(started, mark, st);
      if (e != hipSuccess) return e;
    }
    switch (geo.u) {
      case 1: return launch_scan_xcd<1>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
      case 2: return launch_scan_xcd<2>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
      case 4: return launch_scan_xcd<4>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
      case 8: return launch_scan_xcd<8>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
      case 16: return launch_scan_xcd<16>(pairs, n, geo, code, le, re, touched, tcount, max_blocks, st);
      default: break;
    }
  }
  switch (geo.u) {
    case 4:
      return launch_scan_u<4>(pairs, n, geo, code, le, re, touched, tcount, claim, slot, started,
                              mark, max_blocks, st);
    case 8:
      return launch_scan_u<8>(pairs, n, geo, code, le, re, touched, tcount, claim, slot, started,
                              mark, max_blocks, st);
    default:
      return launch_scan_u<0>(pairs, n, geo, code, le, re, touched, tcount, claim, slot, started,
                              mark, max_blocks, st);
  }
}

// ------------------------------------------------------------------ group
// Fused scan of a monitor group over one pair stream: every pair is loaded
// once (16-byte loads, two pairs per lane), then each member applies its own
// Algorithm 2 -- its hash functions, rows, window-agnostic stamp arrays,
// sampling threshold and sampled-source list -- read from the member table
// with uniform (scalar) loads.  Equivalent to scanning the same pairs into
// every member separately.

template <bool VEC>
__global__ __launch_bounds__(kBlock) void k_scan_group(const uint32_t* __restrict__ pairs,
                                                      uint64_t n,
                                                      const GroupMember* __restrict__ members,
                                                      uint32_t n_members, GroupScanArgs args) {
  for (uint64_t base = (uint64_t)blockIdx.x * kScanTile; base < n;
       base += (uint64_t)gridDim.x * kScanTile) {
    uint32_t a[kScanSteps][2], b[kScanSteps][2];
    bool v[kScanSteps][2];
#pragma unroll
    for (int s = 0; s < kScanSteps; ++s) {
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
    for (uint32_t mi = 0; mi < n_members; ++mi) {
      const GroupMember& m = members[mi];
      const uint32_t par = (uint32_t)(args.parity >> mi) & 1u;
      const uint16_t code = args.code[mi];
#pragma unroll
      for (int s = 0; s < kScanSteps; ++s) {
        scan_one<0>(a[s][0], b[s][0], v[s][0], m.geo, code, m.le, m.re, m.touched[par],
                    m.tcount + par);
        scan_one<0>(a[s][1], b[s][1], v[s][1], m.geo, code, m.le, m.re, m.touched[par],
                    m.tcount + par);
      }
    }
  }
}

hipError_t launch_scan_group(const uint32_t* pairs, uint64_t n, const GroupMember* members,
                             uint32_t n_members, const GroupScanArgs& args, uint32_t max_blocks,
                             hipStream_t st) {
  if (n == 0 || n_members == 0) return hipSuccess;
  uint64_t blocks = (n + kScanTile - 1) / kScanTile;
  if (max_blocks && blocks > max_blocks) blocks = max_blocks;
  if (((uintptr_t)pairs & 15u) == 0)
    hipLaunchKernelGGL(k_scan_group<true>, dim3((uint32_t)blocks), dim3(kBlock), 0, st, pairs, n,
                       members, n_members, args);
  else
    hipLaunchKernelGGL(k_scan_group<false>, dim3((uint32_t)blocks), dim3(kBlock), 0, st, pairs, n,
                       members, n_members, args);
  return hipGetLastError();
}

}  // namespace srla
