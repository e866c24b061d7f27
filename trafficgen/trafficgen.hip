// Seeded synthetic (aip, bip) pair streams on the GPU: the device twin of
// trafficgen/__init__.py, bit-identical to it.  Input generation only -- no
// estimator arithmetic lives here.  One thread writes one output pair.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kSrcSalt = 0x5352435F53524C41ull;
constexpr uint64_t kDstSalt = 0x4453545F53524C41ull;
constexpr uint32_t kIpMult = 0x9E3779B1u;
constexpr uint32_t kIpXor = 0x5A5A5A5Au;
constexpr uint32_t kPoolBits = 18;
constexpr uint32_t kDstPoolXor = 0x6D2B79F5u;

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// output c of SplitMix64 started at base
__device__ __forceinline__ uint64_t sm_at(uint64_t base, uint64_t c) {
  return mix64(base + (c + 1) * kGamma);
}

__device__ __forceinline__ uint32_t perm32(uint32_t key, uint32_t x) {
  x ^= key;
  x ^= x >> 16;
  x *= 0x7FEB352Du;
  x ^= x >> 15;
  x *= 0x846CA68Bu;
  x ^= x >> 16;
  return x;
}

__device__ __forceinline__ uint32_t rank_to_ip(uint64_t r) {
  return ((uint32_t)r * kIpMult) ^ kIpXor;
}

__global__ __launch_bounds__(256) void k_generate(uint32_t* __restrict__ out, uint64_t n,
                                                 uint64_t slice, uint64_t seed, uint64_t pa,
                                                 uint64_t pb, const uint64_t* __restrict__ thr,
                                                 uint32_t n_ranks,
                                                 const uint32_t* __restrict__ off,
                                                 const uint32_t* __restrict__ mp,
                                                 const uint32_t* __restrict__ dp, uint32_t P,
                                                 uint32_t pool_key, uint32_t dst_pool) {
  const uint64_t j = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= n) return;
  const uint64_t i = (pa * j + pb) % n;
  const uint32_t n_planted = P ? off[P] : 0u;
  uint32_t src, dst;
  if (i < n_planted) {
    uint32_t lo = 0, hi = P + 1;  // first off[] entry > i, minus one
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (off[mid] <= i) lo = mid + 1; else hi = mid;
    }
    const uint32_t p = lo - 1;
    const uint64_t x = i - off[p];
    const uint64_t idx = (slice * mp[p] + x) % dp[p];
    src = rank_to_ip((uint64_t)n_ranks + p);
    dst = perm32(pool_key, (p << kPoolBits) | (uint32_t)idx);
  } else {
    const uint64_t ctr = (slice << 32) | i;
    const uint64_t x = sm_at(seed ^ kSrcSalt, ctr) >> 1;
    uint32_t lo = 0, hi = n_ranks;  // number of thresholds <= x
    while (lo < hi) {
      const uint32_t mid = (lo + hi) >> 1;
      if (thr[mid] <= x) lo = mid + 1; else hi = mid;
    }
    src = rank_to_ip(lo);
    dst = (uint32_t)sm_at(seed ^ kDstSalt, ctr);
    if (dst_pool) dst = perm32(pool_key ^ kDstPoolXor, lo * dst_pool + dst % dst_pool);
  }
  out[2 * j] = src;
  out[2 * j + 1] = dst;
}

}  // namespace

extern "C" int tg_generate(uint32_t* out_pairs, uint64_t n, uint64_t slice, uint64_t seed,
                           uint64_t perm_a, uint64_t perm_b, const uint64_t* thr,
                           uint32_t n_ranks, const uint32_t* off, const uint32_t* mp,
                           const uint32_t* dp, uint32_t P, uint32_t pool_key, uint32_t dst_pool,
                           void* stream) {
  if (n == 0) return 0;
  if (!out_pairs || !thr || n_ranks == 0 || (P && (!off || !mp || !dp))) return -1;
  const uint64_t blocks = (n + 255) / 256;
  hipLaunchKernelGGL(k_generate, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream,
                     out_pairs, n, slice, seed, perm_a, perm_b, thr, n_ranks, off, mp, dp, P,
                     pool_key, dst_pool);
  return hipGetLastError() == hipSuccess ? 0 : -5;
}
