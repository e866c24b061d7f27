// Memory-system probes that give the SRLA kernels their ceilings:
// * the rate of random 2-byte stores (or random one-bit atomic ORs into
//   32-bit words, or random 2-byte loads), one per lane, uniform over a
//   footprint of F bytes -- the access pattern of the flat scan (16-bit stamp
//   form, resp. one-bit discrete form) with nothing else;
// * streaming reads and copies of F bytes with 16-byte accesses, consecutive
//   lanes on consecutive words -- the pattern of the slice-end sweeps and of
//   the partitioned scan's passes;
// * coalesced kernel stores into pinned host memory -- the report's path.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// every lane stores `per_lane` 2-byte values at uniform random cells
__global__ __launch_bounds__(256) void k_random_store(uint16_t* __restrict__ buf, uint64_t cells,
                                                     uint32_t per_lane, uint64_t seed,
                                                     uint16_t value) {
  const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  uint64_t s = mix64(seed ^ (t * 0x9E3779B97F4A7C15ull));
  for (uint32_t i = 0; i < per_lane; ++i) {
    s = mix64(s + 0x9E3779B97F4A7C15ull);
    const uint64_t cell = (uint64_t)(((unsigned __int128)s * cells) >> 64);
    buf[cell] = value;
  }
}

// every lane sets `per_lane` random bits with device-scope atomic ORs
__global__ __launch_bounds__(256) void k_random_or(uint32_t* __restrict__ buf, uint64_t words,
                                                  uint32_t per_lane, uint64_t seed) {
  const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  uint64_t s = mix64(seed ^ (t * 0x9E3779B97F4A7C15ull));
  for (uint32_t i = 0; i < per_lane; ++i) {
    s = mix64(s + 0x9E3779B97F4A7C15ull);
    const uint64_t w = (uint64_t)(((unsigned __int128)s * words) >> 64);
    __hip_atomic_fetch_or(buf + w, 1u << (uint32_t)(s & 31u), __ATOMIC_RELAXED,
                          __HIP_MEMORY_SCOPE_AGENT);
  }
}

// every lane loads `per_lane` random 2-byte cells (the test-before-store
// pattern's reads); one sum per lane is written so the loads stay live
__global__ __launch_bounds__(256) void k_random_load(const uint16_t* __restrict__ buf,
                                                    uint64_t cells, uint32_t per_lane,
                                                    uint64_t seed, uint32_t* __restrict__ sink) {
  const uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  uint64_t s = mix64(seed ^ (t * 0x9E3779B97F4A7C15ull));
  uint32_t acc = 0;
  for (uint32_t i = 0; i < per_lane; ++i) {
    s = mix64(s + 0x9E3779B97F4A7C15ull);
    acc += buf[(uint64_t)(((unsigned __int128)s * cells) >> 64)];
  }
  if (acc == 0xFFFFFFFFu) sink[0] = acc;   // practically never; keeps the loads
}

// grid-stride coalesced 16-byte stores of `bytes` into (pinned, mapped)
// host memory: the rate a kernel can push results over PCIe
__global__ __launch_bounds__(256) void k_host_write(uint4* __restrict__ dst, uint64_t n16,
                                                   uint32_t seed) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride)
    dst[i] = make_uint4((uint32_t)i, seed, (uint32_t)(i >> 32), ~seed);
}

// streaming reads: every lane reads 16-byte words grid-stride, four in flight;
// the XOR of what it read goes to the sink only if it matches a value the
// launch never produces (so the loads stay live)
__global__ __launch_bounds__(256) void k_stream_read(const uint4* __restrict__ src, uint64_t n16,
                                                    uint32_t* __restrict__ sink) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  uint32_t acc = 0;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    acc ^= a.x ^ a.y ^ a.z ^ a.w ^ b.x ^ b.y ^ b.z ^ b.w ^ c.x ^ c.y ^ c.z ^ c.w ^ d.x ^ d.y ^
           d.z ^ d.w;
  }
  for (; i < n16; i += stride) {
    const uint4 a = src[i];
    acc ^= a.x ^ a.y ^ a.z ^ a.w;
  }
  if (acc == 0xFFFFFFFFu) sink[0] = acc;   // the buffers hold zeros: never taken
}

// streaming copy: the same reads, each word stored to the same offset of dst
__global__ __launch_bounds__(256) void k_stream_copy(const uint4* __restrict__ src,
                                                    uint4* __restrict__ dst, uint64_t n16) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  for (; i + 3 * stride < n16; i += 4 * stride) {
    const uint4 a = src[i], b = src[i + stride], c = src[i + 2 * stride], d = src[i + 3 * stride];
    dst[i] = a;
    dst[i + stride] = b;
    dst[i + 2 * stride] = c;
    dst[i + 3 * stride] = d;
  }
  for (; i < n16; i += stride) dst[i] = src[i];
}

}  // namespace

// Streaming read (dst == NULL) or copy of `bytes` (a multiple of 16) with
// `blocks` workgroups; returns the kernel time in ms, or a negative value.
extern "C" double probe_stream(const void* src, void* dst, uint64_t bytes, uint32_t blocks,
                               void* sink, void* stream) {
  if (!src || bytes < 16 || blocks == 0 || (!dst && !sink)) return -1.0;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -2.0;
  hipEventRecord(a, st);
  if (dst)
    hipLaunchKernelGGL(k_stream_copy, dim3(blocks), dim3(256), 0, st, (const uint4*)src,
                       (uint4*)dst, bytes / 16);
  else
    hipLaunchKernelGGL(k_stream_read, dim3(blocks), dim3(256), 0, st, (const uint4*)src,
                       bytes / 16, (uint32_t*)sink);
  hipEventRecord(b, st);
  float ms = -3.f;
  if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
    ms = -4.f;
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms;
}

// Returns the kernel time in ms of writing `bytes` (a multiple of 16) to the
// device-visible address of pinned host memory, or a negative value.
extern "C" double probe_host_write(void* dst, uint64_t bytes, uint32_t blocks, void* stream) {
  if (!dst || bytes < 16 || blocks == 0) return -1.0;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -2.0;
  hipEventRecord(a, st);
  hipLaunchKernelGGL(k_host_write, dim3(blocks), dim3(256), 0, st, (uint4*)dst, bytes / 16, 7u);
  hipEventRecord(b, st);
  float ms = -3.f;
  if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
    ms = -4.f;
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms;
}

// Same for random 2-byte loads (footprint in bytes).
extern "C" double probe_random_load(void* buf, uint64_t bytes, uint64_t blocks, uint32_t per_lane,
                                    uint64_t seed, void* stream) {
  if (!buf || bytes < 8 || blocks == 0) return -1.0;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -2.0;
  hipEventRecord(a, st);
  // the sink is the buffer's first word (the cells read are left unchanged)
  hipLaunchKernelGGL(k_random_load, dim3((uint32_t)blocks), dim3(256), 0, st,
                     (const uint16_t*)buf, bytes / 2, per_lane, seed, (uint32_t*)buf);
  hipEventRecord(b, st);
  float ms = -3.f;
  if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
    ms = -4.f;
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms;
}

// Same for the atomic-OR pattern (footprint in bytes, a multiple of 4).
extern "C" double probe_random_or(void* buf, uint64_t bytes, uint64_t blocks, uint32_t per_lane,
                                  uint64_t seed, void* stream) {
  if (!buf || bytes < 4 || blocks == 0) return -1.0;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -2.0;
  hipEventRecord(a, st);
  hipLaunchKernelGGL(k_random_or, dim3((uint32_t)blocks), dim3(256), 0, st, (uint32_t*)buf,
                     bytes / 4, per_lane, seed);
  hipEventRecord(b, st);
  float ms = -3.f;
  if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
    ms = -4.f;
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms;
}

// Returns the kernel time in ms (HIP events) or a negative value on error.
extern "C" double probe_random_store(void* buf, uint64_t bytes, uint64_t blocks, uint32_t per_lane,
                                     uint64_t seed, void* stream) {
  if (!buf || bytes < 2 || blocks == 0) return -1.0;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -2.0;
  hipEventRecord(a, st);
  hipLaunchKernelGGL(k_random_store, dim3((uint32_t)blocks), dim3(256), 0, st, (uint16_t*)buf,
                     bytes / 2, per_lane, seed, (uint16_t)(seed | 1));
  hipEventRecord(b, st);
  float ms = -3.f;
  if (hipEventSynchronize(b) != hipSuccess || hipEventElapsedTime(&ms, a, b) != hipSuccess)
    ms = -4.f;
  hipEventDestroy(a);
  hipEventDestroy(b);
  return ms;
}
