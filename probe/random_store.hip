// Memory-system probes: the rate of random 2-byte stores (or of random
// one-bit atomic ORs into 32-bit words), one per lane, uniform over a
// footprint of F bytes -- the access pattern of the SRLA scan (16-bit stamp
// form, resp. one-bit discrete form) with nothing else (no pair loads, no
// hashing beyond the address).  Used to calibrate the scan kernels'
// achievable ceilings per footprint.
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

// block b writes the id of the XCD (XCC) it runs on to out[b]: a read of a
// hardware register, to check the round-robin placement of workgroups
__global__ __launch_bounds__(64) void k_xcc_of_block(uint32_t* __restrict__ out) {
  if (threadIdx.x == 0) out[blockIdx.x] = __builtin_amdgcn_s_getreg((3 << 11) | 20) & 15u;
}

// grid-stride coalesced 16-byte stores of `bytes` into (pinned, mapped)
// host memory: the rate a kernel can push results over PCIe
__global__ __launch_bounds__(256) void k_host_write(uint4* __restrict__ dst, uint64_t n16,
                                                   uint32_t seed) {
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride)
    dst[i] = make_uint4((uint32_t)i, seed, (uint32_t)(i >> 32), ~seed);
}

// a fixed amount of ALU work per lane (no memory traffic but one store per
// lane at the end, so the loop is not optimized away)
__global__ __launch_bounds__(256) void k_spin(uint32_t* __restrict__ out, uint32_t iters) {
  uint32_t x = threadIdx.x + 1u;
  for (uint32_t i = 0; i < iters; ++i) x = x * 1664525u + 1013904223u;
  out[(uint64_t)blockIdx.x * 256 + threadIdx.x] = x;
}

}  // namespace

// Two spin kernels of `blocks` workgroups each, on two streams at once, and
// then one after the other on one stream: returns the ms of both (via *both)
// and of one alone (the return value), or a negative value on error.  Equal
// times mean the two streams' kernels ran side by side.
extern "C" double probe_two_streams(void* buf, uint32_t blocks, uint32_t iters, void* s1,
                                    void* s2, double* both) {
  if (!buf || blocks == 0 || !both) return -1.0;
  hipStream_t a = (hipStream_t)s1, b = (hipStream_t)s2;
  uint32_t* out = (uint32_t*)buf;
  hipEvent_t e0, e1, e2, ea, eb;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess ||
      hipEventCreate(&e2) != hipSuccess || hipEventCreate(&ea) != hipSuccess ||
      hipEventCreate(&eb) != hipSuccess)
    return -2.0;
  float one = -1.f, two = -1.f;
  // one kernel alone
  hipEventRecord(e0, a);
  hipLaunchKernelGGL(k_spin, dim3(blocks), dim3(256), 0, a, out, iters);
  hipEventRecord(e1, a);
  hipEventSynchronize(e1);
  hipEventElapsedTime(&one, e0, e1);
  // two kernels, one per stream, released together
  hipEventRecord(e0, a);
  hipStreamWaitEvent(b, e0, 0);
  hipLaunchKernelGGL(k_spin, dim3(blocks), dim3(256), 0, a, out, iters);
  hipLaunchKernelGGL(k_spin, dim3(blocks), dim3(256), 0, b, out + (uint64_t)blocks * 256, iters);
  hipEventRecord(eb, b);
  hipStreamWaitEvent(a, eb, 0);
  hipEventRecord(e2, a);
  hipEventSynchronize(e2);
  hipEventElapsedTime(&two, e0, e2);
  hipEventDestroy(e0); hipEventDestroy(e1); hipEventDestroy(e2);
  hipEventDestroy(ea); hipEventDestroy(eb);
  *both = two;
  return one;
}

// Cross-stream ordering: stream 1 runs spin kernel K1, records event E, runs
// spin kernel K2; stream 2 waits for E and runs spin kernel K3 (blocks3
// workgroups of iters3 steps).
// Returns the ms from before K1 to after K3 (about one spin if K3 ran right
// after K1, two if it waited for K2), and the ms of stream 1's two spins
// via *both.
extern "C" double probe_event_order(void* buf, uint32_t blocks, uint32_t iters, void* s1,
                                    void* s2, double* both, uint32_t blocks3, uint32_t iters3) {
  if (!buf || blocks == 0 || !both) return -1.0;
  hipStream_t a = (hipStream_t)s1, b = (hipStream_t)s2;
  uint32_t* out = (uint32_t*)buf;
  hipEvent_t e0, e, ea, eb;
  const bool untimed = (blocks3 & 0x80000000u) != 0;   // E without timing
  blocks3 &= 0x7FFFFFFFu;
  if (hipEventCreate(&e0) != hipSuccess ||
      (untimed ? hipEventCreateWithFlags(&e, hipEventDisableTiming) : hipEventCreate(&e)) !=
          hipSuccess ||
      hipEventCreate(&ea) != hipSuccess || hipEventCreate(&eb) != hipSuccess)
    return -2.0;
  hipEventRecord(e0, a);
  hipLaunchKernelGGL(k_spin, dim3(blocks), dim3(256), 0, a, out, iters);
  hipEventRecord(e, a);
  hipLaunchKernelGGL(k_spin, dim3(blocks), dim3(256), 0, a, out, iters);
  hipEventRecord(ea, a);
  hipStreamWaitEvent(b, e, 0);
  hipLaunchKernelGGL(k_spin, dim3(blocks3), dim3(256), 0, b, out + (uint64_t)blocks * 256,
                     iters3);
  hipEventRecord(eb, b);
  hipEventSynchronize(ea);
  hipEventSynchronize(eb);
  float t3 = -1.f, t12 = -1.f;
  hipEventElapsedTime(&t3, e0, eb);
  hipEventElapsedTime(&t12, e0, ea);
  hipEventDestroy(e0); hipEventDestroy(e); hipEventDestroy(ea); hipEventDestroy(eb);
  *both = t12;
  return t3;
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

extern "C" int probe_xcc_of_blocks(void* out, uint32_t blocks, void* stream) {
  if (!out || blocks == 0) return -1;
  hipLaunchKernelGGL(k_xcc_of_block, dim3(blocks), dim3(64), 0, (hipStream_t)stream,
                     (uint32_t*)out);
  return hipStreamSynchronize((hipStream_t)stream) == hipSuccess ? 0 : -2;
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
