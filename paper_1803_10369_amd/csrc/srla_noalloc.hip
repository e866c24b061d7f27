// Scratch of the allocation-free scan (srla_scan_noalloc): the partitioned
// scan's DR-index blocks, region offsets and marking bitmaps live in one
// file-scope device array of fixed size instead of memory the monitor
// allocates, so that a caller that cannot allocate (code under stream
// capture, a serving loop that forbids it) can scan.
//
// Host code never passes the array's name to a kernel: in host code it only
// stands for the device symbol.  noalloc_setup() looks up the array's device
// address once per device (with that device current) and keeps it;
// noalloc_scratch() hands that address out.  Every call on a device shares
// that device's array, so scans that overlap on one device race.
#include <mutex>

#include "srla_noalloc.h"

namespace srla {

static __device__ __align__(256) uint8_t scratch[kNoAllocScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_lock;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> hold(g_lock);
  if (g_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  if (!ptr) return hipErrorInvalidSymbol;
  g_ptr[device] = ptr;
  return hipSuccess;
}

void* noalloc_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> hold(g_lock);
  return g_ptr[device];
}

}  // namespace srla
