// Static device scratch of the allocation-free forward entry point
// (ur_simulate_noalloc): the transform intermediates, block partials and cell
// tables of one call live in a file-scope device array instead of memory the
// plan allocates, so the call itself never allocates.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ur_kernels.hpp"

namespace ur {

// Every device the library runs on holds its own copy of this array until
// the process ends; every call on a device shares it.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

// Device address of `scratch` on the current device.  On the host the
// array's name is only a stand-in for the symbol, not an address: it is
// resolved once per device (with that device current) and the cached
// address is used everywhere host code hands the memory to a kernel.
hipError_t noalloc_scratch(void** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[dev] = p;
  }
  *ptr = addr[dev];
  return hipSuccess;
}

}  // namespace ur
