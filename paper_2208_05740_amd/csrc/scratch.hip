// Static device workspace of the entry point that allocates nothing
// (gcp_bound_noalloc): a file-scope device array, one copy per device, held
// for the life of the process.  Host code never passes the array's name to
// a kernel: on the host that name is only a stand-in, so its device address
// is looked up once per device with hipGetSymbolAddress and kept.
#include "gcp_internal.h"

#include <hip/hip_runtime.h>

#include <mutex>

namespace gcp {

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

hipError_t scratch_region(void** ptr, size_t* bytes) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static void* addr[kMaxDevices] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(mu);
  if (!addr[dev]) {
    void* q = nullptr;
    e = hipGetSymbolAddress(&q, HIP_SYMBOL(scratch));   // with `dev` current
    if (e != hipSuccess) return e;
    if (!q) return hipErrorInvalidSymbol;
    addr[dev] = q;
  }
  *ptr = addr[dev];
  *bytes = kScratchBytes;
  return hipSuccess;
}

}  // namespace gcp
