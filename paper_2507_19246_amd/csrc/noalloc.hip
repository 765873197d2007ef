// Fixed device workspace of the allocation-free entry point
// (mlmc_level_run_noalloc): one file-scope device array per device that loads
// this library, held until the process ends.  Host code never passes the
// array's name to a kernel or a copy (on the host it is only a stand-in
// symbol); it uses the device address looked up here, once per device, with
// that device current.
#include <hip/hip_runtime.h>

#include <mutex>

#include "mq_internal.h"

static __device__ __align__(256) char scratch[MQ_NOALLOC_WORKSPACE_BYTES];

namespace mq {

hipError_t noalloc_workspace(int device, char** ptr) {
  constexpr int kMaxDevices = 64;
  static std::mutex mu;
  static char* addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(mu);
  if (!addr[device]) {
    int cur = -1;
    hipError_t e = hipGetDevice(&cur);
    if (e != hipSuccess) return e;
    if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
    void* a = nullptr;
    e = hipGetSymbolAddress(&a, HIP_SYMBOL(scratch));
    if (cur != device) (void)hipSetDevice(cur);
    if (e != hipSuccess) return e;
    addr[device] = static_cast<char*>(a);
  }
  *ptr = addr[device];
  return hipSuccess;
}

}  // namespace mq
