// Fixed device scratch for the allocation-free entry point (wh_apply_A_noalloc):
// the state levels and the FP64 filter accumulator of one WaveHoltz
// application live in a file-scope device array instead of the caller's
// workspace, for callers that cannot allocate (code under stream capture,
// serving loops, harnesses that forbid allocation).  Every GPU the library
// runs on holds its own copy of the array until the process ends.
#include <hip/hip_runtime.h>

#include <mutex>

#include "wh_internal.h"

namespace wh {
namespace {

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

}  // namespace

// Device address of `scratch` on `device`, which the caller has made current.
// The address is looked up once per device (each device holds its own copy
// of the array at its own address) and kept; the array's name itself is only
// a host-side stand-in and is never used as a device address.
hipError_t static_scratch(int device, void **ptr) {
  if (device < 0 || device >= kMaxDevices || !ptr) return hipErrorInvalidValue;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return hipSuccess;
}

}  // namespace wh
