// Library-owned device scratch for lsim_decode_noalloc.
//
// A file-scope device array holds the layered decoder's per-check state for
// callers that cannot allocate.  Each GPU the library runs on gets its own
// copy of the array (at its own address) for the life of the process.  In
// host code the array's name is only a host-side stand-in, so its device
// address is looked up once per device with hipGetSymbolAddress while that
// device is current, and every launch takes that address.
#include <hip/hip_runtime.h>

#include <mutex>

#include "lsim_internal.h"

namespace lsim {

namespace {

constexpr int kMaxDevices = 64;

static __device__ __align__(256) uint32_t scratch[LSIM_NOALLOC_SCRATCH_BYTES / 4];

std::mutex g_mu;
void* g_ptr[kMaxDevices] = {};

}  // namespace

hipError_t noalloc_scratch(void** ptr, size_t* bytes) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_ptr[dev] = p;
  }
  *ptr = g_ptr[dev];
  *bytes = LSIM_NOALLOC_SCRATCH_BYTES;
  return hipSuccess;
}

}  // namespace lsim
