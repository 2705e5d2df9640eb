// LDS access by byte offset.  A kernel with no static LDS gets its dynamic
// LDS at offset 0, so an integer byte offset is the LDS address itself: no
// per-access add of the dynamic array's base (which the compiler cannot fold,
// the base being a link-time symbol).  Launchers check the precondition
// with require_lds_at_zero().
#pragma once

#include <hip/hip_runtime.h>

namespace lsim {

template <class T>
__device__ __forceinline__ T lds_ld(int byte_off) {
  return *(const __attribute__((address_space(3))) T*)(size_t)byte_off;
}

template <class T>
__device__ __forceinline__ void lds_st(int byte_off, T v) {
  *(__attribute__((address_space(3))) T*)(size_t)byte_off = v;
}

}  // namespace lsim
