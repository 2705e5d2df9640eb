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

// 16-byte records (one ds_read_b128 / ds_write_b128); HIP's uint4 has no
// assignment in the LDS address space, so go through the native vector.
typedef unsigned int lds_u32x4 __attribute__((ext_vector_type(4)));

template <>
__device__ __forceinline__ uint4 lds_ld<uint4>(int byte_off) {
  const lds_u32x4 v = *(const __attribute__((address_space(3))) lds_u32x4*)(size_t)byte_off;
  return make_uint4(v.x, v.y, v.z, v.w);
}

template <>
__device__ __forceinline__ void lds_st<uint4>(int byte_off, uint4 v) {
  lds_u32x4 w;
  w.x = v.x;
  w.y = v.y;
  w.z = v.z;
  w.w = v.w;
  *(__attribute__((address_space(3))) lds_u32x4*)(size_t)byte_off = w;
}

}  // namespace lsim
