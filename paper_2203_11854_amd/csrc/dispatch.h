// Small device helpers shared by the decoder kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace lsim {

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

// Returns x unchanged in a vector register the optimizer cannot look
// through.  Rotated LDS addresses ((lane_bytes - shift_bytes) & mask) | base
// then stay one subtract and one v_and_or_b32 per edge: with the mask in a
// VGPR the and-or reads a single scalar (the base), and the lane's byte
// offset is not refactored into (lane - shift) & mask followed by a shift.
__device__ __forceinline__ int vreg(int x) {
  asm volatile("" : "+v"(x));
  return x;
}

template <int N>
struct Deg {
  static constexpr int value = N;
};

// Calls f(Deg<d>{}) for the wave-uniform degree d in [1, D]: every degree
// gets its own straight-line body, so all of a check's (or a variable
// node's) LDS reads are issued back to back before the first use.
template <int D, class F>
__device__ __forceinline__ void with_degree(int d, F&& f) {
  if constexpr (D >= 1) {
    if (d == D) {
      f(Deg<D>{});
      return;
    }
    with_degree<D - 1>(d, f);
  }
}

// Global access at an unsigned 32-bit byte offset from a wave-uniform base:
// the zero-extended offset lets the compiler use the scalar-base form of
// global_load/global_store (no 64-bit address arithmetic per lane).
template <class T>
__device__ __forceinline__ T ldg_at(const T* base, uint32_t byte_off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const unsigned char*>(base) + byte_off);
}
template <class T>
__device__ __forceinline__ void stg_at(T* base, uint32_t byte_off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<unsigned char*>(base) + byte_off) = v;
}

// Workgroup barrier that orders LDS only: global loads and stores in flight
// stay in flight across it (a plain __syncthreads() would wait for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace lsim
