// Small device helpers shared by the decoder kernels.
#pragma once

#include <hip/hip_runtime.h>

namespace lsim {

__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }

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

// Workgroup barrier that orders LDS only: global loads and stores in flight
// stay in flight across it (a plain __syncthreads() would wait for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

}  // namespace lsim
