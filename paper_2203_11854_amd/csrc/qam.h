// Square Gray QAM of 3GPP TS 38.211 Sec. 5.1 (the mapper of Listing 1):
// per axis, h bits a0 a1 .. (a0 first) select the level
// (1-2a0)(2^{h-1} - (1-2a1)(2^{h-2} - ...)), scaled so that the complex
// constellation has unit average energy.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsim {

__device__ __forceinline__ float pam_level(const uint32_t* a, int h) {
  int v = 1;
  for (int l = h - 1; l >= 1; --l) v = (1 << (h - l)) - (1 - 2 * (int)a[l]) * v;
  return (float)((1 - 2 * (int)a[0]) * v);
}

// 1 / sqrt(2 (4^h - 1) / 3)
__device__ __forceinline__ float qam_inv_scale(int h) {
  return h == 1 ? 0.70710678118654752f : h == 2 ? 0.31622776601683794f : 0.15430334996209191f;
}

// Unit-energy level of axis label l (h bits, first bit most significant).
__device__ __forceinline__ float pam_unit(int l, int h) {
  uint32_t a[3] = {0, 0, 0};
  for (int q = 0; q < h; ++q) a[q] = (uint32_t)(l >> (h - 1 - q)) & 1u;
  return pam_level(a, h) * qam_inv_scale(h);
}

}  // namespace lsim
