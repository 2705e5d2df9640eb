// Philox4x32-10 counter-based generator (Salmon, Moraes, Dror & Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC'11), device side.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsim {

struct U4 {
  uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox10(U4 c, uint32_t k0, uint32_t k1) {
  constexpr uint32_t kM0 = 0xD2511F53u, kM1 = 0xCD9E8D57u;
  constexpr uint32_t kW0 = 0x9E3779B9u, kW1 = 0xBB67AE85u;
#pragma unroll
  for (int rnd = 0; rnd < 10; ++rnd) {
    const uint32_t hi0 = __umulhi(kM0, c.x), lo0 = kM0 * c.x;
    const uint32_t hi1 = __umulhi(kM1, c.z), lo1 = kM1 * c.z;
    c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
    k0 += kW0;
    k1 += kW1;
  }
  return c;
}

// Stream ids of the link's counters.
enum : uint32_t { kStreamBits = 0, kStreamNoise = 1, kStreamPrior = 2 };

__device__ __forceinline__ U4 philox_at(uint64_t seed, uint32_t block, uint64_t cw,
                                        uint32_t stream) {
  return philox10(U4{block, (uint32_t)cw, (uint32_t)(cw >> 32), stream}, (uint32_t)seed,
                  (uint32_t)(seed >> 32));
}

// Box-Muller pair of standard normals from two Philox words:
// u_a = (x_a + 1) 2^-32 in (0, 1], u_b = x_b 2^-32; radius sqrt(-2 ln u_a),
// angle 2 pi u_b.  The normals are rho*cs and rho*sn.
struct Polar {
  float rho, sn, cs;
};

__device__ __forceinline__ Polar box_muller(uint32_t xa, uint32_t xb) {
  constexpr float kInv32 = 2.3283064365386963e-10f;  // 2^-32
  const float ua = fmaf((float)xa, kInv32, kInv32);
  const float ub = (float)xb * kInv32;
  Polar p;
  p.rho = sqrtf(-2.0f * logf(ua));
  sincospif(2.0f * ub, &p.sn, &p.cs);
  return p;
}

}  // namespace lsim
