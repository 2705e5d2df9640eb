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
enum : uint32_t { kStreamBits = 0, kStreamNoise = 1 };

__device__ __forceinline__ U4 philox_at(uint64_t seed, uint32_t block, uint64_t cw,
                                        uint32_t stream) {
  return philox10(U4{block, (uint32_t)cw, (uint32_t)(cw >> 32), stream}, (uint32_t)seed,
                  (uint32_t)(seed >> 32));
}

}  // namespace lsim
