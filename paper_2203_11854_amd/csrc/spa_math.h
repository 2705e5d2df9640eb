// Sum-product check-node arithmetic in the "1 - prod tanh" domain.
//
// For an input message q, m = 1 - tanh(|q|/2) = 2e / (1 + e) with
// e = exp(-|q|).  For a check with inputs q_1..q_d the magnitude of the
// extrinsic output to edge v is 2 atanh(prod_{j != v} tanh(|q_j|/2)).
// Writing D_v = 1 - prod_{j != v} (1 - m_j), built from exclusive prefix and
// suffix combinations x (+) y = x + y - x y, the output magnitude is
// ln((2 - D_v) / D_v).  This keeps full relative precision both for strong
// inputs (m tiny, D small) and weak ones (D near 1, output near 0), and needs
// one exp and one reciprocal per input and one reciprocal and one log per
// output.  Useful identities for the adjoint: cosh^2(r_v/2) = 1/(D_v (2-D_v)),
// sech^2(q/2) = m (2 - m), |tanh(q/2)| = 1 - m.
#pragma once

#include <hip/hip_runtime.h>

namespace lsim {

constexpr float kLog2e = 1.4426950408889634f;
constexpr float kLn2 = 0.6931471805599453f;

__device__ __forceinline__ float spa_m(float q) {
  const float e = __builtin_amdgcn_exp2f(-fabsf(q) * kLog2e);
  return 2.f * e * __builtin_amdgcn_rcpf(1.f + e);
}

__device__ __forceinline__ float spa_combine(float x, float y) { return x + y - x * y; }

// Unclamped output magnitude ln((2 - D) / D); +inf for D = 0.
__device__ __forceinline__ float spa_mag(float D) {
  return kLn2 * __builtin_amdgcn_logf((2.f - D) * __builtin_amdgcn_rcpf(D));
}

}  // namespace lsim
