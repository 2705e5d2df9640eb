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
  // e2 = 2 exp(-|q|);  m = e2 / (1 + e2 / 2)
  const float e2 = __builtin_amdgcn_exp2f(fmaf(fabsf(q), -kLog2e, 1.f));
  return e2 * __builtin_amdgcn_rcpf(fmaf(e2, 0.5f, 1.f));
}

__device__ __forceinline__ float spa_combine(float x, float y) { return x + y - x * y; }

// Running combination over a sequence: keeps D = 1 - prod(1 - m) and its
// complement C = prod(1 - m); one step is two fused multiply-adds, and
// (+)-ing another running value y onto it is D + y C (one more).
struct SpaAcc {
  float D = 0.f, C = 1.f;
  __device__ __forceinline__ void add(float m) {
    D = fmaf(m, C, D);
    C = fmaf(-C, m, C);
  }
};

// Unclamped output magnitude ln((2 - D) / D); +inf for D = 0.
__device__ __forceinline__ float spa_mag(float D) {
  return kLn2 * __builtin_amdgcn_logf((2.f - D) * __builtin_amdgcn_rcpf(D));
}

// Sum / difference form (flooding decoder).  With e = exp(-|q|) per input,
// tanh(|q|/2) = (1 - e) / (1 + e), so the product over a set of inputs is
// N / Dn with N = prod (1 - e_j) and Dn = prod (1 + e_j).  The decoder keeps
// S and A proportional to Dn + N and Dn - N: one input gives (1, e), and
// each further input maps
//   S' = S + e A,   A' = A + e S
// (positive terms only: no cancellation when every e is tiny).  For the
// inputs other than v, split into a prefix p and a suffix s,
//   S_v ~ Sp Ss + Ap As,   A_v ~ Sp As + Ap Ss,
// and the extrinsic magnitude is 2 atanh(N_v / Dn_v) = ln(S_v / A_v); at
// the ends of a check one side is empty and the ratio is that of the other.
// The flooding kernel keeps messages in log2 units (x log2 e), so e is one
// exp2 of the stored value and the magnitude one log2 of the ratio.
struct SpaSA {
  float S, A;
  __device__ __forceinline__ void add(float e) {
    const float s = fmaf(e, A, S);
    A = fmaf(e, S, A);
    S = s;
  }
};

// e = exp(-|q|) of a message stored in log2 units
__device__ __forceinline__ float spa_e2(float q2) { return __builtin_amdgcn_exp2f(-fabsf(q2)); }

// log2 of num / den clamped to [0, lmax2] (the ratio is >= 1 up to rounding)
__device__ __forceinline__ float spa_log2_ratio(float num, float den, float lmax2) {
  const float l = __builtin_amdgcn_logf(num * __builtin_amdgcn_rcpf(den));
  return __builtin_amdgcn_fmed3f(l, 0.f, lmax2);
}

}  // namespace lsim
