// Flooding FP32 sum-product decoder on a QC Tanner graph (messages clamped
// to +-llr_max; the int8 offset min-sum decoder is k_oms2.hip).
//
// One workgroup decodes one codeword with its whole message state in LDS:
// msg[E] holds, per edge in canonical order (base nonzero e, lift r -> e*Z+r),
// the variable-to-check message q before a check phase and the
// check-to-variable message r after it; lam[n_dec] holds the channel LLRs.
// A round is two phases separated by barriers:
//   check phase     lane = check (i, r); reads the d_i messages of its row
//                   (addresses e*Z + r: consecutive lanes, no bank conflict),
//                   writes r in place;
//   variable phase  lane = variable node (j, c); gathers the column's r
//                   (addresses e*Z + (c - s) mod Z: rotated contiguous
//                   segments), forms APP = lam + sum r and writes
//                   q = clamp(APP - r).
// Work items are (base row or column, 64-lift block); every wavefront works
// on a single row or column at a time, so the degree loop is uniform.  Items
// are sorted heaviest first and dealt round-robin to the wavefronts.
#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "lds.h"
#include "lsim_internal.h"
#include "spa_math.h"

namespace lsim {

namespace {

struct FloodArgs {
  const float* llr;
  int64_t B;
  uint8_t* bits;
  float* lpost;
  const float* q_in;
  float* r_out;
  float* q_out;
  int iters;
  float llr_max;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t spa_lds(const DevCode& c) {
  return align16((size_t)c.E * 4) + align16((size_t)c.n_dec * 4);
}

// ZC: the lift size when it is a compile-time constant (0: read from the
// code), which turns the check phase's row strides into immediate offsets.
// LDS: messages at byte 0, channel LLRs at lam_b (kernel has no static LDS).
template <int NT, int DMAX, int ZC>
__global__ __launch_bounds__(NT) void flood_kernel(DevCode c, FloodArgs a) {
  using M = float;
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  M* msg = reinterpret_cast<M*>(smem);
  M* lam = reinterpret_cast<M*>(smem + align16((size_t)c.E * sizeof(M)));
  const int lam_b = (int)align16((size_t)c.E * sizeof(M));
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = uni(tid >> 6);
  const int Z = ZC ? ZC : c.Z;
  const int64_t b = blockIdx.x;

  // ---- channel LLRs, zero messages (graph tables are read with scalar
  // loads from the code's device tables)
  const int zm = Z - 1;
  const bool zpow2 = (Z & zm) == 0;
  // sum-product messages live in log2 units (x log2 e) inside the kernel
  const float lmax2 = a.llr_max * kLog2e;
  const float* llr = a.llr + b * (int64_t)c.e_tx;
  for (int v = tid; v < c.n_dec; v += NT) {
    const int x = v - c.tx_lo;
    M l = 0;
    if (x >= 0 && x < c.e_tx) l = fminf(fmaxf(-llr[x], -a.llr_max), a.llr_max) * kLog2e;
    lam[v] = l;
  }
  if (a.q_in) {
    const float* qi = a.q_in + b * (int64_t)c.E;
    for (int e = tid; e < c.E; e += NT) msg[e] = qi[e] * kLog2e;
  } else {
    for (int e = tid; e < c.E; e += NT) msg[e] = 0;
  }
  __syncthreads();

  // variable phase; mode 0: q <- clamp(lam + sum r - r), 1: last round
  auto var_phase = [&](bool write_q, bool final_round) {
    for (int ti = wave; ti < c.n_vn_tasks; ti += NW) {
      const int task = uni(ld_const(c.vn_tasks, ti));
      const int j = task >> 16;
      const int cc = (task & 0xffff) + lane;
      const int cb = uni(ld_const(c.col_ptr, j));
      const int dc = uni(ld_const(c.col_ptr, j + 1)) - cb;
      if (cc < Z) {
        const int v = j * Z + cc;
        with_degree<DMAX>(dc, [&](auto deg) {
          constexpr int DC = decltype(deg)::value;
          int idx[DC];
          float rv[DC];
          // byte offset of entry e's edge at lift c: (e*Z + (c - shift) mod Z) * sizeof(M)
          constexpr int SZ = sizeof(M);
          if (zpow2) {
            const int cc_b = vreg(cc * SZ), zm_b = vreg(zm * SZ);
#pragma unroll
            for (int q = 0; q < DC; ++q) {
              const int2 ce = ld_const(c.col_edge, cb + q);
              idx[q] = ((cc_b - ce.y * SZ) & zm_b) | (ce.x * SZ);
            }
          } else {
#pragma unroll
            for (int q = 0; q < DC; ++q) {
              const int2 ce = ld_const(c.col_edge, cb + q);
              int x = cc - ce.y;
              x += x < 0 ? Z : 0;
              idx[q] = (ce.x + x) * SZ;
            }
          }
#pragma unroll
          for (int q = 0; q < DC; ++q) rv[q] = lds_ld<float>(idx[q]);
          float acc = lds_ld<float>(lam_b + v * 4);
#pragma unroll
          for (int q = 0; q < DC; ++q) acc += rv[q];
          if (write_q) {
#pragma unroll
            for (int q = 0; q < DC; ++q)
              lds_st<float>(idx[q], __builtin_amdgcn_fmed3f(acc - rv[q], -lmax2, lmax2));
          }
          if (final_round) {
            if (a.bits && v < c.k) a.bits[b * (int64_t)c.k + v] = acc < 0;
            if (a.lpost) a.lpost[b * (int64_t)c.n_dec + v] = -acc * kLn2;
          }
        });
      }
    }
  };

  auto check_phase = [&]() {
    for (int ti = wave; ti < c.n_cn_tasks; ti += NW) {
      const int task = uni(ld_const(c.cn_tasks, ti));
      const int i = task >> 16;
      const int r = (task & 0xffff) + lane;
      const int e0 = uni(ld_const(c.row_ptr, i));
      const int d = uni(ld_const(c.row_ptr, i + 1)) - e0;
      if (r < Z) {
        const int row_b = (e0 * Z + r) * 4;
        with_degree<DMAX>(d, [&](auto deg) {
          constexpr int D = decltype(deg)::value;
          if constexpr (D >= 2) {  // decoded checks have degree >= 2
          M x[D];
#pragma unroll
          for (int q = 0; q < D; ++q) x[q] = lds_ld<float>(row_b + q * Z * 4);
          // sum-product in the sum / difference form, log2 units
          // (spa_math.h); the output sign is the XOR of the other inputs'
          // sign bits (a zero input only ever receives or sends zero
          // magnitudes, so the sign of a zero is immaterial)
          uint32_t sx = 0;
#pragma unroll
          for (int q = 0; q < D; ++q) sx ^= __float_as_uint(x[q]);
          float ee[D], pS[D], pA[D];
#pragma unroll
          for (int q = 0; q < D; ++q) ee[q] = spa_e2(x[q]);
          SpaSA pre{1.f, ee[0]};
#pragma unroll
          for (int q = 1; q < D; ++q) {
            pS[q] = pre.S;
            pA[q] = pre.A;
            if (q + 1 < D) pre.add(ee[q]);
          }
          SpaSA suf{1.f, ee[D - 1]};
#pragma unroll
          for (int q = D - 1; q >= 0; --q) {
            float num, den;
            if (q == D - 1) {
              num = pS[q];
              den = pA[q];
            } else if (q == 0) {
              num = suf.S;
              den = suf.A;
            } else {
              num = fmaf(pS[q], suf.S, pA[q] * suf.A);
              den = fmaf(pS[q], suf.A, pA[q] * suf.S);
            }
            const float rv = spa_log2_ratio(num, den, lmax2);
            const uint32_t sg = (sx ^ __float_as_uint(x[q])) & 0x80000000u;
            lds_st<float>(row_b + q * Z * 4, __uint_as_float(__float_as_uint(rv) | sg));
            if (q < D - 1 && q > 0) suf.add(ee[q]);
          }
          }
        });
      }
    }
  };

  if (!a.q_in) {
    var_phase(true, false);  // q = lam on every edge
    __syncthreads();
  }
  for (int it = 0; it < a.iters; ++it) {
    const bool last = it + 1 == a.iters;
    check_phase();
    __syncthreads();
    if (last && a.r_out) {
      float* ro = a.r_out + b * (int64_t)c.E;
      for (int e = tid; e < c.E; e += NT) ro[e] = msg[e] * kLn2;
      __syncthreads();
    }
    var_phase(!last || a.q_out != nullptr, last);
    __syncthreads();
  }
  if (a.q_out) {
    float* qo = a.q_out + b * (int64_t)c.E;
    for (int e = tid; e < c.E; e += NT) qo[e] = msg[e] * kLn2;
  }
}

template <int NT, int DMAX, int ZC>
hipError_t launch_t(const DevCode& c, const FloodArgs& a, size_t lds, hipStream_t s) {
  const void* k = (const void*)flood_kernel<NT, DMAX, ZC>;
  hipError_t e = require_lds_at_zero(k);
  if (e == hipSuccess) e = ensure_dyn_lds(k, lds);
  if (e != hipSuccess) return e;
  flood_kernel<NT, DMAX, ZC><<<(unsigned)a.B, NT, lds, s>>>(c, a);
  return hipGetLastError();
}

hipError_t dispatch(const DevCode& c, int nt, const FloodArgs& a, size_t lds, hipStream_t s) {
  const int dmax = c.max_row_deg > c.max_col_deg ? c.max_row_deg : c.max_col_deg;
  // the lift of the BG2-shaped workloads with its own code
  if (c.Z == 128 && nt == 512 && dmax <= 16) return launch_t<512, 16, 128>(c, a, lds, s);
  if (c.Z == 128 && nt == 512 && dmax <= 24) return launch_t<512, 24, 128>(c, a, lds, s);
#define LSIM_FLOOD_CASE(NT_, D_) \
  if (nt == NT_ && dmax <= D_) return launch_t<NT_, D_, 0>(c, a, lds, s);
  LSIM_FLOOD_CASE(256, 16)
  LSIM_FLOOD_CASE(256, 24)
  LSIM_FLOOD_CASE(256, 32)
  LSIM_FLOOD_CASE(512, 16)
  LSIM_FLOOD_CASE(512, 24)
  LSIM_FLOOD_CASE(512, 32)
  LSIM_FLOOD_CASE(1024, 16)
  LSIM_FLOOD_CASE(1024, 24)
  LSIM_FLOOD_CASE(1024, 32)
#undef LSIM_FLOOD_CASE
  return hipErrorInvalidValue;
}

}  // namespace

size_t flood_lds_bytes(const DevCode& c, int algo) {
  if (algo == LSIM_SPA_F32) return spa_lds(c);
  return oms2_lds_bytes(c, 2) <= 160 * 1024 ? oms2_lds_bytes(c, 2) : oms2_lds_bytes(c, 1);
}

hipError_t launch_flood(const DevCode& c, const lsim_decode_params& p, const void* llr, int64_t B,
                        uint8_t* bits, float* lpost, const void* q_in, void* r_out, void* q_out,
                        hipStream_t s, std::string* why) {
  if (p.algo == LSIM_OMS_I8)
    return launch_oms2(c, p, static_cast<const int8_t*>(llr), B, bits, lpost,
                       static_cast<const int8_t*>(q_in), static_cast<int8_t*>(r_out),
                       static_cast<int8_t*>(q_out), s, why);
  const size_t lds = flood_lds_bytes(c, p.algo);
  if (lds > 160 * 1024) {
    *why = "flooding decoder state (" + std::to_string(lds) + " B) exceeds the 160 KiB LDS";
    return hipSuccess;
  }
  FloodArgs a{static_cast<const float*>(llr), B, bits, lpost, static_cast<const float*>(q_in),
              static_cast<float*>(r_out), static_cast<float*>(q_out), p.iters, p.llr_max};
  const int nt = p.threads ? p.threads : 512;
  return dispatch(c, nt, a, lds, s);
}

}  // namespace lsim
