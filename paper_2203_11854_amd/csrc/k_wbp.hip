// Weighted belief propagation (trainable flooding sum-product) and its
// hand-written adjoint.
//
// Forward, T rounds, weights w[t][e] on the check-to-variable messages:
//   r = clamp(CN_SPA(q), +-L);  APP = lam + sum_e w r;  q' = clamp(APP - w r, +-L)
// with q^(1) = lam = clamp(-L_ch, +-L) and output L_post = -APP^(T).  The
// variable-to-check messages entering each round are checkpointed to device
// memory, ckpt[t][b][e]; the backward pass recomputes every check from them.
//
// Backward of round t, given the adjoint of APP^(t) (only for t = T: minus
// dLoss/dL_post) and the adjoint qb' of q^(t+1):
//   g_e   = qb'_e [|APP_v - s_e| <= L]             (s_e = w_e r_e)
//   A_v   = abar_v + sum_{e at v} g_e ;  lam_bar_v += A_v
//   sb_e  = A_v - g_e ;  dw_e = sb_e r_e ;  rb_e = sb_e w_e
//   c_e   = rb_e [|r_e unclamped| <= L]
//   qb_k  = sech^2(q_k/2) sum_{v != k} c_v cosh^2(r_v/2) prod_{j not in {v,k}} tanh(q_j/2)
// The last sum is formed in O(d) per check from prefix/suffix products of
// t_j = tanh(q_j/2) and prefix/suffix sums A of c_v cosh^2 times partial
// products.  Once the reverse pass is through the first round,
// lam_bar_v += sum_e qb_e (q^(1) = lam), and
// dLoss/dL_ch = -lam_bar [|L_ch| <= L].
//
// The weight gradient is summed over the batch in a fixed order: every
// codeword writes its own contribution, a second kernel adds them up.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dispatch.h"
#include "lds.h"
#include "lsim_internal.h"
#include "spa_math.h"

namespace lsim {

namespace {

constexpr int kDMAX = 16;

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__device__ __forceinline__ float chan_lam(const DevCode& c, const float* llr_b, int v,
                                          float lmax) {
  const int x = v - c.tx_lo;
  return (x >= 0 && x < c.e_tx) ? fminf(fmaxf(-llr_b[x], -lmax), lmax) : 0.f;
}

// Clamped check outputs (natural units) of one check of degree D >= 2 from
// its inputs at byte offsets in_b + q*zs of ck (device memory), written to
// LDS at out_b + q*zs: the sum / difference form of spa_math.h.
template <int D>
__device__ __forceinline__ void cn_forward(const float* ck, uint32_t in_b, int zs, int out_b,
                                           float lmax2) {
  float x[D], ee[D], pS[D], pA[D];
#pragma unroll
  for (int q = 0; q < D; ++q) x[q] = ldg_at(ck, in_b + (uint32_t)(q * zs));
  uint32_t sx = 0;
#pragma unroll
  for (int q = 0; q < D; ++q) sx ^= __float_as_uint(x[q]);
#pragma unroll
  for (int q = 0; q < D; ++q) ee[q] = spa_e2(x[q] * kLog2e);
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
    const float rv = spa_log2_ratio(num, den, lmax2) * kLn2;
    lds_st<float>(out_b + q * zs,
                  __uint_as_float(__float_as_uint(rv) | ((sx ^ __float_as_uint(x[q])) & 0x80000000u)));
    if (q < D - 1 && q > 0) suf.add(ee[q]);
  }
}

// Forward.  Same schedule and arithmetic as the flooding sum-product
// decoder (sum / difference check update, messages in log2 units inside
// the kernel, LDS addressed by byte offset from 0); the weights multiply
// the check outputs and the checkpoints are stored in natural units, each
// check writing its inputs as it reads them (coalesced over the lift
// index; no separate copy pass or barrier).  ZC: compile-time lift size or
// 0.
template <int NT, int ZC>
__global__ __launch_bounds__(NT) void wbp_forward_kernel(DevCode c, int T,
                                                         const float* __restrict__ w,
                                                         const float* __restrict__ llr,
                                                         float lmax, float* __restrict__ ckpt,
                                                         float* __restrict__ lpost, int64_t B) {
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  (void)smem;
  const int lam_b = (int)align16((size_t)c.E * 4);
  const int tid = threadIdx.x, lane = tid & 63, wave = uni(tid >> 6);
  const int Z = ZC ? ZC : c.Z;
  const int zm = Z - 1;
  const bool zpow2 = (Z & zm) == 0;
  const float lmax2 = lmax * kLog2e;
  const int64_t b = blockIdx.x;
  const float* llr_b = llr + b * (int64_t)c.e_tx;
  for (int v = tid; v < c.n_dec; v += NT)
    lds_st<float>(lam_b + 4 * v, chan_lam(c, llr_b, v, lmax) * kLog2e);
  __syncthreads();

  // byte offsets of the DC edges of variable node (j, cc)
  auto col_b = [&](auto deg, int cb, int cc, int* off) {
    constexpr int DC = decltype(deg)::value;
    if (zpow2) {
      const int cc_b = vreg(cc * 4), zm_b = vreg(zm * 4);
#pragma unroll
      for (int q = 0; q < DC; ++q) {
        const int2 ce = ld_const(c.col_edge, cb + q);
        off[q] = ((cc_b - ce.y * 4) & zm_b) | (ce.x * 4);
      }
    } else {
#pragma unroll
      for (int q = 0; q < DC; ++q) {
        const int2 ce = ld_const(c.col_edge, cb + q);
        int x = cc - ce.y;
        x += x < 0 ? Z : 0;
        off[q] = (ce.x + x) * 4;
      }
    }
  };

  // q^(1) = lam on every edge
  for (int ti = wave; ti < c.n_vn_tasks; ti += NW) {
    const int task = uni(ld_const(c.vn_tasks, ti));
    const int j = task >> 16, cc = (task & 0xffff) + lane;
    const int cb = uni(ld_const(c.col_ptr, j)), dc = uni(ld_const(c.col_ptr, j + 1)) - cb;
    if (cc < Z) {
      const float l = lds_ld<float>(lam_b + 4 * (j * Z + cc));
      with_degree<kDMAX>(dc, [&](auto deg) {
        constexpr int DC = decltype(deg)::value;
        int off[DC];
        col_b(deg, cb, cc, off);
#pragma unroll
        for (int q = 0; q < DC; ++q) lds_st<float>(off[q], l);
      });
    }
  }
  __syncthreads();
  for (int it = 0; it < T; ++it) {
    const bool last = it + 1 == T;
    // the round's checkpoint: each check writes its inputs as it reads them
    float* ck = ckpt ? ckpt + ((int64_t)it * B + b) * c.E : nullptr;
    for (int ti = wave; ti < c.n_cn_tasks; ti += NW) {
      const int task = uni(ld_const(c.cn_tasks, ti));
      const int i = task >> 16, r = (task & 0xffff) + lane;
      const int e0 = uni(ld_const(c.row_ptr, i)), d = uni(ld_const(c.row_ptr, i + 1)) - e0;
      if (r < Z) {
        const int row_b = (e0 * Z + r) * 4;
        with_degree<kDMAX>(d, [&](auto deg) {
          constexpr int D = decltype(deg)::value;
          float x[D];
#pragma unroll
          for (int q = 0; q < D; ++q) x[q] = lds_ld<float>(row_b + q * Z * 4);
          if (ck) {
#pragma unroll
            for (int q = 0; q < D; ++q) stg_at(ck, (uint32_t)(row_b + q * Z * 4), x[q] * kLn2);
          }
          if constexpr (D >= 2) {  // decoded checks have degree >= 2
            float ee[D], pS[D], pA[D];
            uint32_t sx = 0;
#pragma unroll
            for (int q = 0; q < D; ++q) sx ^= __float_as_uint(x[q]);
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
    lds_barrier();
    const float* wt = w + (int64_t)it * c.E;
    for (int ti = wave; ti < c.n_vn_tasks; ti += NW) {
      const int task = uni(ld_const(c.vn_tasks, ti));
      const int j = task >> 16, cc = (task & 0xffff) + lane;
      const int cb = uni(ld_const(c.col_ptr, j)), dc = uni(ld_const(c.col_ptr, j + 1)) - cb;
      if (cc < Z) {
        const int v = j * Z + cc;
        with_degree<kDMAX>(dc, [&](auto deg) {
          constexpr int DC = decltype(deg)::value;
          int off[DC];
          col_b(deg, cb, cc, off);
          float s[DC], wv[DC];
#pragma unroll
          for (int q = 0; q < DC; ++q) wv[q] = ldg_at(wt, (uint32_t)off[q]);
#pragma unroll
          for (int q = 0; q < DC; ++q) s[q] = lds_ld<float>(off[q]);
          float acc = lds_ld<float>(lam_b + 4 * v);
#pragma unroll
          for (int q = 0; q < DC; ++q) {
            s[q] *= wv[q];
            acc += s[q];
          }
          if (!last) {
#pragma unroll
            for (int q = 0; q < DC; ++q)
              lds_st<float>(off[q], __builtin_amdgcn_fmed3f(acc - s[q], -lmax2, lmax2));
          } else {
            lpost[b * (int64_t)c.n_dec + v] = -acc * kLn2;
          }
        });
      }
    }
    lds_barrier();
  }
}

// LDS (byte offsets from 0; no static LDS): R[E] (recomputed clamped check
// outputs) at 0, QB[E] (adjoints of the variable-to-check messages, then of
// the check outputs) at qb_b, LB[n_dec] at lb_b.  ZC: compile-time lift size
// or 0.  A check output is unclamped, ln((2 - D)/D) <= L, exactly when
// D >= dth = 2 / (1 + e^L), so the clamp mask needs no logarithm.
// Workgroup g takes codewords g, g + G, g + 2G, ... (G = gridDim.x) and adds
// their weight gradients into its own partial gw_part[g][T][E] in that
// order: the first codeword stores, the later ones load and add.  Each edge
// of a round is written by one fixed thread (the column task's lane), so a
// thread only reads back its own earlier stores.
template <int NT, int ZC>
__global__ __launch_bounds__(NT) void wbp_backward_kernel(
    DevCode c, int T, const float* __restrict__ w, const float* __restrict__ llr,
    const float* __restrict__ ckpt, float lmax, float dth, const float* __restrict__ gpost,
    float* __restrict__ gllr, float* __restrict__ gw_part, int64_t B) {
  constexpr int NW = NT / 64;
  const int qb_b = c.E * 4;
  const int lb_b = (int)align16((size_t)2 * c.E * 4);
  const int tid = threadIdx.x, lane = tid & 63, wave = uni(tid >> 6);
  const int Z = ZC ? ZC : c.Z;
  const int zm = Z - 1;
  const bool zpow2 = (Z & zm) == 0;
  const float lmax2 = lmax * kLog2e;

  auto col_b = [&](auto deg, int cb, int cc, int* off) {
    constexpr int DC = decltype(deg)::value;
    if (zpow2) {
      const int cc_b = vreg(cc * 4), zm_b = vreg(zm * 4);
#pragma unroll
      for (int q = 0; q < DC; ++q) {
        const int2 ce = ld_const(c.col_edge, cb + q);
        off[q] = ((cc_b - ce.y * 4) & zm_b) | (ce.x * 4);
      }
    } else {
#pragma unroll
      for (int q = 0; q < DC; ++q) {
        const int2 ce = ld_const(c.col_edge, cb + q);
        int x = cc - ce.y;
        x += x < 0 ? Z : 0;
        off[q] = (ce.x + x) * 4;
      }
    }
  };

  for (int64_t b = blockIdx.x; b < B; b += gridDim.x) {
    const bool first = b == (int64_t)blockIdx.x;
    const float* llr_b = llr + b * (int64_t)c.e_tx;
    for (int v = tid; v < c.n_dec; v += NT) lds_st<float>(lb_b + 4 * v, 0.f);
    for (int e = tid; e < c.E; e += NT) lds_st<float>(qb_b + 4 * e, 0.f);
    __syncthreads();

    for (int it = T - 1; it >= 0; --it) {
      const float* ck = ckpt + ((int64_t)it * B + b) * c.E;
      // A: recompute the clamped check outputs of round it
      for (int ti = wave; ti < c.n_cn_tasks; ti += NW) {
        const int task = uni(ld_const(c.cn_tasks, ti));
        const int i = task >> 16, r = (task & 0xffff) + lane;
        const int e0 = uni(ld_const(c.row_ptr, i)), d = uni(ld_const(c.row_ptr, i + 1)) - e0;
        if (r < Z) {
          with_degree<kDMAX>(d, [&](auto deg) {
            constexpr int D = decltype(deg)::value;
            if constexpr (D >= 2)
              cn_forward<D>(ck, (uint32_t)((e0 * Z + r) * 4), Z * 4, (e0 * Z + r) * 4, lmax2);
          });
        }
      }
      lds_barrier();
      // B: variable-side adjoint
      const float* wt = w + (int64_t)it * c.E;
      float* gwb = gw_part + ((int64_t)blockIdx.x * T + it) * c.E;
      const bool last = it + 1 == T;
      for (int ti = wave; ti < c.n_vn_tasks; ti += NW) {
        const int task = uni(ld_const(c.vn_tasks, ti));
        const int j = task >> 16, cc = (task & 0xffff) + lane;
        const int cb = uni(ld_const(c.col_ptr, j)), dc = uni(ld_const(c.col_ptr, j + 1)) - cb;
        if (cc < Z) {
          const int v = j * Z + cc;
          with_degree<kDMAX>(dc, [&](auto deg) {
            constexpr int DC = decltype(deg)::value;
            int off[DC];
            col_b(deg, cb, cc, off);
            float rr[DC], ww[DC], s[DC], g[DC], gp[DC];
#pragma unroll
            for (int q = 0; q < DC; ++q) ww[q] = ldg_at(wt, (uint32_t)off[q]);
#pragma unroll
            for (int q = 0; q < DC; ++q) gp[q] = first ? 0.f : ldg_at(gwb, (uint32_t)off[q]);
#pragma unroll
            for (int q = 0; q < DC; ++q) rr[q] = lds_ld<float>(off[q]);
            float acc = chan_lam(c, llr_b, v, lmax);
#pragma unroll
            for (int q = 0; q < DC; ++q) {
              s[q] = ww[q] * rr[q];
              acc += s[q];
            }
            float A = last ? -gpost[b * (int64_t)c.n_dec + v] : 0.f;
            if (!last) {
#pragma unroll
              for (int q = 0; q < DC; ++q) {
                const float qv = acc - s[q];
                g[q] = fabsf(qv) <= lmax ? lds_ld<float>(qb_b + off[q]) : 0.f;
                A += g[q];
              }
            } else {
#pragma unroll
              for (int q = 0; q < DC; ++q) g[q] = 0.f;
            }
            lds_st<float>(lb_b + 4 * v, lds_ld<float>(lb_b + 4 * v) + A);
#pragma unroll
            for (int q = 0; q < DC; ++q) {
              const float sb = A - g[q];
              const float gq = sb * rr[q];
              stg_at(gwb, (uint32_t)off[q], first ? gq : gp[q] + gq);
              lds_st<float>(qb_b + off[q], sb * ww[q]);
            }
          });
        }
      }
      lds_barrier();
      // C: check-side adjoint from the checkpointed inputs
      for (int ti = wave; ti < c.n_cn_tasks; ti += NW) {
        const int task = uni(ld_const(c.cn_tasks, ti));
        const int i = task >> 16, r = (task & 0xffff) + lane;
        const int e0 = uni(ld_const(c.row_ptr, i)), d = uni(ld_const(c.row_ptr, i + 1)) - e0;
        if (r < Z) {
          const uint32_t qin_b = (uint32_t)((e0 * Z + r) * 4);
          const int qrow_b = qb_b + (e0 * Z + r) * 4;
          with_degree<kDMAX>(d, [&](auto deg) {
            constexpr int D = decltype(deg)::value;
            float x[D], cbar[D];
#pragma unroll
            for (int q = 0; q < D; ++q) x[q] = ldg_at(ck, qin_b + (uint32_t)(q * Z * 4));
#pragma unroll
            for (int q = 0; q < D; ++q) cbar[q] = lds_ld<float>(qrow_b + q * Z * 4);
            float mm[D], tt[D], pD[D], pC[D], av[D];
            SpaAcc pre;
#pragma unroll
            for (int q = 0; q < D; ++q) {
              const float m = spa_m(x[q]);
              mm[q] = m;
              tt[q] = __uint_as_float(__float_as_uint(1.f - m) |
                                      (__float_as_uint(x[q]) & 0x80000000u));
              pD[q] = pre.D;
              pC[q] = pre.C;
              pre.add(m);
            }
            // a_v = c_v cosh^2(r_v/2) with cosh^2 = 1/(D (2 - D)); zero where clamped
            SpaAcc suf;
#pragma unroll
            for (int q = D - 1; q >= 0; --q) {
              const float Dx = fmaf(suf.D, pC[q], pD[q]);
              av[q] = Dx >= dth ? cbar[q] * __builtin_amdgcn_rcpf(Dx * (2.f - Dx)) : 0.f;
              suf.add(mm[q]);
            }
            // S_k = Apre_k Psuf_k + Ppre_k Asuf_k
            float ap[D], pp[D];
            float P = 1.f, Aacc = 0.f;
#pragma unroll
            for (int q = 0; q < D; ++q) {
              ap[q] = Aacc;
              pp[q] = P;
              Aacc = Aacc * tt[q] + av[q] * P;
              P *= tt[q];
            }
            float Ps = 1.f, As = 0.f;
#pragma unroll
            for (int q = D - 1; q >= 0; --q) {
              const float S = ap[q] * Ps + pp[q] * As;
              lds_st<float>(qrow_b + q * Z * 4, mm[q] * (2.f - mm[q]) * S);
              As = As * tt[q] + av[q] * Ps;
              Ps *= tt[q];
            }
          });
        }
      }
      lds_barrier();
    }
    // D: q^(1) = lam, then the channel clamp
    for (int ti = wave; ti < c.n_vn_tasks; ti += NW) {
      const int task = uni(ld_const(c.vn_tasks, ti));
      const int j = task >> 16, cc = (task & 0xffff) + lane;
      const int cb = uni(ld_const(c.col_ptr, j)), dc = uni(ld_const(c.col_ptr, j + 1)) - cb;
      if (cc < Z) {
        const int v = j * Z + cc;
        float acc = lds_ld<float>(lb_b + 4 * v);
        with_degree<kDMAX>(dc, [&](auto deg) {
          constexpr int DC = decltype(deg)::value;
          int off[DC];
          col_b(deg, cb, cc, off);
#pragma unroll
          for (int q = 0; q < DC; ++q) acc += lds_ld<float>(qb_b + off[q]);
        });
        const int xx = v - c.tx_lo;
        if (xx >= 0 && xx < c.e_tx) {
          const float L = llr_b[xx];
          gllr[b * (int64_t)c.e_tx + xx] = fabsf(L) <= lmax ? -acc : 0.f;
        }
      }
    }
    __syncthreads();  // the next codeword clears the LDS this one still reads
  }
}

// gw[t][e] = sum over rows b of part[b][t][e] (one row per adjoint
// workgroup), in a fixed order: pass 1 sums kSlices contiguous runs of rows
// into slice partials, pass 2 adds the slices in order.  When rows are a multiple of four floats every thread
// reads four adjacent columns with 16-byte loads.
constexpr int kSlices = 32;

__global__ __launch_bounds__(256) void sum_slices_kernel(const float* __restrict__ part, int64_t B,
                                                         int64_t n, float* __restrict__ slices) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int64_t per = (B + kSlices - 1) / kSlices;
  const int64_t b0 = blockIdx.y * per;
  const int64_t b1 = b0 + per < B ? b0 + per : B;
  float acc = 0.f;
#pragma unroll 8
  for (int64_t b = b0; b < b1; ++b) acc += part[b * n + i];
  slices[(int64_t)blockIdx.y * n + i] = acc;
}

__global__ __launch_bounds__(256) void sum_slices4_kernel(const float* __restrict__ part, int64_t B,
                                                         int64_t n, float* __restrict__ slices) {
  const int64_t i4 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // column quad
  if (4 * i4 >= n) return;
  const int64_t per = (B + kSlices - 1) / kSlices;
  const int64_t b0 = blockIdx.y * per;
  const int64_t b1 = b0 + per < B ? b0 + per : B;
  float4 acc = make_float4(0.f, 0.f, 0.f, 0.f);
  const float4* p = reinterpret_cast<const float4*>(part) + i4;
  const int64_t stride = n / 4;
#pragma unroll 8
  for (int64_t b = b0; b < b1; ++b) {
    const float4 x = p[b * stride];
    acc.x += x.x;
    acc.y += x.y;
    acc.z += x.z;
    acc.w += x.w;
  }
  reinterpret_cast<float4*>(slices)[(int64_t)blockIdx.y * stride + i4] = acc;
}

__global__ void sum_final_kernel(const float* __restrict__ slices, int64_t n,
                                 float* __restrict__ out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
  for (int k = 0; k < kSlices; ++k) acc += slices[(int64_t)k * n + i];
  out[i] = acc;
}

size_t fwd_lds(const DevCode& c) { return align16((size_t)c.E * 4) + align16((size_t)c.n_dec * 4); }
size_t bwd_lds(const DevCode& c) {
  return align16((size_t)2 * c.E * 4) + align16((size_t)c.n_dec * 4);
}

constexpr int kFwdNT = 512;
constexpr int kBwdNT = 1024;

const void* bwd_kernel(const DevCode& c) {
  return c.Z == 128 ? (const void*)wbp_backward_kernel<kBwdNT, 128>
                    : (const void*)wbp_backward_kernel<kBwdNT, 0>;
}

// Adjoint workgroups resident at once on the current device: the launch's
// grid and the number of weight-gradient partials it writes.
hipError_t bwd_slots(const DevCode& c, int64_t* slots) {
  const void* k = bwd_kernel(c);
  const size_t lds = bwd_lds(c);
  int dev = 0, ncu = 0, occ = 0;
  hipError_t e = ensure_dyn_lds(k, lds);
  if (e == hipSuccess) e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, k, kBwdNT, lds);
  if (e != hipSuccess) return e;
  *slots = (int64_t)(ncu > 0 ? ncu : 1) * (occ > 0 ? occ : 1);
  return hipSuccess;
}

}  // namespace

// min(B, resident workgroups) partial rows plus the slice sums; where the
// device cannot be asked, one row per codeword (an upper bound)
size_t wbp_work_bytes(const DevCode& c, int T, int64_t B) {
  int64_t slots = B;
  if (bwd_lds(c) > 160 * 1024 || bwd_slots(c, &slots) != hipSuccess) {
    (void)hipGetLastError();
    slots = B;
  }
  const int64_t G = B < slots ? B : slots;
  return ((size_t)G + kSlices) * T * c.E * 4;
}

hipError_t launch_wbp_forward(const DevCode& c, int T, const float* w, const float* llr,
                              int64_t B, float llr_max, float* ckpt, float* lpost, hipStream_t s,
                              std::string* why) {
  const int dmax = c.max_row_deg > c.max_col_deg ? c.max_row_deg : c.max_col_deg;
  if (dmax > kDMAX) {
    *why = "weighted BP supports degrees up to 16";
    return hipSuccess;
  }
  const size_t lds = fwd_lds(c);
  if (lds > 160 * 1024) {
    *why = "weighted BP state exceeds the 160 KiB LDS";
    return hipSuccess;
  }
  const void* k = c.Z == 128 ? (const void*)wbp_forward_kernel<kFwdNT, 128>
                             : (const void*)wbp_forward_kernel<kFwdNT, 0>;
  hipError_t e = require_lds_at_zero(k);
  if (e == hipSuccess) e = ensure_dyn_lds(k, lds);
  if (e != hipSuccess) return e;
  if (c.Z == 128)
    wbp_forward_kernel<kFwdNT, 128><<<(unsigned)B, kFwdNT, lds, s>>>(c, T, w, llr, llr_max, ckpt,
                                                                    lpost, B);
  else
    wbp_forward_kernel<kFwdNT, 0><<<(unsigned)B, kFwdNT, lds, s>>>(c, T, w, llr, llr_max, ckpt,
                                                                  lpost, B);
  return hipGetLastError();
}

hipError_t launch_wbp_backward(const DevCode& c, int T, const float* w, const float* llr,
                               const float* ckpt, int64_t B, float llr_max, const float* gpost,
                               float* gllr, float* gw, void* work, hipStream_t s,
                               std::string* why) {
  const int dmax = c.max_row_deg > c.max_col_deg ? c.max_row_deg : c.max_col_deg;
  if (dmax > kDMAX) {
    *why = "weighted BP supports degrees up to 16";
    return hipSuccess;
  }
  const size_t lds = bwd_lds(c);
  if (lds > 160 * 1024) {
    *why = "weighted BP adjoint state exceeds the 160 KiB LDS";
    return hipSuccess;
  }
  const void* k = bwd_kernel(c);
  hipError_t e = require_lds_at_zero(k);
  if (e == hipSuccess) e = ensure_dyn_lds(k, lds);
  if (e != hipSuccess) return e;
  float* part = reinterpret_cast<float*>(work);
  // one workgroup per resident slot, each summing its codewords' weight
  // gradients into one partial; the partials are then added in a fixed order
  // (the workspace was sized by wbp_work_bytes from the same query)
  int64_t slots = 0;
  e = bwd_slots(c, &slots);
  if (e != hipSuccess) return e;
  const int64_t G = B < slots ? B : slots;
  // the clamp threshold on D: ln((2 - D) / D) <= L  <=>  D >= 2 / (1 + e^L)
  const float dth = (float)(2.0 / (1.0 + std::exp((double)llr_max)));
  if (c.Z == 128)
    wbp_backward_kernel<kBwdNT, 128><<<(unsigned)G, kBwdNT, lds, s>>>(
        c, T, w, llr, ckpt, llr_max, dth, gpost, gllr, part, B);
  else
    wbp_backward_kernel<kBwdNT, 0><<<(unsigned)G, kBwdNT, lds, s>>>(
        c, T, w, llr, ckpt, llr_max, dth, gpost, gllr, part, B);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)T * c.E;
  float* slices = part + (size_t)G * n;
  if ((n & 3) == 0) {
    dim3 grid((unsigned)((n / 4 + 255) / 256), kSlices);
    sum_slices4_kernel<<<grid, 256, 0, s>>>(part, G, n, slices);
  } else {
    dim3 grid((unsigned)((n + 255) / 256), kSlices);
    sum_slices_kernel<<<grid, 256, 0, s>>>(part, G, n, slices);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  sum_final_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(slices, n, gw);
  return hipGetLastError();
}

}  // namespace lsim
