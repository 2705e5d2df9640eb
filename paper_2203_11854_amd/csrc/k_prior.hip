// Demapper with prior, consistent Gaussian a-priori LLRs, the mutual
// information between code bits and LLRs, and the decoder's extrinsic
// output: the pieces of EXIT chart simulations and of iterative demapping
// and decoding (both listed among the FEC features, Sec. III-B).
#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "lsim_internal.h"
#include "philox.h"
#include "qam.h"

namespace lsim {

namespace {

// Extrinsic LLRs of the h Gray bits of one axis at coordinate v, given the
// axis' a-priori LLRs la[h].  For bit q the metric of level l is
// -(v - x_l)^2 / N0 plus the priors of l's other bits that are 1 (bit q's
// own prior is left out, so nothing cancels); exact: log-sum-exp over the
// levels with bit q = 1 minus that over bit q = 0, max-log: max - max.
template <int h>
__device__ __forceinline__ void axis_ext(float v, float inv_no, const float* la, bool exact,
                                         float* out) {
  constexpr int nl = 1 << h;
  float d[nl];
#pragma unroll
  for (int l = 0; l < nl; ++l) {
    const float dv = v - pam_unit(l, h);
    d[l] = -(dv * dv * inv_no);
  }
#pragma unroll
  for (int q = 0; q < h; ++q) {
    float mt[nl];
#pragma unroll
    for (int l = 0; l < nl; ++l) {
      float a = d[l];
#pragma unroll
      for (int r = 0; r < h; ++r)
        if (r != q && ((l >> (h - 1 - r)) & 1)) a += la[r];
      mt[l] = a;
    }
    float m1 = -INFINITY, m0 = -INFINITY;
#pragma unroll
    for (int l = 0; l < nl; ++l) {
      if ((l >> (h - 1 - q)) & 1) m1 = fmaxf(m1, mt[l]);
      else m0 = fmaxf(m0, mt[l]);
    }
    if (!exact) {
      out[q] = m1 - m0;
    } else {
      float s1 = 0.f, s0 = 0.f;
#pragma unroll
      for (int l = 0; l < nl; ++l) {
        if ((l >> (h - 1 - q)) & 1) s1 += expf(mt[l] - m1);
        else s0 += expf(mt[l] - m0);
      }
      out[q] = (m1 - m0) + logf(s1) - logf(s0);
    }
  }
}

template <int M>
__device__ __forceinline__ void load_m(const float* p, float* v) {
  if constexpr (M == 4) {
    const float4 a = *reinterpret_cast<const float4*>(p);
    v[0] = a.x, v[1] = a.y, v[2] = a.z, v[3] = a.w;
  } else if constexpr (M == 2 || M == 6) {
#pragma unroll
    for (int i = 0; i < M / 2; ++i) {
      const float2 a = reinterpret_cast<const float2*>(p)[i];
      v[2 * i] = a.x, v[2 * i + 1] = a.y;
    }
  } else {
    v[0] = p[0];
  }
}

template <int M>
__device__ __forceinline__ void store_m(float* p, const float* v) {
  if constexpr (M == 4) {
    *reinterpret_cast<float4*>(p) = make_float4(v[0], v[1], v[2], v[3]);
  } else if constexpr (M == 2 || M == 6) {
#pragma unroll
    for (int i = 0; i < M / 2; ++i) reinterpret_cast<float2*>(p)[i] = make_float2(v[2 * i], v[2 * i + 1]);
  } else {
    p[0] = v[0];
  }
}

template <int M>
__global__ __launch_bounds__(256) void demap_prior_kernel(bool exact, const float* __restrict__ y,
                                                          const float* __restrict__ no,
                                                          const float* __restrict__ la, int64_t B,
                                                          int64_t S, bool extrinsic,
                                                          float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * S) return;
  const int64_t b = t / S;
  const float2 yy = reinterpret_cast<const float2*>(y)[t];
  const float n0 = no[b];
  float pa[M], L[M];
  load_m<M>(la + t * M, pa);
  if constexpr (M == 1) {
    L[0] = -4.0f * yy.x / n0;
  } else {
    constexpr int h = M / 2;
    const float inv_no = 1.0f / n0;
    float lai[h], laq[h], li[h], lq[h];
#pragma unroll
    for (int q = 0; q < h; ++q) {
      lai[q] = pa[2 * q];
      laq[q] = pa[2 * q + 1];
    }
    axis_ext<h>(yy.x, inv_no, lai, exact, li);
    axis_ext<h>(yy.y, inv_no, laq, exact, lq);
#pragma unroll
    for (int q = 0; q < h; ++q) {
      L[2 * q] = li[q];
      L[2 * q + 1] = lq[q];
    }
  }
  if (!extrinsic) {
#pragma unroll
    for (int i = 0; i < M; ++i) L[i] += pa[i];
  }
  store_m<M>(out + t * M, L);
}

// La = (2c - 1) sigma^2 / 2 + sigma n for the transmitted bits; bits
// 4j .. 4j+3 of a codeword take the two Box-Muller pairs of Philox block j
// of stream 2 (cosine, sine of words (0, 1), then of words (2, 3)).
__global__ __launch_bounds__(256) void apriori_kernel(DevCode c, const uint8_t* __restrict__ cw,
                                                      const float* __restrict__ sigma,
                                                      uint64_t seed, int64_t cw0, int64_t B,
                                                      float* __restrict__ la) {
  const int n = c.e_tx;
  const int nq = (n + 3) >> 2;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * nq) return;
  const int64_t b = t / nq;
  const int j = (int)(t - b * nq);
  const U4 r = philox_at(seed, (uint32_t)j, (uint64_t)(cw0 + b), kStreamPrior);
  const Polar p0 = box_muller(r.x, r.y), p1 = box_muller(r.z, r.w);
  const float nr[4] = {p0.rho * p0.cs, p0.rho * p0.sn, p1.rho * p1.cs, p1.rho * p1.sn};
  const float s = sigma[b];
  const float mu = 0.5f * s * s;
  const uint8_t* bits = cw + b * (int64_t)c.n_mother + c.tx_lo + 4 * j;
  float* o = la + b * (int64_t)n + 4 * j;
#pragma unroll
  for (int q = 0; q < 4; ++q)
    if (4 * j + q < n) o[q] = ((bits[q] & 1) ? mu : -mu) + s * nr[q];
}

// Per-codeword mutual-information estimate, one wavefront per codeword:
// 1 - (1/n) sum_i log2(1 + exp(-(2c_i - 1) L_i)), lane sums then a
// fixed-shape tree.
constexpr int kMiThreads = 256;

__global__ __launch_bounds__(kMiThreads) void mi_rows_kernel(const float* __restrict__ L,
                                                             int64_t L_stride,
                                                             const uint8_t* __restrict__ c,
                                                             int64_t c_stride, int64_t B, int64_t n,
                                                             float* __restrict__ mi) {
  const int lane = threadIdx.x & 63;
  const int64_t b = (int64_t)blockIdx.x * (kMiThreads / 64) + (threadIdx.x >> 6);
  if (b >= B) return;
  const float* Lr = L + b * L_stride;
  const uint8_t* cr = c + b * c_stride;
  float acc = 0.f;
  for (int64_t i = lane; i < n; i += 64) {
    const float x = (cr[i] & 1) ? -Lr[i] : Lr[i];  // -(2c - 1) L
    acc += fmaxf(x, 0.f) + log1pf(expf(-fabsf(x)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) mi[b] = 1.0f - acc * (1.4426950408889634f / (float)n);
}

// Mean of the per-codeword estimates over the codewords of each bin (one
// workgroup per bin, fixed-order sums in double).
__global__ __launch_bounds__(256) void mi_bins_kernel(const float* __restrict__ mi,
                                                      const int32_t* __restrict__ bin, int64_t B,
                                                      double* __restrict__ out) {
  __shared__ double ssum[256];
  __shared__ int64_t scnt[256];
  const int k = blockIdx.x;
  double acc = 0.0;
  int64_t cnt = 0;
  for (int64_t b = threadIdx.x; b < B; b += 256) {
    if (bin == nullptr || bin[b] == k) {
      acc += (double)mi[b];
      ++cnt;
    }
  }
  ssum[threadIdx.x] = acc;
  scnt[threadIdx.x] = cnt;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) {
      ssum[threadIdx.x] += ssum[threadIdx.x + h];
      scnt[threadIdx.x] += scnt[threadIdx.x + h];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[k] = scnt[0] ? ssum[0] / (double)scnt[0] : __builtin_nan("");
}

// Extrinsic output of the decoder on the transmitted bits:
// L_post[tx_lo + i] - L_in[i] with L_in as the decoder used it (clamped to
// +-llr_max when llr_max > 0), zero where the bit is outside the decoded
// graph.
__global__ __launch_bounds__(256) void extrinsic_kernel(const float* __restrict__ app, int64_t n_dec,
                                                        int64_t tx_lo, const float* __restrict__ lin,
                                                        float llr_max, int64_t B, int64_t e_tx,
                                                        float* __restrict__ out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * e_tx) return;
  const int64_t b = t / e_tx;
  const int64_t v = tx_lo + (t - b * e_tx);
  float x = lin[t];
  if (llr_max > 0.f) x = fminf(fmaxf(x, -llr_max), llr_max);
  out[t] = v < n_dec ? app[b * n_dec + v] - x : 0.f;
}

inline unsigned blocks(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

}  // namespace

hipError_t launch_demap_prior(int m, bool exact, const float* y, const float* no, const float* la,
                              int64_t B, int64_t S, bool extrinsic, float* out, hipStream_t s) {
  const unsigned g = blocks(B * S, 256);
  switch (m) {
    case 1: demap_prior_kernel<1><<<g, 256, 0, s>>>(exact, y, no, la, B, S, extrinsic, out); break;
    case 2: demap_prior_kernel<2><<<g, 256, 0, s>>>(exact, y, no, la, B, S, extrinsic, out); break;
    case 4: demap_prior_kernel<4><<<g, 256, 0, s>>>(exact, y, no, la, B, S, extrinsic, out); break;
    case 6: demap_prior_kernel<6><<<g, 256, 0, s>>>(exact, y, no, la, B, S, extrinsic, out); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_apriori(const DevCode& c, const uint8_t* cw, const float* sigma, uint64_t seed,
                          int64_t cw0, int64_t B, float* la, hipStream_t s) {
  apriori_kernel<<<blocks(B * ((c.e_tx + 3) / 4), 256), 256, 0, s>>>(c, cw, sigma, seed, cw0, B, la);
  return hipGetLastError();
}

hipError_t launch_mutual_info(const float* L, int64_t L_stride, const uint8_t* c, int64_t c_stride,
                              int64_t B, int64_t n, const int32_t* bin, int nbins, float* mi_cw,
                              double* mi_bins, hipStream_t s) {
  mi_rows_kernel<<<blocks(B, kMiThreads / 64), kMiThreads, 0, s>>>(L, L_stride, c, c_stride, B, n,
                                                                   mi_cw);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !mi_bins) return e;
  mi_bins_kernel<<<nbins, 256, 0, s>>>(mi_cw, bin, B, mi_bins);
  return hipGetLastError();
}

hipError_t launch_extrinsic(const DevCode& c, const float* app, const float* lin, float llr_max,
                            int64_t B, float* out, hipStream_t s) {
  extrinsic_kernel<<<blocks(B * (int64_t)c.e_tx, 256), 256, 0, s>>>(app, c.n_dec, c.tx_lo, lin,
                                                                    llr_max, B, c.e_tx, out);
  return hipGetLastError();
}

}  // namespace lsim
