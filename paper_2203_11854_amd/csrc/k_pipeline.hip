// Link kernels around the decoder: binary source, QC encoder, Gray QAM
// mapper + AWGN, demappers, quantizer, error counting and syndrome.
#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "lsim_internal.h"
#include "philox.h"
#include "qam.h"

namespace lsim {

namespace {

// ----------------------------------------------------------------- source

// 32 information bits of codeword cw, word w (bit i of the word is
// information bit 32 w + i): Philox block w / 4, lane w % 4, stream 0.
__device__ __forceinline__ uint32_t source_word(uint64_t seed, uint64_t cw, int64_t w) {
  const U4 r = philox_at(seed, (uint32_t)(w >> 2), cw, kStreamBits);
  const uint32_t sel = (uint32_t)(w & 3);
  return sel == 0 ? r.x : sel == 1 ? r.y : sel == 2 ? r.z : r.w;
}

// Writes the n <= 32 low bits of word as bytes 0/1 to dst (4-byte stores
// when all 32 go to a 4-byte aligned address).
__device__ __forceinline__ void expand_word(uint32_t word, int n, uint8_t* dst) {
  if (n == 32 && (((uintptr_t)dst) & 3) == 0) {
    uint32_t* d4 = reinterpret_cast<uint32_t*>(dst);
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const uint32_t nib = word >> (4 * q);
      d4[q] = (nib & 1u) | ((nib >> 1) & 1u) << 8 | ((nib >> 2) & 1u) << 16 | ((nib >> 3) & 1u) << 24;
    }
  } else {
    for (int i = 0; i < n; ++i) dst[i] = (uint8_t)((word >> i) & 1u);
  }
}

__global__ void source_bits_kernel(uint64_t seed, int64_t cw0, int64_t B, int64_t k,
                                   int64_t words_per_cw, uint8_t* __restrict__ u) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * words_per_cw) return;
  const int64_t b = t / words_per_cw;
  const int64_t w = t - b * words_per_cw;  // 32-bit word index within the codeword
  const uint32_t word = source_word(seed, (uint64_t)(cw0 + b), w);
  const int64_t i0 = w * 32;
  expand_word(word, (int)min<int64_t>(32, k - i0), u + b * k + i0);
}

// ---------------------------------------------------------------- encoder

// One workgroup per codeword; the whole mother codeword sits in LDS, one
// byte per bit.  lambda_i (dual-diagonal rows) = XOR over the row's
// information blocks of rotated u_j; p_0 = XOR of all lambda_i;
// p_1 = lambda_0 ^ P^1 p_0; p_{i+1} = lambda_i ^ p_i (^ p_0 at the middle
// row); extension rows (BG shape) then set their own block from columns
// < kb + 4.  XOR rows are dealt to wavefronts as (row, 64-lift chunk) items
// so the row's entry list is read with scalar loads; bits move in and out
// with 16-byte accesses when the rows are aligned.
constexpr int kEncThreads = 256;

constexpr int kEncDMAX = 32;  // straight-line XOR bodies up to this many entries

__device__ __forceinline__ void enc_xor_rows(const DevCode& c, uint8_t* cb, int row0, int nrows,
                                             uint8_t* dst, int dst_stride) {
  const int Z = c.Z;
  const int cpr = (Z + 63) >> 6;
  const int lane = threadIdx.x & 63;
  for (int q = uni(threadIdx.x >> 6); q < nrows * cpr; q += kEncThreads / 64) {
    const int i = q / cpr;
    const int r = (q - i * cpr) * 64 + lane;
    const int e0 = ld_const(c.enc_ptr, row0 + i), e1 = ld_const(c.enc_ptr, row0 + i + 1);
    if (r < Z) {
      uint8_t acc = 0;
      if (e1 - e0 <= kEncDMAX) {
        // all of the row's table loads, then all of its LDS reads, back to back
        with_degree<kEncDMAX>(e1 - e0, [&](auto deg) {
          constexpr int D = decltype(deg)::value;
          int idx[D];
#pragma unroll
          for (int k = 0; k < D; ++k) {
            const int2 cs = ld_const(c.enc_cz, e0 + k);
            int x = r + cs.y;
            x -= x >= Z ? Z : 0;
            idx[k] = cs.x + x;
          }
          uint8_t v[D];
#pragma unroll
          for (int k = 0; k < D; ++k) v[k] = cb[idx[k]];
#pragma unroll
          for (int k = 0; k < D; ++k) acc ^= v[k];
        });
      } else {
        for (int e = e0; e < e1; ++e) {
          const int2 cs = ld_const(c.enc_cz, e);
          int x = r + cs.y;
          x -= x >= Z ? Z : 0;
          acc ^= cb[cs.x + x];
        }
      }
      dst[i * dst_stride + r] = acc;
    }
  }
}

// Bytes [0, n) from src to dst, 16 bytes at a time when both are aligned
// and n is a multiple of 16 (all threads of the workgroup take part).
__device__ __forceinline__ void block_copy(const uint8_t* src, uint8_t* dst, int n, uint32_t mask) {
  if (((n & 15) | ((uintptr_t)src & 15) | ((uintptr_t)dst & 15)) == 0) {
    for (int i = threadIdx.x; i < (n >> 4); i += kEncThreads) {
      uint4 v = reinterpret_cast<const uint4*>(src)[i];
      v.x &= mask;
      v.y &= mask;
      v.z &= mask;
      v.w &= mask;
      reinterpret_cast<uint4*>(dst)[i] = v;
    }
  } else {
    for (int i = threadIdx.x; i < n; i += kEncThreads) dst[i] = src[i] & (uint8_t)mask;
  }
}

// The parity part of the codeword in LDS, from its information bits cb[0,k).
__device__ __forceinline__ void encode_in_lds(const DevCode& c, uint8_t* cb, uint8_t* lam) {
  const int Z = c.Z, kb = c.kb, mb = c.mb;
  const int m = c.family == LSIM_FAMILY_11N ? mb : 4;
  const int mid = m / 2;
  enc_xor_rows(c, cb, 0, m, lam, Z);
  __syncthreads();
  for (int r = threadIdx.x; r < Z; r += kEncThreads) {
    uint8_t p0 = 0;
    for (int i = 0; i < m; ++i) p0 ^= lam[i * Z + r];
    cb[kb * Z + r] = p0;
  }
  __syncthreads();
  for (int r = threadIdx.x; r < Z; r += kEncThreads) {
    const int r1 = r + 1 == Z ? 0 : r + 1;
    const uint8_t p0r = cb[kb * Z + r];
    uint8_t p = lam[r] ^ cb[kb * Z + r1];
    cb[(kb + 1) * Z + r] = p;
    for (int i = 1; i < m - 1; ++i) {
      p = lam[i * Z + r] ^ p ^ (i == mid ? p0r : 0);
      cb[(kb + i + 1) * Z + r] = p;
    }
  }
  __syncthreads();
  if (c.family == LSIM_FAMILY_BG && mb > 4) {
    enc_xor_rows(c, cb, 4, mb - 4, cb + (kb + 4) * Z, Z);
    __syncthreads();
  }
}

__host__ __device__ inline size_t enc_lds_bytes(const DevCode& c) {
  const int m = c.family == LSIM_FAMILY_11N ? c.mb : 4;
  return (((size_t)c.n_mother + 15) & ~(size_t)15) + (size_t)m * c.Z;
}

__global__ __launch_bounds__(kEncThreads) void encode_kernel(DevCode c, const uint8_t* __restrict__ u,
                                                             uint8_t* __restrict__ cw) {
  extern __shared__ __align__(16) uint8_t sm[];
  uint8_t* cb = sm;                                        // n_mother bits
  uint8_t* lam = sm + ((c.n_mother + 15) & ~15);           // m * Z
  const int64_t b = blockIdx.x;
  block_copy(u + b * (int64_t)c.k, cb, c.k, 0x01010101u);
  __syncthreads();
  encode_in_lds(c, cb, lam);
  block_copy(cb, cw + b * (int64_t)c.n_mother, c.n_mother, 0xffffffffu);
}

// ------------------------------------------------------- mapper + channel

// Symbol s of a codeword whose transmitted bits start at `bits`: Gray QAM
// (or BPSK) point plus sqrt(N0/2) times the Box-Muller pair of the Philox
// words (xa, xb).
__device__ __forceinline__ float2 map_symbol(int m, const uint8_t* bits, int s, uint32_t xa,
                                             uint32_t xb, float sig) {
  const Polar bm = box_muller(xa, xb);
  const float rho = bm.rho, sn = bm.sn, cs = bm.cs;
  float xr, xi;
  if (m == 1) {
    xr = 1.0f - 2.0f * (float)bits[s];
    xi = 0.0f;
  } else {
    const int hb = m >> 1;
    uint32_t ai[3], aq[3];
    for (int q = 0; q < hb; ++q) {
      ai[q] = bits[s * m + 2 * q];
      aq[q] = bits[s * m + 2 * q + 1];
    }
    const float inv = qam_inv_scale(hb);
    xr = pam_level(ai, hb) * inv;
    xi = pam_level(aq, hb) * inv;
  }
  float2 out;
  out.x = xr + sig * rho * cs;
  out.y = xi + sig * rho * sn;
  return out;
}

__global__ void map_awgn_kernel(DevCode c, int m, const uint8_t* __restrict__ cw,
                                const float* __restrict__ no, uint64_t seed, int64_t cw0,
                                int64_t B, int S, float* __restrict__ y) {
  const int npair = (S + 1) >> 1;
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * npair) return;
  const int64_t b = t / npair;
  const int j = (int)(t - b * npair);
  const U4 r = philox_at(seed, (uint32_t)j, (uint64_t)(cw0 + b), kStreamNoise);
  const float sig = sqrtf(no[b] * 0.5f);
  const uint8_t* bits = cw + b * (int64_t)c.n_mother + c.tx_lo;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int s = 2 * j + h;
    if (s >= S) break;
    reinterpret_cast<float2*>(y)[b * (int64_t)S + s] =
        map_symbol(m, bits, s, h ? r.z : r.x, h ? r.w : r.y, sig);
  }
}

// --------------------------------------------------------------- demapper

// Unit-energy Gray PAM levels per axis, indexed by the axis label read
// MSB-first (bits a0 a1 ...), for h = 1, 2, 3 bits per axis.
__constant__ float kPam1[2] = {0.70710678118654752f, -0.70710678118654752f};
__constant__ float kPam2[4] = {0.31622776601683794f, 0.94868329805051381f, -0.31622776601683794f,
                               -0.94868329805051381f};
__constant__ float kPam3[8] = {0.46291004988627573f, 0.15430334996209191f, 0.77151674981045953f,
                               1.08012344973464337f, -0.46291004988627573f, -0.15430334996209191f,
                               -0.77151674981045953f, -1.08012344973464337f};

// Per-axis LLRs of h Gray bits for coordinate v: max-log
// (min_{b=0} d^2 - min_{b=1} d^2) / N0, or exact: log-sum-exp of -d^2/N0
// over the levels with bit 1 minus that over bit 0.
template <int h>
__device__ __forceinline__ void axis_llr(float v, float inv_no, bool exact, float* out) {
  constexpr int nl = 1 << h;
  const float* lv = h == 1 ? kPam1 : h == 2 ? kPam2 : kPam3;
  float d2[nl];
#pragma unroll
  for (int l = 0; l < nl; ++l) {
    const float dv = v - lv[l];
    d2[l] = dv * dv * inv_no;
  }
#pragma unroll
  for (int q = 0; q < h; ++q) {
    const int sh = h - 1 - q;
    float m0 = INFINITY, m1 = INFINITY;
#pragma unroll
    for (int l = 0; l < nl; ++l) {
      if ((l >> sh) & 1) m1 = fminf(m1, d2[l]);
      else m0 = fminf(m0, d2[l]);
    }
    if (!exact) {
      out[q] = m0 - m1;
    } else {
      float s0 = 0.f, s1 = 0.f;
#pragma unroll
      for (int l = 0; l < nl; ++l) {
        if ((l >> sh) & 1) s1 += expf(m1 - d2[l]);
        else s0 += expf(m0 - d2[l]);
      }
      out[q] = (m0 - m1) + logf(s1) - logf(s0);
    }
  }
}

template <int M>
__device__ __forceinline__ void symbol_llr(float2 yy, float n0, bool exact, float* L) {
  if constexpr (M == 1) {
    L[0] = -4.0f * yy.x / n0;
  } else {
    constexpr int h = M / 2;
    const float inv_no = 1.0f / n0;
    float li[h], lq[h];
    axis_llr<h>(yy.x, inv_no, exact, li);
    axis_llr<h>(yy.y, inv_no, exact, lq);
#pragma unroll
    for (int i = 0; i < h; ++i) {
      L[2 * i] = li[i];
      L[2 * i + 1] = lq[i];
    }
  }
}

// LLRs of symbol t (M of them) to llr (f32) or, when llr is null, quantized
// to q (clamp(rint(L * scale), +-sat)).
template <int M>
__device__ __forceinline__ void store_llr(const float* L, int64_t t, float* __restrict__ llr,
                                          int8_t* __restrict__ q, float scale, int sat) {
  if (llr) {
    float* o = llr + t * M;
    if constexpr (M == 4) {
      *reinterpret_cast<float4*>(o) = make_float4(L[0], L[1], L[2], L[3]);
    } else if constexpr (M == 2) {
      *reinterpret_cast<float2*>(o) = make_float2(L[0], L[1]);
    } else if constexpr (M == 6) {
      reinterpret_cast<float2*>(o)[0] = make_float2(L[0], L[1]);
      reinterpret_cast<float2*>(o)[1] = make_float2(L[2], L[3]);
      reinterpret_cast<float2*>(o)[2] = make_float2(L[4], L[5]);
    } else {
      o[0] = L[0];
    }
  } else {
    int8_t qq[M];
#pragma unroll
    for (int i = 0; i < M; ++i)
      qq[i] = (int8_t)fminf(fmaxf(rintf(L[i] * scale), (float)-sat), (float)sat);
#pragma unroll
    for (int i = 0; i < M; ++i) q[t * M + i] = qq[i];
  }
}

template <int M>
__global__ void demap_kernel(int method, const float* __restrict__ y, const float* __restrict__ no,
                             int64_t B, int64_t S, float* __restrict__ llr,
                             int8_t* __restrict__ q, float scale, int sat) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * S) return;
  const int64_t b = t / S;
  float L[M];
  symbol_llr<M>(reinterpret_cast<const float2*>(y)[t], no[b], method == LSIM_DEMAP_EXACT, L);
  store_llr<M>(L, t, llr, q, scale, sat);
}

// The link's transmit side for one codeword per workgroup, all in LDS:
// Philox information bits (also written to u), encoder, then per symbol
// pair the Gray map + AWGN and the demapper, written as f32 LLRs or int8.
// Same device functions as the separate kernels, so the same results; the
// codeword (cw) and the channel output (y) are written only when asked.
template <int M>
__global__ __launch_bounds__(kEncThreads) void link_tx_kernel(
    DevCode c, uint64_t seed, int64_t cw0, const float* __restrict__ no, int method,
    uint8_t* __restrict__ u, uint8_t* __restrict__ cw, float* __restrict__ y,
    float* __restrict__ llr, int8_t* __restrict__ q, float scale, int sat) {
  extern __shared__ __align__(16) uint8_t sm[];
  uint8_t* cb = sm;
  uint8_t* lam = sm + ((c.n_mother + 15) & ~15);
  const int64_t b = blockIdx.x;
  const uint64_t cwi = (uint64_t)(cw0 + b);
  const int64_t wpc = (c.k + 31) / 32;
  for (int64_t w = threadIdx.x; w < wpc; w += kEncThreads)
    expand_word(source_word(seed, cwi, w), (int)min<int64_t>(32, c.k - 32 * w), cb + 32 * w);
  __syncthreads();
  block_copy(cb, u + b * (int64_t)c.k, c.k, 0xffffffffu);
  encode_in_lds(c, cb, lam);
  if (cw) block_copy(cb, cw + b * (int64_t)c.n_mother, c.n_mother, 0xffffffffu);
  const int S = c.e_tx / M;
  const int npair = (S + 1) >> 1;
  const float n0 = no[b];
  const float sig = sqrtf(n0 * 0.5f);
  const bool exact = method == LSIM_DEMAP_EXACT;
  const uint8_t* bits = cb + c.tx_lo;
  for (int j = threadIdx.x; j < npair; j += kEncThreads) {
    const U4 r = philox_at(seed, (uint32_t)j, cwi, kStreamNoise);
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int s = 2 * j + h;
      if (s >= S) break;
      const float2 yy = map_symbol(M, bits, s, h ? r.z : r.x, h ? r.w : r.y, sig);
      const int64_t t = b * (int64_t)S + s;
      if (y) reinterpret_cast<float2*>(y)[t] = yy;
      float L[M];
      symbol_llr<M>(yy, n0, exact, L);
      store_llr<M>(L, t, llr, q, scale, sat);
    }
  }
}

__global__ void quantize_kernel(const float* __restrict__ L, int64_t n, float scale, int sat,
                                int8_t* __restrict__ q) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float v = fminf(fmaxf(rintf(L[t] * scale), (float)-sat), (float)sat);
  q[t] = (int8_t)v;
}

// ------------------------------------------------------------ error count

// One wavefront per codeword, four codewords per workgroup (a launch of
// 1024 codewords fills every CU).  Bits are bytes holding 0/1, so the
// population count of the XOR of two words counts 4 bit errors at a time
// (16-byte loads when both rows are 16-byte aligned, 4-byte when 4-byte
// aligned, else bytes).  Up to
// kLdsBins bins are summed in LDS and added to the device counters once per
// workgroup; with more bins each codeword adds its own counts.
constexpr int kCountThreads = 256;
constexpr int kCwPerWave = 1;
constexpr int kCwPerBlock = kCountThreads / 64 * kCwPerWave;
constexpr int kLdsBins = 64;

__device__ __forceinline__ int popc_err(uint32_t a, uint32_t b) {
  return __popc((a ^ b) & 0x01010101u);
}

__global__ __launch_bounds__(kCountThreads) void count_errors_kernel(
    const uint8_t* __restrict__ ref, int64_t ref_stride, const uint8_t* __restrict__ hat,
    int64_t k, int64_t B, const int32_t* __restrict__ bin, int nbins,
    int64_t* __restrict__ counts) {
  __shared__ unsigned long long acc[3 * kLdsBins];
  const bool in_lds = nbins <= kLdsBins;
  for (int t = threadIdx.x; t < 3 * kLdsBins; t += kCountThreads) acc[t] = 0;
  __syncthreads();
  const int lane = threadIdx.x & 63;
  const int64_t first = (int64_t)blockIdx.x * kCwPerBlock + uni(threadIdx.x >> 6) * kCwPerWave;
  for (int j = 0; j < kCwPerWave; ++j) {
    const int64_t b = first + j;
    if (b >= B) break;
    const uint8_t* rr = ref + b * ref_stride;
    const uint8_t* hh = hat + b * k;
    const uintptr_t al = (uintptr_t)rr | (uintptr_t)hh;
    int err = 0;
    int64_t done = 0;
    if ((al & 15) == 0) {
      const int64_t nv = k >> 4;
      const uint4* r4 = reinterpret_cast<const uint4*>(rr);
      const uint4* h4 = reinterpret_cast<const uint4*>(hh);
      for (int64_t i = lane; i < nv; i += 64) {
        const uint4 x = r4[i], y = h4[i];
        err += popc_err(x.x, y.x) + popc_err(x.y, y.y) + popc_err(x.z, y.z) + popc_err(x.w, y.w);
      }
      done = nv << 4;
    } else if ((al & 3) == 0) {
      const int64_t nw = k >> 2;
      const uint32_t* r1 = reinterpret_cast<const uint32_t*>(rr);
      const uint32_t* h1 = reinterpret_cast<const uint32_t*>(hh);
      for (int64_t i = lane; i < nw; i += 64) err += popc_err(r1[i], h1[i]);
      done = nw << 2;
    }
    for (int64_t i = done + lane; i < k; i += 64) err += (rr[i] & 1) != (hh[i] & 1);
    for (int off = 32; off > 0; off >>= 1) err += __shfl_down(err, off, 64);
    if (lane == 0) {
      const int bb = bin ? bin[b] : 0;
      if (bb >= 0 && bb < nbins) {  // codewords outside every bin are not counted
        if (in_lds) {
          atomicAdd(&acc[3 * bb + 0], (unsigned long long)err);
          atomicAdd(&acc[3 * bb + 1], (unsigned long long)(err > 0));
          atomicAdd(&acc[3 * bb + 2], 1ull);
        } else {
          unsigned long long* cnt = reinterpret_cast<unsigned long long*>(counts) + 3 * (int64_t)bb;
          atomicAdd(cnt + 0, (unsigned long long)err);
          atomicAdd(cnt + 1, (unsigned long long)(err > 0));
          atomicAdd(cnt + 2, 1ull);
        }
      }
    }
  }
  if (!in_lds) return;
  __syncthreads();
  unsigned long long* cnt = reinterpret_cast<unsigned long long*>(counts);
  for (int t = threadIdx.x; t < 3 * nbins; t += kCountThreads)
    if (acc[t]) atomicAdd(cnt + t, acc[t]);
}

__global__ __launch_bounds__(256) void syndrome_kernel(DevCode c, const uint8_t* __restrict__ cw,
                                                       int64_t stride, int32_t* __restrict__ unsat) {
  __shared__ int part[4];
  const int64_t b = blockIdx.x;
  const uint8_t* x = cw + b * stride;
  const int Z = c.Z;
  int bad = 0;
  for (int chk = threadIdx.x; chk < c.m_dec; chk += blockDim.x) {
    const int i = chk / Z, r = chk - i * Z;
    uint8_t acc = 0;
    for (int e = c.row_ptr[i]; e < c.row_ptr[i + 1]; ++e) {
      int v = r + c.ent_shift[e];
      v -= v >= Z ? Z : 0;
      acc ^= x[c.ent_col[e] * Z + v] & 1;
    }
    bad += acc;
  }
  for (int off = 32; off > 0; off >>= 1) bad += __shfl_down(bad, off, 64);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = bad;
  __syncthreads();
  if (threadIdx.x == 0) unsat[b] = part[0] + part[1] + part[2] + part[3];
}

inline unsigned grid_for(int64_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

}  // namespace

hipError_t launch_source_bits(uint64_t seed, int64_t cw0, int64_t B, int64_t k, uint8_t* u,
                              hipStream_t s) {
  const int64_t wpc = (k + 31) / 32;
  source_bits_kernel<<<grid_for(B * wpc, 256), 256, 0, s>>>(seed, cw0, B, k, wpc, u);
  return hipGetLastError();
}

hipError_t launch_encode(const DevCode& c, const uint8_t* u, int64_t B, uint8_t* cw,
                         hipStream_t s) {
  hipError_t e = ensure_dyn_lds((const void*)encode_kernel, enc_lds_bytes(c));
  if (e != hipSuccess) return e;
  encode_kernel<<<(unsigned)B, kEncThreads, enc_lds_bytes(c), s>>>(c, u, cw);
  return hipGetLastError();
}

hipError_t launch_link_tx(const DevCode& c, int m, int method, uint64_t seed, int64_t cw0,
                          int64_t B, const float* no, uint8_t* u, uint8_t* cw, float* y,
                          float* llr, int8_t* q, float scale, int sat, hipStream_t s) {
  const size_t lds = enc_lds_bytes(c);
  const unsigned g = (unsigned)B;
  const void* k = m == 1 ? (const void*)link_tx_kernel<1> : m == 2 ? (const void*)link_tx_kernel<2>
                : m == 4 ? (const void*)link_tx_kernel<4> : (const void*)link_tx_kernel<6>;
  hipError_t e = ensure_dyn_lds(k, lds);
  if (e != hipSuccess) return e;
  switch (m) {
    case 1: link_tx_kernel<1><<<g, kEncThreads, lds, s>>>(c, seed, cw0, no, method, u, cw, y, llr, q, scale, sat); break;
    case 2: link_tx_kernel<2><<<g, kEncThreads, lds, s>>>(c, seed, cw0, no, method, u, cw, y, llr, q, scale, sat); break;
    case 4: link_tx_kernel<4><<<g, kEncThreads, lds, s>>>(c, seed, cw0, no, method, u, cw, y, llr, q, scale, sat); break;
    default: link_tx_kernel<6><<<g, kEncThreads, lds, s>>>(c, seed, cw0, no, method, u, cw, y, llr, q, scale, sat); break;
  }
  return hipGetLastError();
}

hipError_t launch_map_awgn(const DevCode& c, int m, const uint8_t* cw, const float* no,
                           uint64_t seed, int64_t cw0, int64_t B, float* y, hipStream_t s) {
  const int S = c.e_tx / m;
  const int64_t n = B * ((S + 1) / 2);
  map_awgn_kernel<<<grid_for(n, 256), 256, 0, s>>>(c, m, cw, no, seed, cw0, B, S, y);
  return hipGetLastError();
}

hipError_t launch_demap(int m, int method, const float* y, const float* no, int64_t B, int64_t S,
                        float* llr, int8_t* q, float scale, int sat, hipStream_t s) {
  const unsigned g = grid_for(B * S, 256);
  switch (m) {
    case 1: demap_kernel<1><<<g, 256, 0, s>>>(method, y, no, B, S, llr, q, scale, sat); break;
    case 2: demap_kernel<2><<<g, 256, 0, s>>>(method, y, no, B, S, llr, q, scale, sat); break;
    case 4: demap_kernel<4><<<g, 256, 0, s>>>(method, y, no, B, S, llr, q, scale, sat); break;
    default: demap_kernel<6><<<g, 256, 0, s>>>(method, y, no, B, S, llr, q, scale, sat); break;
  }
  return hipGetLastError();
}

hipError_t launch_quantize(const float* llr, int64_t n, float scale, int sat, int8_t* q,
                           hipStream_t s) {
  quantize_kernel<<<grid_for(n, 256), 256, 0, s>>>(llr, n, scale, sat, q);
  return hipGetLastError();
}

hipError_t launch_count_errors(const uint8_t* ref, int64_t ref_stride, const uint8_t* hat,
                               int64_t B, int64_t k, const int32_t* bin, int nbins,
                               int64_t* counts, hipStream_t s) {
  count_errors_kernel<<<grid_for(B, kCwPerBlock), kCountThreads, 0, s>>>(ref, ref_stride, hat, k,
                                                                         B, bin, nbins, counts);
  return hipGetLastError();
}

namespace {

// bits[b][v] = [L[b][v] > 0] for the first k columns of each row.
__global__ __launch_bounds__(256) void hard_bits_kernel(const float* __restrict__ L, int64_t stride,
                                                        int64_t B, int64_t k,
                                                        uint8_t* __restrict__ bits) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * k) return;
  const int64_t b = t / k, v = t - b * k;
  bits[t] = L[b * stride + v] > 0.f ? 1 : 0;
}

}  // namespace

hipError_t launch_hard_bits(const float* L, int64_t stride, int64_t B, int64_t k, uint8_t* bits,
                            hipStream_t s) {
  hard_bits_kernel<<<grid_for(B * k, 256), 256, 0, s>>>(L, stride, B, k, bits);
  return hipGetLastError();
}

hipError_t launch_syndrome(const DevCode& c, const uint8_t* cw, int64_t stride, int64_t B,
                           int32_t* unsat, hipStream_t s) {
  syndrome_kernel<<<(unsigned)B, 256, 0, s>>>(c, cw, stride, unsat);
  return hipGetLastError();
}

}  // namespace lsim
