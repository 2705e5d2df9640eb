// Neural demapper (3 -> 64 -> 64 -> 4 MLP per symbol, ReLU), its parameter
// gradient, the binary cross-entropy on logits and an Adam step.
//
// Both passes run the layers as 16x16x4 FP32 matrix-core products
// (v_mfma_f32_16x16x4f32) over tiles of 16 symbols.  Lane l = 16 g + c
// supplies A[c][g] and B[g][c] and receives D[4 g + v][c], v = 0..3.
// Activations are kept in that output layout with hidden units on the rows
// (unit 16 m + 4 g + v of row tile m) and symbols on the columns, and a
// product over hidden units takes its K-steps as (tile, v): step (u, v)
// covers units 16 u + 4 g + v, so the previous layer's output register v is
// the next product's B operand as is and only the weight operand is
// gathered in that order.  The input layer is one K = 4 product of
// [W1 | b1] with [Re y, Im y, ln N0, 1].
//
// Backward (per wavefront, 32 symbols per step): H1, A2 = W2 H1 + b2,
// D2 = (W3^T D3) * [A2 > 0], D1 = (W2^T D2) * [H1 > 0] as above; the
// weight gradient dW2 = D2 H1^T contracts over symbols, so D2 and H1 go
// through an LDS transpose (per-wave tiles) and come back with symbols on
// the K axis.  db2, db1, dW1, dW3, db3 are summed per lane over its symbols
// and across the 16 lanes of a row group at the end.  Every wavefront writes
// one partial-gradient row; rows are then summed in a fixed order, so the
// result is deterministic.  On request the gradient with respect to the
// received symbol, dy = W1[:, 0:2]^T D1, comes out of one more product per
// tile whose weight operand is W1's first two columns padded to 16 rows.
#include <hip/hip_runtime.h>

#include "lsim_internal.h"

namespace lsim {

namespace {

constexpr int H = 64;
constexpr int OW1 = 0, OB1 = 192, OW2 = 256, OB2 = 4352, OW3 = 4416, OB3 = 4672, NP = 4676;

typedef float f4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 relu4(f4 x) {
  f4 r;
#pragma unroll
  for (int v = 0; v < 4; ++v) r[v] = fmaxf(x[v], 0.f);
  return r;
}

constexpr int kNdmFwdThreads = 256;

// Forward: each wavefront takes 16-symbol tiles; the layer-2 weights are
// held in registers in the gathered order (64 values per lane).
__global__ __launch_bounds__(kNdmFwdThreads) void ndm_forward_kernel(
    const float* __restrict__ P, const float* __restrict__ y, const float* __restrict__ no,
    int64_t B, int64_t S, float* __restrict__ llr) {
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  const int64_t n = B * S, ntile = (n + 15) / 16;
  const int64_t w0 = (int64_t)blockIdx.x * (kNdmFwdThreads / 64) + (threadIdx.x >> 6);
  const int64_t nw = (int64_t)gridDim.x * (kNdmFwdThreads / 64);
  float w1a[4], w2a[4][4][4], w3a[4][4];
  f4 b2i[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) w1a[u] = g < 3 ? P[OW1 + 3 * (16 * u + c) + g] : P[OB1 + 16 * u + c];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) w2a[m][u][v] = P[OW2 + (16 * m + c) * H + 16 * u + 4 * g + v];
  // output layer as a 16-row tile whose rows 0..3 are the four LLRs
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) w3a[m][v] = c < 4 ? P[OW3 + c * H + 16 * m + 4 * g + v] : 0.f;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) b2i[m][v] = P[OB2 + 16 * m + 4 * g + v];
  f4 b3i = {0.f, 0.f, 0.f, 0.f};
  if (g == 0) b3i = f4{P[OB3], P[OB3 + 1], P[OB3 + 2], P[OB3 + 3]};
  const f4 zero = {0.f, 0.f, 0.f, 0.f};

  for (int64_t tile = w0; tile < ntile; tile += nw) {
    const int64_t sym = tile * 16 + c;
    const bool on = sym < n;
    float xb = 1.f;
    if (on) xb = g == 0 ? y[2 * sym] : g == 1 ? y[2 * sym + 1] : g == 2 ? logf(no[sym / S]) : 1.f;
    f4 h1[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) h1[u] = relu4(mfma(w1a[u], xb, zero));
    f4 a2[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) a2[m] = b2i[m];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v)
#pragma unroll
        for (int m = 0; m < 4; ++m) a2[m] = mfma(w2a[m][u][v], h1[u][v], a2[m]);
    f4 o = b3i;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const f4 h2 = relu4(a2[m]);
#pragma unroll
      for (int v = 0; v < 4; ++v) o = mfma(w3a[m][v], h2[v], o);
    }
    // rows 0..3 (lanes 0..15) hold the four LLRs of symbol 16 tile + c
    if (g == 0 && on) reinterpret_cast<float4*>(llr)[sym] = make_float4(o[0], o[1], o[2], o[3]);
  }
}

constexpr int kBwdWaves = 4;             // wavefronts per workgroup
constexpr int kBwdThreads = 64 * kBwdWaves;
constexpr int kTS = 32;                  // symbols per wavefront step
constexpr int kPW = H + 4;               // LDS pitch of W2 and W2^T
constexpr int kPS = kTS + 4;             // LDS pitch of the per-wave transposes

constexpr int kW1Rows = 16;              // W1 columns 0, 1 as rows, zero-padded

__host__ __device__ constexpr size_t ndm_bwd_lds() {
  return (size_t)(2 * H * kPW + kBwdWaves * 2 * H * kPS + kW1Rows * kPW) * 4;
}

__global__ __launch_bounds__(kBwdThreads) void ndm_backward_kernel(
    const float* __restrict__ P, const float* __restrict__ y, const float* __restrict__ no,
    const float* __restrict__ gllr, int64_t B, int64_t S, float* __restrict__ part,
    float* __restrict__ gy) {
  extern __shared__ __align__(16) float sm[];
  float* w2s = sm;               // W2[out][in], pitch kPW
  float* w2t = sm + H * kPW;     // W2^T[in][out]
  const int wave = threadIdx.x >> 6;
  const int l = threadIdx.x & 63, g = l >> 4, c = l & 15;
  float* h1u = sm + 2 * H * kPW + wave * 2 * H * kPS;  // H1[in][symbol]
  float* d2u = h1u + H * kPS;                          // D2[out][symbol]
  float* w1p = sm + 2 * H * kPW + kBwdWaves * 2 * H * kPS;  // [k][unit] = W1[unit][k], k < 2
  for (int t = threadIdx.x; t < H * H; t += kBwdThreads) {
    const int o = t >> 6, i = t & 63;
    const float w = P[OW2 + t];
    w2s[o * kPW + i] = w;
    w2t[i * kPW + o] = w;
  }
  for (int t = threadIdx.x; t < kW1Rows * H; t += kBwdThreads) {
    const int k = t >> 6, unit = t & 63;
    w1p[k * kPW + unit] = k < 2 ? P[OW1 + 3 * unit + k] : 0.f;
  }
  __syncthreads();

  float w1a[4], w3a[4];
  f4 b2i[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) w1a[u] = g < 3 ? P[OW1 + 3 * (16 * u + c) + g] : P[OB1 + 16 * u + c];
#pragma unroll
  for (int m = 0; m < 4; ++m) w3a[m] = P[OW3 + g * H + 16 * m + c];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) b2i[m][v] = P[OB2 + 16 * m + 4 * g + v];
  const f4 zero = {0.f, 0.f, 0.f, 0.f};

  f4 gw2[4][4];                   // tile (m, u): dW2[16m + 4g + v][16u + c]
  f4 pb2[4], pb1[4], pw1[4][3], pw3[4][4];
  float pb3[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int m = 0; m < 4; ++m) {
    pb2[m] = zero;
    pb1[m] = zero;
#pragma unroll
    for (int u = 0; u < 4; ++u) gw2[m][u] = zero;
#pragma unroll
    for (int k = 0; k < 3; ++k) pw1[m][k] = zero;
#pragma unroll
    for (int o = 0; o < 4; ++o) pw3[o][m] = zero;
  }

  const int64_t n = B * S, nstep = (n + kTS - 1) / kTS;
  const int64_t gwv = (int64_t)blockIdx.x * kBwdWaves + wave;
  const int64_t nwv = (int64_t)gridDim.x * kBwdWaves;
  for (int64_t st = gwv; st < nstep; st += nwv) {
    float xk[2][3], d3[2][4], xb[2], d3b[2];
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      const int64_t sym = st * kTS + 16 * t + c;
      const bool on = sym < n;
      xk[t][0] = on ? y[2 * sym] : 0.f;
      xk[t][1] = on ? y[2 * sym + 1] : 0.f;
      xk[t][2] = on ? logf(no[sym / S]) : 0.f;
      // a padded symbol has zero output gradient, so it adds nothing
#pragma unroll
      for (int o = 0; o < 4; ++o) d3[t][o] = on ? gllr[4 * sym + o] : 0.f;
      xb[t] = g == 0 ? xk[t][0] : g == 1 ? xk[t][1] : g == 2 ? xk[t][2] : 1.f;
      d3b[t] = g == 0 ? d3[t][0] : g == 1 ? d3[t][1] : g == 2 ? d3[t][2] : d3[t][3];
    }
    f4 h1[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < 2; ++t) h1[u][t] = relu4(mfma(w1a[u], xb[t], zero));
    f4 a2[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m) a2[m][0] = a2[m][1] = b2i[m];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int m = 0; m < 4; ++m) {
        const f4 w = *reinterpret_cast<const f4*>(w2s + (16 * m + c) * kPW + 16 * u + 4 * g);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int t = 0; t < 2; ++t) a2[m][t] = mfma(w[v], h1[u][t][v], a2[m][t]);
      }
    f4 d2[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        d2[m][t] = mfma(w3a[m], d3b[t], zero);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float a = a2[m][t][v];
          d2[m][t][v] = a > 0.f ? d2[m][t][v] : 0.f;
          pb2[m][v] += d2[m][t][v];
          const float h2 = fmaxf(a, 0.f);
#pragma unroll
          for (int o = 0; o < 4; ++o) pw3[o][m][v] += d3[t][o] * h2;
        }
      }
    if (g == 0) {
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int o = 0; o < 4; ++o) pb3[o] += d3[t][o];
    }
    f4 d1[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) d1[u][0] = d1[u][1] = zero;
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const f4 w = *reinterpret_cast<const f4*>(w2t + (16 * u + c) * kPW + 16 * m + 4 * g);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int t = 0; t < 2; ++t) d1[u][t] = mfma(w[v], d2[m][t][v], d1[u][t]);
      }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const float d = h1[u][t][v] > 0.f ? d1[u][t][v] : 0.f;
          d1[u][t][v] = d;
          pb1[u][v] += d;
#pragma unroll
          for (int k = 0; k < 3; ++k) pw1[u][k][v] += d * xk[t][k];
        }
    if (gy) {
      // rows 0, 1 of W1[:, 0:2]^T D1: lanes 0..15 hold (dRe y, dIm y)
      f4 dx[2] = {zero, zero};
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const f4 w = *reinterpret_cast<const f4*>(w1p + c * kPW + 16 * u + 4 * g);
#pragma unroll
        for (int v = 0; v < 4; ++v)
#pragma unroll
          for (int t = 0; t < 2; ++t) dx[t] = mfma(w[v], d1[u][t][v], dx[t]);
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int64_t sym = st * kTS + 16 * t + c;
        if (g == 0 && sym < n) reinterpret_cast<float2*>(gy)[sym] = make_float2(dx[t][0], dx[t][1]);
      }
    }
    // transpose H1 and D2 through this wavefront's LDS tiles
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          h1u[(16 * u + 4 * g + v) * kPS + 16 * t + c] = h1[u][t][v];
          d2u[(16 * u + 4 * g + v) * kPS + 16 * t + c] = d2[u][t][v];
        }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
    // dW2 += D2 H1^T over the step's 32 symbols: K-step k covers symbols
    // 8 g + k of lane group g
    f4 hb[4][2];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      hb[u][0] = *reinterpret_cast<const f4*>(h1u + (16 * u + c) * kPS + 8 * g);
      hb[u][1] = *reinterpret_cast<const f4*>(h1u + (16 * u + c) * kPS + 8 * g + 4);
    }
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const f4 da0 = *reinterpret_cast<const f4*>(d2u + (16 * m + c) * kPS + 8 * g);
      const f4 da1 = *reinterpret_cast<const f4*>(d2u + (16 * m + c) * kPS + 8 * g + 4);
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u) gw2[m][u] = mfma(da0[k], hb[u][0][k], gw2[m][u]);
#pragma unroll
      for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int u = 0; u < 4; ++u) gw2[m][u] = mfma(da1[k], hb[u][1][k], gw2[m][u]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
  }

  // per-lane sums -> sums over the 16 lanes of each row group (fixed order)
  auto red16 = [](float x) {
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) x += __shfl_xor(x, off, 16);
    return x;
  };
  float* out = part + gwv * NP;
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) out[OW2 + (16 * m + 4 * g + v) * H + 16 * u + c] = gw2[m][u][v];
#pragma unroll
  for (int m = 0; m < 4; ++m)
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const int unit = 16 * m + 4 * g + v;
      const float sb2 = red16(pb2[m][v]), sb1 = red16(pb1[m][v]);
      const float s0 = red16(pw1[m][0][v]), s1 = red16(pw1[m][1][v]), s2 = red16(pw1[m][2][v]);
      float s3[4];
#pragma unroll
      for (int o = 0; o < 4; ++o) s3[o] = red16(pw3[o][m][v]);
      if (c == 0) {
        out[OB2 + unit] = sb2;
        out[OB1 + unit] = sb1;
        out[OW1 + 3 * unit + 0] = s0;
        out[OW1 + 3 * unit + 1] = s1;
        out[OW1 + 3 * unit + 2] = s2;
#pragma unroll
        for (int o = 0; o < 4; ++o) out[OW3 + o * H + unit] = s3[o];
      }
    }
#pragma unroll
  for (int o = 0; o < 4; ++o) {
    const float sb3 = red16(pb3[o]);
    if (l == 0) out[OB3 + o] = sb3;
  }
}

// out[i] = sum over rows of part[r][i] in a fixed order: pass 1 sums
// kSlices row slices, pass 2 adds the slices in order.
constexpr int kSlices = 32;

__global__ void sum_slices_kernel(const float* __restrict__ part, int rows, int n,
                                  float* __restrict__ slices) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int per = (rows + kSlices - 1) / kSlices;
  const int r0 = blockIdx.y * per;
  const int r1 = min(rows, r0 + per);
  float acc = 0.f;
  for (int r = r0; r < r1; ++r) acc += part[(int64_t)r * n + i];
  slices[(int64_t)blockIdx.y * n + i] = acc;
}

__global__ void sum_final_kernel(const float* __restrict__ slices, int n, float* __restrict__ out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float acc = 0.f;
  for (int k = 0; k < kSlices; ++k) acc += slices[(int64_t)k * n + i];
  out[i] = acc;
}

constexpr int kBceBlocks = 1024;

__global__ __launch_bounds__(256) void bce_kernel(const float* __restrict__ L,
                                                  const uint8_t* __restrict__ c, int64_t c_stride,
                                                  int64_t B, int64_t n, float scale,
                                                  float* __restrict__ g, float* __restrict__ part) {
  __shared__ float red[4];
  float acc = 0.f;
  const int64_t N = B * n;
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < N;
       t += (int64_t)gridDim.x * blockDim.x) {
    const int64_t b = t / n, v = t - b * n;
    const float x = L[t];
    const float lab = (float)(c[b * c_stride + v] & 1);
    const float e = expf(-fabsf(x));
    const float sig = x >= 0.f ? 1.f / (1.f + e) : e / (1.f + e);
    g[t] = scale * (sig - lab);
    if (part) acc += fmaxf(x, 0.f) + log1pf(e) - lab * x;
  }
  if (!part) return;
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Loss total: a fixed-shape tree over the per-workgroup partials.
__global__ __launch_bounds__(1024) void bce_final_kernel(const float* __restrict__ part, int n,
                                                         float scale, float* __restrict__ loss) {
  __shared__ float red[1024];
  const int tid = threadIdx.x;
  float a = 0.f;
  for (int i = tid; i < n; i += 1024) a += part[i];
  red[tid] = a;
  __syncthreads();
  for (int h = 512; h > 0; h >>= 1) {
    if (tid < h) red[tid] += red[tid + h];
    __syncthreads();
  }
  if (tid == 0) *loss = scale * red[0];
}

__global__ void adam_kernel(float* __restrict__ p, const float* __restrict__ g,
                            float* __restrict__ m, float* __restrict__ v, int64_t n, float lr,
                            float b1, float b2, float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// workgroups of the backward pass: one per CU worth of steps at most
inline int ndm_bwd_blocks(int64_t n) {
  const int64_t nstep = (n + kTS - 1) / kTS;
  const int64_t want = (nstep + kBwdWaves - 1) / kBwdWaves;
  return (int)(want < 256 ? want : 256);
}

}  // namespace

size_t ndm_work_bytes(int64_t B, int64_t S) {
  return ((size_t)ndm_bwd_blocks(B * S) * kBwdWaves + kSlices) * NP * 4;
}

hipError_t launch_ndm_forward(const float* params, const float* y, const float* no, int64_t B,
                              int64_t S, float* llr, hipStream_t s) {
  const int64_t ntile = (B * S + 15) / 16;
  const int64_t waves = ntile < 8192 ? ntile : 8192;
  const unsigned grid = (unsigned)((waves + kNdmFwdThreads / 64 - 1) / (kNdmFwdThreads / 64));
  ndm_forward_kernel<<<grid, kNdmFwdThreads, 0, s>>>(params, y, no, B, S, llr);
  return hipGetLastError();
}

hipError_t launch_ndm_backward(const float* params, const float* y, const float* no,
                               const float* gllr, int64_t B, int64_t S, float* gparams,
                               float* gy, void* work, hipStream_t s) {
  const int nb = ndm_bwd_blocks(B * S);
  const int rows = nb * kBwdWaves;
  float* part = reinterpret_cast<float*>(work);
  hipError_t e = ensure_dyn_lds((const void*)ndm_backward_kernel, ndm_bwd_lds());
  if (e != hipSuccess) return e;
  ndm_backward_kernel<<<nb, kBwdThreads, ndm_bwd_lds(), s>>>(params, y, no, gllr, B, S, part, gy);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  float* slices = part + (size_t)rows * NP;
  dim3 grid((NP + 255) / 256, kSlices);
  sum_slices_kernel<<<grid, 256, 0, s>>>(part, rows, NP, slices);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  sum_final_kernel<<<(NP + 255) / 256, 256, 0, s>>>(slices, NP, gparams);
  return hipGetLastError();
}

size_t bce_work_bytes(int64_t, int64_t) { return (size_t)kBceBlocks * 4; }

hipError_t launch_bce_grad(const float* lpost, const uint8_t* c, int64_t c_stride, int64_t B,
                           int64_t n, float scale, float* g, float* loss, void* work,
                           hipStream_t s) {
  float* part = loss ? reinterpret_cast<float*>(work) : nullptr;
  bce_kernel<<<kBceBlocks, 256, 0, s>>>(lpost, c, c_stride, B, n, scale, g, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || !loss) return e;
  bce_final_kernel<<<1, 1024, 0, s>>>(part, kBceBlocks, scale, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace lsim
