// Neural demapper (3 -> 64 -> 64 -> 4 MLP per symbol, ReLU), its parameter
// gradient, the binary cross-entropy on logits and an Adam step.
//
// Forward: one thread per symbol; the parameters are read with
// wave-uniform addresses (scalar loads), h1 stays in registers and the
// second layer is consumed row by row straight into the 4 outputs.
// Backward: one wavefront handles 64 symbols at a time; each lane recomputes
// its symbol's activations, forms the deltas, and the wavefront reduces the
// outer products through LDS tiles in two phases with every lane owning one
// row of W2 (and of W1, b1, b2, one column of W3).  Per-workgroup partial gradients are then
// summed over workgroups in a fixed order, so the result is deterministic.
#include <hip/hip_runtime.h>

#include "lsim_internal.h"

namespace lsim {

namespace {

constexpr int H = 64;
constexpr int OW1 = 0, OB1 = 192, OW2 = 256, OB2 = 4352, OW3 = 4416, OB3 = 4672, NP = 4676;

__global__ __launch_bounds__(256) void ndm_forward_kernel(const float* __restrict__ P,
                                                          const float* __restrict__ y,
                                                          const float* __restrict__ no,
                                                          int64_t B, int64_t S,
                                                          float* __restrict__ llr) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= B * S) return;
  const int64_t b = t / S;
  const float x0 = y[2 * t], x1 = y[2 * t + 1], x2 = logf(no[b]);
  float h1[H];
#pragma unroll
  for (int i = 0; i < H; ++i) {
    const float a = P[OW1 + 3 * i] * x0 + P[OW1 + 3 * i + 1] * x1 + P[OW1 + 3 * i + 2] * x2 +
                    P[OB1 + i];
    h1[i] = fmaxf(a, 0.f);
  }
  float o0 = P[OB3], o1 = P[OB3 + 1], o2 = P[OB3 + 2], o3 = P[OB3 + 3];
  for (int o = 0; o < H; ++o) {
    float a = P[OB2 + o];
#pragma unroll
    for (int i = 0; i < H; ++i) a += P[OW2 + o * H + i] * h1[i];
    const float h = fmaxf(a, 0.f);
    o0 += P[OW3 + o] * h;
    o1 += P[OW3 + H + o] * h;
    o2 += P[OW3 + 2 * H + o] * h;
    o3 += P[OW3 + 3 * H + o] * h;
  }
  float4 out = make_float4(o0, o1, o2, o3);
  reinterpret_cast<float4*>(llr)[t] = out;
}

constexpr int PAD = H + 1;

// LDS per wavefront: three 64 x 65 float tiles (50 KB), so three
// wavefronts fit on a CU.  delta1 = W2^T delta2 is accumulated while the
// rows of delta2 are produced, so delta2 and h2 never sit in registers.
// Phase 1 reduces dW2 = D2^T H1, db2, dW3 = D3^T H2, db3; phase 2 reuses
// the H1 tile for dW1 = D1^T X and db1.
__global__ __launch_bounds__(64) void ndm_backward_kernel(const float* __restrict__ P,
                                                          const float* __restrict__ y,
                                                          const float* __restrict__ no,
                                                          const float* __restrict__ gllr,
                                                          int64_t B, int64_t S,
                                                          float* __restrict__ part) {
  __shared__ float sA[64 * PAD], sB[64 * PAD], sC[64 * PAD];
  __shared__ float sX[64 * 3], sD3[64 * 4];
  const int lane = threadIdx.x;
  const int64_t n = B * S;
  const int64_t nchunk = (n + 63) / 64;
  // accumulators owned by this lane (row/col `lane`)
  float gW2[H];
#pragma unroll
  for (int i = 0; i < H; ++i) gW2[i] = 0.f;
  float gW1[3] = {0.f, 0.f, 0.f}, gb1 = 0.f, gb2 = 0.f, gW3[4] = {0.f, 0.f, 0.f, 0.f}, gb3 = 0.f;

  for (int64_t ch = blockIdx.x; ch < nchunk; ch += gridDim.x) {
    const int64_t t = ch * 64 + lane;
    const bool on = t < n;
    float x0 = 0.f, x1 = 0.f, x2 = 0.f, d3[4] = {0.f, 0.f, 0.f, 0.f};
    if (on) {
      const int64_t b = t / S;
      x0 = y[2 * t];
      x1 = y[2 * t + 1];
      x2 = logf(no[b]);
#pragma unroll
      for (int j = 0; j < 4; ++j) d3[j] = gllr[4 * t + j];
    }
    float h1[H];
#pragma unroll
    for (int i = 0; i < H; ++i) {
      const float a = P[OW1 + 3 * i] * x0 + P[OW1 + 3 * i + 1] * x1 + P[OW1 + 3 * i + 2] * x2 +
                      P[OB1 + i];
      h1[i] = on ? fmaxf(a, 0.f) : 0.f;
      sA[lane * PAD + i] = h1[i];
    }
    // layer 2 forward, delta2 row by row, delta1 accumulated on the way
    float d1[H];
#pragma unroll
    for (int i = 0; i < H; ++i) d1[i] = 0.f;
    for (int o = 0; o < H; ++o) {
      float a = P[OB2 + o];
#pragma unroll
      for (int i = 0; i < H; ++i) a += P[OW2 + o * H + i] * h1[i];
      const float g = P[OW3 + o] * d3[0] + P[OW3 + H + o] * d3[1] + P[OW3 + 2 * H + o] * d3[2] +
                      P[OW3 + 3 * H + o] * d3[3];
      const float d2 = (on && a > 0.f) ? g : 0.f;
      sC[lane * PAD + o] = on ? fmaxf(a, 0.f) : 0.f;
      sB[lane * PAD + o] = d2;
#pragma unroll
      for (int i = 0; i < H; ++i) d1[i] += P[OW2 + o * H + i] * d2;
    }
    sX[lane * 3 + 0] = on ? x0 : 0.f;
    sX[lane * 3 + 1] = on ? x1 : 0.f;
    sX[lane * 3 + 2] = on ? x2 : 0.f;
#pragma unroll
    for (int j = 0; j < 4; ++j) sD3[lane * 4 + j] = on ? d3[j] : 0.f;
    __syncthreads();
    // phase 1: row `lane` of dW2 and db2, column `lane` of dW3, db3
    for (int s = 0; s < 64; ++s) {
      const float d2 = sB[s * PAD + lane];
#pragma unroll
      for (int i = 0; i < H; ++i) gW2[i] += d2 * sA[s * PAD + i];
      gb2 += d2;
      const float hh = sC[s * PAD + lane];
#pragma unroll
      for (int j = 0; j < 4; ++j) gW3[j] += sD3[s * 4 + j] * hh;
      if (lane < 4) gb3 += sD3[s * 4 + lane];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < H; ++i) sA[lane * PAD + i] = h1[i] > 0.f ? d1[i] : 0.f;
    __syncthreads();
    // phase 2: row `lane` of dW1 and db1
    for (int s = 0; s < 64; ++s) {
      const float d1l = sA[s * PAD + lane];
      gW1[0] += d1l * sX[s * 3 + 0];
      gW1[1] += d1l * sX[s * 3 + 1];
      gW1[2] += d1l * sX[s * 3 + 2];
      gb1 += d1l;
    }
    __syncthreads();
  }
  float* out = part + (int64_t)blockIdx.x * NP;
#pragma unroll
  for (int i = 0; i < H; ++i) out[OW2 + lane * H + i] = gW2[i];
  out[OW1 + 3 * lane + 0] = gW1[0];
  out[OW1 + 3 * lane + 1] = gW1[1];
  out[OW1 + 3 * lane + 2] = gW1[2];
  out[OB1 + lane] = gb1;
  out[OB2 + lane] = gb2;
#pragma unroll
  for (int j = 0; j < 4; ++j) out[OW3 + j * H + lane] = gW3[j];
  if (lane < 4) out[OB3 + lane] = gb3;
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

__global__ void bce_final_kernel(const float* __restrict__ part, int n, float scale,
                                 float* __restrict__ loss) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  float acc = 0.f;
  for (int i = 0; i < n; ++i) acc += part[i];
  *loss = scale * acc;
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

inline int ndm_bwd_blocks(int64_t n) {
  const int64_t nchunk = (n + 63) / 64;
  return (int)(nchunk < 2048 ? nchunk : 2048);
}

}  // namespace

size_t ndm_work_bytes(int64_t B, int64_t S) {
  return ((size_t)ndm_bwd_blocks(B * S) + kSlices) * NP * 4;
}

hipError_t launch_ndm_forward(const float* params, const float* y, const float* no, int64_t B,
                              int64_t S, float* llr, hipStream_t s) {
  const int64_t n = B * S;
  ndm_forward_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(params, y, no, B, S, llr);
  return hipGetLastError();
}

hipError_t launch_ndm_backward(const float* params, const float* y, const float* no,
                               const float* gllr, int64_t B, int64_t S, float* gparams,
                               void* work, hipStream_t s) {
  const int nb = ndm_bwd_blocks(B * S);
  float* part = reinterpret_cast<float*>(work);
  ndm_backward_kernel<<<nb, 64, 0, s>>>(params, y, no, gllr, B, S, part);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  float* slices = part + (size_t)nb * NP;
  dim3 grid((NP + 255) / 256, kSlices);
  sum_slices_kernel<<<grid, 256, 0, s>>>(part, nb, NP, slices);
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
  bce_final_kernel<<<1, 64, 0, s>>>(part, kBceBlocks, scale, loss);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, int step, hipStream_t s) {
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  adam_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(p, g, m, v, n, lr, b1, b2, eps, c1, c2);
  return hipGetLastError();
}

}  // namespace lsim
