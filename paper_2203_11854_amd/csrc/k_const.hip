// Trainable constellation: the mapper with a table of K = 2^m points and
// its adjoint (end-to-end learning with the neural demapper).
//
// Points p[K][2] are indexed by the label of m coded bits, first bit most
// significant, and used scaled to unit average energy,
//   x_k = p_k / s,   s = sqrt(mean_j |p_j|^2).
// Forward: y = x_label + sqrt(N0/2) (normal pair), the normals drawn exactly
// as by the Gray-QAM mapper (same Philox words, same Box-Muller).
// Adjoint: with G_k = sum of dL/dy over the symbols carrying label k,
//   dL/dp_j = (G_j - x_j (sum_k G_k . x_k) / K) / s,
// the second term coming from the normalisation.  The per-label sums are
// formed deterministically: each lane accumulates its own symbols, lanes
// and workgroups are then added in a fixed order.
#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "lsim_internal.h"
#include "philox.h"

namespace lsim {

namespace {

constexpr int kKMax = 64;  // points (m <= 6)

// Normalised points into LDS (every workgroup computes s in the same order).
__device__ __forceinline__ void load_points(const float* p, int K, float2* xs, float* s_out) {
  if (threadIdx.x < 64) {
    float e = 0.f;
    if ((int)threadIdx.x < K) e = p[2 * threadIdx.x] * p[2 * threadIdx.x] +
                                  p[2 * threadIdx.x + 1] * p[2 * threadIdx.x + 1];
    // fixed-shape tree over the 64 lanes of the first wavefront
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) e += __shfl_xor(e, off, 64);
    const float s = sqrtf(e / (float)K);
    if ((int)threadIdx.x < K) xs[threadIdx.x] = make_float2(p[2 * threadIdx.x] / s, p[2 * threadIdx.x + 1] / s);
    if (threadIdx.x == 0) *s_out = s;
  }
  __syncthreads();
}

__device__ __forceinline__ int label_of(const uint8_t* bits, int m) {
  int k = 0;
  for (int q = 0; q < m; ++q) k = (k << 1) | (bits[q] & 1);
  return k;
}

__global__ __launch_bounds__(256) void map_points_kernel(DevCode c, int m, const float* __restrict__ pts,
                                                         const uint8_t* __restrict__ cw,
                                                         const float* __restrict__ no, uint64_t seed,
                                                         int64_t cw0, int64_t B, int S,
                                                         float* __restrict__ y) {
  __shared__ float2 xs[kKMax];
  __shared__ float s_norm;
  load_points(pts, 1 << m, xs, &s_norm);
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
    const Polar bm = box_muller(h ? r.z : r.x, h ? r.w : r.y);
    const float2 x = xs[label_of(bits + s * m, m)];
    float2 out;
    out.x = x.x + sig * bm.rho * bm.cs;
    out.y = x.y + sig * bm.rho * bm.sn;
    reinterpret_cast<float2*>(y)[b * (int64_t)S + s] = out;
  }
}

constexpr int kGradThreads = 256;    // four wavefronts per workgroup
constexpr int kGradBlocks = 1024;    // partial rows at most
constexpr int kFinalThreads = 1024;  // >= kGradBlocks: one row per thread

// Per-workgroup label sums of dL/dy: column col = 2 k + (Re, Im) of row wg
// lands at part[col][wg].  Each lane accumulates its own symbols in its own
// LDS row (pitch 2K + 1); each wavefront then adds its 64 rows in order and
// the four wavefronts are added in order.
__global__ __launch_bounds__(kGradThreads) void points_partial_kernel(
    DevCode c, int m, const uint8_t* __restrict__ cw, const float* __restrict__ gy, int64_t B,
    int S, float* __restrict__ part) {
  extern __shared__ float acc[];
  __shared__ float wsum[kGradThreads / 64][2 * kKMax];
  const int K = 1 << m, pitch = 2 * K + 1;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  float* mine = acc + tid * pitch;
  for (int k = 0; k < 2 * K; ++k) mine[k] = 0.f;
  const int64_t n = B * S;
  for (int64_t t = (int64_t)blockIdx.x * kGradThreads + tid; t < n;
       t += (int64_t)gridDim.x * kGradThreads) {
    const int64_t b = t / S;
    const int s = (int)(t - b * S);
    const int k = label_of(cw + b * (int64_t)c.n_mother + c.tx_lo + (int64_t)s * m, m);
    const float2 g = reinterpret_cast<const float2*>(gy)[t];
    mine[2 * k] += g.x;
    mine[2 * k + 1] += g.y;
  }
  __syncthreads();
  for (int col = lane; col < 2 * K; col += 64) {
    float v = 0.f;
    for (int l = 0; l < 64; ++l) v += acc[(wave * 64 + l) * pitch + col];
    wsum[wave][col] = v;
  }
  __syncthreads();
  if (tid < 2 * K) {
    float v = 0.f;
    for (int w = 0; w < kGradThreads / 64; ++w) v += wsum[w][tid];
    part[(int64_t)tid * gridDim.x + blockIdx.x] = v;
  }
}

// Sums the partial rows (thread r takes row r, then fixed-shape trees over
// each wavefront and the wavefronts in order) and applies the
// normalisation's adjoint.
__global__ __launch_bounds__(kFinalThreads) void points_final_kernel(
    int m, const float* __restrict__ pts, const float* __restrict__ part, int rows,
    float* __restrict__ gp) {
  __shared__ float2 xs[kKMax];
  __shared__ float s_norm;
  __shared__ float wsum[kFinalThreads / 64][2 * kKMax];
  __shared__ float G[2 * kKMax];
  const int K = 1 << m;
  load_points(pts, K, xs, &s_norm);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
#pragma unroll 4
  for (int col = 0; col < 2 * K; ++col) {
    float v = tid < rows ? part[(int64_t)col * rows + tid] : 0.f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if (lane == 0) wsum[wave][col] = v;
  }
  __syncthreads();
  if (tid < 2 * K) {
    float a = 0.f;
    for (int w = 0; w < kFinalThreads / 64; ++w) a += wsum[w][tid];
    G[tid] = a;
  }
  __syncthreads();
  if (tid < 64) {
    const int k = tid;
    // radial term sum_k G_k . x_k, fixed-shape tree
    float d = k < K ? G[2 * k] * xs[k].x + G[2 * k + 1] * xs[k].y : 0.f;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) d += __shfl_xor(d, off, 64);
    if (k < K) {
      const float rad = d / (float)K;
      gp[2 * k] = (G[2 * k] - xs[k].x * rad) / s_norm;
      gp[2 * k + 1] = (G[2 * k + 1] - xs[k].y * rad) / s_norm;
    }
  }
}

inline int64_t grad_rows(int64_t n) {
  const int64_t want = (n + kGradThreads - 1) / kGradThreads;
  return want < kGradBlocks ? want : kGradBlocks;
}

}  // namespace

hipError_t launch_map_points(const DevCode& c, int m, const float* pts, const uint8_t* cw,
                             const float* no, uint64_t seed, int64_t cw0, int64_t B, float* y,
                             hipStream_t s) {
  const int S = c.e_tx / m;
  const int64_t n = B * ((S + 1) / 2);
  map_points_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(c, m, pts, cw, no, seed, cw0, B, S, y);
  return hipGetLastError();
}

size_t points_work_bytes(const DevCode& c, int m, int64_t B) {
  return (size_t)grad_rows(B * (c.e_tx / m)) * 2 * ((size_t)1 << m) * 4;
}

hipError_t launch_points_grad(const DevCode& c, int m, const float* pts, const uint8_t* cw,
                              const float* gy, int64_t B, float* gp, void* work, hipStream_t s) {
  const int S = c.e_tx / m;
  const int64_t rows = grad_rows(B * S);
  float* part = reinterpret_cast<float*>(work);
  const size_t lds = (size_t)kGradThreads * (2 * (1 << m) + 1) * 4;
  hipError_t e = ensure_dyn_lds((const void*)points_partial_kernel, lds);
  if (e != hipSuccess) return e;
  points_partial_kernel<<<(unsigned)rows, kGradThreads, lds, s>>>(c, m, cw, gy, B, S, part);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  points_final_kernel<<<1, kFinalThreads, 0, s>>>(m, pts, part, (int)rows, gp);
  return hipGetLastError();
}

}  // namespace lsim
