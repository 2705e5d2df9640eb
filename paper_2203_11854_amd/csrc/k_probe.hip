// Peak-rate probes for the roofline denominators, run in the same job as the
// decoders: device copy and read (HBM bytes per second), LDS reads and
// writes of 16 bytes per lane (LDS bytes per second), and independent VALU
// chains of fused multiply-adds and of base-2 exponentials (lane operations
// per second).  Every probe writes one word per thread so nothing is
// optimized away.
#include <hip/hip_runtime.h>

#include "lsim_internal.h"

namespace lsim {

namespace {

constexpr int kProbeThreads = 256;
constexpr int kLdsProbeBytes = 64 * 1024;  // per workgroup: two per CU fit

__global__ __launch_bounds__(256) void copy_probe_kernel(const float4* __restrict__ src,
                                                         float4* __restrict__ dst, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride)
    dst[i] = src[i];
}

__global__ __launch_bounds__(256) void read_probe_kernel(const uint4* __restrict__ src, int64_t n4,
                                                         uint32_t* __restrict__ out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint32_t acc = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
    const uint4 v = src[i];
    acc ^= v.x ^ v.y ^ v.z ^ v.w;
  }
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

// Each lane reads (or writes) 16 bytes at lane-consecutive addresses, eight
// accesses in flight per round, walking the workgroup's 64 KB.
__global__ __launch_bounds__(256) void lds_read_probe_kernel(int rounds, uint32_t* __restrict__ out) {
  extern __shared__ __align__(16) uint4 lds[];
  const int t = threadIdx.x;
  for (int i = t; i < kLdsProbeBytes / 16; i += kProbeThreads) lds[i] = make_uint4(i, i + 1, i + 2, i + 3);
  __syncthreads();
  uint4 acc = make_uint4(0u, 0u, 0u, 0u);
  constexpr int kSlots = kLdsProbeBytes / 16;  // 4096 uint4
  for (int r = 0; r < rounds; ++r) {
    // the compiler may not reuse loads of an earlier round
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const uint4 v = lds[(t + (u + 8 * (r & 1)) * kProbeThreads) & (kSlots - 1)];
      acc.x ^= v.x;
      acc.y ^= v.y;
      acc.z ^= v.z;
      acc.w ^= v.w;
    }
  }
  out[(int64_t)blockIdx.x * kProbeThreads + t] = acc.x ^ acc.y ^ acc.z ^ acc.w;
}

__global__ __launch_bounds__(256) void lds_write_probe_kernel(int rounds, uint32_t* __restrict__ out) {
  extern __shared__ __align__(16) uint4 lds[];
  const int t = threadIdx.x;
  constexpr int kSlots = kLdsProbeBytes / 16;
  uint4 v = make_uint4(t, t + 1, t + 2, t + 3);
  for (int r = 0; r < rounds; ++r) {
    // nor drop the stores a later round overwrites
    asm volatile("" ::: "memory");
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      lds[(t + (u + 8 * (r & 1)) * kProbeThreads) & (kSlots - 1)] = v;
      v.x += 1u;
    }
  }
  __syncthreads();
  const uint4 w = lds[(t * 7) & (kSlots - 1)];
  out[(int64_t)blockIdx.x * kProbeThreads + t] = w.x ^ w.y ^ w.z ^ w.w;
}

// Eight independent chains per lane; one fused multiply-add (or one base-2
// exponential) per chain per step is one VALU lane operation.
__global__ __launch_bounds__(256) void fma_probe_kernel(int steps, float a, float b,
                                                        float* __restrict__ out) {
  float x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = (float)(threadIdx.x + j) * 1e-3f;
#pragma unroll 4
  for (int s = 0; s < steps; ++s) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = __builtin_fmaf(x[j], a, b);
  }
  float acc = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) acc += x[j];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

__global__ __launch_bounds__(256) void exp_probe_kernel(int steps, float* __restrict__ out) {
  float x[8];
#pragma unroll
  for (int j = 0; j < 8; ++j) x[j] = -(float)(threadIdx.x + j) * 1e-3f;
#pragma unroll 4
  for (int s = 0; s < steps; ++s) {
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = -__builtin_amdgcn_exp2f(x[j]);
  }
  float acc = 0.f;
#pragma unroll
  for (int j = 0; j < 8; ++j) acc += x[j];
  out[(int64_t)blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace

hipError_t launch_probe(int kind, const void* src, void* dst, int64_t bytes, int rounds, int grid,
                        hipStream_t s, int64_t* units) {
  switch (kind) {
    case 0: {  // copy: bytes read + written
      const int64_t n4 = bytes / 16;
      copy_probe_kernel<<<grid, 256, 0, s>>>((const float4*)src, (float4*)dst, n4);
      *units = 2 * n4 * 16;
      break;
    }
    case 1: {  // read
      const int64_t n4 = bytes / 16;
      read_probe_kernel<<<grid, 256, 0, s>>>((const uint4*)src, n4, (uint32_t*)dst);
      *units = n4 * 16;
      break;
    }
    case 2:
    case 3: {  // LDS read / write bytes
      const void* k = kind == 2 ? (const void*)lds_read_probe_kernel : (const void*)lds_write_probe_kernel;
      hipError_t e = ensure_dyn_lds(k, kLdsProbeBytes);
      if (e != hipSuccess) return e;
      if (kind == 2)
        lds_read_probe_kernel<<<grid, kProbeThreads, kLdsProbeBytes, s>>>(rounds, (uint32_t*)dst);
      else
        lds_write_probe_kernel<<<grid, kProbeThreads, kLdsProbeBytes, s>>>(rounds, (uint32_t*)dst);
      *units = (int64_t)grid * kProbeThreads * rounds * 8 * 16;
      break;
    }
    case 4:  // fused multiply-adds
      fma_probe_kernel<<<grid, 256, 0, s>>>(rounds, 0.999f, 1e-4f, (float*)dst);
      *units = (int64_t)grid * 256 * rounds * 8;
      break;
    case 5:  // base-2 exponentials
      exp_probe_kernel<<<grid, 256, 0, s>>>(rounds, (float*)dst);
      *units = (int64_t)grid * 256 * rounds * 8;
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace lsim
