// Layered normalized min-sum (FP32) and the persistent mixed-shape decoder.
//
// A tile is G codewords of one code decoded by one workgroup: lane
// (g, r) = (tid / Z, tid % Z) owns check r of every layer of codeword g.  The
// posteriors APP[G][n_dec] live in LDS; a QC row block meets each variable
// node at most once, so the Z checks of a layer update APP without
// conflicts and one barrier separates consecutive layers.  The check state
// of the previous iteration is kept compressed per check as
// (alpha*m1, alpha*m2, sign bits | i1 << 27) in three 32-bit words, streamed
// through device memory in [codeword][layer][word][Z] order (coalesced).
//
// Arithmetic follows the layered min-sum update one IEEE single-precision
// operation at a time (no fused multiply-add): t = APP - r_old;
// r_new = sign * (alpha * (v == i1 ? m2 : m1)); APP = t + r_new.
#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "lds.h"
#include "lsim_internal.h"

#pragma clang fp contract(off)

namespace lsim {

namespace {

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

__host__ __device__ inline size_t tile_lds_bytes(const DevCode& c, int G) {
  return align16((size_t)G * c.n_dec * 4);
}

struct TileIO {
  const float* llr;     // [count][e_tx] of this shape
  uint8_t* bits;        // [count][k]
  float* lpost;         // [count][n_dec]
  float* r_out;         // [count][E]
  uint32_t* state;      // [count][rows][3][Z]
  int64_t count;
};

template <int NT, int DMAX>
__device__ __forceinline__ void decode_tile(const DevCode& c, int G, int64_t tile, const TileIO& io, int iters,
                            float alpha, unsigned char* smem) {
  float* app = reinterpret_cast<float*>(smem);
  const int Z = c.Z;
  const int tid = threadIdx.x;
  const int64_t cw0 = tile * G;
  const int gmax = (int)min<int64_t>(G, io.count - cw0);

  for (int idx = tid; idx < G * c.n_dec; idx += NT) {
    const int g = idx / c.n_dec, v = idx - g * c.n_dec;
    const int x = v - c.tx_lo;
    float l = 0.f;
    if (g < gmax && x >= 0 && x < c.e_tx) l = -io.llr[(cw0 + g) * c.e_tx + x];
    app[idx] = l;
  }
  __syncthreads();

  const int g = tid / Z;
  const int r = tid - g * Z;
  const bool active = g < gmax;
  // LDS byte address of this lane's codeword's posteriors (the tile's LDS
  // starts at offset 0: the kernels have no static LDS)
  const int app_b = vreg((active ? g : 0) * c.n_dec * 4);
  const int Z4 = Z * 4, zm4 = (Z - 1) * 4, r4 = vreg(r * 4);
  const bool zpow2 = (Z & (Z - 1)) == 0;
  uint32_t* st = io.state + (size_t)(cw0 + (active ? g : 0)) * c.rows * 3 * Z + r;

  // The check state of the next layer is loaded one layer ahead so its
  // memory latency overlaps the current layer.  A decoded graph has at
  // least three layers, so a prefetched layer was stored at least two
  // layers earlier.
  const int rows = c.rows;
  float n1 = 0.f, n2 = 0.f;
  uint32_t npk_in = 0;
  for (int it = 0; it < iters; ++it) {
    for (int i = 0; i < rows; ++i) {
      const int e0 = uni(ld_const(c.row_ptr, i));
      const int d = uni(ld_const(c.row_ptr, i + 1)) - e0;
      const float a1 = n1, a2 = n2;
      const uint32_t pk = npk_in;
      {
        int ni = i + 1, nit = it;
        if (ni == rows) {
          ni = 0;
          ++nit;
        }
        if (active && nit >= 1 && nit < iters) {
          const uint32_t* s2 = st + (size_t)ni * 3 * Z;
          n1 = __uint_as_float(s2[0]);
          n2 = __uint_as_float(s2[Z]);
          npk_in = s2[2 * Z];
        } else {
          n1 = 0.f;
          n2 = 0.f;
          npk_in = 0;
        }
      }
      if (active) {
        uint32_t* sti = st + (size_t)i * 3 * Z;
        with_degree<DMAX>(d, [&](auto deg) {
          constexpr int D = decltype(deg)::value;
          int addr[D];
          float tv[D];
          // LDS byte address of the variable node of entry e at lift r:
          // app_b + col*Z*4 + ((r + shift) mod Z)*4; the reduction is a mask
          // for a power-of-two lift, else min(x, x - Z*4) on unsigned x
          if (zpow2) {
#pragma unroll
            for (int q = 0; q < D; ++q) {
              const int2 en = ld_const(c.ent_cz, e0 + q);
              addr[q] = app_b + en.x * 4 + ((r4 + en.y * 4) & zm4);
            }
          } else {
#pragma unroll
            for (int q = 0; q < D; ++q) {
              const int2 en = ld_const(c.ent_cz, e0 + q);
              const uint32_t x = (uint32_t)(r4 + en.y * 4);
              addr[q] = app_b + en.x * 4 + (int)min(x, x - (uint32_t)Z4);
            }
          }
#pragma unroll
          for (int q = 0; q < D; ++q) tv[q] = lds_ld<float>(addr[q]);
          const int i1_old = (int)(pk >> 27);
          // sign of a zero never reaches a nonzero value (a zero input forces
          // every other output magnitude to zero), so sign bits are used as is
          uint32_t sx = 0;
          float m1 = INFINITY, m2 = INFINITY;
#pragma unroll
          for (int q = 0; q < D; ++q) {
            const float mag = q == i1_old ? a2 : a1;
            const float rold = __uint_as_float(__float_as_uint(mag) | ((pk << (31 - q)) & 0x80000000u));
            const float t = __fsub_rn(tv[q], rold);
            tv[q] = t;
            sx ^= __float_as_uint(t);
            const float at = fabsf(t);
            m2 = __builtin_amdgcn_fmed3f(m1, at, m2);
            m1 = fminf(m1, at);
          }
          const float b1 = __fmul_rn(alpha, m1);
          const float b2 = __fmul_rn(alpha, m2);
          // Outputs in reverse order: the input at the minimum gets alpha*m2,
          // the others alpha*m1, and i1 ends on the first index at the minimum.
          // A repeated minimum makes m2 == m1, so every tie gets the same value.
          int i1 = 0;
          uint32_t npk = 0;
#pragma unroll
          for (int q = D - 1; q >= 0; --q) {
            const bool at_min = fabsf(tv[q]) == m1;
            const float mag = at_min ? b2 : b1;
            i1 = at_min ? q : i1;
            const uint32_t sg = (sx ^ __float_as_uint(tv[q])) & 0x80000000u;
            lds_st<float>(addr[q], __fadd_rn(tv[q], __uint_as_float(__float_as_uint(mag) | sg)));
            npk |= sg >> (31 - q);
          }
          npk |= (uint32_t)i1 << 27;
          sti[0] = __float_as_uint(b1);
          sti[Z] = __float_as_uint(b2);
          sti[2 * Z] = npk;
        });
      }
      lds_barrier();
    }
  }

  // outputs
  for (int idx = tid; idx < gmax * c.n_dec; idx += NT) {
    const int gg = idx / c.n_dec, v = idx - gg * c.n_dec;
    const float x = app[idx];
    if (io.bits && v < c.k) io.bits[(cw0 + gg) * c.k + v] = x < 0.f;
    if (io.lpost) io.lpost[(cw0 + gg) * c.n_dec + v] = -x;
  }
  if (io.r_out && active) {
    for (int i = 0; i < c.rows; ++i) {
      const uint32_t* sti = st + (size_t)i * 3 * Z;
      const float a1 = __uint_as_float(sti[0]), a2 = __uint_as_float(sti[Z]);
      const uint32_t pk = sti[2 * Z];
      const int i1 = (int)(pk >> 27);
      const int rb = c.row_ptr[i];
      for (int e = rb; e < c.row_ptr[i + 1]; ++e) {
        const int q = e - rb;
        const float mag = q == i1 ? a2 : a1;
        io.r_out[(cw0 + g) * (int64_t)c.E + (int64_t)e * Z + r] = ((pk >> q) & 1u) ? -mag : mag;
      }
    }
  }
}

template <int NT, int DMAX>
__global__ __launch_bounds__(NT) void layered_kernel(DevCode c, int G, TileIO io, int iters,
                                                     float alpha) {
  extern __shared__ __align__(16) unsigned char smem[];
  decode_tile<NT, DMAX>(c, G, blockIdx.x, io, iters, alpha, smem);
}

// Persistent decoder over a work list of (shape, tile) items.  Workgroups
// take items from a device counter until the list is drained; the counter
// is reset by reset_counter_kernel launched just before, so the pair can be
// captured in a graph.
template <int NT, int DMAX>
__global__ __launch_bounds__(NT) void mixed_kernel(const LayerShape* __restrict__ shapes,
                                                   const int* __restrict__ tile_shape,
                                                   const int64_t* __restrict__ tile_local,
                                                   int64_t ntiles, const float* llr,
                                                   uint8_t* bits, float* lpost, uint32_t* state,
                                                   int* counter, int persistent, int iters,
                                                   float alpha, int next_off) {
  // dynamic LDS only (tiles address it from offset 0); the work item taken
  // by thread 0 is broadcast through the word at next_off
  extern __shared__ __align__(16) unsigned char smem[];
  int* next = reinterpret_cast<int*>(smem + next_off);
  int64_t item = persistent ? -1 : (int64_t)blockIdx.x;
  for (;;) {
    if (persistent) {
      if (threadIdx.x == 0) *next = atomicAdd(counter, 1);
      __syncthreads();
      item = *next;
      __syncthreads();
    }
    if (item >= ntiles) break;
    const int s = tile_shape[item];
    const LayerShape& sh = shapes[s];
    TileIO io;
    io.llr = llr + sh.llr_off;
    io.bits = bits ? bits + sh.bits_off : nullptr;
    io.lpost = lpost ? lpost + sh.app_off : nullptr;
    io.r_out = nullptr;
    io.state = state + sh.state_off;
    io.count = sh.count;
    decode_tile<NT, DMAX>(sh.code, sh.G, tile_local[item], io, iters, alpha, smem);
    __syncthreads();
    if (!persistent) break;
  }
}

__global__ void reset_counter_kernel(int* counter) { *counter = 0; }


}  // namespace

size_t layered_state_words(const DevCode& c, int64_t B) { return (size_t)B * c.rows * 3 * c.Z; }

hipError_t launch_layered(const DevCode& c, const lsim_decode_params& p, const float* llr,
                          int64_t B, uint8_t* bits, float* lpost, float* r_out, uint32_t* state,
                          hipStream_t s, std::string* why) {
  int nt = p.threads;
  if (!nt) {
    const int cand[5] = {256, 384, 512, 768, 1024};
    nt = 1024;
    for (int x : cand)
      if (x >= c.Z) {
        nt = x;
        break;
      }
  }
  if (c.Z > nt) {
    *why = "layered decoder needs threads >= Z";
    return hipSuccess;
  }
  int G = nt / c.Z;
  while (G > 1 && tile_lds_bytes(c, G) > 160 * 1024) --G;
  const size_t lds = tile_lds_bytes(c, G);
  if (lds > 160 * 1024) {
    *why = "layered decoder posteriors exceed the 160 KiB LDS";
    return hipSuccess;
  }
  TileIO io{llr, bits, lpost, r_out, state, B};
  const unsigned grid = (unsigned)((B + G - 1) / G);
  const int dmax = c.max_row_deg;
#define LSIM_LAYER_CASE(NT_, D_)                                                   \
  if (nt == NT_ && dmax <= D_) {                                                   \
    hipError_t e = require_lds_at_zero((const void*)layered_kernel<NT_, D_>);   \
    if (e == hipSuccess) e = ensure_dyn_lds((const void*)layered_kernel<NT_, D_>, lds); \
    if (e != hipSuccess) return e;                                                 \
    layered_kernel<NT_, D_><<<grid, NT_, lds, s>>>(c, G, io, p.iters, p.alpha);    \
    return hipGetLastError();                                                      \
  }
  LSIM_LAYER_CASE(256, 16)
  LSIM_LAYER_CASE(256, 24)
  LSIM_LAYER_CASE(256, 27)
  LSIM_LAYER_CASE(384, 16)
  LSIM_LAYER_CASE(384, 24)
  LSIM_LAYER_CASE(384, 27)
  LSIM_LAYER_CASE(512, 16)
  LSIM_LAYER_CASE(512, 24)
  LSIM_LAYER_CASE(512, 27)
  LSIM_LAYER_CASE(768, 16)
  LSIM_LAYER_CASE(768, 24)
  LSIM_LAYER_CASE(768, 27)
  LSIM_LAYER_CASE(1024, 16)
  LSIM_LAYER_CASE(1024, 24)
  LSIM_LAYER_CASE(1024, 27)
#undef LSIM_LAYER_CASE
  return hipErrorInvalidValue;
}

size_t layered_tile_lds(const DevCode& c, int G) { return tile_lds_bytes(c, G); }

hipError_t launch_mixed(const LayerShape* d_shapes, int nshapes, const int* d_tile_shape,
                        const int64_t* d_tile_local, int64_t ntiles, int threads,
                        size_t lds_bytes, const lsim_decode_params& p, const void* llr,
                        uint8_t* bits, float* lpost, uint32_t* state, int* counter,
                        int persistent, int grid, int dmax, hipStream_t s) {
  (void)nshapes;
  if (persistent) {
    reset_counter_kernel<<<1, 1, 0, s>>>(counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const unsigned g = persistent ? (unsigned)grid : (unsigned)ntiles;
  const int next_off = (int)((lds_bytes + 15) & ~(size_t)15);
  const size_t lds_all = (size_t)next_off + 16;
#define LSIM_MIXED_CASE(NT_, D_)                                                           \
  if (threads == NT_ && dmax <= D_) {                                                      \
    hipError_t e = require_lds_at_zero((const void*)mixed_kernel<NT_, D_>);               \
    if (e == hipSuccess) e = ensure_dyn_lds((const void*)mixed_kernel<NT_, D_>, lds_all);  \
    if (e != hipSuccess) return e;                                                         \
    mixed_kernel<NT_, D_><<<g, NT_, lds_all, s>>>(d_shapes, d_tile_shape, d_tile_local,    \
                                                  ntiles, (const float*)llr, bits, lpost,   \
                                                  state, counter, persistent, p.iters,     \
                                                  p.alpha, next_off);                      \
    return hipGetLastError();                                                              \
  }
  LSIM_MIXED_CASE(256, 16)
  LSIM_MIXED_CASE(256, 24)
  LSIM_MIXED_CASE(256, 27)
  LSIM_MIXED_CASE(384, 16)
  LSIM_MIXED_CASE(384, 24)
  LSIM_MIXED_CASE(384, 27)
  LSIM_MIXED_CASE(512, 16)
  LSIM_MIXED_CASE(512, 24)
  LSIM_MIXED_CASE(512, 27)
  LSIM_MIXED_CASE(768, 16)
  LSIM_MIXED_CASE(768, 24)
  LSIM_MIXED_CASE(768, 27)
  LSIM_MIXED_CASE(1024, 16)
  LSIM_MIXED_CASE(1024, 24)
  LSIM_MIXED_CASE(1024, 27)
#undef LSIM_MIXED_CASE
  return hipErrorInvalidValue;
}

}  // namespace lsim
