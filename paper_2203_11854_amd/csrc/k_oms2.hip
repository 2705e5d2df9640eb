// Flooding int8 offset min-sum, two codewords per workgroup in packed
// 16-bit lanes (or one, for codes whose pair state does not fit the LDS).
//
// Every message, channel value and posterior of codeword pair (2w, 2w+1)
// is held as a pair of signed 16-bit integers in one 32-bit word (low half:
// codeword 2w, high half: codeword 2w+1), in LDS and in registers, so one
// packed 16-bit instruction updates both codewords.  The single-codeword
// tile (W = 2 bytes per value) keeps one 16-bit value per edge and variable
// node in LDS, half the pair's state, and runs the same packed instructions
// with the high halves zero.  The values are the
// int8 decoder's exactly: inputs and variable-to-check messages saturate
// at +-sat (<= 127), check outputs are sign * max(min_excl - offset, 0),
// posteriors are channel value + sum of check outputs (at most
// 127 + 27 * 126, far inside 16 bits).
//
// Check update without an argmin: with m1 <= m2 the two smallest input
// magnitudes, the output magnitude for input v is m2 if |x_v| == m1 and m1
// otherwise.  When the minimum occurs twice m2 == m1, so this equals the
// first-argmin rule of the reference.  The selection is done branch-free as
// max(m1', m2' - 64 (|x_v| - m1)) (primes: after the offset; a nonzero
// difference is at least 1 and the magnitudes at most 127 - offset).
//
// Layout, schedule and addressing follow the sum-product flooding kernel:
// one row (check phase) or column (variable phase) per wavefront at a time,
// lane = lift index, messages in canonical edge order e*Z + r.
#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "lds.h"
#include "lsim_internal.h"

namespace lsim {

namespace {

typedef short s16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ s16x2 pk(int lo, int hi) {
  s16x2 v;
  v.x = (short)lo;
  v.y = (short)hi;
  return v;
}
__device__ __forceinline__ uint32_t bits_of(s16x2 v) { return __builtin_bit_cast(uint32_t, v); }
__device__ __forceinline__ s16x2 from_bits(uint32_t u) { return __builtin_bit_cast(s16x2, u); }
__device__ __forceinline__ s16x2 vmin(s16x2 a, s16x2 b) { return __builtin_elementwise_min(a, b); }
__device__ __forceinline__ s16x2 vmax(s16x2 a, s16x2 b) { return __builtin_elementwise_max(a, b); }

struct Oms2Args {
  const int8_t* llr;
  int64_t B;
  uint8_t* bits;
  float* lpost;
  const int8_t* q_in;
  int8_t* r_out;
  int8_t* q_out;
  int iters;
  int offset;
  int sat;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

// LDS of a tile: W bytes per edge and per variable node (4: a codeword
// pair, 2: one codeword).
__host__ __device__ inline size_t oms2_lds(const DevCode& c, int W = 4) {
  return align16((size_t)c.E * W) + align16((size_t)c.n_dec * W);
}

// Values of a tile at an LDS byte offset: the packed pair word (W = 4), or
// one 16-bit value in the low half with the high half zero (W = 2).
template <int W>
__device__ __forceinline__ s16x2 ld_val(int off) {
  if constexpr (W == 4) return lds_ld<s16x2>(off);
  return pk(lds_ld<short>(off), 0);
}
template <int W>
__device__ __forceinline__ void st_val(int off, s16x2 v) {
  if constexpr (W == 4)
    lds_st<s16x2>(off, v);
  else
    lds_st<short>(off, v.x);
}

// Tile `tile` of code c: codewords (2 tile, 2 tile + 1) for W = 4, codeword
// `tile` for W = 2.  ZC: compile-time lift size or 0 (read from the code).
// LDS: messages at byte 0, channel values at lam_b (the calling kernel has
// no static LDS).
template <int NT, int DMAX, int ZC, int W = 4>
__device__ __forceinline__ void oms2_pair(const DevCode& c, const Oms2Args& a, int64_t tile,
                                          unsigned char* smem) {
  constexpr int NW = NT / 64;
  (void)smem;
  const int lam_b = (int)align16((size_t)c.E * W);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = uni(tid >> 6);
  const int Z = ZC ? ZC : c.Z;
  const int zm = Z - 1;
  const bool zpow2 = (Z & zm) == 0;
  const int64_t b0 = W == 4 ? 2 * tile : tile;
  const bool has1 = W == 4 && b0 + 1 < a.B;
  const int sat = a.sat;
  const s16x2 psat = pk(sat, sat), nsat = pk(-sat, -sat);
  const s16x2 poff = pk(a.offset, a.offset), zero = pk(0, 0);

  // ---- channel values (saturated, sign flipped), zero or imported messages
  const int8_t* l0 = a.llr + b0 * (int64_t)c.e_tx;
  const int8_t* l1 = l0 + c.e_tx;
  for (int v = tid; v < c.n_dec; v += NT) {
    const int x = v - c.tx_lo;
    int y0 = 0, y1 = 0;
    if (x >= 0 && x < c.e_tx) {
      y0 = min(max(-(int)l0[x], -sat), sat);
      if (has1) y1 = min(max(-(int)l1[x], -sat), sat);
    }
    st_val<W>(lam_b + v * W, pk(y0, y1));
  }
  if (a.q_in) {
    const int8_t* q0 = a.q_in + b0 * (int64_t)c.E;
    const int8_t* q1 = q0 + c.E;
    for (int e = tid; e < c.E; e += NT) st_val<W>(e * W, pk(q0[e], has1 ? q1[e] : 0));
  } else {
    for (int e = tid; e < c.E; e += NT) st_val<W>(e * W, zero);
  }
  __syncthreads();

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
          s16x2 rv[DC];
          // byte offset of entry e's edge at lift cc: (e*Z + (cc - shift) mod Z) * W
          if (zpow2) {
            const int cc_b = vreg(cc * W), zm_b = vreg(zm * W);
#pragma unroll
            for (int q = 0; q < DC; ++q) {
              const int2 ce = ld_const(c.col_edge, cb + q);
              idx[q] = ((cc_b - ce.y * W) & zm_b) | (ce.x * W);
            }
          } else {
#pragma unroll
            for (int q = 0; q < DC; ++q) {
              const int2 ce = ld_const(c.col_edge, cb + q);
              int x = cc - ce.y;
              x += x < 0 ? Z : 0;
              idx[q] = (ce.x + x) * W;
            }
          }
#pragma unroll
          for (int q = 0; q < DC; ++q) rv[q] = ld_val<W>(idx[q]);
          s16x2 acc = ld_val<W>(lam_b + v * W);
#pragma unroll
          for (int q = 0; q < DC; ++q) acc += rv[q];
          if (write_q) {
            // staged so that independent edges interleave
#pragma unroll
            for (int q = 0; q < DC; ++q) rv[q] = acc - rv[q];
#pragma unroll
            for (int q = 0; q < DC; ++q) rv[q] = vmin(rv[q], psat);
#pragma unroll
            for (int q = 0; q < DC; ++q) rv[q] = vmax(rv[q], nsat);
#pragma unroll
            for (int q = 0; q < DC; ++q) st_val<W>(idx[q], rv[q]);
          }
          if (final_round) {
            if (a.bits && v < c.k) {
              a.bits[b0 * (int64_t)c.k + v] = acc.x < 0;
              if (has1) a.bits[(b0 + 1) * (int64_t)c.k + v] = acc.y < 0;
            }
            if (a.lpost) {
              a.lpost[b0 * (int64_t)c.n_dec + v] = (float)(-(int)acc.x);
              if (has1) a.lpost[(b0 + 1) * (int64_t)c.n_dec + v] = (float)(-(int)acc.y);
            }
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
        const int row_b = (e0 * Z + r) * W;
        with_degree<DMAX>(d, [&](auto deg) {
          constexpr int D = decltype(deg)::value;
          s16x2 x[D], ax[D];
#pragma unroll
          for (int q = 0; q < D; ++q) x[q] = ld_val<W>(row_b + q * Z * W);
          // sign parity in bits 15 and 31, the two smallest magnitudes
          uint32_t sx = 0;
          s16x2 m1 = pk(0x7fff, 0x7fff), m2 = m1;
#pragma unroll
          for (int q = 0; q < D; ++q) {
            sx ^= bits_of(x[q]);
            ax[q] = vmax(x[q], zero - x[q]);
            m2 = vmin(m2, vmax(m1, ax[q]));
            m1 = vmin(m1, ax[q]);
          }
          const s16x2 o1 = vmax(m1 - poff, zero), o2 = vmax(m2 - poff, zero);
          // staged so that independent edges interleave; neg is 0 or -1 per
          // half from the parity of the other inputs' signs
          s16x2 mag[D], neg[D];
#pragma unroll
          for (int q = 0; q < D; ++q) mag[q] = ax[q] - m1;
#pragma unroll
          for (int q = 0; q < D; ++q) neg[q] = from_bits(sx ^ bits_of(x[q])) >> 15;
#pragma unroll
          for (int q = 0; q < D; ++q) mag[q] = o2 - (mag[q] << 6);
#pragma unroll
          for (int q = 0; q < D; ++q) mag[q] = vmax(o1, mag[q]);
#pragma unroll
          for (int q = 0; q < D; ++q) mag[q] = mag[q] ^ neg[q];
#pragma unroll
          for (int q = 0; q < D; ++q) st_val<W>(row_b + q * Z * W, mag[q] - neg[q]);
        });
      }
    }
  };

  if (!a.q_in) {
    var_phase(true, false);  // q = channel value on every edge
    __syncthreads();
  }
  for (int it = 0; it < a.iters; ++it) {
    const bool last = it + 1 == a.iters;
    check_phase();
    __syncthreads();
    if (last && a.r_out) {
      int8_t* r0 = a.r_out + b0 * (int64_t)c.E;
      for (int e = tid; e < c.E; e += NT) {
        const s16x2 m = ld_val<W>(e * W);
        r0[e] = (int8_t)m.x;
        if (has1) r0[c.E + e] = (int8_t)m.y;
      }
      __syncthreads();
    }
    var_phase(!last || a.q_out != nullptr, last);
    __syncthreads();
  }
  if (a.q_out) {
    int8_t* q0 = a.q_out + b0 * (int64_t)c.E;
    for (int e = tid; e < c.E; e += NT) {
      const s16x2 m = ld_val<W>(e * W);
      q0[e] = (int8_t)m.x;
      if (has1) q0[c.E + e] = (int8_t)m.y;
    }
  }
}

__global__ void oms2_reset_counter_kernel(int* counter) { *counter = 0; }

template <int NT, int DMAX, int ZC, int W>
__global__ __launch_bounds__(NT) void oms2_kernel(DevCode c, Oms2Args a) {
  extern __shared__ __align__(16) unsigned char smem[];
  oms2_pair<NT, DMAX, ZC, W>(c, a, blockIdx.x, smem);
}

// Persistent decoder over a work list of (shape, codeword pair) items, as
// the layered mixed kernel: workgroups take items from a device counter
// (reset by oms2_reset_counter_kernel just before, so the pair of launches can
// be captured in a graph); the item taken by thread 0 is broadcast through
// the word at next_off of the dynamic LDS.
template <int NT, int DMAX>
__global__ __launch_bounds__(NT) void oms2_mixed_kernel(
    const LayerShape* __restrict__ shapes, const int* __restrict__ tile_shape,
    const int64_t* __restrict__ tile_local, int64_t ntiles, const int8_t* llr, uint8_t* bits,
    float* lpost, int* counter, int persistent, int iters, int offset, int sat, int next_off) {
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
    const LayerShape& sh = shapes[tile_shape[item]];
    Oms2Args a{llr + sh.llr_off, sh.count, bits ? bits + sh.bits_off : nullptr,
               lpost ? lpost + sh.app_off : nullptr, nullptr, nullptr, nullptr, iters, offset,
               sat};
    // a shape's tile is a codeword pair (G = 2) or one codeword (G = 1)
    if (sh.G == 2)
      oms2_pair<NT, DMAX, 0, 4>(sh.code, a, tile_local[item], smem);
    else
      oms2_pair<NT, DMAX, 0, 2>(sh.code, a, tile_local[item], smem);
    __syncthreads();
    if (!persistent) break;
  }
}

template <int NT, int DMAX, int ZC, int W>
hipError_t launch_tw(const DevCode& c, const Oms2Args& a, size_t lds, hipStream_t s) {
  const void* k = (const void*)oms2_kernel<NT, DMAX, ZC, W>;
  hipError_t e = require_lds_at_zero(k);
  if (e == hipSuccess) e = ensure_dyn_lds(k, lds);
  if (e != hipSuccess) return e;
  const unsigned grid = (unsigned)(W == 4 ? (a.B + 1) / 2 : a.B);
  oms2_kernel<NT, DMAX, ZC, W><<<grid, NT, lds, s>>>(c, a);
  return hipGetLastError();
}

template <int NT, int DMAX, int ZC>
hipError_t launch_t(const DevCode& c, const Oms2Args& a, int W, hipStream_t s) {
  return W == 4 ? launch_tw<NT, DMAX, ZC, 4>(c, a, oms2_lds(c, 4), s)
                : launch_tw<NT, DMAX, ZC, 2>(c, a, oms2_lds(c, 2), s);
}

}  // namespace

size_t oms2_lds_bytes(const DevCode& c, int cw_per_tile) {
  return oms2_lds(c, cw_per_tile == 2 ? 4 : 2);
}

template <int NT, int DMAX>
hipError_t launch_mixed_oms_t(const LayerShape* d_shapes, const int* d_tile_shape,
                              const int64_t* d_tile_local, int64_t ntiles, size_t lds,
                              const lsim_decode_params& p, const int8_t* llr, uint8_t* bits,
                              float* lpost, int* counter, int persistent, int grid,
                              hipStream_t s) {
  const void* k = (const void*)oms2_mixed_kernel<NT, DMAX>;
  const int next_off = (int)align16(lds);
  const size_t lds_all = (size_t)next_off + 16;
  hipError_t e = require_lds_at_zero(k);
  if (e == hipSuccess) e = ensure_dyn_lds(k, lds_all);
  if (e != hipSuccess) return e;
  if (persistent) {
    oms2_reset_counter_kernel<<<1, 1, 0, s>>>(counter);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const unsigned g = persistent ? (unsigned)grid : (unsigned)ntiles;
  oms2_mixed_kernel<NT, DMAX><<<g, NT, lds_all, s>>>(d_shapes, d_tile_shape, d_tile_local, ntiles,
                                                     llr, bits, lpost, counter, persistent,
                                                     p.iters, (int)p.offset, p.sat, next_off);
  return hipGetLastError();
}

hipError_t launch_mixed_oms(const LayerShape* d_shapes, const int* d_tile_shape,
                            const int64_t* d_tile_local, int64_t ntiles, int threads, size_t lds,
                            const lsim_decode_params& p, const int8_t* llr, uint8_t* bits,
                            float* lpost, int* counter, int persistent, int grid, int dmax,
                            hipStream_t s) {
#define LSIM_OMS2_MIXED(NT_, D_)                                                               \
  if (threads == NT_ && dmax <= D_)                                                            \
    return launch_mixed_oms_t<NT_, D_>(d_shapes, d_tile_shape, d_tile_local, ntiles, lds, p,   \
                                       llr, bits, lpost, counter, persistent, grid, s);
  LSIM_OMS2_MIXED(256, 16)
  LSIM_OMS2_MIXED(256, 24)
  LSIM_OMS2_MIXED(256, 32)
  LSIM_OMS2_MIXED(512, 16)
  LSIM_OMS2_MIXED(512, 24)
  LSIM_OMS2_MIXED(512, 32)
  LSIM_OMS2_MIXED(1024, 16)
  LSIM_OMS2_MIXED(1024, 24)
  LSIM_OMS2_MIXED(1024, 32)
#undef LSIM_OMS2_MIXED
  return hipErrorInvalidValue;
}

hipError_t launch_oms2(const DevCode& c, const lsim_decode_params& p, const int8_t* llr, int64_t B,
                       uint8_t* bits, float* lpost, const int8_t* q_in, int8_t* r_out,
                       int8_t* q_out, hipStream_t s, std::string* why) {
  // a codeword pair per workgroup when its state fits the LDS, else one
  const int W = oms2_lds(c, 4) <= 160 * 1024 ? 4 : 2;
  const size_t lds = oms2_lds(c, W);
  if (lds > 160 * 1024) {
    *why = "min-sum decoder state (" + std::to_string(lds) + " B) exceeds the 160 KiB LDS";
    return hipSuccess;
  }
  Oms2Args a{llr, B, bits, lpost, q_in, r_out, q_out, p.iters, (int)p.offset, p.sat};
  const int nt = p.threads ? p.threads : 512;
  const int dmax = c.max_row_deg > c.max_col_deg ? c.max_row_deg : c.max_col_deg;
  if (c.Z == 128 && nt == 512 && dmax <= 16) return launch_t<512, 16, 128>(c, a, W, s);
  if (c.Z == 128 && nt == 512 && dmax <= 24) return launch_t<512, 24, 128>(c, a, W, s);
#define LSIM_OMS2_CASE(NT_, D_) \
  if (nt == NT_ && dmax <= D_) return launch_t<NT_, D_, 0>(c, a, W, s);
  LSIM_OMS2_CASE(256, 16)
  LSIM_OMS2_CASE(256, 24)
  LSIM_OMS2_CASE(256, 32)
  LSIM_OMS2_CASE(512, 16)
  LSIM_OMS2_CASE(512, 24)
  LSIM_OMS2_CASE(512, 32)
  LSIM_OMS2_CASE(1024, 16)
  LSIM_OMS2_CASE(1024, 24)
  LSIM_OMS2_CASE(1024, 32)
#undef LSIM_OMS2_CASE
  return hipErrorInvalidValue;
}

}  // namespace lsim
