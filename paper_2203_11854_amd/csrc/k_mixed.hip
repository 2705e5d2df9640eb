// Persistent mixed-shape layered decoder: codewords of several codes in one
// launch (the tile decoder and its data layout are in layered_tile.h).
#include "layered_tile.h"

namespace lsim {

using namespace layered;

namespace {

// Persistent decoder over a work list of (shape, tile) items.  Workgroups
// take items from a device counter until the list is drained; the counter
// is reset by reset_counter_kernel launched just before, so the pair can be
// captured in a graph.
template <int NT, int DMAX, int WPE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void mixed_kernel(const LayerShape* __restrict__ shapes,
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
    io.lds_rows = sh.lds_rows;
    decode_tile<NT, DMAX, false>(sh.code, sh.G, tile_local[item], io, iters, alpha);
    __syncthreads();
    if (!persistent) break;
  }
}

__global__ void reset_counter_kernel(int* counter) { *counter = 0; }

}  // namespace

hipError_t launch_mixed(const LayerShape* d_shapes, int nshapes, const int* d_tile_shape,
                        const int64_t* d_tile_local, int64_t ntiles, int threads,
                        size_t lds_bytes, const lsim_decode_params& p, const void* llr,
                        uint8_t* bits, float* lpost, uint32_t* state, int* counter,
                        int persistent, int grid, int dmax, int wpe, hipStream_t s) {
  (void)nshapes;
  if (persistent) {
    reset_counter_kernel<<<1, 1, 0, s>>>(counter);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const unsigned g = persistent ? (unsigned)grid : (unsigned)ntiles;
  const int next_off = (int)align16(lds_bytes);
  const size_t lds_all = (size_t)next_off + 16;
  const int D = dmax <= 16 ? 16 : dmax <= 24 ? 24 : 27;
#define LSIM_MIXED_CASE(NT_, D_, W_)                                                   \
  if (threads == NT_ && D == D_ && wpe == W_) {                                        \
    const void* k = (const void*)mixed_kernel<NT_, D_, W_>;                            \
    hipError_t e = require_lds_at_zero(k);                                             \
    if (e == hipSuccess) e = ensure_dyn_lds(k, lds_all);                               \
    if (e != hipSuccess) return e;                                                     \
    mixed_kernel<NT_, D_, W_><<<g, NT_, lds_all, s>>>(d_shapes, d_tile_shape,          \
                                                      d_tile_local, ntiles,            \
                                                      (const float*)llr, bits, lpost,  \
                                                      state, counter, persistent,      \
                                                      p.iters, p.alpha, next_off);     \
    return hipGetLastError();                                                          \
  }
  LSIM_LAYERED_INSTANCES_W(LSIM_MIXED_CASE)
#undef LSIM_MIXED_CASE
  return hipErrorInvalidValue;
}

hipError_t mixed_occupancy(int threads, int dmax, int wpe, size_t lds, int* occ) {
  const size_t lds_all = align16(lds) + 16;
  const int D = dmax <= 16 ? 16 : dmax <= 24 ? 24 : 27;
  *occ = 0;
#define LSIM_MIXED_OCC(NT_, D_, W_)                                                   \
  if (threads == NT_ && D == D_ && wpe == W_) {                                       \
    const void* k = (const void*)mixed_kernel<NT_, D_, W_>;                           \
    hipError_t e = ensure_dyn_lds(k, kLdsBytes); /* the query honours the limit */    \
    if (e != hipSuccess) return e;                                                    \
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(occ, k, NT_, lds_all);        \
  }
  LSIM_LAYERED_INSTANCES_W(LSIM_MIXED_OCC)
#undef LSIM_MIXED_OCC
  return hipErrorInvalidValue;
}

}  // namespace lsim
