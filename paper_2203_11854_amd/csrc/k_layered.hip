// Layered normalized min-sum (FP32) decoder: one launch over a batch of one
// code (the tile decoder and its data layout are in layered_tile.h).
#include "layered_tile.h"

namespace lsim {

using namespace layered;

namespace {

template <int NT, int DMAX>
__global__ __launch_bounds__(NT) void layered_kernel(DevCode c, int G, TileIO io, int iters,
                                                     float alpha) {
  decode_tile<NT, DMAX>(c, G, blockIdx.x, io, iters, alpha);
}

}  // namespace

size_t layered_state_words(const DevCode& c, int64_t B) { return (size_t)B * c.rows * 4 * c.Z; }

size_t layered_tile_lds(const DevCode& c, int G) { return tile_lds_bytes(c, G); }

// Workgroups of whole multiples of four wavefronts spread evenly over a CU's
// four SIMDs; among 256, 512, 768 and 1024 threads take the one whose tile
// (threads / Z codewords, as many as the LDS holds) leaves the fewest lanes
// idle, nearest to 512 threads on a tie.
int layered_default_threads(const DevCode& c) {
  int best = 1024;
  double best_u = -1.0;
  for (int nt : {512, 256, 768, 1024}) {
    if (nt < c.Z) continue;
    int G = nt / c.Z;
    while (G > 1 && tile_lds_bytes(c, G) > 160 * 1024) --G;
    const double u = (double)G * c.Z / nt;
    if (u > best_u + 1e-9) {
      best_u = u;
      best = nt;
    }
  }
  return best;
}

hipError_t launch_layered(const DevCode& c, const lsim_decode_params& p, const float* llr,
                          int64_t B, uint8_t* bits, float* lpost, float* r_out, uint32_t* state,
                          hipStream_t s, std::string* why) {
  const int nt = p.threads ? p.threads : layered_default_threads(c);
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
  TileIO io{llr, bits, lpost, r_out, reinterpret_cast<uint4*>(state), B};
  const unsigned grid = (unsigned)((B + G - 1) / G);
  const int dmax = c.max_row_deg;
  const int D = dmax <= 16 ? 16 : dmax <= 24 ? 24 : 27;
#define LSIM_LAYER_CASE(NT_, D_)                                                    \
  if (nt == NT_ && D == D_ ) {                                                \
    const void* k = (const void*)layered_kernel<NT_, D_>;                           \
    hipError_t e = require_lds_at_zero(k);                                              \
    if (e == hipSuccess) e = ensure_dyn_lds(k, lds);                                    \
    if (e != hipSuccess) return e;                                                      \
    layered_kernel<NT_, D_><<<grid, NT_, lds, s>>>(c, G, io, p.iters, p.alpha);     \
    return hipGetLastError();                                                           \
  }
  LSIM_LAYERED_INSTANCES(LSIM_LAYER_CASE)
#undef LSIM_LAYER_CASE
  return hipErrorInvalidValue;
}

}  // namespace lsim
