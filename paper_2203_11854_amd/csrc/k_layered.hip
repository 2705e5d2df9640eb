// Layered normalized min-sum (FP32) decoder: one launch over a batch of one
// code (the tile decoder and its data layout are in layered_tile.h).
#include <map>
#include <mutex>
#include <tuple>

#include "layered_tile.h"

namespace lsim {

using namespace layered;

namespace {

template <int NT, int DMAX, int WPE>
__global__ __launch_bounds__(NT) __attribute__((amdgpu_waves_per_eu(WPE))) void layered_kernel(
    DevCode c, int G, TileIO io, int iters, float alpha) {
  decode_tile<NT, DMAX, WPE == 6>(c, G, blockIdx.x, io, iters, alpha);
}

}  // namespace

size_t layered_state_words(const DevCode& c, int64_t B) { return (size_t)B * c.rows * 3 * c.Z; }

size_t layered_tile_lds(const DevCode& c, int G, int K) { return tile_lds_bytes(c, G, K); }

// Rows whose check records stay in LDS.  `want` 0: as many as fit in the LDS
// a workgroup can have without fewer workgroups per CU than with the shared
// posteriors alone; -1: none; k > 0: k rows (an error if they do not fit).
hipError_t layered_lds_rows(const void* kernel, const DevCode& c, int G, int threads, int want,
                            int* K, std::string* why) {
  const size_t base = tile_lds_bytes(c, G), per_row = (size_t)G * c.Z * 16;
  *K = 0;
  if (want < 0) return hipSuccess;
  if (want > 0) {
    if (want > c.rows || base + want * per_row > kLdsBytes)
      *why = "lds_rows: the check records of that many rows do not fit the LDS";
    else
      *K = want;
    return hipSuccess;
  }
  static std::mutex mu;
  static std::map<std::tuple<const void*, int, size_t, size_t, int>, int> cache;
  const auto key = std::make_tuple(kernel, threads, base, per_row, c.rows);
  std::lock_guard<std::mutex> lock(mu);
  auto it = cache.find(key);
  if (it != cache.end()) {
    *K = it->second;
    return hipSuccess;
  }
  int occ0 = 0;
  hipError_t e = ensure_dyn_lds(kernel, kLdsBytes);  // the occupancy query honours the limit
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ0, kernel, threads, base);
  if (e != hipSuccess) return e;
  int k = 0;
  if (occ0 > 0) {
    const size_t budget = kLdsBytes / occ0;
    k = (int)std::min<size_t>(c.rows, budget > base ? (budget - base) / per_row : 0);
    for (; k > 0; --k) {
      int occ = 0;
      e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kernel, threads, base + k * per_row);
      if (e != hipSuccess) return e;
      if (occ >= occ0) break;
    }
  }
  cache[key] = k;
  *K = k;
  return hipSuccess;
}

// Workgroups of whole multiples of four wavefronts spread evenly over a CU's
// four SIMDs; among 256, 512, 768 and 1024 threads take the one whose tile
// (threads / Z codewords, as many as the LDS holds) leaves the fewest lanes
// idle, the smallest on a tie (more, smaller workgroups balance better:
// 0.94 ms at 256 against 0.99 ms at 512 threads for the BG2 code at Z = 128).
int layered_default_threads(const DevCode& c) {
  int best = 1024;
  double best_u = -1.0;
  for (int nt : {256, 512, 768, 1024}) {
    if (nt < c.Z) continue;
    int G = nt / c.Z;
    while (G > 1 && tile_lds_bytes(c, G) > kLdsBytes) --G;
    const double u = (double)G * c.Z / nt;
    if (u > best_u + 1e-9) {
      best_u = u;
      best = nt;
    }
  }
  return best;
}

// The kernel instance of a launch shape.
static const void* layered_instance(int nt, int D, int wpe) {
#define LSIM_LAYER_PTR(NT_, D_, W_) \
  if (nt == NT_ && D == D_ && wpe == W_) return (const void*)layered_kernel<NT_, D_, W_>;
  LSIM_LAYERED_INSTANCES_W(LSIM_LAYER_PTR)
#undef LSIM_LAYER_PTR
  return nullptr;
}

static int degree_class(const DevCode& c) {
  return c.max_row_deg <= 16 ? 16 : c.max_row_deg <= 24 ? 24 : 27;
}

// Register budget of a launch: 6 wavefronts per SIMD when that at least
// doubles the workgroups per CU the shared posteriors allow.
hipError_t layered_budget(int nt, int D, size_t base, int* wpe) {
  int occ1 = 0, occ6 = 0;
  const void* k1 = layered_instance(nt, D, 1);
  const void* k6 = layered_instance(nt, D, 6);
  if (!k1 || !k6) return hipErrorInvalidValue;
  hipError_t e = ensure_dyn_lds(k1, kLdsBytes);
  if (e == hipSuccess) e = ensure_dyn_lds(k6, kLdsBytes);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ1, k1, nt, base);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ6, k6, nt, base);
  *wpe = occ6 >= 2 * occ1 ? 6 : 1;
  return e;
}

hipError_t layered_launch_shape(const DevCode& c, const lsim_decode_params& p, int* nt, int* G,
                                int* K, int* wpe, std::string* why) {
  *nt = p.threads ? p.threads : layered_default_threads(c);
  if (c.n_deg1_inner || c.rows < 3) {
    *why = c.rows < 3 ? kLayeredRowsMsg : kLayeredDeg1Msg;
    return hipSuccess;
  }
  if (c.Z > *nt) {
    *why = "layered decoder needs threads >= Z";
    return hipSuccess;
  }
  *G = *nt / c.Z;
  while (*G > 1 && tile_lds_bytes(c, *G) > kLdsBytes) --*G;
  if (tile_lds_bytes(c, *G) > kLdsBytes) {
    *why = "layered decoder posteriors exceed the 160 KiB LDS";
    return hipSuccess;
  }
  const int D = degree_class(c);
  hipError_t e = layered_budget(*nt, D, tile_lds_bytes(c, *G), wpe);
  if (e != hipSuccess) return e;
  return layered_lds_rows(layered_instance(*nt, D, *wpe), c, *G, *nt, p.lds_rows, K, why);
}

hipError_t launch_layered(const DevCode& c, const lsim_decode_params& p, const float* llr,
                          int64_t B, uint8_t* bits, float* lpost, float* r_out, uint32_t* state,
                          hipStream_t s, std::string* why) {
  int nt = 0, G = 1, K = 0, wpe = 1;
  hipError_t e = layered_launch_shape(c, p, &nt, &G, &K, &wpe, why);
  if (e != hipSuccess || !why->empty()) return e;
  const unsigned grid = (unsigned)((B + G - 1) / G);
  const int D = degree_class(c);
  const size_t lds = tile_lds_bytes(c, G, K);
  TileIO io{llr, bits, lpost, r_out, state, B, K};
#define LSIM_LAYER_CASE(NT_, D_, W_)                                                   \
  if (nt == NT_ && D == D_ && wpe == W_) {                                             \
    const void* k = (const void*)layered_kernel<NT_, D_, W_>;                          \
    e = require_lds_at_zero(k);                                                        \
    if (e == hipSuccess) e = ensure_dyn_lds(k, lds);                                   \
    if (e != hipSuccess) return e;                                                     \
    layered_kernel<NT_, D_, W_><<<grid, NT_, lds, s>>>(c, G, io, p.iters, p.alpha);    \
    return hipGetLastError();                                                          \
  }
  LSIM_LAYERED_INSTANCES_W(LSIM_LAYER_CASE)
#undef LSIM_LAYER_CASE
  return hipErrorInvalidValue;
}

}  // namespace lsim
