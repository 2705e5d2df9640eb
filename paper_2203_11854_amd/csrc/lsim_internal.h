// Internal declarations shared by the host API (api.cpp) and the kernel
// translation units.  Not part of the C-ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/lsim.h"
#include "devcode.h"

struct lsim_code {
  lsim::DevCode dev;
  lsim_code_info info;
  std::vector<int16_t> base;
  std::vector<int> row_ptr, ent_col, ent_shift, col_ptr, col_ent;
  // layered schedule: per row the LDS (multi-check) columns it meets and its
  // private column's (LLR offset, shift); the current visiting order and
  // where the schedule table sits in dmem (in ints)
  std::vector<std::vector<int>> row_lds_cols;
  std::vector<int> row_pch;
  std::vector<int> layer_order;
  size_t layer_pos_off = 0;
  void* dmem = nullptr;
  int device = 0;
};

namespace lsim {

void set_error(const std::string& msg);

// Raises a kernel's dynamic-LDS limit to at least `bytes` (once per kernel
// and size; thread-safe).
hipError_t ensure_dyn_lds(const void* kernel, size_t bytes);

// Kernels that address their dynamic LDS by byte offset from 0 (lds.h) are
// valid only without static LDS, which would come first; checked once per
// kernel from its attributes.
hipError_t require_lds_at_zero(const void* kernel);

// Flooding decoders (k_flood.hip)
hipError_t launch_flood(const DevCode& c, const lsim_decode_params& p, const void* llr, int64_t B,
                        uint8_t* bits, float* lpost, const void* q_in, void* r_out, void* q_out,
                        hipStream_t s, std::string* why);
size_t flood_lds_bytes(const DevCode& c, int algo);
// Packed two-codeword int8 offset min-sum (k_oms2.hip); launch_flood routes
// LSIM_OMS_I8 here.
hipError_t launch_oms2(const DevCode& c, const lsim_decode_params& p, const int8_t* llr, int64_t B,
                       uint8_t* bits, float* lpost, const int8_t* q_in, int8_t* r_out,
                       int8_t* q_out, hipStream_t s, std::string* why);
// LDS of one tile: a codeword pair (cw_per_tile 2) or one codeword (1).
size_t oms2_lds_bytes(const DevCode& c, int cw_per_tile = 2);

// Device address (on the current device) and size of the library-owned
// scratch of lsim_decode_noalloc (k_noalloc.hip); looked up once per device.
hipError_t noalloc_scratch(void** ptr, size_t* bytes);

// Layered decoder and mixed batches (k_layered.hip)
struct LayerShape {
  DevCode code;
  int G;               // codewords per tile
  int64_t count;       // codewords of this shape
  int64_t tile0;       // first global tile index of this shape
  int64_t llr_off;     // offset (elements) of the shape's LLRs in the concatenated input
  int64_t bits_off;    // offset of the shape's bits
  int64_t app_off;     // offset of the shape's posteriors
  int64_t state_off;   // offset (in 32-bit words) of the shape's check state
  int lds_rows;        // layered decoder: rows whose check records stay in LDS
};
// Three words per check record: [B][rows][Z][3].
size_t layered_state_words(const DevCode& c, int64_t B);
// The layered decoder takes the message of a degree-one variable node to be
// its channel value, which it reads per row; a code with such a column that
// does not close its row is outside that layout.
constexpr const char* kLayeredDeg1Msg =
    "layered decoder: a column of degree one must be the last entry of its row";
// Its check records are read back two layers after they are stored, so it
// needs three layers (code creation already requires three rows).
constexpr const char* kLayeredRowsMsg = "layered decoder: fewer than three decoded rows";
size_t layered_tile_lds(const DevCode& c, int G, int K = 0);
// Launch shape of the layered decoder: threads, codewords per workgroup,
// rows whose check records stay in LDS, register budget (k_layered.hip).
hipError_t layered_launch_shape(const DevCode& c, const lsim_decode_params& p, int* nt, int* G,
                                int* K, int* wpe, std::string* why);
// Rows whose check records a launch keeps in LDS (k_layered.hip).
hipError_t layered_lds_rows(const void* kernel, const DevCode& c, int G, int threads, int want,
                            int* K, std::string* why);
int layered_default_threads(const DevCode& c);
hipError_t launch_layered(const DevCode& c, const lsim_decode_params& p, const float* llr,
                          int64_t B, uint8_t* bits, float* lpost, float* r_out, uint32_t* state,
                          hipStream_t s, std::string* why);
hipError_t launch_mixed_oms(const LayerShape* d_shapes, const int* d_tile_shape,
                            const int64_t* d_tile_local, int64_t ntiles, int threads, size_t lds,
                            const lsim_decode_params& p, const int8_t* llr, uint8_t* bits,
                            float* lpost, int* counter, int persistent, int grid, int dmax,
                            hipStream_t s);
hipError_t launch_mixed(const LayerShape* d_shapes, int nshapes, const int* d_tile_shape,
                        const int64_t* d_tile_local, int64_t ntiles, int threads,
                        size_t lds_bytes, const lsim_decode_params& p, const void* llr,
                        uint8_t* bits, float* lpost, uint32_t* state, int* counter,
                        int persistent, int grid, int dmax, int wpe, hipStream_t s);
// Workgroups per CU of the mixed layered kernel (register budget wpe: 1 or
// 6 wavefronts per SIMD) with `lds` bytes of tile LDS.
hipError_t mixed_occupancy(int threads, int dmax, int wpe, size_t lds, int* occ);

// Peak-rate probes (k_probe.hip)
hipError_t launch_probe(int kind, const void* src, void* dst, int64_t bytes, int rounds, int grid,
                        hipStream_t s, int64_t* units);

// Pipeline kernels (k_pipeline.hip)
hipError_t launch_source_bits(uint64_t seed, int64_t cw0, int64_t B, int64_t k, uint8_t* u,
                              hipStream_t s);
hipError_t launch_encode(const DevCode& c, const uint8_t* u, int64_t B, uint8_t* cw,
                         hipStream_t s);
// Source bits -> encoder -> map + AWGN -> demapper for one codeword per
// workgroup (cw and y nullable; q instead of llr for int8 output).
hipError_t launch_link_tx(const DevCode& c, int m, int method, uint64_t seed, int64_t cw0,
                          int64_t B, const float* no, uint8_t* u, uint8_t* cw, float* y,
                          float* llr, int8_t* q, float scale, int sat, hipStream_t s);
hipError_t launch_map_awgn(const DevCode& c, int m, const uint8_t* cw, const float* no,
                           uint64_t seed, int64_t cw0, int64_t B, float* y, hipStream_t s);
hipError_t launch_demap(int m, int method, const float* y, const float* no, int64_t B, int64_t S,
                        float* llr, int8_t* q, float scale, int sat, hipStream_t s);
hipError_t launch_quantize(const float* llr, int64_t n, float scale, int sat, int8_t* q,
                           hipStream_t s);
hipError_t launch_count_errors(const uint8_t* ref, int64_t ref_stride, const uint8_t* hat,
                               int64_t B, int64_t k, const int32_t* bin, int nbins,
                               int64_t* counts, hipStream_t s);
hipError_t launch_hard_bits(const float* L, int64_t stride, int64_t B, int64_t k, uint8_t* bits,
                            hipStream_t s);
hipError_t launch_syndrome(const DevCode& c, const uint8_t* cw, int64_t stride, int64_t B,
                           int32_t* unsat, hipStream_t s);

// Differentiable forms (k_wbp.hip, k_ndm.hip)
size_t wbp_work_bytes(const DevCode& c, int T, int64_t B);
hipError_t launch_wbp_forward(const DevCode& c, int T, const float* w, const float* llr,
                              int64_t B, float llr_max, float* ckpt, float* lpost, hipStream_t s,
                              std::string* why);
hipError_t launch_wbp_backward(const DevCode& c, int T, const float* w, const float* llr,
                               const float* ckpt, int64_t B, float llr_max, const float* gpost,
                               float* gllr, float* gw, void* work, hipStream_t s,
                               std::string* why);
size_t ndm_work_bytes(int64_t B, int64_t S);
hipError_t launch_ndm_forward(const float* params, const float* y, const float* no, int64_t B,
                              int64_t S, float* llr, hipStream_t s);
hipError_t launch_ndm_backward(const float* params, const float* y, const float* no,
                               const float* gllr, int64_t B, int64_t S, float* gparams,
                               float* gy, void* work, hipStream_t s);
size_t bce_work_bytes(int64_t B, int64_t n);
hipError_t launch_bce_grad(const float* lpost, const uint8_t* c, int64_t c_stride, int64_t B,
                           int64_t n, float scale, float* g, float* loss, void* work,
                           hipStream_t s);
// Polar codes (k_polar.hip)
struct DevPolar {
  int n, N, K, r;
  const uint8_t* mask;      // N: 1 at information indices
  const int16_t* info;      // K: information indices, increasing
  const uint32_t* crc_tab;  // K - r: CRC remainder contributed by each data bit
};
size_t polar_decode_lds(int list, int N, int K);
hipError_t launch_polar_decode(const DevPolar& pc, int list, int use_crc, const float* llr,
                               int64_t B, uint8_t* bits, float* pm, hipStream_t s);
hipError_t launch_polar_encode(const DevPolar& pc, const uint8_t* data, int64_t B, uint8_t* x,
                               hipStream_t s);
// Demapper with prior, EXIT pieces (k_prior.hip)
hipError_t launch_demap_prior(int m, bool exact, const float* y, const float* no, const float* la,
                              int64_t B, int64_t S, bool extrinsic, float* out, hipStream_t s);
hipError_t launch_apriori(const DevCode& c, const uint8_t* cw, const float* sigma, uint64_t seed,
                          int64_t cw0, int64_t B, float* la, hipStream_t s);
hipError_t launch_mutual_info(const float* L, int64_t L_stride, const uint8_t* c, int64_t c_stride,
                              int64_t B, int64_t n, const int32_t* bin, int nbins, float* mi_cw,
                              double* mi_bins, hipStream_t s);
hipError_t launch_extrinsic(const DevCode& c, const float* app, const float* lin, float llr_max,
                            int64_t B, float* out, hipStream_t s);
// Trainable constellation (k_const.hip)
hipError_t launch_map_points(const DevCode& c, int m, const float* pts, const uint8_t* cw,
                             const float* no, uint64_t seed, int64_t cw0, int64_t B, float* y,
                             hipStream_t s);
size_t points_work_bytes(const DevCode& c, int m, int64_t B);
hipError_t launch_points_grad(const DevCode& c, int m, const float* pts, const uint8_t* cw,
                              const float* gy, int64_t B, float* gp, void* work, hipStream_t s);
hipError_t launch_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr,
                       float b1, float b2, float eps, int step, hipStream_t s);

}  // namespace lsim
