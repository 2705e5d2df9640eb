// C-ABI entry points of liblsim: host-side validation, code objects and
// dispatch to the HIP kernels.  See include/lsim.h for the contract of each
// call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include "lsim_internal.h"

namespace lsim {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

}  // namespace lsim

using lsim::DevCode;
using lsim::set_error;

namespace {

lsim_status fail(lsim_status st, const std::string& msg) {
  set_error(msg);
  return st;
}

lsim_status dev_status(hipError_t e, const char* what) {
  if (e == hipSuccess) return LSIM_OK;
  set_error(std::string(what) + ": " + hipGetErrorString(e));
  return e == hipErrorOutOfMemory ? LSIM_E_NOMEM : LSIM_E_DEVICE;
}

hipStream_t as_stream(lsim_stream s) { return reinterpret_cast<hipStream_t>(s); }

// Checks that the parity part of `base` has the structure of `family`.
bool check_family(const std::vector<int16_t>& H, int mb, int nb, int family, std::string* why) {
  const int kb = nb - mb;
  auto at = [&](int i, int j) { return (int)H[(size_t)i * nb + j]; };
  const int m = family == LSIM_FAMILY_11N ? mb : 4;
  if (m < 3 || m > mb) {
    *why = "too few rows for the dual-diagonal parity part";
    return false;
  }
  const int mid = m / 2;
  for (int i = 0; i < mb; ++i) {
    for (int j = kb; j < nb; ++j) {
      int want = -1;
      const int pj = j - kb;
      // extension rows of the BG shape may touch the core parity columns
      if (family == LSIM_FAMILY_BG && i >= 4 && pj < 4) continue;
      if (pj == 0) {
        if (i == 0 || i == m - 1) want = 1;
        else if (i == mid) want = 0;
      } else if (pj < m) {
        if (i == pj - 1 || i == pj) want = 0;
      } else {
        if (i == pj) want = 0;
      }
      if (at(i, j) != want) {
        *why = "parity column " + std::to_string(j) + " row " + std::to_string(i) +
               " does not match the family layout";
        return false;
      }
    }
    if (family == LSIM_FAMILY_BG && i >= 4) {
      // extension rows touch only columns < kb+4 besides their own
      for (int j = kb + 4; j < nb; ++j)
        if (j != kb + i && at(i, j) >= 0) {
          *why = "extension row reaches a later parity column";
          return false;
        }
    }
  }
  return true;
}

std::vector<int> make_tasks(int n, int Z, const std::vector<int>& deg) {
  std::vector<int> order(n);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return deg[a] > deg[b]; });
  std::vector<int> tasks;
  for (int idx : order)
    for (int l0 = 0; l0 < Z; l0 += 64) tasks.push_back((idx << 16) | l0);
  return tasks;
}

bool is_pow2_scale(float s) {
  if (!(s > 0.f) || !std::isfinite(s)) return false;
  int e;
  float f = std::frexp(s, &e);
  return f == 0.5f;
}

lsim_status check_params(const lsim_code* code, const lsim_decode_params* p) {
  if (!code || !p) return fail(LSIM_E_INVAL, "null code or params");
  if (p->iters < 1 || p->iters > 1000) return fail(LSIM_E_INVAL, "iters must be in 1..1000");
  switch (p->algo) {
    case LSIM_SPA_F32:
      if (!(p->llr_max > 0.f)) return fail(LSIM_E_INVAL, "llr_max must be > 0");
      break;
    case LSIM_OMS_I8:
      if (p->sat < 1 || p->sat > 127) return fail(LSIM_E_INVAL, "sat must be in 1..127");
      if (!(p->offset >= 0.f) || p->offset != std::floor(p->offset) || p->offset > 127.f)
        return fail(LSIM_E_INVAL, "offset must be a non-negative integer");
      break;
    case LSIM_NMS_F32:
      if (!(p->alpha > 0.f && p->alpha <= 1.f)) return fail(LSIM_E_INVAL, "alpha must be in (0,1]");
      break;
    default:
      return fail(LSIM_E_INVAL, "unknown algo");
  }
  const int t = p->threads;
  const bool layered_ok = t == 384 || t == 768;
  if (t != 0 && t != 256 && t != 512 && t != 1024 && !(layered_ok && p->algo == LSIM_NMS_F32))
    return fail(LSIM_E_INVAL, "threads must be 0, 256, 512 or 1024 (384, 768 also for NMS)");
  return LSIM_OK;
}

}  // namespace

extern "C" {

const char* lsim_last_error(void) { return lsim::g_err.c_str(); }

const char* lsim_version(void) { return "lsim 0.1 gfx950"; }

lsim_status lsim_code_create(const int16_t* base, int mb, int nb, int Z, int family,
                             int n_punct_cols, int64_t e_tx, lsim_code** out) {
  if (!base || !out) return fail(LSIM_E_INVAL, "null base or out");
  *out = nullptr;
  if (mb < 1 || nb <= mb || mb > 4096 || nb > 4096) return fail(LSIM_E_INVAL, "bad mb/nb");
  if (Z < 1) return fail(LSIM_E_INVAL, "Z must be >= 1");
  if (Z > 1024) return fail(LSIM_E_UNSUPPORTED, "Z > 1024");
  if (family != LSIM_FAMILY_11N && family != LSIM_FAMILY_BG)
    return fail(LSIM_E_INVAL, "unknown family");
  const int kb = nb - mb;
  if (n_punct_cols < 0 || n_punct_cols > kb) return fail(LSIM_E_INVAL, "bad n_punct_cols");
  const int64_t tx_lo = (int64_t)n_punct_cols * Z;
  if (e_tx < 1 || tx_lo + e_tx > (int64_t)nb * Z) return fail(LSIM_E_INVAL, "bad e_tx");
  std::vector<int16_t> H(base, base + (size_t)mb * nb);
  for (int16_t v : H)
    if (v < -1 || v >= Z) return fail(LSIM_E_INVAL, "shift out of [-1, Z)");
  std::string why;
  if (!check_family(H, mb, nb, family, &why)) return fail(LSIM_E_INVAL, why);

  // decoded part: core rows plus extension rows whose own column is sent
  int rows = mb, cols = nb;
  if (family == LSIM_FAMILY_BG) {
    const int64_t end = tx_lo + e_tx;
    rows = 4;
    for (int r = 4; r < mb; ++r)
      if ((int64_t)(kb + r) * Z < end) rows = r + 1;
    cols = kb + rows;
  }
  auto* c = new lsim_code();
  c->base = H;
  c->row_ptr.assign(rows + 1, 0);
  std::vector<int> row_deg(rows, 0), col_deg(cols, 0);
  for (int i = 0; i < rows; ++i) {
    for (int j = 0; j < cols; ++j) {
      const int s = H[(size_t)i * nb + j];
      if (s < 0) continue;
      c->ent_col.push_back(j);
      c->ent_shift.push_back(s);
      row_deg[i]++;
      col_deg[j]++;
    }
    c->row_ptr[i + 1] = (int)c->ent_col.size();
  }
  const int nnz = (int)c->ent_col.size();
  int max_row = 0, max_col = 0, min_row = 1 << 30;
  for (int d : row_deg) max_row = std::max(max_row, d), min_row = std::min(min_row, d);
  for (int d : col_deg) max_col = std::max(max_col, d);
  if (min_row < 2) {
    delete c;
    return fail(LSIM_E_INVAL, "a decoded check row has degree < 2");
  }
  if (max_row > 27 || max_col > 27) {
    delete c;
    return fail(LSIM_E_UNSUPPORTED, "decoded degree > 27");
  }
  c->col_ptr.assign(cols + 1, 0);
  for (int j = 0; j < cols; ++j) c->col_ptr[j + 1] = c->col_ptr[j] + col_deg[j];
  c->col_ent.assign(nnz, 0);
  {
    std::vector<int> fill(c->col_ptr.begin(), c->col_ptr.end() - 1);
    for (int e = 0; e < nnz; ++e) c->col_ent[fill[c->ent_col[e]]++] = e;  // rows ascending
  }
  std::vector<int> cn = make_tasks(rows, Z, row_deg);
  std::vector<int> vn = make_tasks(cols, Z, col_deg);

  // one device allocation for every table
  std::vector<int> blob;
  auto push = [&](const std::vector<int>& v) {
    size_t off = blob.size();
    blob.insert(blob.end(), v.begin(), v.end());
    return off;
  };
  size_t o_row = push(c->row_ptr), o_col = push(c->ent_col), o_sh = push(c->ent_shift),
         o_cp = push(c->col_ptr), o_ce = push(c->col_ent), o_cn = push(cn), o_vn = push(vn);
  size_t o_base = blob.size();
  blob.resize(blob.size() + ((size_t)mb * nb + 1) / 2, 0);
  std::memcpy(blob.data() + o_base, H.data(), H.size() * sizeof(int16_t));
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipMalloc(&c->dmem, blob.size() * sizeof(int));
  if (e == hipSuccess)
    e = hipMemcpy(c->dmem, blob.data(), blob.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (c->dmem) (void)hipFree(c->dmem);
    delete c;
    return dev_status(e, "code table upload");
  }
  const int* d = reinterpret_cast<const int*>(c->dmem);
  DevCode& dc = c->dev;
  dc.Z = Z;
  dc.mb = mb;
  dc.nb = nb;
  dc.kb = kb;
  dc.rows = rows;
  dc.cols = cols;
  dc.nnz = nnz;
  dc.E = nnz * Z;
  dc.n_dec = cols * Z;
  dc.m_dec = rows * Z;
  dc.k = kb * Z;
  dc.n_mother = nb * Z;
  dc.tx_lo = (int)tx_lo;
  dc.e_tx = (int)e_tx;
  dc.family = family;
  dc.max_row_deg = max_row;
  dc.max_col_deg = max_col;
  dc.n_cn_tasks = (int)cn.size();
  dc.n_vn_tasks = (int)vn.size();
  dc.row_ptr = d + o_row;
  dc.ent_col = d + o_col;
  dc.ent_shift = d + o_sh;
  dc.col_ptr = d + o_cp;
  dc.col_ent = d + o_ce;
  dc.cn_tasks = d + o_cn;
  dc.vn_tasks = d + o_vn;
  dc.base = reinterpret_cast<const int16_t*>(d + o_base);
  lsim_code_info& in = c->info;
  in.k = dc.k;
  in.n_mother = dc.n_mother;
  in.e_tx = e_tx;
  in.n_dec = dc.n_dec;
  in.m_dec = dc.m_dec;
  in.n_edges = dc.E;
  in.Z = Z;
  in.mb = mb;
  in.nb = nb;
  in.kb = kb;
  in.rows = rows;
  in.cols = cols;
  in.n_punct_cols = n_punct_cols;
  in.max_row_deg = max_row;
  in.max_col_deg = max_col;
  *out = c;
  return LSIM_OK;
}

void lsim_code_destroy(lsim_code* code) {
  if (!code) return;
  if (code->dmem) (void)hipFree(code->dmem);
  delete code;
}

lsim_status lsim_code_query(const lsim_code* code, lsim_code_info* info) {
  if (!code || !info) return fail(LSIM_E_INVAL, "null code or info");
  *info = code->info;
  return LSIM_OK;
}

lsim_status lsim_source_bits(uint64_t seed, int64_t cw0, int64_t B, int64_t k, uint8_t* d_u,
                             lsim_stream stream) {
  if (!d_u || B < 1 || k < 1 || cw0 < 0) return fail(LSIM_E_INVAL, "bad source_bits arguments");
  return dev_status(lsim::launch_source_bits(seed, cw0, B, k, d_u, as_stream(stream)),
                    "source_bits");
}

lsim_status lsim_encode(const lsim_code* code, const uint8_t* d_u, int64_t B, uint8_t* d_c,
                        lsim_stream stream) {
  if (!code || !d_u || !d_c || B < 1) return fail(LSIM_E_INVAL, "bad encode arguments");
  if ((int64_t)code->dev.n_mother > 48 * 1024)
    return fail(LSIM_E_UNSUPPORTED, "mother code too long for the encoder's LDS tile");
  return dev_status(lsim::launch_encode(code->dev, d_u, B, d_c, as_stream(stream)), "encode");
}

lsim_status lsim_map_awgn(const lsim_code* code, int bits_per_sym, const uint8_t* d_c,
                          const float* d_no, uint64_t seed, int64_t cw0, int64_t B, float* d_y,
                          lsim_stream stream) {
  if (!code || !d_c || !d_no || !d_y || B < 1 || cw0 < 0)
    return fail(LSIM_E_INVAL, "bad map_awgn arguments");
  const int m = bits_per_sym;
  if (m != 1 && m != 2 && m != 4 && m != 6)
    return fail(LSIM_E_UNSUPPORTED, "bits_per_sym must be 1, 2, 4 or 6");
  if (code->dev.e_tx % m) return fail(LSIM_E_INVAL, "e_tx is not a multiple of bits_per_sym");
  return dev_status(
      lsim::launch_map_awgn(code->dev, m, d_c, d_no, seed, cw0, B, d_y, as_stream(stream)),
      "map_awgn");
}

static lsim_status check_demap(int m, int method, const void* y, const float* no, int64_t B,
                               int64_t S, const void* out) {
  if (!y || !no || !out || B < 1 || S < 1) return fail(LSIM_E_INVAL, "bad demap arguments");
  if (m != 1 && m != 2 && m != 4 && m != 6)
    return fail(LSIM_E_UNSUPPORTED, "bits_per_sym must be 1, 2, 4 or 6");
  if (method != LSIM_DEMAP_EXACT && method != LSIM_DEMAP_MAXLOG)
    return fail(LSIM_E_INVAL, "unknown demap method");
  return LSIM_OK;
}

lsim_status lsim_demap(int bits_per_sym, int method, const float* d_y, const float* d_no,
                       int64_t B, int64_t S, float* d_llr, lsim_stream stream) {
  lsim_status st = check_demap(bits_per_sym, method, d_y, d_no, B, S, d_llr);
  if (st != LSIM_OK) return st;
  return dev_status(lsim::launch_demap(bits_per_sym, method, d_y, d_no, B, S, d_llr, nullptr,
                                       0.f, 0, as_stream(stream)),
                    "demap");
}

lsim_status lsim_demap_q8(int bits_per_sym, int method, const float* d_y, const float* d_no,
                          int64_t B, int64_t S, float scale, int sat, int8_t* d_q,
                          lsim_stream stream) {
  lsim_status st = check_demap(bits_per_sym, method, d_y, d_no, B, S, d_q);
  if (st != LSIM_OK) return st;
  if (!is_pow2_scale(scale)) return fail(LSIM_E_INVAL, "scale must be a power of two");
  if (sat < 1 || sat > 127) return fail(LSIM_E_INVAL, "sat must be in 1..127");
  return dev_status(lsim::launch_demap(bits_per_sym, method, d_y, d_no, B, S, nullptr, d_q, scale,
                                       sat, as_stream(stream)),
                    "demap_q8");
}

lsim_status lsim_quantize(const float* d_llr, int64_t count, float scale, int sat, int8_t* d_q,
                          lsim_stream stream) {
  if (!d_llr || !d_q || count < 1) return fail(LSIM_E_INVAL, "bad quantize arguments");
  if (!is_pow2_scale(scale)) return fail(LSIM_E_INVAL, "scale must be a power of two");
  if (sat < 1 || sat > 127) return fail(LSIM_E_INVAL, "sat must be in 1..127");
  return dev_status(lsim::launch_quantize(d_llr, count, scale, sat, d_q, as_stream(stream)),
                    "quantize");
}

lsim_status lsim_decode_workspace(const lsim_code* code, const lsim_decode_params* p, int64_t B,
                                  size_t* bytes) {
  lsim_status st = check_params(code, p);
  if (st != LSIM_OK) return st;
  if (!bytes || B < 1) return fail(LSIM_E_INVAL, "bad workspace query");
  *bytes = p->algo == LSIM_NMS_F32 ? lsim::layered_state_words(code->dev, B) * 4 : 0;
  return LSIM_OK;
}

static lsim_status decode_common(const lsim_code* code, const lsim_decode_params* p,
                                 const void* d_llr, int64_t B, uint8_t* d_bits, float* d_app,
                                 const void* q_in, void* r_out, void* q_out, void* d_work,
                                 size_t work_bytes, lsim_stream stream) {
  lsim_status st = check_params(code, p);
  if (st != LSIM_OK) return st;
  if (!d_llr || B < 1) return fail(LSIM_E_INVAL, "null llr or B < 1");
  if (B > (int64_t)1 << 31) return fail(LSIM_E_INVAL, "B too large");
  std::string why;
  hipError_t e;
  if (p->algo == LSIM_NMS_F32) {
    if (q_in || q_out) return fail(LSIM_E_INVAL, "layered decoder takes no q_in/q_out");
    const size_t need = lsim::layered_state_words(code->dev, B) * 4;
    if (!d_work || work_bytes < need)
      return fail(LSIM_E_NOMEM, "workspace smaller than lsim_decode_workspace()");
    e = lsim::launch_layered(code->dev, *p, (const float*)d_llr, B, d_bits, d_app, (float*)r_out,
                             (uint32_t*)d_work, as_stream(stream), &why);
  } else {
    e = lsim::launch_flood(code->dev, *p, d_llr, B, d_bits, d_app, q_in, r_out, q_out,
                           as_stream(stream), &why);
  }
  if (!why.empty()) return fail(LSIM_E_UNSUPPORTED, why);
  return dev_status(e, "decode");
}

lsim_status lsim_decode(const lsim_code* code, const lsim_decode_params* p, const void* d_llr,
                        int64_t B, uint8_t* d_bits, float* d_app, void* d_work, size_t work_bytes,
                        lsim_stream stream) {
  return decode_common(code, p, d_llr, B, d_bits, d_app, nullptr, nullptr, nullptr, d_work,
                       work_bytes, stream);
}

lsim_status lsim_decode_state(const lsim_code* code, const lsim_decode_params* p,
                              const void* d_llr, int64_t B, const void* d_q_in, void* d_r_out,
                              void* d_q_out, float* d_app, void* d_work, size_t work_bytes,
                              lsim_stream stream) {
  return decode_common(code, p, d_llr, B, nullptr, d_app, d_q_in, d_r_out, d_q_out, d_work,
                       work_bytes, stream);
}

lsim_status lsim_count_errors(const uint8_t* d_ref, int64_t ref_stride, const uint8_t* d_hat,
                              int64_t B, int64_t k, const int32_t* d_bin, int nbins,
                              int64_t* d_counts, lsim_stream stream) {
  if (!d_ref || !d_hat || !d_counts || B < 1 || k < 1 || nbins < 1 || ref_stride < k)
    return fail(LSIM_E_INVAL, "bad count_errors arguments");
  return dev_status(lsim::launch_count_errors(d_ref, ref_stride, d_hat, B, k, d_bin, nbins,
                                              d_counts, as_stream(stream)),
                    "count_errors");
}

lsim_status lsim_syndrome(const lsim_code* code, const uint8_t* d_c, int64_t stride, int64_t B,
                          int32_t* d_unsat, lsim_stream stream) {
  if (!code || !d_c || !d_unsat || B < 1 || stride < code->dev.n_dec)
    return fail(LSIM_E_INVAL, "bad syndrome arguments");
  return dev_status(lsim::launch_syndrome(code->dev, d_c, stride, B, d_unsat, as_stream(stream)),
                    "syndrome");
}

}  // extern "C"
