// C-ABI entry points of liblsim: host-side validation, code objects and
// dispatch to the HIP kernels.  See include/lsim.h for the contract of each
// call.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <numeric>
#include <unordered_map>
#include <string>
#include <vector>

#include "lsim_internal.h"

namespace lsim {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

hipError_t require_lds_at_zero(const void* kernel) {
  static std::mutex mu;
  static std::unordered_map<const void*, bool> ok;
  std::lock_guard<std::mutex> lock(mu);
  auto it = ok.find(kernel);
  if (it == ok.end()) {
    hipFuncAttributes attr;
    hipError_t e = hipFuncGetAttributes(&attr, kernel);
    if (e != hipSuccess) return e;
    it = ok.emplace(kernel, attr.sharedSizeBytes == 0).first;
  }
  return it->second ? hipSuccess : hipErrorInvalidDeviceFunction;
}

hipError_t ensure_dyn_lds(const void* kernel, size_t bytes) {
  static std::mutex mu;
  static std::unordered_map<const void*, size_t> done;
  if (bytes <= 64 * 1024) return hipSuccess;
  std::lock_guard<std::mutex> lock(mu);
  auto it = done.find(kernel);
  if (it != done.end() && it->second >= bytes) return hipSuccess;
  hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes);
  if (e == hipSuccess) done[kernel] = bytes;
  return e;
}

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

// Conflict graph of the decoded rows: rows that meet a common LDS column,
// as an n x n byte matrix built from the column lists.
std::vector<char> row_conflicts(const lsim_code& c) {
  const int n = (int)c.row_lds_cols.size();
  const int cols = (int)c.col_ptr.size() - 1;
  std::vector<std::vector<int>> col_rows(cols);
  for (int i = 0; i < n; ++i)
    for (int j : c.row_lds_cols[i]) col_rows[j].push_back(i);
  std::vector<char> m((size_t)n * n, 0);
  for (const auto& rs : col_rows)
    for (int a : rs)
      for (int b : rs)
        if (a != b) m[(size_t)a * n + b] = 1;
  return m;
}

// The layered schedule table for a visiting order: per position (row,
// private LLR offset, shift, barrier after).  A barrier follows position p
// when the layer at p + 1 meets an LDS column of a layer visited since the
// last barrier (only then can one lane read a posterior another lane of
// the previous layers writes), and always after the last position, so every
// iteration starts from the same state of the schedule.
std::vector<int> layer_table(const lsim_code& c, const std::vector<int>& order) {
  const int n = (int)order.size();
  const std::vector<char> meet = row_conflicts(c);
  std::vector<int> t(4 * (size_t)n);
  std::vector<int> run;
  for (int p = 0; p < n; ++p) {
    const int i = order[p];
    run.push_back(i);
    bool sync = p == n - 1;
    if (!sync)
      for (int j : run)
        if (meet[(size_t)j * n + order[p + 1]]) {
          sync = true;
          break;
        }
    if (sync) run.clear();
    t[4 * p] = i;
    t[4 * p + 1] = c.row_pch[2 * i];
    t[4 * p + 2] = c.row_pch[2 * i + 1];
    t[4 * p + 3] = sync ? 1 : 0;
  }
  return t;
}

// Groups of mutually disjoint layers (rows that meet no common LDS column)
// by DSatur greedy colouring of the conflict graph, visited group after
// group (rows ascending inside a group): a barrier is then needed only
// between groups.
std::vector<int> grouped_order(const lsim_code& c) {
  const int n = (int)c.row_lds_cols.size();
  const std::vector<char> meet = row_conflicts(c);
  std::vector<std::vector<int>> adj(n);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      if (meet[(size_t)a * n + b]) adj[a].push_back(b);
  // saturation: distinct colours among a row's coloured neighbours, kept
  // with a per-row colour mark (at most n colours)
  std::vector<int> colour(n, -1), sat(n, 0);
  std::vector<char> has((size_t)n * n, 0);
  for (int step = 0; step < n; ++step) {
    int best = -1;
    for (int i = 0; i < n; ++i) {
      if (colour[i] >= 0) continue;
      if (best < 0 || sat[i] > sat[best] ||
          (sat[i] == sat[best] && adj[i].size() > adj[best].size()))
        best = i;
    }
    int col = 0;
    while (has[(size_t)best * n + col]) ++col;
    colour[best] = col;
    for (int j : adj[best])
      if (!has[(size_t)j * n + col]) {
        has[(size_t)j * n + col] = 1;
        ++sat[j];
      }
  }
  std::vector<int> order;
  const int ng = n ? *std::max_element(colour.begin(), colour.end()) + 1 : 0;
  for (int g = 0; g < ng; ++g)
    for (int i = 0; i < n; ++i)
      if (colour[i] == g) order.push_back(i);
  return order;
}

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
  if (p->lds_rows < -1) return fail(LSIM_E_INVAL, "lds_rows must be >= -1");
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
  std::vector<int> ce2(2 * (size_t)nnz);
  for (int i = 0; i < nnz; ++i) {
    const int e = c->col_ent[i];
    ce2[2 * i] = e * Z;
    ce2[2 * i + 1] = c->ent_shift[e];
  }
  std::vector<int> ecz(2 * (size_t)nnz);
  for (int e = 0; e < nnz; ++e) {
    ecz[2 * e] = c->ent_col[e] * Z;
    ecz[2 * e + 1] = c->ent_shift[e];
  }
  // layered decoder: private rows (last entry in a column of degree one) and
  // LDS slots of the shared columns
  std::vector<int> row_priv(rows, -1), priv_row, shared_col;
  std::vector<char> is_priv_col(cols, 0);
  for (int i = 0; i < rows; ++i) {
    const int j = c->ent_col[c->row_ptr[i + 1] - 1];
    if (col_deg[j] == 1) {
      row_priv[i] = (int)priv_row.size();
      priv_row.push_back(i);
      is_priv_col[j] = 1;
    }
  }
  int deg1_inner = 0;
  for (int j = 0; j < cols; ++j) deg1_inner += col_deg[j] == 1 && !is_priv_col[j];
  std::vector<int> col_slot(cols, -1);
  for (int j = 0; j < cols; ++j)
    if (!is_priv_col[j]) {
      col_slot[j] = (int)shared_col.size();
      shared_col.push_back(j);
    }
  std::vector<int> elz(2 * (size_t)nnz);
  for (int e = 0; e < nnz; ++e) {
    const int j = c->ent_col[e];
    elz[2 * e] = (is_priv_col[j] ? j : col_slot[j]) * Z;
    elz[2 * e + 1] = c->ent_shift[e];
  }
  size_t o_rp = push(row_priv), o_sc = push(shared_col), o_pr = push(priv_row);
  if (blob.size() & 1) blob.push_back(0);  // 8-byte alignment of the int2 tables
  // encoder lists: the dual-diagonal rows (all rows of the 11n family, the
  // four core rows of the BG shape) XOR information columns; extension rows
  // XOR information and core parity columns
  const int m_core = family == LSIM_FAMILY_11N ? mb : 4;
  std::vector<int> enc_ptr(mb + 1, 0), enc_cz;
  for (int i = 0; i < mb; ++i) {
    const int lim = i < m_core ? kb : kb + 4;
    for (int j = 0; j < lim; ++j) {
      const int sh = H[(size_t)i * nb + j];
      if (sh < 0) continue;
      enc_cz.push_back(j * Z);
      enc_cz.push_back(sh);
    }
    enc_ptr[i + 1] = (int)(enc_cz.size() / 2);
  }
  size_t o_ce2 = push(ce2);
  size_t o_ecz = push(ecz);
  size_t o_encz = push(enc_cz);
  size_t o_encp = push(enc_ptr);
  // per row: where lane r finds the channel LLR of the row's private column,
  // as (col * Z - tx_lo, shift) (rows without one get an offset that no lane
  // reaches from below), and the LDS columns the row meets; the layered
  // schedule table starts in natural order
  c->row_pch.assign(2 * (size_t)rows, 0);
  c->row_lds_cols.assign(rows, {});
  for (int i = 0; i < rows; ++i) {
    const int e = c->row_ptr[i + 1] - 1;
    const bool pv = row_priv[i] >= 0;
    c->row_pch[2 * i] = pv ? (int)(c->ent_col[e] * (int64_t)Z - tx_lo) : -(1 << 30);
    c->row_pch[2 * i + 1] = pv ? c->ent_shift[e] : 0;
    for (int q = c->row_ptr[i]; q < c->row_ptr[i + 1]; ++q)
      if (!is_priv_col[c->ent_col[q]]) c->row_lds_cols[i].push_back(c->ent_col[q]);
  }
  c->layer_order.resize(rows);
  for (int i = 0; i < rows; ++i) c->layer_order[i] = i;
  if (blob.size() & 1) blob.push_back(0);
  size_t o_elz = push(elz);
  while (blob.size() & 3) blob.push_back(0);  // 16-byte alignment of the int4 table
  size_t o_pos = push(layer_table(*c, c->layer_order));
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
  dc.enc_ptr = d + o_encp;
  dc.enc_cz = reinterpret_cast<const int2*>(d + o_encz);
  dc.col_edge = reinterpret_cast<const int2*>(d + o_ce2);
  dc.ent_cz = reinterpret_cast<const int2*>(d + o_ecz);
  dc.n_shared = (int)shared_col.size();
  dc.n_priv = (int)priv_row.size();
  dc.n_deg1_inner = deg1_inner;
  dc.row_priv = d + o_rp;
  dc.shared_col = d + o_sc;
  dc.priv_row = d + o_pr;
  dc.ent_lz = reinterpret_cast<const int2*>(d + o_elz);
  dc.layer_pos = reinterpret_cast<const int4*>(d + o_pos);
  c->layer_pos_off = o_pos;
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
  in.n_shared_cols = dc.n_shared;
  in.n_private_rows = dc.n_priv;
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

lsim_status lsim_code_set_layer_order(lsim_code* code, int mode, const int* order) {
  if (!code) return fail(LSIM_E_INVAL, "null code");
  const int n = code->dev.rows;
  std::vector<int> ord;
  if (mode == LSIM_LAYERS_NATURAL) {
    ord.resize(n);
    std::iota(ord.begin(), ord.end(), 0);
  } else if (mode == LSIM_LAYERS_GROUPED) {
    ord = grouped_order(*code);
  } else if (mode == LSIM_LAYERS_CUSTOM) {
    if (!order) return fail(LSIM_E_INVAL, "custom layer order needs an order");
    ord.assign(order, order + n);
    std::vector<char> seen(n, 0);
    for (int i : ord) {
      if (i < 0 || i >= n || seen[i]) return fail(LSIM_E_INVAL, "layer order is not a permutation of the decoded rows");
      seen[i] = 1;
    }
  } else {
    return fail(LSIM_E_INVAL, "unknown layer order mode");
  }
  const std::vector<int> t = layer_table(*code, ord);
  int* dst = reinterpret_cast<int*>(code->dmem) + code->layer_pos_off;
  int cur = 0;
  hipError_t e = hipGetDevice(&cur);
  if (e == hipSuccess && cur != code->device) e = hipSetDevice(code->device);
  if (e == hipSuccess) e = hipMemcpy(dst, t.data(), t.size() * sizeof(int), hipMemcpyHostToDevice);
  if (cur != code->device) (void)hipSetDevice(cur);
  if (e != hipSuccess) return dev_status(e, "layer order upload");
  code->layer_order = ord;
  return LSIM_OK;
}

lsim_status lsim_code_layer_order(const lsim_code* code, int* order, int* barriers) {
  if (!code) return fail(LSIM_E_INVAL, "null code");
  if (order) std::copy(code->layer_order.begin(), code->layer_order.end(), order);
  if (barriers) {
    const std::vector<int> t = layer_table(*code, code->layer_order);
    int nb = 0;
    for (size_t p = 0; p < code->layer_order.size(); ++p) nb += t[4 * p + 3];
    *barriers = nb;
  }
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

lsim_status lsim_map_points(const lsim_code* code, int bits_per_sym, const float* d_points,
                            const uint8_t* d_c, const float* d_no, uint64_t seed, int64_t cw0,
                            int64_t B, float* d_y, lsim_stream stream) {
  if (!code || !d_points || !d_c || !d_no || !d_y || B < 1 || cw0 < 0)
    return fail(LSIM_E_INVAL, "bad map_points arguments");
  const int m = bits_per_sym;
  if (m < 1 || m > 6) return fail(LSIM_E_UNSUPPORTED, "bits_per_sym must be 1..6");
  if (code->dev.e_tx % m) return fail(LSIM_E_INVAL, "e_tx is not a multiple of bits_per_sym");
  if (((uintptr_t)d_y) & 7) return fail(LSIM_E_INVAL, "d_y must be 8-byte aligned");
  return dev_status(lsim::launch_map_points(code->dev, m, d_points, d_c, d_no, seed, cw0, B, d_y,
                                            as_stream(stream)),
                    "map_points");
}

lsim_status lsim_points_workspace(const lsim_code* code, int bits_per_sym, int64_t B,
                                  size_t* bytes) {
  if (!code || !bytes || B < 1 || bits_per_sym < 1 || bits_per_sym > 6)
    return fail(LSIM_E_INVAL, "bad workspace query");
  *bytes = lsim::points_work_bytes(code->dev, bits_per_sym, B);
  return LSIM_OK;
}

lsim_status lsim_points_grad(const lsim_code* code, int bits_per_sym, const float* d_points,
                             const uint8_t* d_c, const float* d_gy, int64_t B, float* d_gpoints,
                             void* d_work, size_t work_bytes, lsim_stream stream) {
  if (!code || !d_points || !d_c || !d_gy || !d_gpoints || B < 1)
    return fail(LSIM_E_INVAL, "bad points_grad arguments");
  const int m = bits_per_sym;
  if (m < 1 || m > 6) return fail(LSIM_E_UNSUPPORTED, "bits_per_sym must be 1..6");
  if (code->dev.e_tx % m) return fail(LSIM_E_INVAL, "e_tx is not a multiple of bits_per_sym");
  if (((uintptr_t)d_gy) & 7) return fail(LSIM_E_INVAL, "d_gy must be 8-byte aligned");
  if (!d_work || work_bytes < lsim::points_work_bytes(code->dev, m, B))
    return fail(LSIM_E_NOMEM, "workspace smaller than lsim_points_workspace()");
  return dev_status(lsim::launch_points_grad(code->dev, m, d_points, d_c, d_gy, B, d_gpoints,
                                             d_work, as_stream(stream)),
                    "points_grad");
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

static bool llr_aligned(int m, const void* p) {
  const uintptr_t a = (uintptr_t)p;
  return m == 4 ? (a & 15) == 0 : (m == 2 || m == 6) ? (a & 7) == 0 : (a & 3) == 0;
}

lsim_status lsim_demap(int bits_per_sym, int method, const float* d_y, const float* d_no,
                       int64_t B, int64_t S, float* d_llr, lsim_stream stream) {
  lsim_status st = check_demap(bits_per_sym, method, d_y, d_no, B, S, d_llr);
  if (st != LSIM_OK) return st;
  if (!llr_aligned(bits_per_sym, d_llr) || ((uintptr_t)d_y & 7))
    return fail(LSIM_E_INVAL, "d_llr must be aligned to 4*m bytes (16 for m=4, 8 for m=2,6), d_y to 8");
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

lsim_status lsim_decode_launch(const lsim_code* code, const lsim_decode_params* p,
                               int* threads, int* codewords_per_tile, int* lds_rows,
                               int* waves_per_simd) {
  lsim_status st = check_params(code, p);
  if (st != LSIM_OK) return st;
  if (!threads || !codewords_per_tile || !lds_rows || !waves_per_simd)
    return fail(LSIM_E_INVAL, "null output");
  if (p->algo != LSIM_NMS_F32)
    return fail(LSIM_E_UNSUPPORTED, "launch shapes are reported for the layered decoder");
  std::string why;
  hipError_t e = lsim::layered_launch_shape(code->dev, *p, threads, codewords_per_tile, lds_rows,
                                            waves_per_simd, &why);
  if (e != hipSuccess) return dev_status(e, "layered launch shape");
  if (!why.empty()) return fail(LSIM_E_UNSUPPORTED, why);
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
    if ((uintptr_t)d_work & 15) return fail(LSIM_E_INVAL, "d_work must be 16-byte aligned");
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

lsim_status lsim_decode_noalloc(const lsim_code* code, const lsim_decode_params* p,
                                const void* d_llr, int64_t B, uint8_t* d_bits, float* d_app,
                                lsim_stream stream) {
  lsim_status st = check_params(code, p);
  if (st != LSIM_OK) return st;
  if (!d_llr || B < 1) return fail(LSIM_E_INVAL, "null llr or B < 1");
  if (p->algo != LSIM_NMS_F32)  // the flooding decoders need no workspace
    return decode_common(code, p, d_llr, B, d_bits, d_app, nullptr, nullptr, nullptr, nullptr, 0,
                         stream);
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return dev_status(e, "decode_noalloc");
  if (dev != code->device)
    return fail(LSIM_E_INVAL, "decode_noalloc: the current device is not the code's device");
  const size_t need = lsim::layered_state_words(code->dev, B) * 4;
  if (need > LSIM_NOALLOC_SCRATCH_BYTES)
    return fail(LSIM_E_NOMEM, "decode_noalloc: the layered decoder state for this batch (" +
                                  std::to_string(need) + " bytes) exceeds the " +
                                  std::to_string((size_t)LSIM_NOALLOC_SCRATCH_BYTES) +
                                  "-byte device scratch; split the batch");
  void* scratch = nullptr;
  size_t bytes = 0;
  e = lsim::noalloc_scratch(&scratch, &bytes);
  if (e != hipSuccess) return dev_status(e, "decode_noalloc scratch lookup");
  return decode_common(code, p, d_llr, B, d_bits, d_app, nullptr, nullptr, nullptr, scratch, bytes,
                       stream);
}

lsim_status lsim_decode_state(const lsim_code* code, const lsim_decode_params* p,
                              const void* d_llr, int64_t B, const void* d_q_in, void* d_r_out,
                              void* d_q_out, float* d_app, void* d_work, size_t work_bytes,
                              lsim_stream stream) {
  return decode_common(code, p, d_llr, B, nullptr, d_app, d_q_in, d_r_out, d_q_out, d_work,
                       work_bytes, stream);
}

lsim_status lsim_demap_prior(int bits_per_sym, int method, const float* d_y, const float* d_no,
                             const float* d_la, int64_t B, int64_t S, int extrinsic, float* d_llr,
                             lsim_stream stream) {
  lsim_status st = check_demap(bits_per_sym, method, d_y, d_no, B, S, d_llr);
  if (st != LSIM_OK) return st;
  if (!d_la) return fail(LSIM_E_INVAL, "null a-priori LLRs");
  if (!llr_aligned(bits_per_sym, d_llr) || !llr_aligned(bits_per_sym, d_la) || ((uintptr_t)d_y & 7))
    return fail(LSIM_E_INVAL,
                "d_llr and d_la must be aligned to 4*m bytes (16 for m=4, 8 for m=2,6), d_y to 8");
  return dev_status(lsim::launch_demap_prior(bits_per_sym, method == LSIM_DEMAP_EXACT, d_y, d_no,
                                             d_la, B, S, extrinsic != 0, d_llr, as_stream(stream)),
                    "demap_prior");
}

lsim_status lsim_apriori_llrs(const lsim_code* code, const uint8_t* d_c, const float* d_sigma,
                              uint64_t seed, int64_t cw0, int64_t B, float* d_la,
                              lsim_stream stream) {
  if (!code || !d_c || !d_sigma || !d_la || B < 1 || cw0 < 0)
    return fail(LSIM_E_INVAL, "bad apriori_llrs arguments");
  return dev_status(lsim::launch_apriori(code->dev, d_c, d_sigma, seed, cw0, B, d_la,
                                         as_stream(stream)),
                    "apriori_llrs");
}

lsim_status lsim_mutual_info(const float* d_llr, int64_t llr_stride, const uint8_t* d_c,
                             int64_t c_stride, int64_t B, int64_t n, const int32_t* d_bin,
                             int nbins, float* d_mi_cw, double* d_mi_bins, lsim_stream stream) {
  if (!d_llr || !d_c || !d_mi_cw || B < 1 || n < 1 || llr_stride < n || c_stride < n)
    return fail(LSIM_E_INVAL, "bad mutual_info arguments");
  if (d_mi_bins && (nbins < 1 || nbins > 65535 || (!d_bin && nbins != 1)))
    return fail(LSIM_E_INVAL, "nbins must be 1..65535 (1 without d_bin)");
  return dev_status(lsim::launch_mutual_info(d_llr, llr_stride, d_c, c_stride, B, n, d_bin, nbins,
                                             d_mi_cw, d_mi_bins, as_stream(stream)),
                    "mutual_info");
}

lsim_status lsim_extrinsic(const lsim_code* code, const float* d_app, const float* d_llr_in,
                           float llr_max, int64_t B, float* d_out, lsim_stream stream) {
  if (!code || !d_app || !d_llr_in || !d_out || B < 1 || !(llr_max >= 0.f))
    return fail(LSIM_E_INVAL, "bad extrinsic arguments");
  return dev_status(lsim::launch_extrinsic(code->dev, d_app, d_llr_in, llr_max, B, d_out,
                                           as_stream(stream)),
                    "extrinsic");
}

lsim_status lsim_map_awgn_bits(int bits_per_sym, const uint8_t* d_bits, int64_t stride, int64_t n,
                               const float* d_no, uint64_t seed, int64_t cw0, int64_t B,
                               float* d_y, lsim_stream stream) {
  if (!d_bits || !d_no || !d_y || B < 1 || n < 1 || stride < n || cw0 < 0 || n > (1 << 30) ||
      stride > (1 << 30))
    return fail(LSIM_E_INVAL, "bad map_awgn_bits arguments");
  const int m = bits_per_sym;
  if (m != 1 && m != 2 && m != 4 && m != 6)
    return fail(LSIM_E_UNSUPPORTED, "bits_per_sym must be 1, 2, 4 or 6");
  if (n % m) return fail(LSIM_E_INVAL, "n is not a multiple of bits_per_sym");
  // the mapper reads row b's bits at b * n_mother + tx_lo .. + e_tx
  DevCode dc{};
  dc.n_mother = (int)stride;
  dc.tx_lo = 0;
  dc.e_tx = (int)n;
  return dev_status(lsim::launch_map_awgn(dc, m, d_bits, d_no, seed, cw0, B, d_y, as_stream(stream)),
                    "map_awgn_bits");
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

lsim_status lsim_probe(int kind, const void* d_src, void* d_dst, int64_t bytes, int rounds,
                       int grid, int64_t* units, lsim_stream stream) {
  if (kind < LSIM_PROBE_COPY || kind > LSIM_PROBE_EXP2 || grid < 1 || grid > 65536 || rounds < 1 ||
      !d_dst || !units)
    return fail(LSIM_E_INVAL, "bad probe arguments");
  if (kind <= LSIM_PROBE_READ && (!d_src || bytes < 16 || (bytes & 15)))
    return fail(LSIM_E_INVAL, "copy and read probes take a source of a positive multiple of 16 bytes");
  return dev_status(lsim::launch_probe(kind, d_src, d_dst, bytes, rounds, grid, as_stream(stream),
                                       units),
                    "probe");
}

lsim_status lsim_ebn0_to_n0(const double* ebn0_db, int64_t n, double rate, int bits_per_sym,
                            double* no) {
  if (!ebn0_db || !no || n < 0 || !(rate > 0.0 && rate <= 1.0) || bits_per_sym < 1)
    return fail(LSIM_E_INVAL, "bad ebn0_to_n0 arguments");
  for (int64_t i = 0; i < n; ++i) {
    // energy per information bit = symbol energy (1) / (rate * m)
    const double v = 1.0 / (rate * bits_per_sym * std::pow(10.0, ebn0_db[i] / 10.0));
    if (!std::isfinite(v)) return fail(LSIM_E_INVAL, "Eb/N0 gives a non-finite noise variance");
    no[i] = v;
  }
  return LSIM_OK;
}

lsim_status lsim_hard_bits(const float* d_llr, int64_t stride, int64_t B, int64_t k,
                           uint8_t* d_bits, lsim_stream stream) {
  if (!d_llr || !d_bits || B < 1 || k < 1 || stride < k)
    return fail(LSIM_E_INVAL, "bad hard_bits arguments");
  return dev_status(lsim::launch_hard_bits(d_llr, stride, B, k, d_bits, as_stream(stream)),
                    "hard_bits");
}

lsim_status lsim_syndrome(const lsim_code* code, const uint8_t* d_c, int64_t stride, int64_t B,
                          int32_t* d_unsat, lsim_stream stream) {
  if (!code || !d_c || !d_unsat || B < 1 || stride < code->dev.n_dec)
    return fail(LSIM_E_INVAL, "bad syndrome arguments");
  return dev_status(lsim::launch_syndrome(code->dev, d_c, stride, B, d_unsat, as_stream(stream)),
                    "syndrome");
}

}  // extern "C"

// ------------------------------------------------------- mixed-shape plans

struct lsim_plan {
  std::vector<lsim::LayerShape> shapes;
  lsim_decode_params p;
  int threads = 0;
  int dmax = 0;
  int wpe = 1;  // layered kernel's register budget (wavefronts per SIMD)
  size_t lds = 0;
  int grid = 0;
  int64_t ntiles = 0;
  size_t state_words = 0;
  void* dmem = nullptr;
  lsim::LayerShape* d_shapes = nullptr;
  int* d_tile_shape = nullptr;
  int64_t* d_tile_local = nullptr;
};

namespace {
constexpr size_t kCounterBytes = 256;
}

extern "C" {

lsim_status lsim_mixed_plan_create(const lsim_code* const* codes, const int64_t* counts,
                                   int nshapes, const lsim_decode_params* p,
                                   const int32_t* codewords_per_tile, int threads,
                                   lsim_plan** out) {
  if (!codes || !counts || !p || !out || nshapes < 1 || nshapes > 4096)
    return fail(LSIM_E_INVAL, "bad mixed plan arguments");
  *out = nullptr;
  lsim_status st = check_params(codes[0], p);
  if (st != LSIM_OK) return st;
  if (p->algo != LSIM_NMS_F32 && p->algo != LSIM_OMS_I8)
    return fail(LSIM_E_UNSUPPORTED,
                "mixed batches decode with the layered NMS or the flooding int8 OMS decoder");
  const bool oms = p->algo == LSIM_OMS_I8;
  int zmax = 0, dmax = 0;
  for (int s = 0; s < nshapes; ++s) {
    if (!codes[s] || counts[s] < 0) return fail(LSIM_E_INVAL, "null code or negative count");
    zmax = std::max(zmax, codes[s]->dev.Z);
    dmax = std::max(dmax, oms ? std::max(codes[s]->dev.max_row_deg, codes[s]->dev.max_col_deg)
                              : codes[s]->dev.max_row_deg);
  }
  if (oms) {
    // flooding OMS: a tile is a codeword pair in packed 16-bit lanes; the
    // waves stride over (row, lift chunk) tasks, so any Z fits any width
    if (threads == 0) threads = 512;
    if (threads != 256 && threads != 512 && threads != 1024)
      return fail(LSIM_E_INVAL, "threads must be 256, 512 or 1024 for the OMS decoder");
    if (dmax > 32) return fail(LSIM_E_UNSUPPORTED, "node degree > 32");
  } else if (threads == 0) {
    // the default launch shape of the shape with the largest lift
    for (int s = 0; s < nshapes; ++s)
      if (codes[s]->dev.Z == zmax) {
        threads = lsim::layered_default_threads(codes[s]->dev);
        break;
      }
  }
  if (!oms && threads != 256 && threads != 384 && threads != 512 && threads != 768 &&
      threads != 1024)
    return fail(LSIM_E_INVAL, "threads must be 256, 384, 512, 768 or 1024");
  if (!oms && threads < zmax) return fail(LSIM_E_INVAL, "threads < largest Z");
  const size_t lds_cap = 160 * 1024 - 64;  // room for the kernel's static LDS
  auto* plan = new lsim_plan();
  plan->p = *p;
  plan->threads = threads;
  int64_t llr_off = 0, bits_off = 0, app_off = 0, state_off = 0, tile0 = 0;
  for (int s = 0; s < nshapes; ++s) {
    const DevCode& c = codes[s]->dev;
    int G;
    size_t tile_lds;
    if (oms) {
      // a codeword pair per tile when its packed state fits the LDS, else
      // one codeword (16-bit values, half the state)
      const int want = codewords_per_tile && codewords_per_tile[s] > 0 ? codewords_per_tile[s] : 0;
      G = want ? want : (lsim::oms2_lds_bytes(c, 2) <= lds_cap - 16 ? 2 : 1);
      tile_lds = G == 1 || G == 2 ? lsim::oms2_lds_bytes(c, G) : 0;
      if ((G != 1 && G != 2) || tile_lds > lds_cap - 16) {
        delete plan;
        return fail(LSIM_E_INVAL,
                    "the OMS decoder takes one codeword or a codeword pair per tile, within the LDS");
      }
    } else {
      if (c.n_deg1_inner || c.rows < 3) {
        delete plan;
        return fail(LSIM_E_UNSUPPORTED, c.rows < 3 ? lsim::kLayeredRowsMsg : lsim::kLayeredDeg1Msg);
      }
      G = codewords_per_tile && codewords_per_tile[s] > 0 ? codewords_per_tile[s] : threads / c.Z;
      if (!codewords_per_tile || codewords_per_tile[s] <= 0)
        while (G > 1 && lsim::layered_tile_lds(c, G) > lds_cap / 2) --G;  // two workgroups per CU
      if (G < 1 || G * c.Z > threads || lsim::layered_tile_lds(c, G) > lds_cap) {
        delete plan;
        return fail(LSIM_E_INVAL, "codewords_per_tile does not fit the workgroup or the LDS");
      }
      tile_lds = lsim::layered_tile_lds(c, G);
    }
    lsim::LayerShape sh;
    sh.code = c;
    sh.G = G;
    sh.count = counts[s];
    sh.tile0 = tile0;
    sh.llr_off = llr_off;
    sh.bits_off = bits_off;
    sh.app_off = app_off;
    sh.state_off = state_off;
    sh.lds_rows = 0;
    plan->lds = std::max(plan->lds, tile_lds);
    llr_off += counts[s] * c.e_tx;
    bits_off += counts[s] * c.k;
    app_off += counts[s] * c.n_dec;
    if (!oms) state_off += (int64_t)lsim::layered_state_words(c, counts[s]);
    tile0 += (counts[s] + G - 1) / G;
    plan->shapes.push_back(sh);
  }
  plan->ntiles = tile0;
  plan->state_words = (size_t)state_off;
  plan->dmax = dmax;
  int occ = 0;
  hipError_t e = hipSuccess;
  if (!oms) {
    // check records kept in LDS (p->lds_rows): by default as many rows per
    // shape as fit the LDS a workgroup has at the occupancy the shared
    // posteriors allow
    // register budget: 6 wavefronts per SIMD when that at least doubles
    // the workgroups per CU
    int occ6 = 0;
    e = lsim::mixed_occupancy(threads, dmax, 1, plan->lds, &occ);
    if (e == hipSuccess) e = lsim::mixed_occupancy(threads, dmax, 6, plan->lds, &occ6);
    if (e == hipSuccess && occ6 >= 2 * occ) {
      plan->wpe = 6;
      occ = occ6;
    }
    if (e == hipSuccess && occ < 1) e = hipErrorInvalidConfiguration;
    if (e != hipSuccess) {
      delete plan;
      return dev_status(e, "mixed plan occupancy");
    }
    const size_t budget = std::min(lds_cap, (size_t)(160 * 1024) / occ) - 32;  // 32: the work-item word
    for (int shrink = 0;; ++shrink) {
      size_t lds = 0;
      for (auto& sh : plan->shapes) {
        const DevCode& c = sh.code;
        const size_t base = lsim::layered_tile_lds(c, sh.G), per_row = (size_t)sh.G * c.Z * 16;
        int K = 0;
        if (p->lds_rows == 0)
          K = std::max(0, (int)std::min<size_t>(c.rows, budget > base ? (budget - base) / per_row
                                                                      : 0) - shrink);
        else if (p->lds_rows > 0)
          K = std::min(p->lds_rows, c.rows);
        sh.lds_rows = K;
        lds = std::max(lds, lsim::layered_tile_lds(c, sh.G, K));
      }
      if (lds > lds_cap) {
        delete plan;
        return fail(LSIM_E_INVAL, "lds_rows: the check records of that many rows do not fit the LDS");
      }
      int occ2 = 0;
      e = lsim::mixed_occupancy(threads, dmax, plan->wpe, lds, &occ2);
      if (e != hipSuccess) {
        delete plan;
        return dev_status(e, "mixed plan occupancy");
      }
      if (occ2 >= occ || p->lds_rows != 0 || shrink > 64) {
        plan->lds = lds;
        occ = occ2;
        break;
      }
    }
  }
  // work list, heaviest tiles first: a tile costs about one pass over the
  // base nonzeros plus one barrier per layer, per iteration
  std::vector<int> order(nshapes);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    const DevCode &ca = plan->shapes[a].code, &cb = plan->shapes[b].code;
    return ca.nnz + 2 * ca.rows > cb.nnz + 2 * cb.rows;
  });
  std::vector<int> tile_shape;
  std::vector<int64_t> tile_local;
  for (int s : order) {
    const lsim::LayerShape& sh = plan->shapes[s];
    const int64_t nt = (sh.count + sh.G - 1) / sh.G;
    for (int64_t t = 0; t < nt; ++t) {
      tile_shape.push_back(s);
      tile_local.push_back(t);
    }
  }
  int dev = 0, ncu = 256;
  e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (oms) {
    const int by_lds = std::max(1, (int)((160 * 1024) / (plan->lds + 64)));
    const int by_waves = std::max(1, 32 / (threads / 64));
    plan->grid = ncu * std::min(by_lds, by_waves);
  } else {
    plan->grid = ncu * std::max(1, occ);  // every workgroup resident at once
  }
  const size_t b_shapes = nshapes * sizeof(lsim::LayerShape);
  const size_t b_ts = tile_shape.size() * sizeof(int);
  const size_t b_tl = tile_local.size() * sizeof(int64_t);
  const size_t o_ts = (b_shapes + 255) & ~(size_t)255;
  const size_t o_tl = (o_ts + b_ts + 255) & ~(size_t)255;
  if (e == hipSuccess) e = hipMalloc(&plan->dmem, o_tl + b_tl + 8);
  if (e == hipSuccess) {
    char* d = (char*)plan->dmem;
    plan->d_shapes = (lsim::LayerShape*)d;
    plan->d_tile_shape = (int*)(d + o_ts);
    plan->d_tile_local = (int64_t*)(d + o_tl);
    e = hipMemcpy(plan->d_shapes, plan->shapes.data(), b_shapes, hipMemcpyHostToDevice);
    if (e == hipSuccess && b_ts)
      e = hipMemcpy(plan->d_tile_shape, tile_shape.data(), b_ts, hipMemcpyHostToDevice);
    if (e == hipSuccess && b_tl)
      e = hipMemcpy(plan->d_tile_local, tile_local.data(), b_tl, hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) {
    if (plan->dmem) (void)hipFree(plan->dmem);
    delete plan;
    return dev_status(e, "mixed plan upload");
  }
  *out = plan;
  return LSIM_OK;
}

void lsim_mixed_plan_destroy(lsim_plan* plan) {
  if (!plan) return;
  if (plan->dmem) (void)hipFree(plan->dmem);
  delete plan;
}

lsim_status lsim_mixed_workspace(const lsim_plan* plan, size_t* bytes) {
  if (!plan || !bytes) return fail(LSIM_E_INVAL, "null plan or bytes");
  *bytes = kCounterBytes + plan->state_words * 4;
  return LSIM_OK;
}

lsim_status lsim_mixed_decode(lsim_plan* plan, const void* d_llr_concat, uint8_t* d_bits_concat,
                              float* d_app_concat, void* d_work, size_t work_bytes,
                              int persistent, lsim_stream stream) {
  if (!plan || !d_llr_concat || (!d_bits_concat && !d_app_concat))
    return fail(LSIM_E_INVAL, "bad mixed decode arguments");
  const size_t need = kCounterBytes + plan->state_words * 4;
  if (!d_work || work_bytes < need)
    return fail(LSIM_E_NOMEM, "workspace smaller than lsim_mixed_workspace()");
  if ((uintptr_t)d_work & 15) return fail(LSIM_E_INVAL, "d_work must be 16-byte aligned");
  if (plan->ntiles == 0) return LSIM_OK;
  char* w = (char*)d_work;
  if (plan->p.algo == LSIM_OMS_I8)
    return dev_status(
        lsim::launch_mixed_oms(plan->d_shapes, plan->d_tile_shape, plan->d_tile_local, plan->ntiles,
                               plan->threads, plan->lds, plan->p, (const int8_t*)d_llr_concat,
                               d_bits_concat, d_app_concat, (int*)w, persistent ? 1 : 0,
                               plan->grid, plan->dmax, as_stream(stream)),
        "mixed decode");
  hipError_t e = lsim::launch_mixed(
      plan->d_shapes, (int)plan->shapes.size(), plan->d_tile_shape, plan->d_tile_local,
      plan->ntiles, plan->threads, plan->lds, plan->p, d_llr_concat, d_bits_concat, d_app_concat,
      (uint32_t*)(w + kCounterBytes), (int*)w, persistent ? 1 : 0, plan->grid, plan->dmax,
      plan->wpe, as_stream(stream));
  return dev_status(e, "mixed decode");
}

}  // extern "C"

// ------------------------------------------------------ differentiable forms

extern "C" {

static lsim_status check_wbp(const lsim_code* code, int T, const float* w, const float* llr,
                             int64_t B, float llr_max) {
  if (!code || !w || !llr || B < 1 || B > ((int64_t)1 << 31))
    return fail(LSIM_E_INVAL, "bad weighted BP arguments");
  if (T < 1 || T > 100) return fail(LSIM_E_INVAL, "T must be in 1..100");
  if (!(llr_max > 0.f)) return fail(LSIM_E_INVAL, "llr_max must be > 0");
  return LSIM_OK;
}

lsim_status lsim_wbp_forward(const lsim_code* code, int T, const float* d_w, const float* d_llr,
                             int64_t B, float llr_max, float* d_ckpt, float* d_lpost,
                             lsim_stream stream) {
  lsim_status st = check_wbp(code, T, d_w, d_llr, B, llr_max);
  if (st != LSIM_OK) return st;
  if (!d_lpost) return fail(LSIM_E_INVAL, "null lpost");
  std::string why;
  hipError_t e = lsim::launch_wbp_forward(code->dev, T, d_w, d_llr, B, llr_max, d_ckpt, d_lpost,
                                          as_stream(stream), &why);
  if (!why.empty()) return fail(LSIM_E_UNSUPPORTED, why);
  return dev_status(e, "wbp_forward");
}

lsim_status lsim_wbp_workspace(const lsim_code* code, int T, int64_t B, size_t* bytes) {
  if (!code || !bytes || T < 1 || B < 1) return fail(LSIM_E_INVAL, "bad workspace query");
  *bytes = lsim::wbp_work_bytes(code->dev, T, B);
  return LSIM_OK;
}

lsim_status lsim_wbp_backward(const lsim_code* code, int T, const float* d_w, const float* d_llr,
                              const float* d_ckpt, int64_t B, float llr_max, const float* d_gpost,
                              float* d_gllr, float* d_gw, void* d_work, size_t work_bytes,
                              lsim_stream stream) {
  lsim_status st = check_wbp(code, T, d_w, d_llr, B, llr_max);
  if (st != LSIM_OK) return st;
  if (!d_ckpt || !d_gpost || !d_gllr || !d_gw)
    return fail(LSIM_E_INVAL, "null checkpoint or gradient buffer");
  if (!d_work || work_bytes < lsim::wbp_work_bytes(code->dev, T, B))
    return fail(LSIM_E_NOMEM, "workspace smaller than lsim_wbp_workspace()");
  std::string why;
  hipError_t e = lsim::launch_wbp_backward(code->dev, T, d_w, d_llr, d_ckpt, B, llr_max, d_gpost,
                                           d_gllr, d_gw, d_work, as_stream(stream), &why);
  if (!why.empty()) return fail(LSIM_E_UNSUPPORTED, why);
  return dev_status(e, "wbp_backward");
}

lsim_status lsim_ndm_forward(const float* d_params, const float* d_y, const float* d_no,
                             int64_t B, int64_t S, float* d_llr, lsim_stream stream) {
  if (!d_params || !d_y || !d_no || !d_llr || B < 1 || S < 1)
    return fail(LSIM_E_INVAL, "bad ndm_forward arguments");
  if (((uintptr_t)d_llr) & 15) return fail(LSIM_E_INVAL, "d_llr must be 16-byte aligned");
  return dev_status(lsim::launch_ndm_forward(d_params, d_y, d_no, B, S, d_llr, as_stream(stream)),
                    "ndm_forward");
}

lsim_status lsim_ndm_workspace(int64_t B, int64_t S, size_t* bytes) {
  if (!bytes || B < 1 || S < 1) return fail(LSIM_E_INVAL, "bad workspace query");
  *bytes = lsim::ndm_work_bytes(B, S);
  return LSIM_OK;
}

lsim_status lsim_ndm_backward(const float* d_params, const float* d_y, const float* d_no,
                              const float* d_gllr, int64_t B, int64_t S, float* d_gparams,
                              float* d_gy, void* d_work, size_t work_bytes, lsim_stream stream) {
  if (!d_params || !d_y || !d_no || !d_gllr || !d_gparams || B < 1 || S < 1)
    return fail(LSIM_E_INVAL, "bad ndm_backward arguments");
  if (((uintptr_t)d_gy) & 7) return fail(LSIM_E_INVAL, "d_gy must be 8-byte aligned");
  if (!d_work || work_bytes < lsim::ndm_work_bytes(B, S))
    return fail(LSIM_E_NOMEM, "workspace smaller than lsim_ndm_workspace()");
  return dev_status(lsim::launch_ndm_backward(d_params, d_y, d_no, d_gllr, B, S, d_gparams, d_gy,
                                              d_work, as_stream(stream)),
                    "ndm_backward");
}

lsim_status lsim_bce_workspace(int64_t B, int64_t n, size_t* bytes) {
  if (!bytes || B < 1 || n < 1) return fail(LSIM_E_INVAL, "bad workspace query");
  *bytes = lsim::bce_work_bytes(B, n);
  return LSIM_OK;
}

lsim_status lsim_bce_grad(const float* d_lpost, const uint8_t* d_c, int64_t c_stride, int64_t B,
                          int64_t n, float scale, float* d_g, float* d_loss, void* d_work,
                          size_t work_bytes, lsim_stream stream) {
  if (!d_lpost || !d_c || !d_g || B < 1 || n < 1 || c_stride < n)
    return fail(LSIM_E_INVAL, "bad bce_grad arguments");
  if (d_loss && (!d_work || work_bytes < lsim::bce_work_bytes(B, n)))
    return fail(LSIM_E_NOMEM, "workspace smaller than lsim_bce_workspace()");
  return dev_status(lsim::launch_bce_grad(d_lpost, d_c, c_stride, B, n, scale, d_g, d_loss,
                                          d_work, as_stream(stream)),
                    "bce_grad");
}

lsim_status lsim_adam_step(float* d_p, const float* d_g, float* d_m, float* d_v, int64_t n,
                           float lr, float beta1, float beta2, float eps, int step,
                           lsim_stream stream) {
  if (!d_p || !d_g || !d_m || !d_v || n < 1 || step < 1)
    return fail(LSIM_E_INVAL, "bad adam arguments");
  if (!(beta1 >= 0.f && beta1 < 1.f && beta2 >= 0.f && beta2 < 1.f && eps > 0.f))
    return fail(LSIM_E_INVAL, "bad adam hyper-parameters");
  return dev_status(lsim::launch_adam(d_p, d_g, d_m, d_v, n, lr, beta1, beta2, eps, step,
                                      as_stream(stream)),
                    "adam_step");
}

}  // extern "C"

// ------------------------------------------------------------- whole link

extern "C" lsim_status lsim_link_run(const lsim_link_args* a, lsim_stream stream) {
  if (!a) return fail(LSIM_E_INVAL, "null link arguments");
  const lsim_code* code = a->code;
  lsim_status st = check_params(code, &a->dec);
  if (st != LSIM_OK) return st;
  const int m = a->bits_per_sym;
  if (!a->d_no || !a->d_u || !a->d_llr || !a->d_bits || !a->d_counts || a->B < 1 || a->cw0 < 0 ||
      a->nbins < 1)
    return fail(LSIM_E_INVAL, "bad link arguments");
  if (m != 1 && m != 2 && m != 4 && m != 6)
    return fail(LSIM_E_UNSUPPORTED, "bits_per_sym must be 1, 2, 4 or 6");
  if (a->demap_method != LSIM_DEMAP_EXACT && a->demap_method != LSIM_DEMAP_MAXLOG)
    return fail(LSIM_E_INVAL, "unknown demap method");
  const DevCode& c = code->dev;
  if (c.e_tx % m) return fail(LSIM_E_INVAL, "e_tx is not a multiple of bits_per_sym");
  if ((int64_t)c.n_mother > 48 * 1024)
    return fail(LSIM_E_UNSUPPORTED, "mother code too long for the encoder's LDS tile");
  const bool q8 = a->dec.algo == LSIM_OMS_I8;
  if ((!q8 && !llr_aligned(m, a->d_llr)) || ((uintptr_t)a->d_y & 7))
    return fail(LSIM_E_INVAL, "d_llr must be aligned to 4*m bytes (16 for m=4, 8 for m=2,6), d_y to 8");
  if (q8 && !is_pow2_scale(a->q_scale)) return fail(LSIM_E_INVAL, "q_scale must be a power of two");
  if (a->dec.algo == LSIM_NMS_F32) {
    const size_t need = lsim::layered_state_words(c, a->B) * 4;
    if (!a->d_work || a->work_bytes < need)
      return fail(LSIM_E_NOMEM, "workspace smaller than lsim_decode_workspace()");
    if ((uintptr_t)a->d_work & 15) return fail(LSIM_E_INVAL, "d_work must be 16-byte aligned");
  }
  hipStream_t s = as_stream(stream);
  const int64_t S = c.e_tx / m;
  (void)S;
  hipError_t e = lsim::launch_link_tx(c, m, a->demap_method, a->seed, a->cw0, a->B, a->d_no,
                                      a->d_u, a->d_c, a->d_y, q8 ? nullptr : (float*)a->d_llr,
                                      q8 ? (int8_t*)a->d_llr : nullptr, a->q_scale, a->dec.sat, s);
  std::string why;
  if (e == hipSuccess) {
    if (a->dec.algo == LSIM_NMS_F32)
      e = lsim::launch_layered(c, a->dec, (const float*)a->d_llr, a->B, a->d_bits, nullptr,
                               nullptr, (uint32_t*)a->d_work, s, &why);
    else
      e = lsim::launch_flood(c, a->dec, a->d_llr, a->B, a->d_bits, nullptr, nullptr, nullptr,
                             nullptr, s, &why);
  }
  if (!why.empty()) return fail(LSIM_E_UNSUPPORTED, why);
  if (e == hipSuccess)
    e = lsim::launch_count_errors(a->d_u, c.k, a->d_bits, a->B, c.k, a->d_bin, a->nbins,
                                  a->d_counts, s);
  return dev_status(e, "link_run");
}

// ------------------------------------------------------------------ Polar

struct lsim_polar {
  lsim::DevPolar dev{};
  void* dmem = nullptr;
  uint32_t poly = 0;
};

extern "C" {

lsim_status lsim_polar_construct(int n, int K, double design_ebn0_db, uint8_t* mask) {
  if (n < 1 || n > 10 || K < 1 || K > (1 << n) || !mask || !std::isfinite(design_ebn0_db))
    return fail(LSIM_E_INVAL, "bad polar_construct arguments");
  const int N = 1 << n;
  std::vector<double> z(1, std::exp(-(double)K / N * std::pow(10.0, design_ebn0_db / 10.0)));
  for (int st = 0; st < n; ++st) {
    std::vector<double> nz(2 * z.size());
    for (size_t q = 0; q < z.size(); ++q) {
#pragma clang fp contract(off)
      const double a = 2.0 * z[q];
      const double b = z[q] * z[q];
      nz[2 * q] = a - b;
      nz[2 * q + 1] = b;
    }
    z.swap(nz);
  }
  std::vector<int> order(N);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) {
    return z[a] < z[b] || (z[a] == z[b] && a > b);
  });
  std::memset(mask, 0, N);
  for (int k = 0; k < K; ++k) mask[order[k]] = 1;
  return LSIM_OK;
}

lsim_status lsim_polar_create(int n, const uint8_t* mask, int crc_degree, uint32_t crc_poly,
                              lsim_polar** out) {
  if (!out || !mask || n < 1 || n > 10) return fail(LSIM_E_INVAL, "bad polar_create arguments");
  *out = nullptr;
  const int N = 1 << n, r = crc_degree;
  std::vector<int16_t> info;
  for (int i = 0; i < N; ++i)
    if (mask[i]) info.push_back((int16_t)i);
  const int K = (int)info.size();
  if (K < 1) return fail(LSIM_E_INVAL, "no information index in the mask");
  if (r < 0 || r > 24 || r >= K) return fail(LSIM_E_INVAL, "crc_degree must be 0..24 and below K");
  if (r == 0 ? crc_poly != 0 : (crc_poly >> r) != 0)
    return fail(LSIM_E_INVAL, "crc_poly must have its bits below x^crc_degree (0 without CRC)");
  // remainder of x^(D-1-k+r) mod g for data bit k, by running the CRC
  // register backwards from the last data bit
  const int D = K - r;
  std::vector<uint32_t> tab(std::max(D, 1), 0);
  if (r) {
    const uint32_t msk = r == 32 ? 0xffffffffu : ((1u << r) - 1);
    uint32_t v = crc_poly;
    for (int k = D - 1; k >= 0; --k) {
      tab[k] = v;
      const uint32_t fb = (v >> (r - 1)) & 1u;
      v = (v << 1) & msk;
      if (fb) v ^= crc_poly;
    }
  }
  auto* pc = new lsim_polar;
  const size_t o_mask = 0, o_info = (size_t)N, o_tab = ((o_info + 2 * K) + 3) & ~(size_t)3;
  const size_t bytes = o_tab + tab.size() * 4;
  std::vector<unsigned char> blob(bytes, 0);
  std::memcpy(blob.data() + o_mask, mask, N);
  for (int i = 0; i < N; ++i) blob[o_mask + i] = mask[i] ? 1 : 0;
  std::memcpy(blob.data() + o_info, info.data(), 2 * (size_t)K);
  std::memcpy(blob.data() + o_tab, tab.data(), tab.size() * 4);
  hipError_t e = hipMalloc(&pc->dmem, bytes);
  if (e == hipSuccess) e = hipMemcpy(pc->dmem, blob.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    if (pc->dmem) (void)hipFree(pc->dmem);
    delete pc;
    return dev_status(e, "polar table upload");
  }
  auto* d = reinterpret_cast<unsigned char*>(pc->dmem);
  pc->dev.n = n;
  pc->dev.N = N;
  pc->dev.K = K;
  pc->dev.r = r;
  pc->dev.mask = d + o_mask;
  pc->dev.info = reinterpret_cast<const int16_t*>(d + o_info);
  pc->dev.crc_tab = reinterpret_cast<const uint32_t*>(d + o_tab);
  pc->poly = crc_poly;
  *out = pc;
  return LSIM_OK;
}

void lsim_polar_destroy(lsim_polar* pc) {
  if (!pc) return;
  if (pc->dmem) (void)hipFree(pc->dmem);
  delete pc;
}

lsim_status lsim_polar_query(const lsim_polar* pc, int* N, int* K, int* crc_degree) {
  if (!pc) return fail(LSIM_E_INVAL, "null polar code");
  if (N) *N = pc->dev.N;
  if (K) *K = pc->dev.K;
  if (crc_degree) *crc_degree = pc->dev.r;
  return LSIM_OK;
}

lsim_status lsim_polar_encode(const lsim_polar* pc, const uint8_t* d_data, int64_t B,
                              uint8_t* d_x, lsim_stream stream) {
  if (!pc || !d_data || !d_x || B < 1) return fail(LSIM_E_INVAL, "bad polar_encode arguments");
  return dev_status(lsim::launch_polar_encode(pc->dev, d_data, B, d_x, as_stream(stream)),
                    "polar_encode");
}

lsim_status lsim_polar_decode(const lsim_polar* pc, int list, int use_crc, const float* d_llr,
                              int64_t B, uint8_t* d_bits, float* d_pm, lsim_stream stream) {
  if (!pc || !d_llr || !d_bits || B < 1) return fail(LSIM_E_INVAL, "bad polar_decode arguments");
  if (list != 1 && list != 2 && list != 4 && list != 8 && list != 16 && list != 32)
    return fail(LSIM_E_UNSUPPORTED, "list size must be 1, 2, 4, 8, 16 or 32");
  if (use_crc && pc->dev.r == 0) return fail(LSIM_E_INVAL, "the code has no CRC");
  if (lsim::polar_decode_lds(list, pc->dev.N, pc->dev.K) > 160 * 1024)
    return fail(LSIM_E_UNSUPPORTED, "list state does not fit in LDS");
  return dev_status(lsim::launch_polar_decode(pc->dev, list, use_crc, d_llr, B, d_bits, d_pm,
                                              as_stream(stream)),
                    "polar_decode");
}

}  // extern "C"
