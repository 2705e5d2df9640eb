// Device view of an LDPC code, shared by the kernels and the host API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lsim {

// Device view of a code: the decoded Tanner graph plus encoder tables.  All
// pointers are device memory owned by the lsim_code.
struct DevCode {
  int Z, mb, nb, kb, rows, cols, nnz, E, n_dec, m_dec, k, n_mother, tx_lo, e_tx, family;
  int max_row_deg, max_col_deg, n_cn_tasks, n_vn_tasks;
  const int* row_ptr;    // rows+1; entries of base row i: row_ptr[i]..row_ptr[i+1]-1 (row-major)
  const int* ent_col;    // nnz
  const int* ent_shift;  // nnz
  const int* col_ptr;    // cols+1
  const int* col_ent;    // entry ids of each column, rows ascending
  const int* cn_tasks;   // (row << 16) | lift0, heaviest first
  const int* vn_tasks;   // (col << 16) | lift0, heaviest first
  const int* enc_ptr;    // mb+1; encoder entries of base row i: enc_ptr[i]..enc_ptr[i+1]-1
  const int2* enc_cz;    // (col * Z, shift) of the row's entries the encoder XORs: information
                         // columns for the dual-diagonal rows, columns < kb+4 for extension rows
  const int2* col_edge;  // per column entry (col_ptr order): (e * Z, shift of e)
  const int2* ent_cz;    // per entry (row-major): (col * Z, shift)
  // Layered decoder: a row whose last entry lies in a column of degree one
  // owns that column ("private"); its posteriors need no LDS and travel with
  // the row's check state.  Every other column is "shared" and gets an LDS
  // slot.
  int n_shared, n_priv;
  int n_deg1_inner;        // degree-one columns that do not close their row
  const int* row_priv;    // rows: private slot of the row (0..n_priv-1) or -1
  const int* shared_col;  // n_shared: column of each LDS slot, ascending
  const int* priv_row;    // n_priv: row of each private slot, ascending
  const int2* ent_lz;     // per entry (row-major): (LDS slot * Z, shift) of a shared
                          // column; (col * Z, shift) of a private one
  // Layered schedule, one entry per position p of the visiting order: (row,
  // col * Z - tx_lo and shift of the row's private column -- its node at lane
  // r has channel LLR offset col * Z - tx_lo + (r + shift) mod Z -- or
  // (-2^30, 0) without one, and 1 when a barrier must follow position p
  // because the next layer shares an LDS column with a layer since the last
  // barrier; the last position always has one).
  const int4* layer_pos;
};


// Read-only device tables through the constant address space: with a
// wave-uniform index the compiler emits scalar loads (no VALU, no LDS).
__device__ __forceinline__ int ld_const(const int* p, int i) {
  return ((const __attribute__((address_space(4))) int*)p)[i];
}
__device__ __forceinline__ int2 ld_const(const int2* p, int i) {
  const __attribute__((address_space(4))) int* q =
      (const __attribute__((address_space(4))) int*)p;
  return make_int2(q[2 * i], q[2 * i + 1]);
}
__device__ __forceinline__ int4 ld_const(const int4* p, int i) {
  const __attribute__((address_space(4))) int* q =
      (const __attribute__((address_space(4))) int*)p;
  return make_int4(q[4 * i], q[4 * i + 1], q[4 * i + 2], q[4 * i + 3]);
}

}  // namespace lsim
