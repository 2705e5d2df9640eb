// Layered normalized min-sum (FP32) tile decoder shared by the one-code
// launch (k_layered.hip) and the persistent mixed-shape launch (k_mixed.hip).
//
// A tile is G codewords of one code decoded by one workgroup: lane
// (g, r) = (tid / Z, tid % Z) owns check r of every layer of codeword g.  A
// QC row block meets each variable node at most once, so the Z checks of a
// layer update the posteriors without conflicts; a barrier separates a
// layer from the next one only where they (or a layer since the last
// barrier) meet a common LDS column, as the code's schedule table says.
//
// Posteriors live where their readers are.  A column met by several rows is
// read by every lane of those rows, so its Z posteriors sit in LDS ("shared"
// columns, one LDS slot each).  A column of degree one that is the last entry
// of its row (the extension parity columns of a BG-shaped code) is read and
// written only by lane r of that row ("private" column).  Such a variable
// node has no other check, so the message it sends is its channel value in
// every iteration: lane r reads it from the channel LLRs and keeps no
// posterior for it until the last iteration writes lam + r_new out.  For
// the BG1-shaped workload (26 shared of 68 columns at Z = 384) a codeword's
// LDS shrinks from 104 KB to 39 KB, so more codewords are resident per CU.
//
// The state of check (i, r) between iterations is one 12-byte record
// (alpha*m1, alpha*m2, sign bits | i1 << 27) streamed through device memory
// in [codeword][layer][Z] order: one coalesced three-word load and store per
// lane and layer, plus the four-byte channel value of a private column.
//
// Arithmetic follows the layered min-sum update one IEEE single-precision
// operation at a time (no fused multiply-add): t = APP - r_old (the channel
// value for a private column); r_new = sign * (alpha * (v == i1 ? m2 : m1));
// APP = t + r_new.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "dispatch.h"
#include "lds.h"
#include "lsim_internal.h"

// one IEEE single-precision operation at a time in everything below
#pragma clang fp contract(off)

namespace lsim {
namespace layered {

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

constexpr size_t kLdsBytes = 160 * 1024;  // LDS per CU (and per workgroup) on gfx950

// LDS of a tile: the shared posteriors of its G codewords, then the check
// records of the rows kept in LDS (K of them per codeword).
__host__ __device__ inline size_t tile_lds_bytes(const DevCode& c, int G, int K = 0) {
  return align16((size_t)G * c.n_shared * c.Z * 4) + (size_t)G * K * c.Z * 16;
}

struct TileIO {
  const float* llr;     // [count][e_tx] of this shape
  uint8_t* bits;        // [count][k]
  float* lpost;         // [count][n_dec]
  float* r_out;         // [count][E]
  uint32_t* state;      // [count][rows][Z][3] check records (rows >= lds_rows)
  int64_t count;
  int lds_rows;         // rows whose records stay in LDS
};

// A check record in device memory: three consecutive words, 4-byte aligned.
struct Rec3 {
  uint32_t x, y, z;
};

// Record at word `off` from a base common to the workgroup (the byte offset
// is formed in 32 bits: the scalar-base plus lane-offset access form).
__device__ __forceinline__ uint4 ld_rec(const uint32_t* base, uint32_t off) {
  const Rec3 v = ldg_at(reinterpret_cast<const Rec3*>(base), off * 4u);
  return make_uint4(v.x, v.y, v.z, 0u);
}

__device__ __forceinline__ void st_rec(uint32_t* base, uint32_t off, uint32_t x, uint32_t y,
                                       uint32_t z) {
  stg_at(reinterpret_cast<Rec3*>(base), off * 4u, Rec3{x, y, z});
}

__device__ __forceinline__ int rot_lift(int r, int s, int Z) {
  const int x = r + s;
  return x >= Z ? x - Z : x;
}

template <int NT, int DMAX, bool LATE_STORE>
__device__ __forceinline__ void decode_tile(const DevCode& c, int G, int64_t tile, const TileIO& io,
                                            int iters, float alpha) {
  const int Z = c.Z;
  const int tid = threadIdx.x;
  const int64_t cw0 = tile * G;
  const int gmax = (int)min<int64_t>(G, io.count - cw0);
  const int nsz = c.n_shared * Z;  // shared posteriors per codeword

  // shared posteriors from the channel (punctured and unsent nodes: 0); the
  // tile's LDS starts at byte 0 (the kernels have no static LDS)
  for (int idx = tid; idx < G * nsz; idx += NT) {
    const int g = idx / nsz, rem = idx - g * nsz;
    const int slot = rem / Z, z = rem - slot * Z;
    const int x = c.shared_col[slot] * Z + z - c.tx_lo;
    float l = 0.f;
    if (g < gmax && x >= 0 && x < c.e_tx) l = -io.llr[(cw0 + g) * c.e_tx + x];
    lds_st<float>(idx * 4, l);
  }
  __syncthreads();

  const int g = tid / Z;
  const int r = tid - g * Z;
  const bool active = g < gmax;
  const int64_t cw = cw0 + (active ? g : 0);
  // LDS byte address of this lane's codeword's shared posteriors
  const int app_b = vreg((active ? g : 0) * nsz * 4);
  const int Z4 = Z * 4, zm4 = (Z - 1) * 4, r4 = vreg(r * 4);
  const bool zpow2 = (Z & (Z - 1)) == 0;
  // Device addresses as a base common to the workgroup (scalar registers)
  // plus a 32-bit per-lane offset: a per-lane 64-bit pointer costs two
  // VGPRs, and under the six-wavefront budget it would be spilled and its
  // reload would wait on the record prefetch.
  const int ga = active ? g : 0;
  uint32_t* const st_t = io.state + (size_t)cw0 * c.rows * Z * 3;
  const uint32_t st_l = (uint32_t)((ga * c.rows * Z + r) * 3);
  const uint32_t* const llr_t = reinterpret_cast<const uint32_t*>(io.llr) + cw0 * c.e_tx;
  const uint32_t llr_l = (uint32_t)(ga * c.e_tx);
  uint8_t* const bits_t = io.bits ? io.bits + cw0 * c.k : nullptr;
  float* const lpost_t = io.lpost ? io.lpost + cw0 * c.n_dec : nullptr;
  const int Z3 = Z * 3;
  // records of rows 0 .. K-1 in LDS after the shared posteriors, lane-private
  // (written and read back by the same lane, so no barrier orders them)
  const int K = io.lds_rows;
  const int rec_b = (int)align16((size_t)G * nsz * 4) + (((active ? g : 0) * K) * Z + r) * 16;

  // Variable node of the private entry of row i at this lane.
  auto priv_vn = [&](int i) {
    const int2 en = ld_const(c.ent_lz, uni(ld_const(c.row_ptr, i + 1)) - 1);
    return en.x + rot_lift(r, en.y, Z);
  };

  // Layers are visited in the code's schedule order (one table entry per
  // position: row, private column's LLR offset and shift, barrier after).
  // The record of the next layer (and the channel value of its private
  // column) is loaded one layer ahead so its memory latency overlaps the
  // current layer.  A decoded graph has at least three layers, so a
  // prefetched layer was stored at least two layers earlier.  In the first
  // iteration the check state is zero.
  const int rows = c.rows;
  uint4 nrec = make_uint4(0u, 0u, 0u, 0u);
  // The channel value is kept as loaded and negated where it is used
  // (arithmetic on it here would wait for the load); a node without one
  // reads as -0 and so enters as +0.  One table entry gives the row and its
  // private column (an offset below zero without one), so the addresses wait
  // on a single scalar load.
  auto fetch = [&](const int4 pe, int nit) {
    uint4 v = make_uint4(0u, 0u, 0u, 0x80000000u);
    if (active && nit < iters) {
      const int ni = pe.x;
      if (nit >= 1) {
        const uint4 rr = ni < K ? lds_ld<uint4>(rec_b + ni * Z * 16) : ld_rec(st_t, st_l + (uint32_t)(ni * Z3));
        v.x = rr.x;
        v.y = rr.y;
        v.z = rr.z;
      }
      // (r + shift) mod Z as min(x, x - Z) on unsigned x; one unsigned
      // compare covers both ends of the range and the rows without a
      // private column
      const uint32_t xr = (uint32_t)(r + pe.z);
      const int x = pe.y + (int)min(xr, xr - (uint32_t)Z);
      if ((uint32_t)x < (uint32_t)c.e_tx) v.w = ldg_at(llr_t, (llr_l + (uint32_t)x) * 4u);
    }
    return v;
  };
  int4 pos_n = ld_const(c.layer_pos, 0);
  nrec = fetch(pos_n, 0);
  // With LATE_STORE the record a layer computes is stored at the start of
  // the next layer, beside that layer's prefetch.  Stores and loads share
  // one counter, so the wait for the prefetched record at the top of a layer
  // also waits for every store in flight; a store issued at the end of the
  // layer it was computed in stalls the next layer, one issued a layer
  // earlier has had the whole layer to complete.  The same lane reads the
  // record back at least two layers later (a decoded graph has at least
  // three layers).  Carrying the record across the degree-specialised
  // bodies costs register copies, and only the six-wavefront one-code
  // launch gains (BG1-shaped code at Z = 384: 1.91 -> 1.85 ms; the
  // persistent mixed launch loses 5 %, the 256-thread BG2 launch 1 %).
  bool pend = false;
  uint32_t pend_off = 0, pend_x = 0, pend_y = 0, pend_z = 0;
  for (int it = 0; it < iters; ++it) {
    for (int p = 0; p < rows; ++p) {
      const int4 pe = pos_n;
      const int i = uni(pe.x);
      const int e0 = uni(ld_const(c.row_ptr, i));
      const int d = uni(ld_const(c.row_ptr, i + 1)) - e0;
      const bool priv = uni(ld_const(c.row_priv, i)) >= 0;
      const uint4 rec = nrec;
      {
        int np = p + 1, nit = it;
        if (np == rows) {
          np = 0;
          ++nit;
        }
        pos_n = ld_const(c.layer_pos, np);
        // Take this layer's record (loaded a layer ago) before the next
        // prefetch is issued.  Loads and stores share one counter and the
        // compiler waits for all of them at once, so a first use after the
        // next prefetch would wait for that prefetch too (mixed batch 1.23 ->
        // 1.18 ms).
        asm volatile("" ::"v"(rec.x), "v"(rec.y), "v"(rec.z), "v"(rec.w));
        nrec = fetch(pos_n, nit);
        if (LATE_STORE && pend) st_rec(st_t, pend_off, pend_x, pend_y, pend_z);
        pend = false;
      }
      const float a1 = __uint_as_float(rec.x), a2 = __uint_as_float(rec.y);
      const uint32_t pk = rec.z;
      // One check update of degree D; with PRIV the last entry's message is
      // its channel value (prefetched with the record), the others' posteriors
      // are in LDS.
      auto update = [&](auto deg, auto privc) {
        constexpr int D = decltype(deg)::value;
        constexpr bool PRIV = decltype(privc)::value;
        constexpr int DL = PRIV ? D - 1 : D;  // entries whose posterior is in LDS
        if constexpr (DL >= 1) {
          int addr[DL];
          float tv[D];
          // LDS byte address of the variable node of entry e at lift r:
          // app_b + slot*Z*4 + ((r + shift) mod Z)*4; the reduction is a mask
          // for a power-of-two lift, else min(x, x - Z*4) on unsigned x
          if (zpow2) {
#pragma unroll
            for (int q = 0; q < DL; ++q) {
              const int2 en = ld_const(c.ent_lz, e0 + q);
              addr[q] = app_b + en.x * 4 + ((r4 + en.y * 4) & zm4);
            }
          } else {
#pragma unroll
            for (int q = 0; q < DL; ++q) {
              const int2 en = ld_const(c.ent_lz, e0 + q);
              const uint32_t x = (uint32_t)(r4 + en.y * 4);
              addr[q] = app_b + en.x * 4 + (int)min(x, x - (uint32_t)Z4);
            }
          }
#pragma unroll
          for (int q = 0; q < DL; ++q) tv[q] = lds_ld<float>(addr[q]);
          if constexpr (PRIV) tv[D - 1] = -__uint_as_float(rec.w);
          const int i1_old = (int)(pk >> 27);
          // sign of a zero never reaches a nonzero value (a zero input forces
          // every other output magnitude to zero), so sign bits are used as is
          uint32_t sx = 0;
          float m1 = INFINITY, m2 = INFINITY;
#pragma unroll
          for (int q = 0; q < D; ++q) {
            float t = tv[q];
            if (!(PRIV && q == D - 1)) {
              const float mag = q == i1_old ? a2 : a1;
              const float rold =
                  __uint_as_float(__float_as_uint(mag) | ((pk << (31 - q)) & 0x80000000u));
              t = __fsub_rn(t, rold);
              tv[q] = t;
            }
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
          float pout = 0.f;
#pragma unroll
          for (int q = D - 1; q >= 0; --q) {
            const bool at_min = fabsf(tv[q]) == m1;
            const float mag = at_min ? b2 : b1;
            i1 = at_min ? q : i1;
            const uint32_t sg = (sx ^ __float_as_uint(tv[q])) & 0x80000000u;
            const float out = __fadd_rn(tv[q], __uint_as_float(__float_as_uint(mag) | sg));
            if (PRIV && q == D - 1)
              pout = out;
            else
              lds_st<float>(addr[q < DL ? q : 0], out);
            npk = (npk << 1) | (sg >> 31);  // descending q: bit q ends at q
          }
          npk |= (uint32_t)i1 << 27;
          if (i < K)
            lds_st<uint4>(rec_b + i * Z * 16,
                          make_uint4(__float_as_uint(b1), __float_as_uint(b2), npk, 0u));
          else if (it < iters - 1 || io.r_out) {  // the last records serve only the export
            if constexpr (LATE_STORE) {
              pend = true;
              pend_off = st_l + (uint32_t)(i * Z3);
              pend_x = __float_as_uint(b1);
              pend_y = __float_as_uint(b2);
              pend_z = npk;
            } else {
              st_rec(st_t, st_l + (uint32_t)(i * Z3), __float_as_uint(b1), __float_as_uint(b2),
                     npk);
            }
          }
          if (PRIV && it == iters - 1) {
            // the private posterior is final: write it out now
            const int v = priv_vn(i);
            if (bits_t && v < c.k) stg_at(bits_t, (uint32_t)(ga * c.k + v), (uint8_t)(pout < 0.f));
            if (lpost_t) stg_at(lpost_t, (uint32_t)(ga * c.n_dec + v) * 4u, -pout);
          }
        }
      };
      if (active) {
        with_degree<DMAX>(d, [&](auto deg) {
          if (priv)
            update(deg, std::true_type{});
          else
            update(deg, std::false_type{});
        });
      }
      // only between layers that meet a common LDS column (and at the end
      // of the iteration): the others' posteriors are disjoint
      if (uni(pe.w)) lds_barrier();
    }
  }

  if (LATE_STORE && pend) st_rec(st_t, pend_off, pend_x, pend_y, pend_z);

  // shared posteriors out of LDS (private ones were written in the last
  // iteration)
  for (int idx = tid; idx < gmax * nsz; idx += NT) {
    const int gg = idx / nsz, rem = idx - gg * nsz;
    const int slot = rem / Z, z = rem - slot * Z;
    const int v = c.shared_col[slot] * Z + z;
    const float x = lds_ld<float>(idx * 4);
    if (io.bits && v < c.k) io.bits[(cw0 + gg) * c.k + v] = x < 0.f;
    if (io.lpost) io.lpost[(cw0 + gg) * c.n_dec + v] = -x;
  }
  if (io.r_out && active) {
    for (int i = 0; i < c.rows; ++i) {
      const uint4 rc = i < K ? lds_ld<uint4>(rec_b + i * Z * 16) : ld_rec(st_t, st_l + (uint32_t)(i * Z3));
      const float a1 = __uint_as_float(rc.x), a2 = __uint_as_float(rc.y);
      const uint32_t pk = rc.z;
      const int i1 = (int)(pk >> 27);
      const int rb = c.row_ptr[i];
      for (int e = rb; e < c.row_ptr[i + 1]; ++e) {
        const int q = e - rb;
        const float mag = q == i1 ? a2 : a1;
        io.r_out[cw * (int64_t)c.E + (int64_t)e * Z + r] = ((pk >> q) & 1u) ? -mag : mag;
      }
    }
  }
}

// Instances: threads x largest row degree.
#define LSIM_LAYERED_INSTANCES(X) \
  X(256, 16) X(256, 24) X(256, 27) X(384, 16) X(384, 24) X(384, 27) X(512, 16) X(512, 24) \
  X(512, 27) X(768, 16) X(768, 24) X(768, 27) X(1024, 16) X(1024, 24) X(1024, 27)

// Every instance comes in two register budgets: the compiler's own (WPE 1)
// and at most 80 VGPRs, six wavefronts per SIMD (WPE 6), where the largest
// degree bodies spill a few values to scratch.  The launchers take the
// second when it at least doubles the workgroups a CU holds (the BG1 code
// at Z = 384: two 768-thread workgroups instead of one).
#define LSIM_LAYERED_INSTANCES_W(X) \
  X(256, 16, 1) X(256, 24, 1) X(256, 27, 1) X(384, 16, 1) X(384, 24, 1) X(384, 27, 1) \
  X(512, 16, 1) X(512, 24, 1) X(512, 27, 1) X(768, 16, 1) X(768, 24, 1) X(768, 27, 1) \
  X(1024, 16, 1) X(1024, 24, 1) X(1024, 27, 1) X(256, 16, 6) X(256, 24, 6) X(256, 27, 6) \
  X(384, 16, 6) X(384, 24, 6) X(384, 27, 6) X(512, 16, 6) X(512, 24, 6) X(512, 27, 6) \
  X(768, 16, 6) X(768, 24, 6) X(768, 27, 6) X(1024, 16, 6) X(1024, 24, 6) X(1024, 27, 6)

}  // namespace layered
}  // namespace lsim
