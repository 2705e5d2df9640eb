// Flooding belief-propagation decoders on a QC Tanner graph:
//   SPA  FP32 sum-product (messages clamped to +-llr_max)
//   OMS  int8 offset min-sum (offset, saturation)
//
// One workgroup decodes one codeword with its whole message state in LDS:
// M[E] holds, per edge in canonical order (base nonzero e, lift r -> e*Z+r),
// the variable-to-check message q before a check phase and the
// check-to-variable message r after it; lam[n_dec] holds the channel LLRs.
// A round is two phases separated by barriers:
//   check phase     lane = check (i, r); reads the d_i messages of its row
//                   (addresses e*Z + r: consecutive lanes, no bank conflict),
//                   writes r in place;
//   variable phase  lane = variable node (j, c); gathers the column's r
//                   (addresses e*Z + (c - s) mod Z: rotated contiguous
//                   segments), forms APP = lam + sum r and writes
//                   q = clamp(APP - r).
// Work items are (base row or column, 64-lift block); every wavefront works
// on a single row or column at a time, so the degree loop is uniform.  Items
// are sorted heaviest first and dealt round-robin to the wavefronts.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "dispatch.h"
#include "lsim_internal.h"
#include "spa_math.h"

namespace lsim {

namespace {

struct FloodArgs {
  const void* llr;
  int64_t B;
  uint8_t* bits;
  float* lpost;
  const void* q_in;
  void* r_out;
  void* q_out;
  int iters;
  float llr_max;
  int offset;
  int sat;
};

template <int ALG>
struct Traits;
template <>
struct Traits<LSIM_SPA_F32> {
  using Msg = float;
  using In = float;
};
template <>
struct Traits<LSIM_OMS_I8> {
  using Msg = int8_t;
  using In = int8_t;
};

__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

template <int ALG>
__host__ __device__ inline size_t lds_bytes_for(const DevCode& c) {
  using M = typename Traits<ALG>::Msg;
  return align16((size_t)c.E * sizeof(M)) + align16((size_t)c.n_dec * sizeof(M));
}

template <int NT, int DMAX, int ALG>
__global__ __launch_bounds__(NT) void flood_kernel(DevCode c, FloodArgs a) {
  using M = typename Traits<ALG>::Msg;
  using In = typename Traits<ALG>::In;
  constexpr int NW = NT / 64;
  extern __shared__ __align__(16) unsigned char smem[];
  M* msg = reinterpret_cast<M*>(smem);
  M* lam = reinterpret_cast<M*>(smem + align16((size_t)c.E * sizeof(M)));
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = uni(tid >> 6);
  const int Z = c.Z;
  const int64_t b = blockIdx.x;

  // ---- channel LLRs, zero messages (graph tables are read with scalar
  // loads from the code's device tables)
  const int zm = Z - 1;
  const bool zpow2 = (Z & zm) == 0;
  // sum-product messages live in log2 units (x log2 e) inside the kernel
  const float lmax2 = a.llr_max * kLog2e;
  const In* llr = reinterpret_cast<const In*>(a.llr) + b * (int64_t)c.e_tx;
  for (int v = tid; v < c.n_dec; v += NT) {
    const int x = v - c.tx_lo;
    M l = 0;
    if (x >= 0 && x < c.e_tx) {
      if constexpr (ALG == LSIM_SPA_F32) {
        l = fminf(fmaxf(-llr[x], -a.llr_max), a.llr_max) * kLog2e;
      } else {
        l = (M)min(max(-(int)llr[x], -a.sat), a.sat);
      }
    }
    lam[v] = l;
  }
  if (a.q_in) {
    const M* qi = reinterpret_cast<const M*>(a.q_in) + b * (int64_t)c.E;
    for (int e = tid; e < c.E; e += NT) {
      if constexpr (ALG == LSIM_SPA_F32)
        msg[e] = qi[e] * kLog2e;
      else
        msg[e] = qi[e];
    }
  } else {
    for (int e = tid; e < c.E; e += NT) msg[e] = 0;
  }
  __syncthreads();

  // variable phase; mode 0: q <- clamp(lam + sum r - r), 1: last round
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
          using Acc = typename std::conditional<ALG == LSIM_SPA_F32, float, int>::type;
          Acc rv[DC];
          // byte offset of entry e's edge at lift c: (e*Z + (c - shift) mod Z) * sizeof(M)
          constexpr int SZ = sizeof(M);
          if (zpow2) {
#pragma unroll
            for (int q = 0; q < DC; ++q) {
              const int2 ce = ld_const(c.col_edge, cb + q);
              idx[q] = ((cc * SZ - ce.y * SZ) & (zm * SZ)) | (ce.x * SZ);
            }
          } else {
#pragma unroll
            for (int q = 0; q < DC; ++q) {
              const int2 ce = ld_const(c.col_edge, cb + q);
              int x = cc - ce.y;
              x += x < 0 ? Z : 0;
              idx[q] = (ce.x + x) * SZ;
            }
          }
          unsigned char* mb = reinterpret_cast<unsigned char*>(msg);
#pragma unroll
          for (int q = 0; q < DC; ++q) rv[q] = *reinterpret_cast<M*>(mb + idx[q]);
          Acc acc = lam[v];
#pragma unroll
          for (int q = 0; q < DC; ++q) acc += rv[q];
          if (write_q) {
#pragma unroll
            for (int q = 0; q < DC; ++q) {
              if constexpr (ALG == LSIM_SPA_F32)
                *reinterpret_cast<M*>(mb + idx[q]) =
                    __builtin_amdgcn_fmed3f(acc - rv[q], -lmax2, lmax2);
              else
                *reinterpret_cast<M*>(mb + idx[q]) = (M)min(max(acc - rv[q], -a.sat), a.sat);
            }
          }
          if (final_round) {
            if (a.bits && v < c.k) a.bits[b * (int64_t)c.k + v] = acc < 0;
            if (a.lpost) {
              if constexpr (ALG == LSIM_SPA_F32)
                a.lpost[b * (int64_t)c.n_dec + v] = -acc * kLn2;
              else
                a.lpost[b * (int64_t)c.n_dec + v] = (float)(-acc);
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
        M* row = msg + (size_t)e0 * Z + r;
        with_degree<DMAX>(d, [&](auto deg) {
          constexpr int D = decltype(deg)::value;
          M x[D];
#pragma unroll
          for (int q = 0; q < D; ++q) x[q] = row[q * Z];
          if constexpr (ALG == LSIM_SPA_F32) {
            // sum-product in the sum / difference form, log2 units
            // (spa_math.h); the output sign is the XOR of the other inputs'
            // sign bits (a zero input only ever receives or sends zero
            // magnitudes, so the sign of a zero is immaterial)
            uint32_t sx = 0;
#pragma unroll
            for (int q = 0; q < D; ++q) sx ^= __float_as_uint(x[q]);
            float ee[D], pS[D], pA[D];
#pragma unroll
            for (int q = 0; q < D; ++q) ee[q] = spa_e2(x[q]);
            SpaSA pre{1.f, ee[0]};
#pragma unroll
            for (int q = 1; q < D; ++q) {
              pS[q] = pre.S;
              pA[q] = pre.A;
              if (q + 1 < D) pre.add(ee[q]);
            }
            SpaSA suf{1.f, ee[D - 1]};
#pragma unroll
            for (int q = D - 1; q >= 0; --q) {
              float num, den;
              if (q == D - 1) {
                num = pS[q];
                den = pA[q];
              } else if (q == 0) {
                num = suf.S;
                den = suf.A;
              } else {
                num = fmaf(pS[q], suf.S, pA[q] * suf.A);
                den = fmaf(pS[q], suf.A, pA[q] * suf.S);
              }
              const float rv = spa_log2_ratio(num, den, lmax2);
              const uint32_t sg = (sx ^ __float_as_uint(x[q])) & 0x80000000u;
              row[q * Z] = __uint_as_float(__float_as_uint(rv) | sg);
              if (q < D - 1 && q > 0) suf.add(ee[q]);
            }
          } else {
            uint32_t neg = 0;
#pragma unroll
            for (int q = 0; q < D; ++q) neg |= (x[q] < 0 ? 1u : 0u) << q;
            const uint32_t par = __popc(neg) & 1u;
            int m1 = 255, m2 = 255, i1 = 0;
#pragma unroll
            for (int q = 0; q < D; ++q) {
              const int ax = x[q] < 0 ? -(int)x[q] : (int)x[q];
              m2 = min(m2, max(m1, ax));
              i1 = ax < m1 ? q : i1;
              m1 = min(m1, ax);
            }
#pragma unroll
            for (int q = 0; q < D; ++q) {
              const int mag = max((q == i1 ? m2 : m1) - a.offset, 0);
              row[q * Z] = (M)((par ^ ((neg >> q) & 1u)) ? -mag : mag);
            }
          }
        });
      }
    }
  };

  if (!a.q_in) {
    var_phase(true, false);  // q = lam on every edge
    __syncthreads();
  }
  for (int it = 0; it < a.iters; ++it) {
    const bool last = it + 1 == a.iters;
    check_phase();
    __syncthreads();
    if (last && a.r_out) {
      M* ro = reinterpret_cast<M*>(a.r_out) + b * (int64_t)c.E;
      for (int e = tid; e < c.E; e += NT) {
        if constexpr (ALG == LSIM_SPA_F32)
          ro[e] = msg[e] * kLn2;
        else
          ro[e] = msg[e];
      }
      __syncthreads();
    }
    var_phase(!last || a.q_out != nullptr, last);
    __syncthreads();
  }
  if (a.q_out) {
    M* qo = reinterpret_cast<M*>(a.q_out) + b * (int64_t)c.E;
    for (int e = tid; e < c.E; e += NT) {
      if constexpr (ALG == LSIM_SPA_F32)
        qo[e] = msg[e] * kLn2;
      else
        qo[e] = msg[e];
    }
  }
}

template <int NT, int DMAX, int ALG>
hipError_t launch_t(const DevCode& c, const FloodArgs& a, size_t lds, hipStream_t s) {
  hipError_t e = ensure_dyn_lds((const void*)flood_kernel<NT, DMAX, ALG>, lds);
  if (e != hipSuccess) return e;
  flood_kernel<NT, DMAX, ALG><<<(unsigned)a.B, NT, lds, s>>>(c, a);
  return hipGetLastError();
}

template <int ALG>
hipError_t dispatch(const DevCode& c, int nt, const FloodArgs& a, size_t lds, hipStream_t s) {
  const int dmax = c.max_row_deg > c.max_col_deg ? c.max_row_deg : c.max_col_deg;
#define LSIM_FLOOD_CASE(NT_, D_) \
  if (nt == NT_ && dmax <= D_) return launch_t<NT_, D_, ALG>(c, a, lds, s);
  LSIM_FLOOD_CASE(256, 16)
  LSIM_FLOOD_CASE(256, 24)
  LSIM_FLOOD_CASE(256, 32)
  LSIM_FLOOD_CASE(512, 16)
  LSIM_FLOOD_CASE(512, 24)
  LSIM_FLOOD_CASE(512, 32)
  LSIM_FLOOD_CASE(1024, 16)
  LSIM_FLOOD_CASE(1024, 24)
  LSIM_FLOOD_CASE(1024, 32)
#undef LSIM_FLOOD_CASE
  return hipErrorInvalidValue;
}

}  // namespace

size_t flood_lds_bytes(const DevCode& c, int algo) {
  return algo == LSIM_SPA_F32 ? lds_bytes_for<LSIM_SPA_F32>(c) : lds_bytes_for<LSIM_OMS_I8>(c);
}

hipError_t launch_flood(const DevCode& c, const lsim_decode_params& p, const void* llr, int64_t B,
                        uint8_t* bits, float* lpost, const void* q_in, void* r_out, void* q_out,
                        hipStream_t s, std::string* why) {
  const size_t lds = flood_lds_bytes(c, p.algo);
  if (lds > 160 * 1024) {
    *why = "flooding decoder state (" + std::to_string(lds) + " B) exceeds the 160 KiB LDS";
    return hipSuccess;
  }
  FloodArgs a{llr, B, bits, lpost, q_in, r_out, q_out, p.iters, p.llr_max,
              (int)p.offset, p.sat};
  const int nt = p.threads ? p.threads : (p.algo == LSIM_SPA_F32 ? 512 : 256);
  if (p.algo == LSIM_SPA_F32) return dispatch<LSIM_SPA_F32>(c, nt, a, lds, s);
  return dispatch<LSIM_OMS_I8>(c, nt, a, lds, s);
}

}  // namespace lsim
