// Polar codes: encoder (CRC attachment + transform) and the SC / SCL /
// SCL-CRC decoders (Polar codes and these decoders are among the FEC
// features, Sec. III-B; the SCL decoder is the paper's example of an
// algorithm that needs a custom kernel, Sec. IV-A).
//
// Decoder: one wavefront per codeword, everything in LDS.  Per list slot p
// the LLRs of the current node at stage s (2^s values, s <= n - 2) sit at
// alpha[p][2^s .. 2^{s+1}); stage n - 1 is never stored: it is read only
// while stage n - 2 is computed (four times per codeword) and is formed on
// the fly from the channel LLRs (f for the first half of the leaves, g with
// the first half's partial sums for the second).  The partial sums of the
// pending left child at stage s sit at bl[p][2^s ..]; the channel LLRs are
// shared.  Leaf i recomputes stages ctz(i) .. 0 (g at the top stage from
// the left sibling's sums, f below), decides, and writes the merged
// partial sums of its trailing-ones subtree in one step:
// x[e] = u_i xor (xor over s < t with bit s of e clear of bl[s][e mod 2^s]),
// t the number of trailing ones of i.  With lambda = ln P(0)/P(1):
// f(a, b) = sgn(a) sgn(b) min(|a|, |b|), g(a, b, x) = b + (1 - 2x) a, the
// path metric adds |lambda| when a bit disagrees with [lambda < 0].  At an
// information leaf the 2 * nact candidates are ranked by (metric, parent
// slot, bit) against each other's metrics read with readlane, the best L
// survive; a parent whose two children survive keeps bit 0 and copies its
// state to the lowest free slot for bit 1 (only the stages still to be
// read: alpha above stage ctz(i + 1) and the pending left sums of the set
// bits of i).  Active slots are always 0 .. nact - 1.
#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "lsim_internal.h"

namespace lsim {

namespace {

constexpr int kPolThreads = 64;

struct PolarLds {
  float* ch;
  float* al;
  uint8_t* bl;
  uint8_t* rec;  // [K][L]: (parent slot << 1) | bit of every slot at each information leaf
  int astr;
};

__host__ __device__ inline int polar_kpad(int K) { return (K + 15) & ~15; }
// alpha stride per slot: stages 0 .. n-2 need N/2 values (N = 2: stage 0)
__host__ __device__ inline int polar_astr(int N) { return N >= 4 ? N / 2 : 2; }

template <int L>
__host__ __device__ inline size_t polar_lds_bytes(int N, int K) {
  return (size_t)N * 4 + (size_t)L * polar_astr(N) * 4 + (size_t)L * N + (size_t)L * polar_kpad(K);
}

template <int L>
__device__ __forceinline__ PolarLds polar_lds(unsigned char* sm, int N, int K) {
  PolarLds s;
  s.astr = polar_astr(N);
  s.ch = reinterpret_cast<float*>(sm);
  s.al = s.ch + N;
  s.bl = reinterpret_cast<uint8_t*>(s.al + (size_t)L * s.astr);
  s.rec = s.bl + (size_t)L * N;
  return s;
}

__device__ __forceinline__ float pol_f(float a, float c) {
  const float m = fminf(fabsf(a), fabsf(c));
  return ((a < 0.f) != (c < 0.f)) ? -m : m;
}

__device__ __forceinline__ float pol_g(float a, float c, uint8_t x) { return x ? c - a : c + a; }

template <int L>
__global__ __launch_bounds__(kPolThreads) void polar_decode_kernel(DevPolar pc,
                                                                   const float* __restrict__ llr,
                                                                   int64_t B, int use_crc,
                                                                   uint8_t* __restrict__ bits,
                                                                   float* __restrict__ pm_out) {
  extern __shared__ __align__(16) unsigned char sm[];
  __shared__ float pm[L];
  __shared__ int pass[L];
  const int N = pc.N, n = pc.n, K = pc.K, r = pc.r;
  const PolarLds s = polar_lds<L>(sm, N, K);
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x;
  for (int e = lane; e < N; e += kPolThreads) s.ch[e] = -llr[b * N + e];
  if (lane < L) pm[lane] = 0.f;
  __syncthreads();
  int nact = 1, j = 0;
  const int A = s.astr;
  const int lgA = N >= 4 ? n - 1 : 1;  // A = 1 << lgA
  for (int i = 0; i < N; ++i) {
    // ---- LLRs down to the leaf (stage n - 1 only on the fly when n >= 2)
    const int top = i == 0 ? n - 1 : __builtin_ctz(i);
    for (int st = top; st >= 0; --st) {
      if (n >= 2 && st == n - 1) continue;
      const int h = 1 << st;
      const int cnt = nact << st;
      const bool use_g = st == top && i != 0;
      if (st + 2 < n) {
        // parent stored at stage st + 1 (the common case): separate f and g
        // loops, slot rows addressed by shifts
        if (use_g) {
          for (int idx = lane; idx < cnt; idx += kPolThreads) {
            const int p = idx >> st, e = idx & (h - 1);
            const float* par = s.al + (p << lgA) + 2 * h;
            s.al[(p << lgA) + h + e] = pol_g(par[e], par[e + h], s.bl[(p << n) + h + e]);
          }
        } else {
          for (int idx = lane; idx < cnt; idx += kPolThreads) {
            const int p = idx >> st, e = idx & (h - 1);
            const float* par = s.al + (p << lgA) + 2 * h;
            s.al[(p << lgA) + h + e] = pol_f(par[e], par[e + h]);
          }
        }
      } else if (st + 2 == n) {
        // parent is stage n - 1, formed here from the channel (f for the
        // first half of the leaves, g with the first half's sums after)
        const int Q = N >> 1;
        const bool second = i >= Q;
        for (int idx = lane; idx < cnt; idx += kPolThreads) {
          const int p = idx >> st, e = idx & (h - 1);
          float a, c;
          if (second) {
            a = pol_g(s.ch[e], s.ch[e + Q], s.bl[(p << n) + Q + e]);
            c = pol_g(s.ch[e + h], s.ch[e + h + Q], s.bl[(p << n) + Q + e + h]);
          } else {
            a = pol_f(s.ch[e], s.ch[e + Q]);
            c = pol_f(s.ch[e + h], s.ch[e + h + Q]);
          }
          s.al[(p << lgA) + h + e] =
              use_g ? pol_g(a, c, s.bl[(p << n) + h + e]) : pol_f(a, c);
        }
      } else {
        // n == 1: the parent is the channel
        for (int idx = lane; idx < cnt; idx += kPolThreads) {
          const int p = idx >> st, e = idx & (h - 1);
          const float a = s.ch[e], c = s.ch[e + h];
          s.al[(p << lgA) + h + e] = use_g ? pol_g(a, c, s.bl[(p << n) + h + e]) : pol_f(a, c);
        }
      }
      __syncthreads();
    }
    // ---- decision
    const bool info = pc.mask[i] != 0;
    if (!info) {
      if (lane < nact) {
        const float l = s.al[lane * A + 1];
        if (l < 0.f) pm[lane] = pm[lane] + (-l);
      }
      __syncthreads();
    } else {
      const int ncand = 2 * nact;
      float mc = INFINITY;
      if (lane < ncand) {
        const int p = lane >> 1, bit = lane & 1;
        const float l = s.al[p * A + 1];
        const int hard = l < 0.f;
        mc = bit == hard ? pm[p] : pm[p] + fabsf(l);
      }
      int rank = 0;
      for (int c2 = 0; c2 < ncand; ++c2) {
        const float m2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mc), c2));
        rank += (m2 < mc) || (m2 == mc && c2 < lane);
      }
      const uint32_t sv = (uint32_t)__ballot(lane < ncand && rank < L);
      // parents with a surviving child / with both children surviving
      uint32_t anyp = 0, bothp = 0;
#pragma unroll
      for (int p = 0; p < L; ++p) {
        const uint32_t two = (sv >> (2 * p)) & 3u;
        anyp |= (two != 0u) << p;
        bothp |= (two == 3u) << p;
      }
      uint32_t freem = ~anyp & ((1u << L) - 1u);
      __syncthreads();  // every lane has read pm and the leaf LLRs
      // each parent with two survivors copies the state still to be read
      // (LLR stages above ctz(i + 1), and here simply its whole row of left
      // sums) to the lowest free slot, in parent order
      const int t = i + 1 < N ? __builtin_ctz(i + 1) : n;
      const int alo = 2 << t;
      int mydest = -1;
      for (uint32_t mb = bothp; mb; mb &= mb - 1u) {
        const int p = __builtin_ctz(mb);
        const int d = __builtin_ctz(freem);
        freem &= freem - 1u;
        if ((lane >> 1) == p) mydest = d;
        float* ad = s.al + d * A;
        const float* as = s.al + p * A;
        if (lane >= alo && lane < 4 && lane < A) ad[lane] = as[lane];
        if (A >= 4) {  // 16-byte rows from offset 4 on
          const int q0 = (alo > 4 ? alo : 4) >> 2;
          for (int q = q0 + lane; q < (A >> 2); q += kPolThreads)
            reinterpret_cast<float4*>(ad)[q] = reinterpret_cast<const float4*>(as)[q];
        }
        uint8_t* bd = s.bl + d * N;
        const uint8_t* bs = s.bl + p * N;
        if (N >= 16) {
          for (int q = lane; q < (N >> 4); q += kPolThreads)
            reinterpret_cast<uint4*>(bd)[q] = reinterpret_cast<const uint4*>(bs)[q];
        } else if (lane < N) {
          bd[lane] = bs[lane];
        }
      }
      // metrics and the new bit of every surviving candidate
      if (lane < ncand && ((sv >> lane) & 1u)) {
        const int p = lane >> 1, bit = lane & 1;
        const bool both = (bothp >> p) & 1u;
        const int slot = (both && bit) ? mydest : p;
        pm[slot] = mc;
        s.rec[j * L + slot] = (uint8_t)((p << 1) | bit);
      }
      nact = min(2 * nact, L);
      ++j;
      __syncthreads();
    }
    // ---- partial sums of the trailing-ones subtree, one step
    const int t = __builtin_ctz(~i);
    if (t < n) {
      const int cnt = nact << t;
      for (int idx = lane; idx < cnt; idx += kPolThreads) {
        const int p = idx >> t, e = idx & ((1 << t) - 1);
        uint8_t x = info ? (uint8_t)(s.rec[(j - 1) * L + p] & 1) : 0;
        for (int st = 0; st < t; ++st)
          if (!((e >> st) & 1)) x ^= s.bl[p * N + (1 << st) + (e & ((1 << st) - 1))];
        s.bl[p * N + (1 << t) + e] = x;
      }
      __syncthreads();
    }
  }
  // ---- each slot's information bits by tracing its history back, into
  // the (now unused) LLR area; then CRC checks and the decision
  uint8_t* tb = reinterpret_cast<uint8_t*>(s.al);  // [L][K] bytes <= L * A * 4
  if (lane < nact) {
    int slot = lane;
    for (int jj = K - 1; jj >= 0; --jj) {
      const int v = s.rec[jj * L + slot];
      tb[lane * K + jj] = (uint8_t)(v & 1);
      slot = v >> 1;
    }
  }
  __syncthreads();
  if (use_crc && r > 0) {
    const int D = K - r;
    for (int p = 0; p < nact; ++p) {
      uint32_t acc = 0;
      for (int k = lane; k < D; k += kPolThreads)
        if (tb[p * K + k]) acc ^= pc.crc_tab[k];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
      if (lane == 0) {
        uint32_t got = 0;
        for (int q = 0; q < r; ++q) got = (got << 1) | tb[p * K + D + q];
        pass[p] = got == acc;
      }
    }
  }
  __syncthreads();
  int choice = 0;
  {
    // slots ordered by (metric, slot); first passing one under CRC
    int best = -1, first = -1;
    for (int q = 0; q < nact; ++q) {
      // q-th slot in the order
      int sel = -1;
      for (int p = 0; p < nact; ++p) {
        int rk = 0;
        for (int p2 = 0; p2 < nact; ++p2)
          rk += (pm[p2] < pm[p]) || (pm[p2] == pm[p] && p2 < p);
        if (rk == q) sel = p;
      }
      if (first < 0) first = sel;
      if (use_crc && r > 0 && best < 0 && pass[sel]) best = sel;
    }
    choice = best >= 0 ? best : first;
  }
  const int D = K - r;
  for (int k = lane; k < D; k += kPolThreads) bits[b * D + k] = tb[choice * K + k];
  if (pm_out && lane < L) pm_out[b * L + lane] = lane < nact ? pm[lane] : INFINITY;
}

constexpr int kEncThreadsP = 256;

// u: data at the first K - r information indices, CRC (data bits times the
// precomputed remainders, XOR-reduced) at the last r, frozen 0; then the
// transform, stage by stage (first half of each block ^= second half).
__global__ __launch_bounds__(kEncThreadsP) void polar_encode_kernel(DevPolar pc,
                                                                    const uint8_t* __restrict__ data,
                                                                    int64_t B,
                                                                    uint8_t* __restrict__ x) {
  extern __shared__ __align__(16) unsigned char u[];
  __shared__ uint32_t red[kEncThreadsP / 64];
  const int N = pc.N, K = pc.K, r = pc.r, D = K - r;
  const int tid = threadIdx.x;
  const int64_t b = blockIdx.x;
  for (int e = tid; e < N; e += kEncThreadsP) u[e] = 0;
  __syncthreads();
  uint32_t acc = 0;
  for (int k = tid; k < D; k += kEncThreadsP) {
    const uint8_t bit = data[b * D + k] & 1;
    u[pc.info[k]] = bit;
    if (bit && r) acc ^= pc.crc_tab[k];
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
  if ((tid & 63) == 0) red[tid >> 6] = acc;
  __syncthreads();
  if (tid < r) {
    uint32_t c = 0;
    for (int w = 0; w < kEncThreadsP / 64; ++w) c ^= red[w];
    u[pc.info[D + tid]] = (uint8_t)((c >> (r - 1 - tid)) & 1u);
  }
  __syncthreads();
  for (int st = 0; st < pc.n; ++st) {
    const int h = 1 << st;
    for (int idx = tid; idx < N / 2; idx += kEncThreadsP) {
      const int blk = idx >> st, e = idx & (h - 1);
      const int pos = blk * 2 * h + e;
      u[pos] ^= u[pos + h];
    }
    __syncthreads();
  }
  for (int e = tid; e < N; e += kEncThreadsP) x[b * N + e] = u[e];
}

template <int L>
hipError_t launch_dec(const DevPolar& pc, const float* llr, int64_t B, int use_crc, uint8_t* bits,
                      float* pm, hipStream_t s) {
  const size_t lds = polar_lds_bytes<L>(pc.N, pc.K);
  hipError_t e = ensure_dyn_lds((const void*)polar_decode_kernel<L>, lds);
  if (e != hipSuccess) return e;
  polar_decode_kernel<L><<<(unsigned)B, kPolThreads, lds, s>>>(pc, llr, B, use_crc, bits, pm);
  return hipGetLastError();
}

}  // namespace

size_t polar_decode_lds(int list, int N, int K) {
  switch (list) {
    case 1: return polar_lds_bytes<1>(N, K);
    case 2: return polar_lds_bytes<2>(N, K);
    case 4: return polar_lds_bytes<4>(N, K);
    case 8: return polar_lds_bytes<8>(N, K);
    default: return 0;
  }
}

hipError_t launch_polar_decode(const DevPolar& pc, int list, int use_crc, const float* llr,
                               int64_t B, uint8_t* bits, float* pm, hipStream_t s) {
  switch (list) {
    case 1: return launch_dec<1>(pc, llr, B, use_crc, bits, pm, s);
    case 2: return launch_dec<2>(pc, llr, B, use_crc, bits, pm, s);
    case 4: return launch_dec<4>(pc, llr, B, use_crc, bits, pm, s);
    case 8: return launch_dec<8>(pc, llr, B, use_crc, bits, pm, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_polar_encode(const DevPolar& pc, const uint8_t* data, int64_t B, uint8_t* x,
                               hipStream_t s) {
  polar_encode_kernel<<<(unsigned)B, kEncThreadsP, (size_t)pc.N, s>>>(pc, data, B, x);
  return hipGetLastError();
}

}  // namespace lsim
