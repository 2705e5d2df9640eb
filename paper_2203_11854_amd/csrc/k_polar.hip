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
  uint8_t* ui;
  int astr, kpad;
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
  s.kpad = polar_kpad(K);
  s.ch = reinterpret_cast<float*>(sm);
  s.al = s.ch + N;
  s.bl = reinterpret_cast<uint8_t*>(s.al + (size_t)L * s.astr);
  s.ui = s.bl + (size_t)L * N;
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
  for (int i = 0; i < N; ++i) {
    // ---- LLRs down to the leaf (stage n - 1 only on the fly when n >= 2)
    const int top = i == 0 ? n - 1 : __builtin_ctz(i);
    for (int st = top; st >= 0; --st) {
      if (n >= 2 && st == n - 1) continue;
      const int h = 1 << st;
      const int cnt = nact << st;
      const bool use_g = st == top && i != 0;
      for (int idx = lane; idx < cnt; idx += kPolThreads) {
        const int p = idx >> st, e = idx & (h - 1);
        float a, c;
        if (st + 1 == n) {  // n == 1: the parent is the channel
          a = s.ch[e];
          c = s.ch[e + h];
        } else if (st + 1 == n - 1) {  // the parent is stage n - 1, formed here
          const int Q = N >> 1;
          if (i < Q) {
            a = pol_f(s.ch[e], s.ch[e + Q]);
            c = pol_f(s.ch[e + h], s.ch[e + h + Q]);
          } else {
            a = pol_g(s.ch[e], s.ch[e + Q], s.bl[p * N + Q + e]);
            c = pol_g(s.ch[e + h], s.ch[e + h + Q], s.bl[p * N + Q + e + h]);
          }
        } else {
          const float* par = s.al + p * A + 2 * h;
          a = par[e];
          c = par[e + h];
        }
        s.al[p * A + h + e] = use_g ? pol_g(a, c, s.bl[p * N + h + e]) : pol_f(a, c);
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
      const uint64_t sv = __ballot(lane < ncand && rank < L);
      // slot plan, the same in every lane
      int dest[L];
      uint32_t freem = 0;
#pragma unroll
      for (int p = 0; p < L; ++p) {
        const bool any = p < nact && ((sv >> (2 * p)) & 3u);
        if (!any) freem |= 1u << p;
      }
#pragma unroll
      for (int p = 0; p < L; ++p) {
        dest[p] = -1;
        if (p < nact && ((sv >> (2 * p)) & 3u) == 3u) {
          const int d = __builtin_ctz(freem);
          freem &= freem - 1;
          dest[p] = d;
        }
      }
      __syncthreads();  // every lane has read pm and the leaf LLRs
      // copies of the state still to be read
      const int t = i + 1 < N ? __builtin_ctz(i + 1) : n;
      const int alo = 2 << t;  // alpha stages above t (stored ones end at A)
      int mydest = -1;
#pragma unroll
      for (int p = 0; p < L; ++p) {
        const int d = dest[p];
        if ((lane >> 1) == p) mydest = d;
        if (d < 0) continue;
        for (int e = alo + lane; e < A; e += kPolThreads) s.al[d * A + e] = s.al[p * A + e];
        for (int st = 0; st < n; ++st) {
          if (!((i >> st) & 1)) continue;
          const int h = 1 << st;
          for (int e = lane; e < h; e += kPolThreads) s.bl[d * N + h + e] = s.bl[p * N + h + e];
        }
        for (int e = lane; e < j; e += kPolThreads) s.ui[d * s.kpad + e] = s.ui[p * s.kpad + e];
      }
      // metrics and the new bit of every surviving candidate
      if (lane < ncand && ((sv >> lane) & 1u)) {
        const int p = lane >> 1, bit = lane & 1;
        const bool both = ((sv >> (2 * p)) & 3u) == 3u;
        const int slot = (both && bit) ? mydest : p;
        pm[slot] = mc;
        s.ui[slot * s.kpad + j] = (uint8_t)bit;
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
        uint8_t x = info ? s.ui[p * s.kpad + j - 1] : 0;
        for (int st = 0; st < t; ++st)
          if (!((e >> st) & 1)) x ^= s.bl[p * N + (1 << st) + (e & ((1 << st) - 1))];
        s.bl[p * N + (1 << t) + e] = x;
      }
      __syncthreads();
    }
  }
  // ---- selection
  if (use_crc && r > 0) {
    const int D = K - r;
    for (int p = 0; p < nact; ++p) {
      uint32_t acc = 0;
      for (int k = lane; k < D; k += kPolThreads)
        if (s.ui[p * s.kpad + k]) acc ^= pc.crc_tab[k];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
      if (lane == 0) {
        uint32_t got = 0;
        for (int q = 0; q < r; ++q) got = (got << 1) | s.ui[p * s.kpad + D + q];
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
  for (int k = lane; k < D; k += kPolThreads) bits[b * D + k] = s.ui[choice * s.kpad + k];
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
