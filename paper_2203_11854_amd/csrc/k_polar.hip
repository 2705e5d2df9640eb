// Polar codes: encoder (CRC attachment + transform) and the SC / SCL /
// SCL-CRC decoders (Polar codes and these decoders are among the FEC
// features, Sec. III-B; the SCL decoder is the paper's example of an
// algorithm that needs a custom kernel, Sec. IV-A).
//
// Decoder: one wavefront per codeword, everything in LDS.  The node LLRs
// of stage s (2^s values) are stored for 1 <= s < S0 = n - V, per list slot at
// alpha[p][2^s .. 2^{s+1}); the top V stages (up to 4 in the list
// decoders, 1 in SC) are never stored: they are read only while stage
// S0 - 1 is computed (2^{V+1} times per codeword) and are formed there on
// the fly from the channel LLRs.  A node at stage s
// is the left (f) or right (g) child of its parent as bit s of the leaf
// index is 0 or 1.  The partial sums of the pending left child of every
// stage are bit-packed per slot in the list decoders (stage s in its own
// words: 1 word for s < 5, 2^{s-5} words above, so a stage's word is
// written by one lane) and one byte each in SC.  Leaf i recomputes the
// stored stages from min(ctz(i), S0 - 1) down to stage 1,
// decides, and writes the merged partial sums of its trailing-ones subtree
// in one step: x[e] = u_i xor (xor over s < t with bit s of e clear of
// bl[s][e mod 2^s]), t the number of trailing ones of i, as word
// operations (for s < 5 the stage's 2^s bits replicated across the word
// and masked to the positions with bit s clear).  With
// lambda = ln P(0)/P(1): f(a, b) = sgn(a) sgn(b) min(|a|, |b|),
// g(a, b, x) = b + (1 - 2x) a, the path metric adds |lambda| when a bit
// disagrees with [lambda < 0].  At an information leaf the 2 * nact
// candidates are ranked by (metric, parent slot, bit) against each other's
// metrics read with readlane, the best L survive; a parent whose two
// children survive keeps bit 0 and copies its state to the lowest free
// slot for bit 1 (the stored LLR stages above ctz(i + 1) and its partial-
// sum words).  Every information leaf records (parent slot, bit) per slot;
// at the end each slot's path is traced back into bit-packed words,
// checking its CRC on the way.  The leaf LLR (stage 0) is
// never stored: each lane that needs it forms it from its path's two
// stage-1 values; the list decoders do not store stage-0 partial sums
// either (an odd leaf's left sibling bit is the path's bit at leaf i - 1,
// found in the history).  Active slots are always 0 .. nact - 1.
#include <hip/hip_runtime.h>

#include "dispatch.h"
#include "lsim_internal.h"

namespace lsim {

namespace {

constexpr int kPolThreads = 64;

__host__ __device__ inline int polar_kpad(int K) { return (K + 15) & ~15; }
// top stages formed on the fly: up to vmax, leaving at least stage 1
// stored (n <= 2: none formed; n = 1 stores nothing, its leaves read the
// channel)
__host__ __device__ inline int polar_virt(int n, int vmax) {
  return n <= 2 ? 0 : (n - 2 < vmax ? n - 2 : vmax);
}
// alpha row per slot: stored stages 1 .. n-V-1 at [2^s, 2^{s+1}); stage 0
// (the leaf LLR) is never stored, each lane that needs it forms it from
// stage 1
__host__ __device__ inline int polar_astr(int n, int vmax) {
  const int s0 = n - polar_virt(n, vmax);
  return s0 >= 2 ? (1 << s0) : 4;
}
// list decoders form four stages on the fly (an eighth of the LLR state
// of forming one: more codewords per CU, which hides the latency of the
// dependent LDS steps); SC, whose state is small anyway, forms one
template <int L>
constexpr int polar_vmax() { return L == 1 ? 1 : 4; }
// first word of stage s's partial sums, and words per slot
__host__ __device__ inline int polar_ws(int s) { return s < 5 ? s : 4 + (1 << (s - 5)); }
__host__ __device__ inline int polar_wrow(int n) {
  return n - 1 < 5 ? n : polar_ws(n - 1) + (1 << (n - 1 - 5));
}

// SC keeps its partial sums one byte per bit (fewer instructions; its state
// is small), the list decoders bit-packed (less LDS, more codewords per CU)
template <int L>
constexpr bool polar_bytes() { return L == 1; }

template <int L>
__host__ __device__ inline size_t polar_lds_bytes(int n, int K) {
  const int N = 1 << n;
  const size_t sums = (size_t)L * 4 * (polar_bytes<L>() ? (N + 3) / 4 : polar_wrow(n));
  return (size_t)N * 4 + (size_t)L * polar_astr(n, polar_vmax<L>()) * 4 + sums +
         (size_t)L * polar_kpad(K);
}

__device__ __forceinline__ float pol_f(float a, float c) {
  const float m = fminf(fabsf(a), fabsf(c));
  return ((a < 0.f) != (c < 0.f)) ? -m : m;
}

__device__ __forceinline__ float pol_g(float a, float c, uint32_t x) { return x ? c - a : c + a; }

// Value at position x of the stage-(n - D) node on leaf i's path, formed
// from the channel LLRs through the D stages above it; bl(st, x) is the
// slot's pending partial sum of stage st at x.
template <int D, class BL>
__device__ __forceinline__ float top_node(const float* ch, int n, int i, int x, const BL& bl) {
  if constexpr (D == 0) {
    return ch[x];
  } else {
    const int st = n - D;
    const float a = top_node<D - 1>(ch, n, i, x, bl);
    const float c = top_node<D - 1>(ch, n, i, x + (1 << st), bl);
    return ((i >> st) & 1) ? pol_g(a, c, bl(st, x)) : pol_f(a, c);
  }
}

// The 2^S-bit pattern of stage S < 5 replicated across a word, kept at the
// positions whose bit S is clear.
template <int S>
__device__ __forceinline__ uint32_t low_stage_term(uint32_t v) {
  constexpr int w = 1 << S;
  constexpr uint32_t clear[5] = {0x55555555u, 0x33333333u, 0x0F0F0F0Fu, 0x00FF00FFu, 0x0000FFFFu};
  v &= (1u << w) - 1u;
#pragma unroll
  for (int k = w; k < 32; k <<= 1) v |= v << k;
  return v & clear[S];
}

// The decoder's workgroup is one wavefront, whose LDS operations the hardware
// performs in program order: ordering its cross-lane LDS traffic only needs
// the compiler not to move accesses across this point (no s_barrier, no
// wait for outstanding LDS operations).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront", "local");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront", "local");
}

template <int L>
__global__ __launch_bounds__(kPolThreads) void polar_decode_kernel(DevPolar pc,
                                                                   const float* __restrict__ llr,
                                                                   int64_t B, int use_crc,
                                                                   uint8_t* __restrict__ bits,
                                                                   float* __restrict__ pm_out) {
  extern __shared__ __align__(16) unsigned char sm[];
  __shared__ float pm[L];
  const int N = pc.N, n = pc.n, K = pc.K, r = pc.r;
  const int V = polar_virt(n, polar_vmax<L>()), S0 = n - V;
  const int A = polar_astr(n, polar_vmax<L>()), lgA = 31 - __builtin_clz(A);
  constexpr bool kBytes = polar_bytes<L>();
  const int W = kBytes ? (N + 3) / 4 : polar_wrow(n);  // 32-bit words of partial sums per slot
  float* ch = reinterpret_cast<float*>(sm);
  float* al = ch + N;
  uint32_t* bw = reinterpret_cast<uint32_t*>(al + L * A);
  uint8_t* bb = reinterpret_cast<uint8_t*>(bw);  // byte form: stage s at [p][2^s ..]
  uint8_t* rec = reinterpret_cast<uint8_t*>(bw + L * W);  // [K][L]: (parent << 1) | bit
  const int lane = threadIdx.x;
  const int64_t b = blockIdx.x;
  // NaN reads as 0 and the channel is clamped to +-2^100, so no node LLR or
  // metric is ever inf - inf (at most 2N clamped terms add up)
  for (int e = lane; e < N; e += kPolThreads) {
    const float v = -llr[b * N + e];
    ch[e] = v != v ? 0.f : fminf(fmaxf(v, -0x1p100f), 0x1p100f);
  }
  if (lane < L) pm[lane] = 0.f;
  wave_sync();
  auto blbit = [&](int p, int st, int e) -> uint32_t {
    if constexpr (kBytes) return bb[p * N + (1 << st) + e];
    return (bw[p * W + polar_ws(st) + (e >> 5)] >> (e & 31)) & 1u;
  };
  // The stage-0 partial sum (the left sibling's bit of an odd leaf) is not
  // stored: it is the bit the path decided at leaf i - 1, read from the
  // history (0 when that leaf is frozen).  `jr` is the history index of
  // leaf i - 1 for the slot's path and `q` its slot there.
  auto prev_bit = [&](bool prev_info, int jr, int q) -> uint32_t {
    return prev_info ? (uint32_t)(rec[jr * L + q] & 1) : 0u;
  };
  // leaf LLR of slot p at leaf i: f or g of the two stage-1 values (the
  // channel when n = 1) with the leaf's left sibling's bit
  auto leaf_llr = [&](int p, int i, uint32_t ub) -> float {
    float a, c;
    if (n == 1) {
      a = ch[0];
      c = ch[1];
    } else {
      a = al[(p << lgA) + 2];
      c = al[(p << lgA) + 3];
    }
    return (i & 1) ? pol_g(a, c, ub) : pol_f(a, c);
  };
  int nact = 1, j = 0;
  for (int i = 0; i < N; ++i) {
    // ---- LLRs down to the leaf
    const int top = i == 0 ? n - 1 : __builtin_ctz(i);
    for (int st = min(top, S0 - 1); st >= 1; --st) {
      const int h = 1 << st;
      const int cnt = nact << st;
      const bool use_g = (i >> st) & 1;
      if (st + 1 < S0) {  // parent stored
        if (use_g) {
          for (int idx = lane; idx < cnt; idx += kPolThreads) {
            const int p = idx >> st, e = idx & (h - 1);
            const float* par = al + (p << lgA) + 2 * h;
            al[(p << lgA) + h + e] = pol_g(par[e], par[e + h], blbit(p, st, e));
          }
        } else {
          for (int idx = lane; idx < cnt; idx += kPolThreads) {
            const int p = idx >> st, e = idx & (h - 1);
            const float* par = al + (p << lgA) + 2 * h;
            al[(p << lgA) + h + e] = pol_f(par[e], par[e + h]);
          }
        }
      } else {
        // parent at stage S0: the channel (V = 0) or formed from it
        for (int idx = lane; idx < cnt; idx += kPolThreads) {
          const int p = idx >> st, e = idx & (h - 1);
          auto bl = [&](int s2, int x) { return blbit(p, s2, x); };
          float a, c;
          switch (V) {
            case 0:
              a = ch[e];
              c = ch[e + h];
              break;
            case 1:
              a = top_node<1>(ch, n, i, e, bl);
              c = top_node<1>(ch, n, i, e + h, bl);
              break;
            case 2:
              a = top_node<2>(ch, n, i, e, bl);
              c = top_node<2>(ch, n, i, e + h, bl);
              break;
            case 3:
              a = top_node<3>(ch, n, i, e, bl);
              c = top_node<3>(ch, n, i, e + h, bl);
              break;
            default:
              a = top_node<4>(ch, n, i, e, bl);
              c = top_node<4>(ch, n, i, e + h, bl);
              break;
          }
          al[(p << lgA) + h + e] = use_g ? pol_g(a, c, blbit(p, st, e)) : pol_f(a, c);
        }
      }
      wave_sync();
    }
    // ---- decision
    const bool info = pc.mask[i] != 0;
    const bool prev_info = i > 0 && pc.mask[i - 1] != 0;
    // the left sibling's bit of an odd leaf for slot p (before this leaf's
    // slot changes): stored by SC, from the history for the lists
    auto left_bit = [&](int p) -> uint32_t {
      if constexpr (kBytes) return bb[p * N + 1];
      return prev_bit(prev_info, j - 1, p);
    };
    if (!info) {
      if (lane < nact) {
        const float l = leaf_llr(lane, i, (i & 1) ? left_bit(lane) : 0u);
        if (l < 0.f) pm[lane] = pm[lane] + (-l);
      }
      wave_sync();
    } else {
      const int ncand = 2 * nact;
      float mc = INFINITY;
      if (lane < ncand) {
        const int p = lane >> 1, bit = lane & 1;
        const float l = leaf_llr(p, i, (i & 1) ? left_bit(p) : 0u);
        const int hard = l < 0.f;
        mc = bit == hard ? pm[p] : pm[p] + fabsf(l);
      }
      // lanes >= ncand hold +inf, which never ranks ahead of a candidate
      int rank = 0;
#pragma unroll
      for (int c2 = 0; c2 < 2 * L; ++c2) {
        const float m2 = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mc), c2));
        rank += (m2 < mc) || (m2 == mc && c2 < lane);
      }
      const uint64_t sv = __ballot(lane < ncand && rank < L);
      // parents with a surviving child / with both children surviving
      uint32_t anyp = 0, bothp = 0;
#pragma unroll
      for (int p = 0; p < L; ++p) {
        const uint32_t two = (uint32_t)(sv >> (2 * p)) & 3u;
        anyp |= (two != 0u) << p;
        bothp |= (two == 3u) << p;
      }
      uint32_t freem = ~anyp & (L == 32 ? 0xffffffffu : ((1u << L) - 1u));
      wave_sync();  // every lane has read pm and the leaf LLRs
      // each parent with two survivors copies the state still to be read to
      // the lowest free slot, in parent order
      const int t = i + 1 < N ? __builtin_ctz(i + 1) : n;
      const int alo = 2 << t;
      int mydest = -1;
      for (uint32_t mb = bothp; mb; mb &= mb - 1u) {
        const int p = __builtin_ctz(mb);
        const int d = __builtin_ctz(freem);
        freem &= freem - 1u;
        if ((lane >> 1) == p) mydest = d;
        float* ad = al + (d << lgA);
        const float* as = al + (p << lgA);
        if (lane >= alo && lane < 4 && lane < A) ad[lane] = as[lane];
        if (A >= 4) {  // 16-byte rows from offset 4 on
          const int q0 = (alo > 4 ? alo : 4) >> 2;
          for (int q = q0 + lane; q < (A >> 2); q += kPolThreads)
            reinterpret_cast<float4*>(ad)[q] = reinterpret_cast<const float4*>(as)[q];
        }
        for (int q = lane; q < W; q += kPolThreads) bw[d * W + q] = bw[p * W + q];
      }
      // metrics and the history of every surviving candidate
      if (lane < ncand && ((sv >> lane) & 1ull)) {
        const int p = lane >> 1, bit = lane & 1;
        const bool both = (bothp >> p) & 1u;
        const int slot = (both && bit) ? mydest : p;
        pm[slot] = mc;
        rec[j * L + slot] = (uint8_t)((p << 1) | bit);
      }
      nact = min(2 * nact, L);
      ++j;
      wave_sync();
    }
    // ---- partial sums of the trailing-ones subtree, one step (for the
    // lists an even leaf stores none: its bit is read from the history)
    const int t = __builtin_ctz(~i);
    // the path now in slot p came from slot q at leaf i - 1
    auto from_slot = [&](int p) { return info ? (int)(rec[(j - 1) * L + p] >> 1) : p; };
    const int jprev = info ? j - 2 : j - 1;
    if (t < n && (kBytes || t >= 1)) {
      if constexpr (kBytes) {
        const int cnt = nact << t;
        for (int idx = lane; idx < cnt; idx += kPolThreads) {
          const int p = idx >> t, e = idx & ((1 << t) - 1);
          uint8_t x = info ? (uint8_t)(rec[(j - 1) * L + p] & 1) : 0;
          for (int st = 0; st < t; ++st)
            if (!((e >> st) & 1)) x ^= bb[p * N + (1 << st) + (e & ((1 << st) - 1))];
          bb[p * N + (1 << t) + e] = x;
        }
      } else {
        // as words: stage t's words written by one lane each
        const int lgw = t < 5 ? 0 : t - 5;  // 2^lgw words of stage t per slot
        const int cnt = nact << lgw;
        for (int idx = lane; idx < cnt; idx += kPolThreads) {
          const int p = idx >> lgw, w = idx & ((1 << lgw) - 1);
          const uint32_t u = info ? (uint32_t)(rec[(j - 1) * L + p] & 1) : 0u;
          uint32_t x = u ? 0xffffffffu : 0u;
          const uint32_t* row = bw + p * W;
          x ^= low_stage_term<0>(prev_bit(prev_info, jprev, from_slot(p)));
          if (t > 1) x ^= low_stage_term<1>(row[1]);
          if (t > 2) x ^= low_stage_term<2>(row[2]);
          if (t > 3) x ^= low_stage_term<3>(row[3]);
          if (t > 4) x ^= low_stage_term<4>(row[4]);
          for (int st = 5; st < t; ++st)
            if (!((w >> (st - 5)) & 1)) x ^= row[polar_ws(st) + (w & ((1 << (st - 5)) - 1))];
          if (t < 5) x &= (1u << (1 << t)) - 1u;
          bw[p * W + polar_ws(t) + w] = x;
        }
      }
      wave_sync();
    }
  }
  // ---- each slot's path traced back through its history (lane p, slot
  // p) into bit-packed words in the (no longer read) LLR area: kw words
  // per slot, L * kw <= L * A since K <= N and A >= N / 16.  Under CRC
  // each path's data bits times their precomputed remainders, XOR the
  // received CRC bits, must vanish.  The slots are ranked by (metric,
  // slot) with a wavefront minimum over (rank, slot) keys; the decision
  // is rank 0, or under CRC the passing slot of smallest rank.
  const int D = K - r, kw = (K + 31) >> 5;
  const bool crc_on = L > 1 && use_crc && r > 0;
  uint32_t* tw = reinterpret_cast<uint32_t*>(al);
  if (lane < nact) {
    int slot = lane;
    uint32_t word = 0;
    for (int jj = K - 1; jj >= 0; --jj) {
      const int v = rec[jj * L + slot];
      word |= (uint32_t)(v & 1) << (jj & 31);
      if ((jj & 31) == 0) {
        tw[lane * kw + (jj >> 5)] = word;
        word = 0;
      }
      slot = v >> 1;
    }
  }
  wave_sync();
  bool passes = false;
  if (crc_on) {
    for (int p = 0; p < nact; ++p) {
      uint32_t acc = 0;
      for (int k = lane; k < K; k += kPolThreads)
        if ((tw[p * kw + (k >> 5)] >> (k & 31)) & 1u) acc ^= k < D ? pc.crc_tab[k] : 1u << (K - 1 - k);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc ^= __shfl_xor(acc, off, 64);
      if (lane == p) passes = acc == 0u;
    }
  }
  int key = 0x7fffffff, key_crc = 0x7fffffff;
  if (lane < nact) {
    int rk = 0;
    for (int p2 = 0; p2 < nact; ++p2)
      rk += (pm[p2] < pm[lane]) || (pm[p2] == pm[lane] && p2 < lane);
    key = (rk << 8) | lane;
    if (passes) key_crc = key;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    key = min(key, __shfl_xor(key, off, 64));
    key_crc = min(key_crc, __shfl_xor(key_crc, off, 64));
  }
  const int choice = (key_crc != 0x7fffffff ? key_crc : key) & 0xff;
  for (int k = lane; k < D; k += kPolThreads)
    bits[b * D + k] = (uint8_t)((tw[choice * kw + (k >> 5)] >> (k & 31)) & 1u);
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
  const size_t lds = polar_lds_bytes<L>(pc.n, pc.K);
  hipError_t e = ensure_dyn_lds((const void*)polar_decode_kernel<L>, lds);
  if (e != hipSuccess) return e;
  polar_decode_kernel<L><<<(unsigned)B, kPolThreads, lds, s>>>(pc, llr, B, use_crc, bits, pm);
  return hipGetLastError();
}

}  // namespace

size_t polar_decode_lds(int list, int N, int K) {
  const int n = 31 - __builtin_clz((unsigned)N);
  switch (list) {
    case 1: return polar_lds_bytes<1>(n, K);
    case 2: return polar_lds_bytes<2>(n, K);
    case 4: return polar_lds_bytes<4>(n, K);
    case 8: return polar_lds_bytes<8>(n, K);
    case 16: return polar_lds_bytes<16>(n, K);
    case 32: return polar_lds_bytes<32>(n, K);
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
    case 16: return launch_dec<16>(pc, llr, B, use_crc, bits, pm, s);
    case 32: return launch_dec<32>(pc, llr, B, use_crc, bits, pm, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_polar_encode(const DevPolar& pc, const uint8_t* data, int64_t B, uint8_t* x,
                               hipStream_t s) {
  polar_encode_kernel<<<(unsigned)B, kEncThreadsP, (size_t)pc.N, s>>>(pc, data, B, x);
  return hipGetLastError();
}

}  // namespace lsim
