/*
 * lsim.h — C-ABI of liblsim, a gfx950 (MI355X) implementation of the LDPC
 * link-level simulation hot path: binary source -> QC-LDPC encoder -> Gray
 * QAM mapper -> AWGN -> LLR demapper -> belief-propagation decoder -> error
 * count, in the order of the Sionna white paper's "Hello, World!" example
 * (arXiv 2203.11854, Sec. III-C, Listing 1), plus a persistent mixed-shape
 * decoder and a differentiable weighted-BP / neural-demapper pair
 * (Sec. II-A "Native support of NNs", Sec. III-A, Listings 2-3, Sec. IV-A).
 *
 * Conventions (every entry point):
 *  - Status codes only; nothing crosses the ABI as an exception.  Arguments
 *    are validated on the host before any launch; a non-OK status means no
 *    work was enqueued.  lsim_last_error() returns a thread-local message.
 *  - Every d_* pointer is device memory owned by the caller.  Calls enqueue
 *    asynchronously on `stream` (a hipStream_t; NULL = the null stream) and
 *    never synchronize.  Decode-path calls allocate nothing; code and plan
 *    creation allocate device tables and may synchronize.
 *  - Row-major, batch-first layouts (Sec. III-A: the first dimension is the
 *    batch of independent Monte-Carlo trials).  Complex values are
 *    interleaved (re, im) float pairs.
 *  - Boundary LLRs are logits of bit = 1, L = ln P(b=1)/P(b=0) (Listing 2
 *    feeds them to a binary cross-entropy with the code bits as labels).
 *    Hard decision: bit = [L_post > 0].
 *  - Codeword index: the Philox counters of bits and noise include the
 *    global codeword index cw0 + b, so a batch can be split anywhere and
 *    reproduce the same data.
 */
#ifndef LSIM_H
#define LSIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  LSIM_OK = 0,
  LSIM_E_INVAL = 1,        /* bad argument: null pointer, bad size, bad table */
  LSIM_E_NOMEM = 2,        /* workspace too small or device allocation failed */
  LSIM_E_UNSUPPORTED = 3,  /* valid but not implemented (e.g. odd-m QAM) */
  LSIM_E_DEVICE = 4        /* a HIP call failed */
} lsim_status;

typedef struct lsim_code lsim_code; /* opaque, immutable after create */
typedef struct lsim_plan lsim_plan; /* opaque mixed-batch plan */
typedef void* lsim_stream;          /* hipStream_t */

/* ---------------------------------------------------------------- codes */

enum { LSIM_FAMILY_11N = 0, LSIM_FAMILY_BG = 1 };

/*
 * Build a quasi-cyclic LDPC code (Sec. III-B lists 5G LDPC codes with rate
 * matching; the base matrices here are synthetic dual-diagonal QC codes).
 *  base          host int16[mb*nb], row-major; -1 = zero block, s in [0,Z) =
 *                identity shifted right by s (check (i,r) joins variable node
 *                (j, (r+s) mod Z)).  Copied; the caller keeps ownership.
 *  family        LSIM_FAMILY_11N: parity part dual-diagonal over all mb rows
 *                (weight-3 column kb with shifts 1/0/1 at rows 0, mb/2, mb-1);
 *                LSIM_FAMILY_BG: 4 dual-diagonal core rows, extension rows r
 *                with an identity at column kb+r.  kb = nb - mb.
 *  n_punct_cols  leading information blocks never transmitted (0 or 2).
 *  e_tx          transmitted bits: mother-code bits n_punct_cols*Z ..
 *                n_punct_cols*Z + e_tx - 1 (column-order rate matching).  The
 *                decoder keeps the core rows plus every extension row whose own
 *                column carries a transmitted bit; untransmitted and punctured
 *                variable nodes get LLR 0.
 * Errors: LSIM_E_INVAL on a table that is not of the stated family, a shift
 * out of range, a decoded row of degree < 2, e_tx out of range or not
 * positive; LSIM_E_UNSUPPORTED when Z > 1024 or a decoded degree > 27;
 * LSIM_E_DEVICE / LSIM_E_NOMEM on device-table upload failure.  The code's
 * device tables live on the device current at creation.
 */
lsim_status lsim_code_create(const int16_t* base, int mb, int nb, int Z, int family,
                             int n_punct_cols, int64_t e_tx, lsim_code** out);
void lsim_code_destroy(lsim_code* code);

typedef struct {
  int64_t k;          /* information bits, kb*Z (punctured ones included) */
  int64_t n_mother;   /* nb*Z */
  int64_t e_tx;       /* transmitted bits */
  int64_t n_dec;      /* decoded variable nodes */
  int64_t m_dec;      /* decoded checks */
  int64_t n_edges;    /* edges of the decoded graph, E */
  int32_t Z, mb, nb, kb, rows, cols, n_punct_cols, max_row_deg, max_col_deg;
  /* layered decoder's placement: columns whose posteriors it keeps in LDS,
   * rows whose last column (degree one) travels with the check state */
  int32_t n_shared_cols, n_private_rows;
} lsim_code_info;

lsim_status lsim_code_query(const lsim_code* code, lsim_code_info* info);

/*
 * Order in which the layered decoder (LSIM_NMS_F32) visits the decoded rows
 * of `code` in every iteration (Sec. III-B lists the BP decoder and its
 * variants; the layered schedule's order is not fixed by it and changes
 * the decoder's output).  Default LSIM_LAYERS_NATURAL: rows 0, 1, ...
 * LSIM_LAYERS_GROUPED: groups of rows that meet no common multi-check
 * column (greedy DSatur colouring of the rows' conflict graph), group after
 * group, rows ascending in a group.  LSIM_LAYERS_CUSTOM: `order` (host,
 * `rows` ints) is a permutation of 0..rows-1.  Whatever the order, the
 * decoder synchronises its workgroup only between a layer and the next one
 * that meets an LDS column of a layer since the last synchronisation (and
 * at the end of each iteration), so an order with fewer such conflicts
 * needs fewer barriers.  The table is copied to the code's device memory
 * synchronously: call it while no decode of this code is in flight.
 * Errors: LSIM_E_INVAL on an unknown mode or an order that is not a
 * permutation; LSIM_E_DEVICE on upload failure.
 */
enum { LSIM_LAYERS_NATURAL = 0, LSIM_LAYERS_GROUPED = 1, LSIM_LAYERS_CUSTOM = 2 };
lsim_status lsim_code_set_layer_order(lsim_code* code, int mode, const int* order);
/* The current order (host, `rows` ints, nullable) and the workgroup barriers
 * it takes per iteration (nullable). */
lsim_status lsim_code_layer_order(const lsim_code* code, int* order, int* barriers);

/* ------------------------------------------------------------- pipeline */

/*
 * BinarySource (Listing 1): d_u u8[B][k], bit i of codeword cw0+b is bit
 * i%32 of word (i/32)%4 of Philox4x32-10(key=(seed lo, seed hi),
 * counter=(i/128, cw lo, cw hi, 0)) (Salmon et al., SC'11).
 */
lsim_status lsim_source_bits(uint64_t seed, int64_t cw0, int64_t B, int64_t k, uint8_t* d_u,
                             lsim_stream stream);

/*
 * LDPC encoder (Listing 1): systematic back-substitution through the
 * dual-diagonal parity part, then the extension parities.
 * d_u u8[B][k] (values 0/1) -> d_c u8[B][n_mother].
 */
lsim_status lsim_encode(const lsim_code* code, const uint8_t* d_u, int64_t B, uint8_t* d_c,
                        lsim_stream stream);

/*
 * Noise variance of the AWGN channel for an Eb/N0 in dB (Listing 1 passes
 * the channel its noise variance `no`; the link's symbols have unit average
 * energy, so one information bit carries 1 / (rate * m) of a symbol's energy):
 * no[i] = 1 / (rate * m * 10^(ebn0_db[i] / 10)).  Host arrays ebn0_db[n] ->
 * no[n] (double), rate = k / e_tx of the code, m = bits per symbol.  Runs on
 * the host, touches no device memory.  Errors: LSIM_E_INVAL on a null
 * pointer, n < 0, rate not in (0, 1], m < 1 or a non-finite result.
 */
lsim_status lsim_ebn0_to_n0(const double* ebn0_db, int64_t n, double rate, int bits_per_sym,
                            double* no);

/*
 * Mapper + AWGN (Listing 1, AWGN takes the noise variance N0): takes the
 * transmitted slice of d_c u8[B][n_mother], maps m = bits_per_sym bits per
 * symbol (1 = BPSK x = 1-2c; 2, 4, 6 = square Gray QAM of 3GPP TS 38.211
 * Sec. 5.1, unit energy; I bits c0,c2,.. Q bits c1,c3,..) and adds
 * sqrt(N0/2)(g_re + j g_im) with Box-Muller normals from Philox counter
 * (j, cw lo, cw hi, 1) for symbols 2j, 2j+1.  d_no f32[B] per-codeword N0.
 * d_y f32[B][S][2], S = e_tx / m.  e_tx % m != 0 -> LSIM_E_INVAL; m not in
 * {1,2,4,6} -> LSIM_E_UNSUPPORTED.
 */
lsim_status lsim_map_awgn(const lsim_code* code, int bits_per_sym, const uint8_t* d_c,
                          const float* d_no, uint64_t seed, int64_t cw0, int64_t B, float* d_y,
                          lsim_stream stream);

/*
 * Mapper with a trainable constellation (Sec. III-C "Hello, World!": the
 * constellation's points become trainable variables, Listing 2) + AWGN.
 * d_points f32[K][2] (Re, Im), K = 2^m, m = bits_per_sym in 1..6, indexed
 * by the label of the symbol's m transmitted bits read first bit most
 * significant; the mapper uses them scaled to unit average energy,
 * x_k = p_k / sqrt(mean_j |p_j|^2) (a table of all zeros gives NaN).  The
 * noise is that of lsim_map_awgn, bit for bit (same Philox counters and
 * Box-Muller), so with the Gray QAM points of lsim_map_awgn the outputs
 * agree to rounding.  d_y f32[B][S][2], S = e_tx / m, 8-byte aligned.
 */
lsim_status lsim_map_points(const lsim_code* code, int bits_per_sym, const float* d_points,
                            const uint8_t* d_c, const float* d_no, uint64_t seed, int64_t cw0,
                            int64_t B, float* d_y, lsim_stream stream);
/*
 * Adjoint of lsim_map_points with respect to the points (the noise does
 * not depend on them): d_gpoints f32[K][2] (overwritten) = dLoss/dp for the
 * upstream d_gy = dLoss/dy f32[B][S][2].  With G_k the sum of d_gy over the
 * symbols of label k and s the normalisation,
 * dLoss/dp_j = (G_j - x_j sum_k <G_k, x_k> / K) / s.  Sums run in a fixed
 * order (deterministic).  d_work needs lsim_points_workspace() bytes.
 */
lsim_status lsim_points_workspace(const lsim_code* code, int bits_per_sym, int64_t B,
                                  size_t* bytes);
lsim_status lsim_points_grad(const lsim_code* code, int bits_per_sym, const float* d_points,
                             const uint8_t* d_c, const float* d_gy, int64_t B, float* d_gpoints,
                             void* d_work, size_t work_bytes, lsim_stream stream);

enum { LSIM_DEMAP_EXACT = 0, LSIM_DEMAP_MAXLOG = 1 };

/*
 * Demapper (Listing 1, "app" = exact; max-log): per-bit LLRs of each symbol
 * given N0.  d_y f32[B][S][2], d_no f32[B] -> d_llr f32[B][S*m].  Both
 * methods separate per I/Q axis for this labelling.  No clipping.  d_y must
 * be 8-byte aligned and d_llr aligned to 16 bytes for m = 4, 8 bytes for
 * m = 2 and 6 (vector stores), else LSIM_E_INVAL.
 */
lsim_status lsim_demap(int bits_per_sym, int method, const float* d_y, const float* d_no,
                       int64_t B, int64_t S, float* d_llr, lsim_stream stream);

/*
 * Demapper with prior (Sec. III-B lists it among the FEC features):
 * bitwise LLRs given a-priori LLRs d_la f32[B][S*m] (logits of bit 1, the
 * symbol's bits in mapping order).  Each point's metric is
 * -|y-x|^2/N0 + sum_j b_j(x) La_j; exact: log-sum-exp over the points with
 * bit i = 1 minus that over bit i = 0; max-log: max - max.  extrinsic != 0
 * writes L_i - La_i (computed with bit i's own prior left out of the
 * metric), else the a-posteriori L_i.  Gray QAM and BPSK as lsim_demap;
 * d_la and d_llr aligned as lsim_demap's d_llr.
 */
lsim_status lsim_demap_prior(int bits_per_sym, int method, const float* d_y, const float* d_no,
                             const float* d_la, int64_t B, int64_t S, int extrinsic, float* d_llr,
                             lsim_stream stream);

/* Demapper fused with the int8 quantizer below: d_q i8[B][S*m]. */
lsim_status lsim_demap_q8(int bits_per_sym, int method, const float* d_y, const float* d_no,
                          int64_t B, int64_t S, float scale, int sat, int8_t* d_q,
                          lsim_stream stream);

/*
 * LLR quantizer: q = clamp(rint(L*scale), -sat, sat), round half to even.
 * scale must be a power of two (so L*scale is exact) and 1 <= sat <= 127.
 */
lsim_status lsim_quantize(const float* d_llr, int64_t count, float scale, int sat, int8_t* d_q,
                          lsim_stream stream);

/* ------------------------------------------------------------- decoders */

enum {
  LSIM_SPA_F32 = 0, /* flooding sum-product, FP32, messages clamped to +-llr_max */
  LSIM_OMS_I8 = 1,  /* flooding offset min-sum on int8 LLRs (offset, sat) */
  LSIM_NMS_F32 = 2  /* layered normalized min-sum, FP32, scale alpha */
};

typedef struct {
  int algo;      /* LSIM_SPA_F32 | LSIM_OMS_I8 | LSIM_NMS_F32 */
  int iters;     /* full iterations, no early stop, 1..1000 */
  float offset;  /* OMS offset (integer-valued, >= 0) */
  float alpha;   /* NMS normalization, (0, 1] */
  float llr_max; /* SPA clamp, > 0 */
  int sat;       /* OMS saturation, 1..127 */
  int threads;   /* workgroup size; 0 = library default */
  int lds_rows;  /* layered decoder: rows 0 .. lds_rows-1 keep their check records
                    in LDS between iterations instead of device memory; 0 = library
                    default (as many as fit without fewer workgroups per CU), -1 =
                    none; more rows than fit the LDS -> LSIM_E_INVAL */
} lsim_decode_params;

/*
 * Belief-propagation decoder (Sec. III-B "BP decoder and variants";
 * Sec. IV-A names the min-sum BP decoder).  d_llr is f32[B][e_tx]
 * (SPA, NMS) or i8[B][e_tx] (OMS, quantized LLRs).  Outputs: d_bits
 * u8[B][k] hard decisions [L_post > 0] of the information bits (nullable),
 * d_app f32[B][n_dec] posteriors L_post (nullable; integers for OMS).
 * d_work: device workspace of at least lsim_decode_workspace() bytes,
 * 16-byte aligned (the layered decoder keeps one 12-byte record per check
 * there; the others need 0 bytes).  An unaligned or short workspace for the
 * layered decoder -> LSIM_E_INVAL / LSIM_E_NOMEM.
 * The layered decoder takes the message of a degree-one variable node to
 * its check to be the node's channel LLR in every iteration (it has no other
 * check); a code with a degree-one column that is not the last entry of its
 * row -> LSIM_E_UNSUPPORTED for LSIM_NMS_F32.
 */
lsim_status lsim_decode_workspace(const lsim_code* code, const lsim_decode_params* p, int64_t B,
                                  size_t* bytes);
lsim_status lsim_decode(const lsim_code* code, const lsim_decode_params* p, const void* d_llr,
                        int64_t B, uint8_t* d_bits, float* d_app, void* d_work,
                        size_t work_bytes, lsim_stream stream);

/*
 * Launch shape lsim_decode takes for the layered decoder (LSIM_NMS_F32) with
 * these parameters: workgroup size, codewords per workgroup, rows whose
 * check records stay in LDS (rows >= lds_rows stream through d_work) and
 * the register budget the kernel is compiled for (waves_per_simd 6: at most
 * 80 VGPRs, taken when it at least doubles the workgroups per CU; 1: the
 * compiler's own).  Needs the code's device current (it asks the runtime for
 * occupancy).  Errors: LSIM_E_UNSUPPORTED for the flooding decoders or a
 * shape that does not fit; LSIM_E_INVAL on bad parameters.
 */
lsim_status lsim_decode_launch(const lsim_code* code, const lsim_decode_params* p,
                               int* threads, int* codewords_per_tile, int* lds_rows,
                               int* waves_per_simd);

/*
 * lsim_decode without a workspace argument, for callers that cannot
 * allocate device memory: code under hipGraph capture, tight serving loops,
 * harnesses that forbid allocation.  Arguments and outputs as lsim_decode.
 * The layered decoder (LSIM_NMS_F32) keeps its per-check state in a
 * library-owned static device buffer of LSIM_NOALLOC_SCRATCH_BYTES, one per
 * GPU, held from the library's load until the process ends; the flooding
 * decoders need none.  The call runs on the current device, which must be
 * the code's device.  Nothing in the buffer has to start at zero (the state
 * is written before it is read), so calls need no clearing in between.
 * Calls that overlap in time on one GPU (other streams, other host threads)
 * share the buffer and race: serialize them.
 * Errors: LSIM_E_NOMEM when lsim_decode_workspace() for (code, p, B)
 * exceeds LSIM_NOALLOC_SCRATCH_BYTES (nothing is launched; split the
 * batch); LSIM_E_INVAL when the current device is not the code's; otherwise
 * as lsim_decode.  Allocates nothing (no hipMalloc, no library allocation).
 */
#define LSIM_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
lsim_status lsim_decode_noalloc(const lsim_code* code, const lsim_decode_params* p,
                                const void* d_llr, int64_t B, uint8_t* d_bits, float* d_app,
                                lsim_stream stream);

/*
 * Decoder state in canonical edge order (base nonzeros row-major, edge
 * e*Z + r for lift index r), for per-iteration parity checks.  Flooding
 * decoders: d_q_in (nullable, f32 or i8 [B][E]) replaces the initial
 * variable-to-check messages; after p->iters rounds d_r_out holds the last
 * check-to-variable messages and d_q_out the variable-to-check messages
 * (both nullable, message type).  Layered: d_q_in and d_q_out must be NULL;
 * d_r_out f32[B][E] gets the stored check messages.  d_app (nullable) as
 * in lsim_decode (L_post).  The decoder input d_q_in is taken as given (no
 * clamp); OMS channel LLRs are clamped to +-sat.
 */
lsim_status lsim_decode_state(const lsim_code* code, const lsim_decode_params* p,
                              const void* d_llr, int64_t B, const void* d_q_in, void* d_r_out,
                              void* d_q_out, float* d_app, void* d_work, size_t work_bytes,
                              lsim_stream stream);

/*
 * Error count (compute_ber, Listing 1): per codeword, bit errors between
 * d_ref (row stride ref_stride bytes) and d_hat u8[B][k]; adds (bit errors,
 * block errors, codewords) into d_counts i64[nbins][3] at bin d_bin[b]
 * (d_bin nullable = bin 0).  The caller zeroes d_counts.  Integer atomics:
 * deterministic.
 */
lsim_status lsim_count_errors(const uint8_t* d_ref, int64_t ref_stride, const uint8_t* d_hat,
                              int64_t B, int64_t k, const int32_t* d_bin, int nbins,
                              int64_t* d_counts, lsim_stream stream);

/*
 * Hard decisions of boundary LLRs (e.g. lsim_wbp_forward's posteriors):
 * d_bits u8[B][k] = [L > 0] for the first k columns of d_llr f32 rows of
 * `stride` floats.
 */
lsim_status lsim_hard_bits(const float* d_llr, int64_t stride, int64_t B, int64_t k,
                           uint8_t* d_bits, lsim_stream stream);

/*
 * Syndrome weight of hard decisions over the decoded graph: d_c u8[B][n_dec]
 * (row stride `stride` bytes) -> d_unsat i32[B] unsatisfied checks.
 */
lsim_status lsim_syndrome(const lsim_code* code, const uint8_t* d_c, int64_t stride, int64_t B,
                          int32_t* d_unsat, lsim_stream stream);

/* ------------------------------------------------------- whole link */

/*
 * One Monte-Carlo batch through the whole link of Listing 1 in a single
 * call: source bits (seed, cw0) -> encoder -> mapper + AWGN (d_no) ->
 * demapper (fused with the quantizer for LSIM_OMS_I8, scale q_scale and
 * saturation dec.sat) -> decoder -> error count.  Buffers are the ones of
 * the individual calls; d_llr is f32[B][e_tx] or, for LSIM_OMS_I8,
 * i8[B][e_tx].  d_c (codewords) and d_y (channel output) are nullable: the
 * transmit side runs as one kernel per batch with the codeword in LDS and
 * writes them only when given.  d_work / work_bytes as for lsim_decode.
 * d_counts receives (bit errors, block errors, codewords) per bin (d_bin
 * nullable = bin 0), accumulated.  Results equal issuing the six calls in
 * order on `stream`.
 */
typedef struct {
  const lsim_code* code;
  int bits_per_sym;
  int demap_method;
  lsim_decode_params dec;
  float q_scale;
  uint64_t seed;
  int64_t cw0;
  int64_t B;
  const float* d_no;
  uint8_t* d_u;
  uint8_t* d_c;
  float* d_y;
  void* d_llr;
  uint8_t* d_bits;
  void* d_work;
  size_t work_bytes;
  const int32_t* d_bin;
  int nbins;
  int64_t* d_counts;
} lsim_link_args;

lsim_status lsim_link_run(const lsim_link_args* args, lsim_stream stream);

/* ------------------------------------------------- mixed-shape batching */

/*
 * Plan for decoding codewords of several codes in one persistent launch
 * with the layered NMS decoder (LSIM_NMS_F32, f32 LLRs) or the flooding
 * int8 offset min-sum decoder (LSIM_OMS_I8, i8 LLRs, codeword pairs in
 * packed 16-bit lanes, or one codeword per tile where a pair's state does not
 * fit the LDS); LSIM_SPA_F32 returns LSIM_E_UNSUPPORTED.  Results
 * per codeword are those of lsim_decode with the same parameters.
 * counts[s] codewords of codes[s].  The plan owns a device work list and
 * descriptor table.  `codewords_per_tile` (nullable) fixes, per shape, how
 * many codewords share one workgroup (NMS: 0 = choose from Z and LDS; OMS:
 * 0 = a pair where it fits the LDS, else one; 1; 2); `threads` (0 = default) the workgroup size (NMS 256, 384, 512,
 * 768 or 1024 and at least every Z; OMS 256, 512 or 1024).  LLRs and bits
 * are concatenated by shape: shape s starts at sum_{t<s} counts[t]*e_tx[t]
 * LLRs and sum_{t<s} counts[t]*k[t] bits.
 */
lsim_status lsim_mixed_plan_create(const lsim_code* const* codes, const int64_t* counts,
                                   int nshapes, const lsim_decode_params* p,
                                   const int32_t* codewords_per_tile, int threads,
                                   lsim_plan** out);
void lsim_mixed_plan_destroy(lsim_plan* plan);
/* Bytes of device workspace the plan's decode needs (pass it 16-byte
 * aligned). */
lsim_status lsim_mixed_workspace(const lsim_plan* plan, size_t* bytes);
/*
 * One persistent launch over the plan's work list: a small kernel resets the
 * work counter (kept in d_work), then workgroups pull tiles until the list is
 * drained.  No allocation and no memset node: graph-capturable.
 * persistent = 0 launches one workgroup per tile instead (same results).
 */
lsim_status lsim_mixed_decode(lsim_plan* plan, const void* d_llr_concat, uint8_t* d_bits_concat,
                              float* d_app_concat, void* d_work, size_t work_bytes,
                              int persistent, lsim_stream stream);

/* ------------------------------------------------ differentiable forms */

/*
 * Weighted BP forward (trainable decoder; Sec. II-A "gradients can be
 * backpropagated through an entire system"): flooding sum-product, T rounds,
 * check-to-variable message of edge e in round t scaled by d_w[t][e].
 * d_llr f32[B][e_tx] channel LLRs; d_app f32[B][n_dec] -> L_post.
 * d_ckpt f32[T][B][E] (nullable) receives the variable-to-check messages
 * entering each round, which the backward pass reads.
 */
lsim_status lsim_wbp_forward(const lsim_code* code, int T, const float* d_w, const float* d_llr,
                             int64_t B, float llr_max, float* d_ckpt, float* d_lpost,
                             lsim_stream stream);
/*
 * Weighted BP backward (custom gradient, Sec. IV-A): given d_gpost =
 * dLoss/dL_post f32[B][n_dec] and the forward checkpoints, writes
 * d_gllr = dLoss/dL f32[B][e_tx] and d_gw = dLoss/dw f32[T][E]
 * (overwritten; reduced over the batch in an order fixed for a given GPU:
 * each of the workgroups the GPU holds at once adds its codewords in index
 * order, then their partial sums are added in workgroup order, so repeated
 * calls give identical bits).  d_work needs lsim_wbp_workspace() bytes:
 * (min(B, resident workgroups) + 32) * T * E floats, asked of the device
 * current at the query (run the call on that device); where the device
 * cannot be asked, the query returns the upper bound (B + 32) * T * E floats.
 */
lsim_status lsim_wbp_workspace(const lsim_code* code, int T, int64_t B, size_t* bytes);
lsim_status lsim_wbp_backward(const lsim_code* code, int T, const float* d_w, const float* d_llr,
                              const float* d_ckpt, int64_t B, float llr_max, const float* d_gpost,
                              float* d_gllr, float* d_gw, void* d_work, size_t work_bytes,
                              lsim_stream stream);

/*
 * Neural demapper (Listing 3): per symbol, input [Re y, Im y, ln N0] ->
 * Dense 64 ReLU -> Dense 64 ReLU -> Dense 4 (LLRs of the symbol's 4 bits).
 * d_params f32[4676]: W1[64][3], b1[64], W2[64][64], b2[64], W3[4][64], b3[4].
 * d_y f32[B][S][2], d_no f32[B] -> d_llr f32[B][S*4].
 */
#define LSIM_NDM_PARAMS 4676
lsim_status lsim_ndm_forward(const float* d_params, const float* d_y, const float* d_no,
                             int64_t B, int64_t S, float* d_llr, lsim_stream stream);
/* dLoss/dparams for upstream d_gllr f32[B][S*4]; d_gparams overwritten
 * (fixed-order reduction); d_gy (nullable, 8-byte aligned) receives
 * dLoss/dy f32[B][S][2], the gradient that flows on into a trainable
 * mapper.  d_work needs lsim_ndm_workspace() bytes. */
lsim_status lsim_ndm_workspace(int64_t B, int64_t S, size_t* bytes);
lsim_status lsim_ndm_backward(const float* d_params, const float* d_y, const float* d_no,
                              const float* d_gllr, int64_t B, int64_t S, float* d_gparams,
                              float* d_gy, void* d_work, size_t work_bytes, lsim_stream stream);

/*
 * Binary cross-entropy on logits (Listing 2 loss) against code bits:
 * d_g[b][v] = scale*(sigmoid(L[b][v]) - c[b][v]) for L = d_lpost f32[B][n]
 * and c = d_c u8 (row stride c_stride bytes); d_loss (nullable, f32[1])
 * receives scale * sum(softplus(L) - c L), reduced in a fixed order.
 * d_work needs lsim_bce_workspace() bytes when d_loss is given.
 */
lsim_status lsim_bce_workspace(int64_t B, int64_t n, size_t* bytes);
lsim_status lsim_bce_grad(const float* d_lpost, const uint8_t* d_c, int64_t c_stride, int64_t B,
                          int64_t n, float scale, float* d_g, float* d_loss, void* d_work,
                          size_t work_bytes, lsim_stream stream);

/* Adam (Kingma & Ba 2015) on n parameters; step >= 1 (bias correction). */
lsim_status lsim_adam_step(float* d_p, const float* d_g, float* d_m, float* d_v, int64_t n,
                           float lr, float beta1, float beta2, float eps, int step,
                           lsim_stream stream);

/* ------------------------------------------------------ EXIT pieces */

/*
 * A-priori LLRs for EXIT chart simulations (Sec. III-B): consistent
 * Gaussian LLRs La = (2c - 1) sigma^2/2 + sigma n of the transmitted bits
 * of d_c u8[B][n_mother], sigma = d_sigma[b] per codeword, n standard
 * normal from Philox stream 2: bits 4j..4j+3 take Box-Muller on words
 * (0, 1) then (2, 3) of counter (j, cw lo, cw hi, 2) (cosine, sine).
 * d_la f32[B][e_tx].
 */
lsim_status lsim_apriori_llrs(const lsim_code* code, const uint8_t* d_c, const float* d_sigma,
                              uint64_t seed, int64_t cw0, int64_t B, float* d_la,
                              lsim_stream stream);
/*
 * Mutual information between code bits and LLRs (EXIT charts): per row b,
 * d_mi_cw[b] = 1 - (1/n) sum_i log2(1 + exp(-(2c_i - 1) L_i)) for
 * L = d_llr f32 (row stride llr_stride) and c = d_c u8 (row stride
 * c_stride).  d_mi_bins (nullable) f64[nbins] gets the mean of d_mi_cw over
 * the rows with d_bin[b] == k (all rows when d_bin is NULL and nbins = 1;
 * NaN for an empty bin); rows with a bin outside [0, nbins) are left out.
 * Fixed-order sums (deterministic).
 */
lsim_status lsim_mutual_info(const float* d_llr, int64_t llr_stride, const uint8_t* d_c,
                             int64_t c_stride, int64_t B, int64_t n, const int32_t* d_bin,
                             int nbins, float* d_mi_cw, double* d_mi_bins, lsim_stream stream);
/*
 * Extrinsic output of a decoder on the transmitted bits (iterative
 * demapping and decoding): d_out[b][i] = L_post[b][tx_lo + i] - L_in[b][i]
 * for d_app = L_post f32[B][n_dec] (lsim_decode's d_app) and its input
 * d_llr_in f32[B][e_tx], with L_in as the decoder used it: clamped to
 * +-llr_max when llr_max > 0 (pass the decoder's llr_max for the float
 * decoders, 0 for none); 0 where tx_lo + i >= n_dec.
 */
lsim_status lsim_extrinsic(const lsim_code* code, const float* d_app, const float* d_llr_in,
                           float llr_max, int64_t B, float* d_out, lsim_stream stream);

/* ------------------------------------------------------------ Polar */

/*
 * Polar codes (Sec. III-B lists Polar codes and the SC, SCL and SCL-CRC
 * decoders; Sec. IV-A names the SCL decoder as a custom-kernel case).
 * Length N = 2^n (1 <= n <= 10), x = u F^{(x)n} with F = [[1,0],[1,1]]
 * (natural order, no bit reversal), no rate matching.
 *
 * lsim_polar_construct (host only): writes mask u8[N] with 1 at the K most
 * reliable indices by the Bhattacharyya parameters of the synthetic
 * channels, z0 = exp(-(K/N) 10^(design_ebn0_db/10)) and z -> (2z - z^2,
 * z^2) per stage (first stage = most significant index bit); equal values
 * rank the larger index first.
 *
 * lsim_polar_create: mask u8[N] (host, any nonzero = information);
 * crc_degree r in 0..24 (< K) and crc_poly = the generator's coefficients
 * below x^r (bit j = x^j; 0 when r = 0).  The K information indices in
 * increasing order carry K - r data bits then the r CRC bits of the data
 * (remainder of d(x) x^r mod g(x), first data bit = highest degree, zero
 * initial value, highest-degree CRC bit first).
 */
typedef struct lsim_polar lsim_polar; /* opaque, immutable after create */
lsim_status lsim_polar_construct(int n, int K, double design_ebn0_db, uint8_t* mask);
lsim_status lsim_polar_create(int n, const uint8_t* mask, int crc_degree, uint32_t crc_poly,
                              lsim_polar** out);
void lsim_polar_destroy(lsim_polar* pc);
lsim_status lsim_polar_query(const lsim_polar* pc, int* N, int* K, int* crc_degree);
/* d_data u8[B][K - r] (0/1) -> codewords d_x u8[B][N]. */
lsim_status lsim_polar_encode(const lsim_polar* pc, const uint8_t* d_data, int64_t B,
                              uint8_t* d_x, lsim_stream stream);
/*
 * SC (list = 1), SCL (list 2, 4, 8, 16, 32) and SCL-CRC (use_crc != 0) decoding of
 * d_llr f32[B][N] (boundary LLRs of x; NaN is read as 0 and values are
 * clamped to +-2^100, so infinite inputs decode) into the data bits d_bits
 * u8[B][K - r].  LLR form with lambda = -L: f(a, b) = sgn(a) sgn(b)
 * min(|a|, |b|) to the left child, g(a, b, x) = b + (1 - 2x) a to the right
 * child; a path's metric adds |lambda| at a leaf whose bit disagrees with
 * [lambda < 0]; at an information leaf the L candidates with the smallest
 * metric survive (ties: lower parent slot, then bit 0; a parent whose two
 * children survive keeps bit 0 in its slot and sends bit 1 to the lowest
 * free slot).  The decision is the slot with the smallest metric (ties:
 * lowest slot); SCL-CRC takes, in that order, the first slot whose CRC
 * checks, else the first.  d_pm (nullable) f32[B][list] receives the final
 * metrics by slot (+inf for unused slots).  One workgroup per codeword
 * holds the list state in LDS (about 7 N + K bytes for SC, 4 N + list
 * (0.4 N + K) for the lists: 32.5 KiB at N = 1024, K = 512, list 32);
 * LSIM_E_UNSUPPORTED if it exceeds 160 KiB.  use_crc on a code without CRC
 * -> LSIM_E_INVAL.
 */
lsim_status lsim_polar_decode(const lsim_polar* pc, int list, int use_crc, const float* d_llr,
                              int64_t B, uint8_t* d_bits, float* d_pm, lsim_stream stream);

/*
 * Mapper + AWGN for rows of bits that are not LDPC codewords (e.g. Polar
 * codewords): maps bits 0 .. n-1 of each row of d_bits (row stride
 * `stride` bytes) exactly as lsim_map_awgn maps a codeword's transmitted
 * bits (same labelling, same Philox counters and Box-Muller noise).
 * d_y f32[B][n/m][2].
 */
lsim_status lsim_map_awgn_bits(int bits_per_sym, const uint8_t* d_bits, int64_t stride, int64_t n,
                               const float* d_no, uint64_t seed, int64_t cw0, int64_t B,
                               float* d_y, lsim_stream stream);

/* ---------------------------------------------------------------- misc */

/* ------------------------------------------------------ peak-rate probes */

/*
 * Roofline denominators measured on the device itself (the decoders' rates
 * are reported as fractions of these beside the published peaks).  One
 * launch of `grid` workgroups of 256 threads on `stream`; *units receives
 * the work the launch does, to be divided by its event-timed duration:
 *  LSIM_PROBE_COPY   d_src -> d_dst, `bytes` (a multiple of 16) each; units =
 *                    bytes read + written.
 *  LSIM_PROBE_READ   reads `bytes` of d_src; d_dst u32[grid*256] receives one
 *                    word per thread; units = bytes read.
 *  LSIM_PROBE_LDS_READ / LSIM_PROBE_LDS_WRITE  each thread reads / writes 16
 *                    bytes of its workgroup's 64 KB of LDS 8*rounds times,
 *                    lane-consecutive (no bank conflicts); d_dst u32[grid*256];
 *                    units = LDS bytes.
 *  LSIM_PROBE_FMA / LSIM_PROBE_EXP2  8 independent chains per thread of
 *                    `rounds` fused multiply-adds / base-2 exponentials;
 *                    d_dst f32[grid*256]; units = VALU lane operations.
 * Errors: LSIM_E_INVAL on an unknown kind, grid outside 1..65536, rounds < 1,
 * a null d_dst, or (copy, read) a null d_src or bytes not a positive multiple
 * of 16.
 */
enum {
  LSIM_PROBE_COPY = 0,
  LSIM_PROBE_READ = 1,
  LSIM_PROBE_LDS_READ = 2,
  LSIM_PROBE_LDS_WRITE = 3,
  LSIM_PROBE_FMA = 4,
  LSIM_PROBE_EXP2 = 5
};
lsim_status lsim_probe(int kind, const void* d_src, void* d_dst, int64_t bytes, int rounds,
                       int grid, int64_t* units, lsim_stream stream);

const char* lsim_last_error(void);
const char* lsim_version(void);

#ifdef __cplusplus
}
#endif
#endif /* LSIM_H */
