/*
 * cider.h -- C ABI of the MI355X (gfx950) CIDER refinement library.
 *
 * CIDER decodes K superposed codewords of a shared binary LDPC code from one
 * noisy aggregate: y_l = sum_k x_{k,l} + noise, x = +1 for bit 0 and -1 for
 * bit 1.  The decoder keeps a K x n grid of symbols {0, 1, MASK} and repeats a
 * masked-diffusion refinement step (paper: method section, refinement loop):
 *
 *   evidence  p[l, a] = normalised Pr(some user sent a at slot l | y_l)
 *                       (Appendix, evidence interface; exact for BPSK)
 *   denoiser  embedding -> Module A (row competition for the evidence) ->
 *             L blocks of {row attention over slots, attention across the K
 *             rows of each slot, GELU MLP} -> final LayerNorm -> logits
 *   Module B  soft parity messages over the Tanner graph of H added to the
 *             logits as a bias (method section, check message and update)
 *   reveal    the most confident masked sites take their argmax symbol;
 *             first-reveal on step 1 (Appendix, masked-diffusion inference)
 *   final pass and quality-guided remasking of parity-failing or
 *             low-confidence rows (Appendix, PRISM-style remasking; here with
 *             a fixed row criterion instead of a learned head)
 *
 * Conventions for every entry point:
 *   - Pointers documented "device" must point to memory on the current HIP
 *     device; "host" pointers are read during the call only.
 *   - `stream` is a hipStream_t (NULL = default stream).  Work is enqueued on
 *     it and the call returns before the work completes, except where noted;
 *     outputs are valid once the stream has reached the enqueued work.
 *   - Return value: CIDER_OK (0) or a negative CIDER_E* code.  Argument errors
 *     are detected before anything is enqueued.  A HIP error is reported as
 *     CIDER_EDEVICE; cider_last_error() gives a readable message for the
 *     calling thread.  No C++ exception crosses this interface.
 *   - Handles (weights, code, server) are owned by the library and freed with
 *     the matching *_destroy.  Weights and code handles are immutable after
 *     creation and may be shared between threads.  Decode calls that use the
 *     library's internal workspace (opts->workspace == NULL) on the same
 *     weights handle must not run concurrently on different streams; pass a
 *     caller-owned workspace to run them concurrently.
 */
#ifndef CIDER_H
#define CIDER_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CIDER_OK            0
#define CIDER_EINVAL       -1   /* bad argument or sizes                        */
#define CIDER_ENOMEM       -2   /* device or host allocation failed             */
#define CIDER_EDEVICE      -3   /* HIP runtime error                            */
#define CIDER_EUNSUPPORTED -4   /* valid request this build does not implement  */
#define CIDER_EAGAIN       -5   /* server queue full, retry later               */

#define CIDER_MAX_K      16     /* users per bin                                */
#define CIDER_MAX_N    1024     /* slots per bin (also the positional table)    */
#define CIDER_MASK        2     /* grid value of a masked site                  */

enum cider_precision {
  CIDER_FP32 = 0,   /* every contraction in FP32 (MFMA 16x16x4 f32)            */
  CIDER_BF16 = 1,   /* GEMM/attention operands BF16, FP32 accumulate           */
  CIDER_FP8  = 2,   /* LayerNorm-fed GEMM operands OCP e4m3 with per-tensor    */
                    /* weight scale and per-token activation scale, FP32       */
                    /* accumulate; at d = 256 (head width 32, binary codes,    */
                    /* fused blocks on) the BF16 token-resident kernels run    */
                    /* with only the MLP up projection in e4m3                 */
  CIDER_FP64 = 3    /* every value in double, from the evidence to the reveal  */
                    /* keys (binary path, no quality head): the integer        */
                    /* decisions of a decode come out as an FP64 reference's   */
                    /* whenever they are farther from a tie than double        */
                    /* rounding.  cider_step_debug then writes its logits and  */
                    /* residual outputs as doubles                             */
};

enum cider_schedule {
  CIDER_SCHED_LINEAR = 0,  /* R_t = floor(t N / T) revealed after step t       */
  CIDER_SCHED_COSINE = 1   /* R_t = floor(rho(t) N), rho = (1 - cos(pi t/T))/2, */
                           /* at least one site per step (Appendix, cosine     */
                           /* reveal schedule)                                  */
};

/* Denoiser sizes.  d % heads == 0, d / heads in {16, 32, 64}, d % 64 == 0,
 * d <= 512, mlp_mult * d <= 2048, n_max <= CIDER_MAX_N. */
typedef struct {
  int32_t n_layers;
  int32_t d;
  int32_t heads;
  int32_t mlp_mult;   /* MLP hidden width = mlp_mult * d (the workloads use 4) */
  int32_t n_max;      /* rows of the positional table P                      */
  int32_t q;          /* symbols Q: 0 or 2 = the binary path (cider_decode);  */
                      /* 4, 8, 16, 32 or 64 = GF(Q) codes (cider_decode_q_batch) */
} cider_model_cfg;

/* Decoding options; cider_opts_default() fills the values in brackets. */
typedef struct {
  int32_t precision;          /* cider_precision                       [BF16]   */
  int32_t schedule;           /* cider_schedule                        [LINEAR] */
  int32_t first_reveal;       /* step 1 of the initial pass (first-reveal      */
                              /* stabilisation, inference appendix):           */
                              /*  1: candidates narrowed to each slot's most   */
                              /*     confident masked row, count from the      */
                              /*     schedule (hybrid)                   [1]   */
                              /*  2: every slot's selected site is revealed    */
                              /*     (verbatim); the schedule resumes after    */
                              /*  0: off                                       */
  int32_t remask;             /* 1: quality-guided remasking on          [0]   */
  int32_t remask_max_rounds;  /* rounds of remasking                     [2]   */
  int32_t final_argmax;       /* 1: output argmax of the last final pass       */
                              /* 0: output the held-fixed grid           [0]   */
  int32_t use_graph;          /* 1: replay each refinement step as a hipGraph  */
                              /*    captured on `stream`                 [1]   */
  float   remask_thr;         /* low row: mean max-prob < thr           [0.9]  */
  float   tau;                /* Module A responsibility temperature    [1.0]  */
  float   eta;                /* Module B bias gain                     [1.0]  */
  float   lam_max;            /* LLR clip and revealed-site LLR         [20]   */
  float   lam_min;            /* |LLR| floor inside phi                 [1e-6] */
  float   tau_max;            /* inference temperature, cosine-annealed from   */
  float   tau_min;            /* tau_max (step 1) to tau_min (step T), per the */
                              /* inference appendix [1, 1].  With two symbols  */
                              /* the temperature does not change the reveal    */
                              /* ranking; tau_min sets the final pass's        */
                              /* confidence in the remask test                 */
  int32_t autotune;           /* 1: before the first decode of a new batch     */
                              /*    size, time every GEMM tile shape on it and */
                              /*    keep the fastest (results do not depend on */
                              /*    the tile)                            [1]   */
                              /*    2 + t: use tile t everywhere (tests)       */
  int32_t profile;            /* 1: time every kernel launch with HIP events   */
                              /*    on `stream` (eager launches, no graph);    */
                              /*    read with cider_profile_read         [0]   */
  int32_t fused_blocks;       /* 1: BF16 runs each attention sublayer (QKV,    */
                              /*    attention, output projection, residual,    */
                              /*    next LayerNorm) as one kernel where the    */
                              /*    shapes allow (d in {64,128,192}; row       */
                              /*    attention needs n <= 128)            [1]   */
                              /*    0: separate GEMM / attention kernels       */
  void*   workspace;          /* device scratch owned by the caller, or NULL   */
  size_t  workspace_bytes;    /* size of `workspace`; see cider_workspace_size */
  /* PRISM-style quality head (Appendix, PRISM-style quality head and
   * remasking plug-in) as the remask criterion, in place of the syndrome /
   * confidence test above.  NULL [default]: not used.  Else a device FP32
   * vector owned by the caller, live until the decode completes: W1 [H][d]
   * row-major, b1 [H], LayerNorm gain [H], LayerNorm bias [H], w2 [H], b2;
   * per token omega = sigmoid(w2 . GELU(LN(W1 LN_f(Z) + b1)) + b2) at the
   * final pass, a row's confidence is its mean omega, and after pass s the
   * rows below remask_phi[s] are remasked, for at most remask_stages rounds
   * (remask_max_rounds and remask_thr are then unused; remask must be 1,
   * else CIDER_EINVAL; d > 1024 gives CIDER_EUNSUPPORTED).  The syndrome
   * still sets out_row_valid. */
  const float* qhead;
  int32_t qhead_hidden;       /* H, 1..64                                  [0] */
  int32_t remask_stages;      /* number of thresholds, 1..4                [3] */
  float   remask_phi[4];      /* thresholds            [0.96, 0.90, 0.85, 0]   */
} cider_opts;

typedef struct cider_weights cider_weights;
typedef struct cider_code    cider_code;

/* One bin of a batch (cider_decode_batch). */
typedef struct {
  const float*      y;             /* device [n] FP32 received aggregate        */
  float             sigma2;        /* noise variance, > 0                        */
  const cider_code* code;          /* parity-check matrix, code->n == n          */
  int32_t           K;             /* users, 1..CIDER_MAX_K                      */
  int32_t           n;             /* slots, 1..min(n_max, CIDER_MAX_N)          */
  uint8_t*          out_symbols;   /* device [K][n] row-major, values {0,1}      */
  float*            out_logits;    /* device [K][n][2] FP32 logits of the last   */
                                   /* final pass, or NULL                        */
  uint8_t*          out_row_valid; /* device [K]: 1 iff H x_k = 0, or NULL       */
  int32_t*          out_rounds;    /* device [1]: remask rounds run, or NULL     */
} cider_bin;

/* Fills `opts` with the defaults listed above. */
void cider_opts_default(cider_opts* opts);   /* opts: host, not NULL */

/* Number of floats a weights blob for `cfg` holds (layout below), or 0 if cfg
 * is invalid.  Blob layout, all row-major FP32, a linear map is y = x W^T + b,
 * Q = cfg->q (2 when 0):
 *   E[Q+1][d] (row Q = mask token), P[n_max][d], u[d], W[Q][d], v[Q][d],
 *   Wg1[d][2d], bg1[d], Wg2[d][d], bg2[d],
 *   per layer: ln1_g[d] ln1_b[d] Wqkv_r[3d][d] bqkv_r[3d] Wo_r[d][d] bo_r[d]
 *              ln2_g[d] ln2_b[d] Wqkv_u[3d][d] bqkv_u[3d] Wo_u[d][d] bo_u[d]
 *              ln3_g[d] ln3_b[d] W1[F][d] b1[F] W2[d][F] b2[d]   (F = mlp_mult d)
 *   lnf_g[d], lnf_b[d].
 * q, k, v of an attention are the three consecutive d-row blocks of Wqkv;
 * head h uses rows h*d/heads .. (h+1)*d/heads - 1 of each block. */
size_t cider_weights_blob_floats(const cider_model_cfg* cfg);

/* The denoiser's parameters: the embedding table E (two symbols and the
 * mask token), the shared symbol projection W, the evidence embeddings v_a
 * and the gate MLP of Module A (Appendix, CIDER architecture: latent
 * parameterisation and slot-competition demixing; method section, Module A
 * equations), the L pre-LN blocks the workload defines, and the final
 * LayerNorm feeding the logit projection.
 * Uploads a host FP32 blob (read during the call only) to the current
 * device and prepares the FP32, BF16 and FP8 copies of every matrix.
 * Synchronous.  `n_floats` must equal cider_weights_blob_floats(cfg), else
 * CIDER_EINVAL; an invalid cfg is CIDER_EINVAL, a failed device allocation
 * CIDER_ENOMEM.  *out is owned by the caller until cider_weights_destroy. */
int cider_weights_create(const cider_model_cfg* cfg, const float* host_blob, size_t n_floats,
                         cider_weights** out);
void cider_weights_destroy(cider_weights* w);

/* The shared code's parity-check matrix, which the parity-aware decoder is
 * given (Appendix, Q-ary LDPC code: H over F_Q with its Tanner graph, taken
 * here at Q = 2; multiuser-code families and parity-check metadata).
 * Binary H (m checks x n slots) given as host CSR (read during the call):
 * row_ptr[m+1], col_idx[row_ptr[m]] with ascending, distinct column indices
 * in [0, n).  Rows may have any degree up to 32; every slot may appear in
 * at most 32 checks.  Copied to the device; synchronous. */
int cider_code_create(int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* col_idx,
                      cider_code** out);
void cider_code_destroy(cider_code* code);

/* A parity-check matrix over GF(Q), Q = 2^q_bits, 2 <= q_bits <= 6 (Appendix,
 * Q-ary LDPC code: H in F_Q^{P x L} with i.i.d. nonzero coefficients on its
 * Tanner-graph edges).  CSR as in cider_code_create plus coef[row_ptr[m]],
 * the nonzero coefficient H[j, l] of each edge; field in polynomial basis
 * with primitive polynomial x^2+x+1, x^3+x+1, x^4+x+1, x^5+x^2+1 or x^6+x+1,
 * symbol index = the element's coefficient bits.  Check degrees 1..16.
 * Host arrays, read during the call; synchronous. */
int cider_code_create_q(int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* col_idx,
                        const uint8_t* coef, int32_t q_bits, cider_code** out);

/* Bytes of caller workspace a batch of `num_bins` bins with `total_tokens`
 * = sum of K*n and `total_slots` = sum of n needs under `opts`: the
 * per-token residual stream and activations of one denoiser forward plus the
 * per-bin grid, logit and schedule state of the refinement loop (method
 * section, refinement loop).  Writes *bytes; CIDER_EINVAL for NULL or
 * negative arguments.  No device work. */
int cider_workspace_size(const cider_weights* w, int32_t num_bins, int64_t total_tokens,
                         int64_t total_slots, const cider_opts* opts, size_t* bytes);

/* Decodes one bin: evidence from y, then the map from evidence S to an
 * unordered K x n grid (Appendix, multiuser decoding objective and
 * set-valued output), computed by the refinement loop of the method section
 * with the final pass and remasking of the inference appendix.  y: device [n] FP32; out_symbols: device [K][n] uint8.
 * steps = T of the initial pass, 1 <= steps <= K*n.  opts may be NULL for the
 * defaults.  Returns after enqueueing, except that with remasking on the
 * call synchronises `stream` once per remask round to learn whether any bin
 * still needs work. */
int cider_decode(const float* y, float sigma2, const cider_code* code, int32_t K, int32_t n,
                 const cider_weights* w, int32_t steps, uint8_t* out_symbols,
                 const cider_opts* opts, void* stream);

/* Allocation-free variant of cider_decode, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, rules and result as cider_decode (bit-identical
 * symbols), but the call allocates nothing, on the device or on the host:
 * its workspace, per-bin metadata and reveal-schedule table live in a
 * library-owned device array of CIDER_NOALLOC_SCRATCH_BYTES per GPU, held
 * from the first call on that GPU until the process ends.  Launches are
 * eager (opts->use_graph is ignored: a graph would allocate) and no tile is
 * autotuned (a tile tuned earlier on the weights handle, or forced with
 * autotune >= 2, is used).  Every call on a GPU shares that GPU's array, which
 * keeps the last call's contents: calls that overlap on one GPU (any stream,
 * any thread) race and must be serialised by the caller.
 * CIDER_EINVAL, before anything is enqueued, when the bin's workspace exceeds
 * the array (roughly K*n*d*(30 + 6*mlp_mult) bytes at BF16 must fit in
 * 64 MiB: every bin of K*n <= 4096 tokens at d = 256), when
 * opts->workspace is set, or when opts->profile = 1 (timing events allocate);
 * otherwise as cider_decode.  With remasking on, the call synchronises
 * `stream` once per remask round, as cider_decode does. */
#define CIDER_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int cider_decode_noalloc(const float* y, float sigma2, const cider_code* code, int32_t K, int32_t n,
                         const cider_weights* w, int32_t steps, uint8_t* out_symbols,
                         const cider_opts* opts, void* stream);

/* Decodes `num_bins` independent bins of possibly different K, n and code in
 * one packed pass per step.  Bins share no state: each preamble bin of the
 * random-access protocol is decoded on its own (Appendix, protocol-level
 * scalability: per-bin decoding), so a batch is only a launch-level grouping
 * of cider_decode calls.  bins: host array [num_bins] (read during the
 * call); its device buffers follow cider_decode's rules.  The result of
 * every bin is bit-identical to decoding it alone with cider_decode and the
 * same opts.  CIDER_EINVAL if any bin fails cider_decode's checks (nothing
 * enqueued). */
int cider_decode_batch(int32_t num_bins, const cider_bin* bins, const cider_weights* w,
                       int32_t steps, const cider_opts* opts, void* stream);

/* ---- GF(Q) codes: the paper's main setting ------------------------------
 * Decoding over a Q-ary LDPC code from the slot-wise evidence S[l][a] =
 * log Pr(symbol a present at slot l | Y_l) (Appendix, per-slot channel model
 * and symbol-level soft evidence; cider_amp_evidence computes it), with the
 * Q-symbol forms of the method: embedding table E[Q+1] (row Q = mask),
 * Module A over the Q symbols with p = softmax_a S, Module B's extrinsic
 * check messages from the exact check-to-variable rule over GF(Q) (the
 * other edges' weighted sum, applied through each edge's coefficient)
 * added to the logits as eta times their centred logarithm, and a reveal
 * ranked by the confidence max_a softmax(L / tau_t)_a at the annealed
 * temperature (masked-diffusion inference appendix).  The grid holds
 * symbols 0..Q-1 and Q = mask.  The weights need cfg.q == Q and every code
 * q_bits == log2 Q.  Precision FP32 or BF16; remasking, the quality head and
 * final_argmax are CIDER_EUNSUPPORTED on this path. */
typedef struct {
  const float*      S;             /* device [n][Q] FP32 log evidence            */
  const cider_code* code;          /* cider_code_create_q, code->n == n          */
  int32_t           K;             /* users, 1..CIDER_MAX_K                      */
  int32_t           n;             /* slots, 1..min(n_max, CIDER_MAX_N)          */
  uint8_t*          out_symbols;   /* device [K][n], values 0..Q-1               */
  float*            out_logits;    /* device [K][n][Q] last final-pass logits,   */
                                   /* or NULL                                    */
  uint8_t*          out_row_valid; /* device [K]: 1 iff H x_k = 0 over GF(Q)     */
} cider_qbin;

/* Decodes `num_bins` independent bins over GF(Q) codes in one packed pass
 * per step, like cider_decode_batch: each bin's result is the same as
 * decoding it alone.  bins: host array (read during the call). */
int cider_decode_q_batch(int32_t num_bins, const cider_qbin* bins, const cider_weights* w,
                         int32_t steps, const cider_opts* opts, void* stream);

/* Teacher-forced GF(Q) step, as cider_step_debug: X_in device [K][n] in
 * 0..Q (Q = mask); out_lbar / out_logits device [K][n][Q] (either NULL);
 * X_out, if not NULL, receives X_in with `reveal_count` sites revealed by the
 * confidence ranking at temperature opts->tau_max (first-reveal if `first`). */
int cider_step_debug_q(const uint8_t* X_in, uint8_t* X_out, const float* S, const cider_code* code,
                       int32_t K, int32_t n, const cider_weights* w, float gamma, int32_t reveal_count,
                       int32_t first, const cider_opts* opts, float* out_lbar, float* out_logits,
                       void* stream);

/* Test entry point: one refinement step (method section, refinement loop:
 * denoiser forward with Modules A and B, then the confidence-ranked reveal
 * of the masked-diffusion inference appendix) on a given grid, teacher
 * forced: the caller supplies the grid instead of the previous step.
 * X_in: device [K][n] uint8 in {0,1,2}; gamma: mask-ratio input.
 * Writes out_lbar (logits before Module B) and out_logits (after), device
 * [K][n][2] FP32, either may be NULL; out_z: device [K][n][d] FP32 residual
 * stream before the final LayerNorm, or NULL.  If X_out is not NULL the
 * reveal rule is applied to a copy of X_in with `reveal_count` sites and
 * first-reveal flag `first` and the result written to X_out [K][n]. */
int cider_step_debug(const uint8_t* X_in, uint8_t* X_out, const float* y, float sigma2,
                     const cider_code* code, int32_t K, int32_t n, const cider_weights* w,
                     float gamma, int32_t reveal_count, int32_t first, const cider_opts* opts,
                     float* out_lbar, float* out_logits, float* out_z, void* stream);

/* Per-slot evidence alone (Appendix, per-slot channel model and symbol-level
 * soft evidence): out_S and out_p device [n][2] FP32 (either may be NULL).
 * S[l,a] = log Pr(symbol a present at slot l | y_l), exact over the number
 * of users sending bit 1; p = softmax_a S.  y: device [n] FP32.
 * CIDER_EINVAL for K outside 1..CIDER_MAX_K, n outside 1..CIDER_MAX_N,
 * sigma2 <= 0 or a NULL y. */
int cider_evidence(const float* y, float sigma2, int32_t K, int32_t n, float* out_S, float* out_p,
                   void* stream);

/* ---- slot-wise AMP-MMSE detector (the non-binary evidence front end) ------
 * Appendix, slot-wise AMP-MMSE detector and sensing-matrix construction.  For
 * each slot: Y = A U + noise in C^{n_s}, A[j][a] = exp(-2 pi i R_j a / Q) /
 * sqrt(n_s) (rows R_j of the Q-point DFT), a Bernoulli-Gaussian prior
 * (1 - rho) delta_0 + rho CN(0, su2) on each U_a.  Runs `iters` AMP
 * iterations with the MMSE denoiser and its Onsager correction (effective
 * noise nu = ||residual||^2 / n_s) and writes S[slot][a] = log Pr(U_a != 0 |
 * Y) from the final pseudo-observation, FP32.
 *   y      device float [slots][n_s][2]: Y, real and imaginary parts
 *   rows   device int32 [slots][n_s]: DFT row indices (taken modulo Q)
 *   out_S  device float [slots][Q]
 * 1 <= n_s <= 64, 2 <= Q <= 64, 0 <= slots < 2^31, 0 <= iters <= 10000,
 * 0 < rho < 1, su2 > 0.  The caller owns every buffer; the call is enqueued
 * on `stream` (a hipStream_t, NULL = default) and does not synchronise.
 * CIDER_EINVAL for bad sizes, parameters or NULL pointers (nothing
 * enqueued), CIDER_EDEVICE if the launch fails. */
int cider_amp_evidence(const float* y, const int32_t* rows, int64_t slots, int32_t n_s, int32_t Q, float rho,
                       float su2, int32_t iters, float* out_S, void* stream);

/* Check-node update of the GF(64) parity layer (Appendix, Q-ary LDPC code
 * over F_Q; FFT-BP's Walsh-Hadamard check update).  For every check
 * sum_i alpha_i x_i = 0 (row j of H, edges row_ptr[j] .. row_ptr[j+1]-1 in
 * CSR order) and every edge o of it, writes the message to the variable of
 * edge o: m_o(a) proportional to the probability, under the other edges'
 * distributions, that their weighted sum equals alpha_o a; normalised, FP32.
 * Field: GF(2^6) in polynomial basis with primitive polynomial x^6 + x + 1,
 * symbol index = the element's coefficient bits.
 *   p_edge   device float [edges][64]: variable-to-check distribution of each edge
 *   row_ptr  device int32 [checks + 1], row_ptr[0] = 0, row_ptr[checks] = edges
 *   coef     device uint8 [edges]: the edge's coefficient alpha, 1..63
 *   out_msg  device float [edges][64]
 * Check degrees 1..32.  A row whose bounds fall outside 0..edges or whose
 * degree is outside 1..32 is left unwritten (no access outside the
 * buffers); a zero coefficient gives unspecified values.  The caller owns
 * every buffer; the call is enqueued on `stream` and does not synchronise.
 * CIDER_EINVAL for negative or too large sizes or NULL buffers (nothing
 * enqueued), CIDER_EDEVICE if the launch fails. */
int cider_gf64_check_update(const float* p_edge, const int32_t* row_ptr, const uint8_t* coef, int64_t checks,
                            int64_t edges, float* out_msg, void* stream);

/* ---- serving: continuous batching of arriving bins ---------------------- */
typedef struct cider_server cider_server;

typedef struct {
  const cider_weights* weights;
  cider_opts           opts;
  int32_t              steps;          /* T of every request                    */
  int32_t              max_slots;      /* bins resident on the device at once   */
  int32_t              max_queue;      /* waiting requests before EAGAIN        */
  size_t               hbm_budget;     /* device bytes the server may hold: the */
                                       /* per-slot bin state of max_slots bins   */
                                       /* plus the step workspace, which takes   */
                                       /* the rest; a waiting bin is admitted    */
                                       /* (in arrival order) when a slot is free */
                                       /* and the workspace the resident set     */
                                       /* would need with it -- laid out for its */
                                       /* exact K, n mix -- fits.  0: workspace  */
                                       /* sized for max_tokens                   */
  int64_t              max_tokens;     /* cap on the sum of K*n over resident   */
                                       /* bins                                   */
} cider_server_cfg;

typedef struct {
  uint64_t id;           /* request id from cider_server_submit            */
  int32_t  K, n;
  int32_t  status;       /* CIDER_OK or an error                           */
  int32_t  rounds;       /* remask rounds run                              */
  double   t_submit;     /* seconds, monotonic clock                       */
  double   t_admit;
  double   t_done;
} cider_result;

/* Continuous batching of arriving bins, each decoded as cider_decode would
 * decode it alone (Appendix, protocol-level scalability: bins arrive from
 * the preamble stage and are decoded independently).
 * Creates a server with its own HIP stream and worker thread on the current
 * device.  Resident bins advance one refinement step per iteration; a newly
 * admitted bin joins at its own step 1 while others are mid-decode. */
int cider_server_create(const cider_server_cfg* cfg, cider_server** out);
/* Smallest hbm_budget cider_server_create accepts for `cfg`: the per-slot
 * bin state of max_slots bins plus the step workspace of one largest bin
 * (K = CIDER_MAX_K, n = the model's n_max).  No device work. */
int cider_server_budget_floor(const cider_server_cfg* cfg, size_t* bytes);
/* Queues a request.  y_host: host [n] FP32 (copied).  out_symbols_host:
 * host [K][n], written before the request is reported done; it must stay
 * valid until then.  Returns CIDER_EAGAIN when the queue is full. */
int cider_server_submit(cider_server* s, const float* y_host, float sigma2, const cider_code* code,
                        int32_t K, int32_t n, uint8_t* out_symbols_host, uint64_t* id);
/* Moves up to `max` finished results into `out`; *n_done receives the count.
 * Non-blocking. */
int cider_server_poll(cider_server* s, cider_result* out, int32_t max, int32_t* n_done);
/* Blocks until every submitted request has finished. */
int cider_server_drain(cider_server* s);
void cider_server_destroy(cider_server* s);

/* Introspection (no step of the method): per-kernel timings gathered by
 * decode calls made with opts->profile = 1 on
 * this weights handle.  Synchronises the device.  Kernels are named by their
 * role in the step (e.g. "gemm_mlp_up", "attn_row", "step_tail").  `reset`
 * clears the accumulated figures after reading. */
typedef struct {
  char    name[32];
  int64_t launches;
  double  total_ms;     /* summed launch durations between the bracketing events */
} cider_kernel_stat;
int cider_profile_read(const cider_weights* w, cider_kernel_stat* out, int32_t max, int32_t* n_out,
                       int32_t reset);

/* Introspection (no step of the method): the GEMM tile shapes and the
 * token-resident kernel variants the autotuner chose on this weights handle:
 * one entry per (role, N, Kd, token-count bucket 2^bucket) with the tile
 * index and the best measured launch time.  GEMM roles: tile indices are
 * those of the library's GEMM (0 = the default shape).  Roles "user_mlp_tr"
 * and "oproj_mlp3" (the fused sublayer + MLP kernels): n is d, kd the hidden
 * width, tile the variant (0 = the default; variants change the waves per
 * workgroup, the weights' layout in LDS, the weight-ring depth or the
 * fragment prefetch depth, never a result). */
typedef struct {
  char    role[24];
  int32_t n, kd, bucket, tile;
  double  best_ms;
  double  default_ms;
} cider_tuning_entry;
int cider_tuning_read(const cider_weights* w, cider_tuning_entry* out, int32_t max, int32_t* n_out);

/* Message for a status code, and the last error detail of this thread. */
const char* cider_strerror(int status);
const char* cider_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* CIDER_H */
