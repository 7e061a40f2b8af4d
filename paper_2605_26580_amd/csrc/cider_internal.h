// Internal declarations shared by the HIP kernels and the host engine of the
// CIDER refinement library (gfx950 only).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace cider {

constexpr int kMask = 2;
constexpr int kMaxK = 16;
constexpr int kMaxN = 1024;
constexpr int kMaxDeg = 32;
// Fused attention blocks: token slots per workgroup (row attention holds a
// whole row, so rows longer than kBlkRowSlots use the unfused kernels).
constexpr int kBlkRowSlots = 128;
constexpr int kBlkUserSlots = 64;

typedef __bf16 bf16;
typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef __bf16 bf16x4 __attribute__((__vector_size__(4 * sizeof(__bf16))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));

enum Phase : int { kReveal = 0, kFinal = 1, kDone = 2 };
enum Prec : int { kF32 = 0, kBF16 = 1, kFP8 = 2 };

// Per-bin decoding state, device resident, advanced by the step-tail kernel.
struct BinState {
  int phase;      // Phase
  int t;          // next reveal step of the current pass, 1-based
  int pass_T;     // reveal steps in the current pass
  int n_masked;   // sites masked when the current pass started
  int revealed;   // sites revealed so far in the current pass
  int masked;     // sites currently masked (gamma = masked / (K n))
  int first;      // first-reveal applies to step 1 of this pass
  int round;      // remask rounds started
  int sched_j;    // schedule table in use: 0 initial pass, j = rows remasked
  int low_rows;   // bitmask of the rows remasked in the current round
  int valid_rows; // bitmask of rows with zero syndrome in the output
  int pad;
};

// Static description of one bin inside a packed batch.
struct DevBin {
  int tok_off;          // first token of the bin in the packed token arrays
  int K, n, m;
  int slot_off;         // first slot of the bin in per-slot arrays
  int row_off;          // first row of the bin in per-row arrays
  const int* row_ptr;   // check -> slots CSR of H (device)
  const int* col_idx;
  const int* var_ptr;   // slot -> edges of H, ascending check order
  const int* var_edge;  // edge index into col_idx for each (slot, check)
  const int* sched;     // [K+1] offsets, [K+1] lengths, cumulative reveal targets
  const float* y;
  float sigma2;
  uint8_t* X;           // grid [K][n], persistent across steps
  uint8_t* out_sym;     // [K][n]
  float* out_logits;    // [K][n][2] or null
  uint8_t* out_valid;   // [K] or null
  int32_t* out_rounds;  // [1] remask rounds run, or null
  BinState* st;
  // GF(Q) path (null / 0 on the binary path)
  const float* S;       // [n][Q] log evidence
  const uint8_t* coef;  // [nnz] coefficient of each edge of H
  int q_bits;           // Q = 2^q_bits
  int msg_off;          // first check message of the bin in StepCtx::msg, in units of Q floats
};

// Everything a refinement step needs besides the weights.
struct StepCtx {
  int num_bins;
  const DevBin* bins;       // device [num_bins]
  const int* slot_bin;      // device [total_slots]
  const int* row_bin;       // device [total_rows]
  const int* ugrp;          // device [total_ugrp][2]: (bin, first column) of each user-attention block
  const int* tile_bin;      // device [ceil(T / 256)]: bin holding token 256 i
  const int* ugrp32;        // device [total_ugrp32][2]: (bin, first column) of each 32-slot user group
  int total_slots;
  int total_rows;
  int total_ugrp;
  int total_ugrp32;
  long total_tokens;
  int max_n;                // largest n in the batch (in the launch's rows, for row launches)
  int row_first;            // first row of a row launch (rows row_first .. row_first + total_rows - 1)
  int schedule, remask, max_rounds, final_argmax;
  int first_verbatim;       // first-reveal step reveals every slot's selected site
  float remask_thr, tau, eta, lam_max, lam_min;
  float q_inv_tau;          // 1 / tau_min: temperature of the remask confidence
  const float* qhead;       // quality-head parameters (NULL: syndrome / confidence criterion)
  int qh_hidden;
  float phi[4];             // per-round thresholds of the quality head
  const float* qw;          // per-token head output omega [T] (written for bins in their final pass)
  // symbols: 2 on the binary path, Q = 2^m on the GF(Q) path (grid value `mask` = masked)
  int q, mask;
  float tau_max, tau_min;   // inference temperature, annealed over a pass (GF(Q) ranking)
  float* msg;               // GF(Q) Module B: per row and edge, the centred log check message [Q]
  unsigned* rank;           // GF(Q) reveal: per token, confidence rank (larger = more confident)
  uint8_t* sym;             // GF(Q) reveal: per token, argmax symbol
  float gamma_override;     // >= 0: mask-ratio input for every bin (teacher-forced step)
  int reveal_override;      // >= 0: reveal this many sites instead of the schedule's count
  int first_override;       // first-reveal flag used with reveal_override
};

// Device copies of one weight matrix.
struct Mat {
  const float* f32 = nullptr;
  const bf16* b16 = nullptr;
  const uint8_t* f8 = nullptr;
  float f8_scale = 1.f;   // W ~= f8_scale * fp8(W)
  const uint8_t* f8p = nullptr;   // W1 only: f8 with each row's columns reordered for the token-resident up projection
  // BF16 with each row's columns reordered within every 16-column block as
  // 0-3, 8-11, 4-7, 12-15: the k order of an operand held in the 32 x 32
  // accumulator layout, so that a lane's 8 k-values are one 16-byte read
  const bf16* b16k = nullptr;
  // BF16 in MFMA-fragment order for the four-wave kernels (om4_fragment_copy):
  // at d = 256 W_o, W1, W2 (output projection + MLP), W_o (row) and the user
  // Wqkv (row output projection + user attention); at d = 128 the user Wqkv
  // and W_o, W1, W2 (user sublayer + MLP) and the row Wqkv and W_o
  const bf16* b16f = nullptr;
  const uint8_t* f8f = nullptr;   // W1 only: f8p in the four-wave kernel's fragment order
  int rows = 0, cols = 0;
};

struct DevLayer {
  const float *ln1_g, *ln1_b, *bqkv_r, *bo_r;
  const float *ln2_g, *ln2_b, *bqkv_u, *bo_u;
  const float *ln3_g, *ln3_b, *b1, *b2;
  Mat Wqkv_r, Wo_r, Wqkv_u, Wo_u, W1, W2;
};

// The small-vector weights the per-slot and per-token kernels read.
struct EmbedW {
  int d;
  const float *E, *P, *u, *W, *v, *lnf_g, *lnf_b;
  int q;                // symbols: E has q + 1 rows, W and v q rows
};

struct DevModel {
  int n_layers, d, heads, mlp_mult, n_max, q;
  const float *E, *P, *u, *W, *v, *bg1, *bg2, *lnf_g, *lnf_b;
  Mat Wg1, Wg2;
  const float* ug;      // [2][d]: Wg1[:, d:2d] v_a, the gate's e input folded into two vectors
  DevLayer layer[64];
};

// Transient buffers of one forward pass over a packed batch of T tokens.
struct Work {
  float* R;        // [T][d]     FP32 residual stream
  float* Ebuf;     // [T][d]     Module A evidence summary e
  void* ZE;        // [T][2d]    gate MLP input [Z ; e]        (compute type)
  void* H1;        // [T][d]     gate MLP hidden               (compute type)
  void* XN;        // [T][d]     LayerNorm output              (compute type)
  uint8_t* XN8;    // [T][d]     LayerNorm output, OCP e4m3 (FP8 precision)
  float* xscale;   // [T]        per-token scale of XN8
  void* QKV;       // [T][3d]    attention projections         (compute type)
  void* O;         // [T][d]     attention output              (compute type)
  void* HID;       // [T][F]     MLP hidden                    (compute type)
  float* ascale;   // [T]        per-token FP8 activation scales (FP8 only)
  float* lbar;     // [T][2]     logits before Module B
  float* logits;   // [T][2]     logits after Module B
  float* qw;       // [T]        quality-head omega (final passes)
  float* p;        // [slots][2] per-slot beliefs
  float* S;        // [slots][2] per-slot log evidence
};

// ---- FP64 precision mode (kernels_f64.hip) --------------------------------
constexpr int kFP64 = 3;
struct DevLayer64 {
  const double *ln1_g, *ln1_b, *Wqkv_r, *bqkv_r, *Wo_r, *bo_r;
  const double *ln2_g, *ln2_b, *Wqkv_u, *bqkv_u, *Wo_u, *bo_u;
  const double *ln3_g, *ln3_b, *W1, *b1, *W2, *b2;
};
// Double copies of every parameter of the model.
struct DevModel64 {
  const double *E, *P, *u, *W, *v, *Wg1, *bg1, *Wg2, *bg2, *lnf_g, *lnf_b;
  DevLayer64 layer[64];
};
// out = epi(A W^T + bias) in double: Store / GELU into out, residual add into
// R, or the gate blend R = g R + (1 - g) E with g = sigmoid(.).
struct Gemm64 {
  long M;
  int N, Kd;
  const double* A;
  const double* bias;
  double* out;
  double* R;
  const double* E;
};
hipError_t launch_evidence64(const StepCtx& c, double* p, hipStream_t s);
hipError_t launch_embed_demix64(const StepCtx& c, const DevModel64& m, int d, double* R, double* E, double* ZE,
                                const double* p, hipStream_t s);
hipError_t launch_gemm64(int epi, const Gemm64& g, const double* W, hipStream_t s);
hipError_t launch_layernorm64(long T, int d, const double* R, const double* g, const double* b, double* out,
                              hipStream_t s);
hipError_t launch_row_attn64(const StepCtx& c, const double* QKV, double* O, int d, int heads, int max_n,
                             hipStream_t s);
hipError_t launch_user_attn64(const StepCtx& c, const double* QKV, double* O, int d, int heads, int max_K,
                              hipStream_t s);
hipError_t launch_final_proj64(long T, int d, const DevModel64& m, const double* R, double* lbar, hipStream_t s);
hipError_t launch_module_b64(const StepCtx& c, const double* lbar, double* logits, hipStream_t s);
hipError_t launch_step_tail64(const StepCtx& c, const double* logits, hipStream_t s);

// ---- GF(Q) path (kernels_qary.hip) ---------------------------------------
constexpr int kQaryMaxDeg = 16;   // check degree bound of the GF(Q) Module B
// p = softmax_a S per slot ([slots][Q])
hipError_t launch_evidence_q(const StepCtx& c, float* p, hipStream_t s);
// embedding + Module A over Q symbols: R = Z, Ebuf = e, ZE = [Z ; e]
hipError_t launch_embed_demix_q(const StepCtx& c, const EmbedW& m, const Work& w, int prec, hipStream_t s);
// lbar[t][a] = <LN_f(R[t]), w_a>, a < Q
hipError_t launch_final_proj_q(const StepCtx& c, const EmbedW& m, const Work& w, hipStream_t s);
// Module B over GF(Q): check messages into c.msg, then logits = lbar + eta sum
hipError_t launch_module_b_q(const StepCtx& c, const Work& w, int max_checks, hipStream_t s);
// reveal keys: per token confidence rank at the pass's temperature and argmax symbol
hipError_t launch_site_key_q(const StepCtx& c, const Work& w, hipStream_t s);

// GF(64) check-node update: per-edge distributions in, per-edge messages out.
struct GfCheckArgs {
  const float* p;          // [edges][64] variable-to-check distributions, CSR edge order
  const int32_t* row_ptr;  // [checks + 1]
  const uint8_t* coef;     // [edges] nonzero GF(64) coefficients
  long checks, edges;
  float* out;              // [edges][64] check-to-variable messages
};
hipError_t launch_gf64_check(const GfCheckArgs& g, hipStream_t s);

// ---- launchers (kernels_*.hip) --------------------------------------------
hipError_t launch_evidence(const StepCtx& c, float* S, float* p, hipStream_t s);
hipError_t launch_init_bins(const StepCtx& c, int T, int first_reveal, hipStream_t s);
hipError_t launch_embed_demix(const StepCtx& c, const EmbedW& m, const Work& w, int prec,
                              hipStream_t s);
hipError_t launch_final_proj(const StepCtx& c, const EmbedW& m, const Work& w, hipStream_t s);
hipError_t launch_module_b(const StepCtx& c, const Work& w, hipStream_t s);
hipError_t launch_step_tail(const StepCtx& c, const Work& w, hipStream_t s);
// PRISM-style quality head: omega per token from the final residual into c.qw.
hipError_t launch_quality_head(const StepCtx& c, const EmbedW& m, const Work& w, hipStream_t s);

// GEMM: out = epi(pro(A) W^T + bias).  A rows are tokens.
enum Pro : int { kProNone = 0, kProLN = 1 };
enum Epi : int { kEpiStore = 0, kEpiGelu = 1, kEpiResid = 2, kEpiGate = 3 };
struct GemmArgs {
  long M;
  int N, Kd;
  const void* A;        // [M][Kd]: FP32 when pro == LN, else compute type
  const float* ln_g;    // LN gain/bias over Kd (pro == LN)
  const float* ln_b;
  const float* bias;    // [N]
  void* out;            // [M][N] compute type (Store, Gelu)
  float* R;             // [M][N] FP32 residual (Resid, Gate)
  const float* E;       // [M][N] FP32 (Gate)
  const float* a_scale; // [M] per-token activation scale (FP8 input)
  float* out_scale;     // [M] per-token scale of `out` (FP8 LayerNorm output)
  const float* proj_w;  // [2][N] symbol projection applied after the final LayerNorm
  float* proj_out;      // [M][2] logits before Module B (final-projection epilogue)
};
hipError_t launch_gemm(int prec, int pro, int epi, const GemmArgs& g, const Mat& W, hipStream_t s);

hipError_t launch_layernorm(int prec, long T, int d, const float* R, const float* g, const float* b, void* out,
                            hipStream_t s);
hipError_t launch_gemm_bf16(int epi, const GemmArgs& g, const Mat& W, hipStream_t s, int tile);
int gemm_tile_count(int epi, int N, bool ln);
hipError_t launch_mlp_bf16(const GemmArgs& g, const Mat& W1, const float* b1, const Mat& W2, int F, hipStream_t s,
                           int tile, void* hid);
int mlp_tile_count(int D);
int mlp_default_tile(int D);
int gemm_default_tile(int epi, int N, bool ln);
bool gate_fusable(int d);
bool mlp3_ok(int d, int F);
bool qkv3_ok(int d);
bool proj3_ok(int d);
hipError_t launch_proj3_bf16(const GemmArgs& g, const Mat& W, hipStream_t s, bool gelu = false);
hipError_t launch_oproj3_bf16(const GemmArgs& g, const Mat& W, hipStream_t s, bool gate = false);
hipError_t launch_mlp3_bf16(const GemmArgs& g, const Mat& W1, const float* b1, const Mat& W2, int F, hipStream_t s);
bool attn_block_ok(int d, int heads, int max_n, bool user);
hipError_t launch_attn_block(const StepCtx& c, bool user, void* XN, const DevLayer& L, const float* ln_g,
                             const float* ln_b, float* R, int d, int heads, hipStream_t s);
bool oproj_user_attn_ok(int d, int heads);
hipError_t launch_oproj_user_attn(const StepCtx& c, const void* Orow, const Mat& Wo, const float* bo,
                                  const float* ln_g, const float* ln_b, float* R, const Mat& Wqkv, const float* bqkv,
                                  void* O, int d, int heads, hipStream_t s);
bool oproj_mlp3_ok(int d, int F);
hipError_t launch_oproj_mlp3_bf16(const GemmArgs& g, const Mat& Wo, const float* bo, const float* lnx_g,
                                  const float* lnx_b, const Mat& W1, const float* b1, const Mat& W2, int F,
                                  hipStream_t s, int variant = 0, bool f8_up = false);
int oproj_mlp3_variants();
void om4_fragment_copy(int role, int d, int F, const float* src, uint16_t* dst, uint16_t (*to_bf16)(float));
void om4_fragment_copy_f8(int d, int F, const uint8_t* w1p, uint8_t* dst);
bool mlp16_ok(int d, int F);
hipError_t launch_mlp16_bf16(const GemmArgs& g, const Mat& W1, const float* b1, const Mat& W2, int F, hipStream_t s);
bool user_mlp_tr_ok(int d, int heads, int F);
hipError_t launch_user_mlp_tr(const StepCtx& c, void* XN, const DevLayer& L, const GemmArgs& g2, int d, int heads,
                              int F, hipStream_t s, int variant = 0);
int user_mlp_tr_variants();
bool row_qkv_attn_ok(int d, int heads, int max_n);
hipError_t launch_row_qkv_attn(const StepCtx& c, const void* XN, const Mat& Wqkv, const float* bqkv, void* O, int d,
                               int heads, hipStream_t s);
bool row_block_tr_ok(int d, int heads, int max_n);
hipError_t launch_row_block_tr(const StepCtx& c, void* XN, const DevLayer& L, const float* ln_g, const float* ln_b,
                               float* R, int d, int heads, hipStream_t s);
bool user_block_tr_ok(int d, int heads);
hipError_t launch_user_block_tr(const StepCtx& c, void* XN, const DevLayer& L, const float* ln_g, const float* ln_b,
                                float* R, int d, int heads, hipStream_t s);
bool user_qkv_attn_ok(int d, int heads);
hipError_t launch_user_qkv_attn(const StepCtx& c, const void* XN, const Mat& Wqkv, const float* bqkv, void* O,
                                int d, int heads, hipStream_t s);
// Columns of one K-row bin that one user-attention block covers.
inline int ugrp_cols(int K) { return (kBlkUserSlots / 16) * (16 / K); }
// Embedding + Module A + the first LayerNorm in one kernel (BF16, d = 128).
struct EmbedGateArgs {
  const bf16* Wg1;      // [d][2d]
  const float* bg1;     // [d]
  const bf16* Wg2;      // [d][d]
  const float* bg2;     // [d]
  const float* ln_g;    // first layer's LayerNorm 1
  const float* ln_b;
  const float* p;       // [slots][2] per-slot beliefs
  float* R;             // [T][d] FP32 residual stream (out)
  bf16* XN;             // [T][d] LayerNorm output (out)
  const float* ug;      // [2][d]: Wg1's e half times v_a (d = 256 kernel)
};
bool embed_gate3_ok(int d);
hipError_t launch_embed_gate3(const StepCtx& c, const EmbedW& m, const EmbedGateArgs& a, hipStream_t s);
// Slot-wise AMP-MMSE detector (kernels_amp.hip).
struct AmpArgs {
  const float* y;        // [slots][ns][2]
  const int32_t* rows;   // [slots][ns]
  long slots;
  int ns, Q;
  float rho, su2;
  int iters;
  float* S;              // [slots][Q]
};
hipError_t launch_amp_evidence(const AmpArgs& g, hipStream_t s);
bool embed_gate_z_ok(int d);
hipError_t launch_embed_gate_z(const StepCtx& c, const EmbedW& m, const EmbedGateArgs& a, hipStream_t s);
hipError_t launch_gate_bf16(const GemmArgs& g, const Mat& Wg1, const float* bg1, const Mat& Wg2, hipStream_t s);
hipError_t launch_gemm_fp8(const GemmArgs& g, const Mat& W, hipStream_t s);
hipError_t launch_mlp_fp8(const GemmArgs& g, const Mat& W1, const float* b1, const Mat& W2, int F, hipStream_t s);
hipError_t launch_row_attn_mfma(const StepCtx& c, const void* QKV, void* O, int d, int heads, int max_n,
                                hipStream_t s);
hipError_t launch_user_attn_mfma(const StepCtx& c, const void* QKV, void* O, int d, int heads, hipStream_t s);
size_t row_attn_mfma_lds(int max_n, int dh);
hipError_t launch_row_attn(const StepCtx& c, int prec, const void* QKV, void* O, int d, int heads,
                           int max_n, hipStream_t s);
hipError_t launch_user_attn(const StepCtx& c, int prec, const void* QKV, void* O, int d, int heads,
                            hipStream_t s);

}  // namespace cider
