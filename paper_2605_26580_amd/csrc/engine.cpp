// Host side of the CIDER refinement library: handles, argument checks, packed
// batch layout, reveal-schedule tables, the per-step launch sequence (eager or
// replayed as a captured hipGraph) and the C ABI declared in cider.h.
#include "cider.h"
#include "cider_internal.h"

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

using namespace cider;

namespace {

// Last error of the calling thread, kept in a fixed buffer so that reporting
// an error never allocates.
thread_local char g_err[512];

void set_err(const char* what, const char* detail = nullptr) {
  std::snprintf(g_err, sizeof(g_err), "%s%s%s", what, detail ? ": " : "", detail ? detail : "");
}

int fail(int code, const char* msg) {
  set_err(msg);
  // a refused allocation leaves HIP's last-error state set; clear it so that
  // the next launch's error check does not report it again
  if (code == CIDER_ENOMEM) (void)hipGetLastError();
  return code;
}

int fail(int code, const std::string& msg) { return fail(code, msg.c_str()); }

int hip_fail(hipError_t e, const char* what) {
  set_err(what, hipGetErrorString(e));
  return CIDER_EDEVICE;
}

#define HIPCHK(expr)                                      \
  do {                                                    \
    hipError_t e__ = (expr);                              \
    if (e__ != hipSuccess) return hip_fail(e__, #expr);   \
  } while (0)

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

uint16_t f32_to_bf16_bits(float f) {
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);                                     // round to nearest even
  return (uint16_t)(u >> 16);
}

// float -> OCP FP8 e4m3 (bias 7, no infinities, largest finite 448), round to
// nearest even, saturating at +-448.
uint8_t f32_to_e4m3(float x) {
  const uint8_t sign = std::signbit(x) ? 0x80 : 0x00;
  const float a = std::fabs(x);
  if (std::isnan(a)) return 0x7F;
  if (a >= 448.0f) return sign | 0x7E;
  if (a < 0.015625f) {                              // below 2^-6: subnormal m * 2^-9
    const int m = (int)std::nearbyint(a * 512.0f);  // 0..8, ties to even
    return sign | (uint8_t)(m >= 8 ? 0x08 : m);
  }
  int e = 0;
  const float f = std::frexp(a, &e);                // a = f 2^e, f in [0.5, 1)
  int E = e - 1;
  int m = (int)std::nearbyint((f * 2.0f - 1.0f) * 8.0f);
  if (m == 8) { m = 0; E += 1; }
  const int ef = E + 7;
  if (ef > 15 || (ef == 15 && m > 6)) return sign | 0x7E;
  return sign | (uint8_t)((ef << 3) | m);
}

bool cfg_ok(const cider_model_cfg* c, std::string* why) {
  if (!c) { *why = "null cfg"; return false; }
  if (c->n_layers < 1 || c->n_layers > 64) { *why = "n_layers must be 1..64"; return false; }
  if (c->d < 64 || c->d > 512 || c->d % 64) { *why = "d must be a multiple of 64 in 64..512"; return false; }
  if (c->heads < 1 || c->d % c->heads) { *why = "heads must divide d"; return false; }
  int dh = c->d / c->heads;
  if (dh != 16 && dh != 32 && dh != 64) { *why = "d/heads must be 16, 32 or 64"; return false; }
  if (c->mlp_mult < 1 || c->mlp_mult * c->d > 2048) { *why = "mlp_mult*d must be <= 2048"; return false; }
  if (c->n_max < 1 || c->n_max > CIDER_MAX_N) { *why = "n_max must be 1..1024"; return false; }
  if (!(c->q == 0 || c->q == 2 || c->q == 4 || c->q == 8 || c->q == 16 || c->q == 32 || c->q == 64)) {
    *why = "q must be 0 or 2 (binary) or 4, 8, 16, 32, 64";
    return false;
  }
  return true;
}

size_t blob_floats(const cider_model_cfg* c) {
  size_t d = c->d, F = (size_t)c->mlp_mult * c->d;
  const size_t Q = c->q > 2 ? (size_t)c->q : 2;
  size_t head = (Q + 1) * d + (size_t)c->n_max * d + d + Q * d + Q * d + d * 2 * d + d + d * d + d;
  size_t per = 2 * d + 3 * d * d + 3 * d + d * d + d + 2 * d + 3 * d * d + 3 * d + d * d + d + 2 * d +
               F * d + F + d * F + d;
  return head + per * c->n_layers + 2 * d;
}

}  // namespace

// ---------------------------------------------------------------------------
struct cider_code {
  int n = 0, m = 0, nnz = 0, device = 0;
  int q_bits = 0;              // 0: binary code; m: GF(2^m) coefficients in d_coef
  uint8_t* d_coef = nullptr;
  int* d_row_ptr = nullptr;
  int* d_col_idx = nullptr;
  int* d_var_ptr = nullptr;
  int* d_var_edge = nullptr;
  std::vector<int> row_ptr, col_idx;
};

struct GraphSlot {
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;
  std::vector<char> key;
};

struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};

struct TuneKey {
  int epi, ln, N, Kd, bucket;
  bool operator<(const TuneKey& o) const {
    return std::tie(epi, ln, N, Kd, bucket) < std::tie(o.epi, o.ln, o.N, o.Kd, o.bucket);
  }
};
struct TuneVal {
  int tile;
  double best_ms, default_ms;
  std::string role;
};

struct cider_weights {
  std::map<TuneKey, TuneVal> tune;
  bool tuning = false;          // true while candidates are being timed
  std::vector<ProfRec> prof_pending;
  std::map<std::string, std::pair<long, double>> prof_stats;
  bool prof_on = false;
  cider_model_cfg cfg{};
  int device = 0;
  std::vector<void*> allocs;
  DevModel dm{};
  DevModel64 dm64{};            // double copies (FP64 precision mode)
  EmbedW ew{};
  std::mutex mu;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  void* pinned = nullptr;
  size_t pinned_bytes = 0;
  hipEvent_t meta_done = nullptr;
  std::map<std::tuple<int, int, int, int>, int*> sched;
  GraphSlot graph;
};

namespace {

// Reveal targets for a bin shape: header [K+1] offsets and [K+1] lengths,
// then, for the initial pass (j = 0, T steps over K n sites) and for every
// remask pass over j rows (T_rm = max(1, floor(T j / K)) steps over j n
// sites), the cumulative number of sites revealed after each step.
// Emits the table's ints in order through put(int).
template <class Put>
void schedule_emit(int K, int n, int T, int kind, Put put) {
  auto pass_T = [&](int j) { return (j == 0) ? T : std::max(1, (int)((long)T * j / K)); };
  int off = 0;
  for (int j = 0; j <= K; ++j) {
    put(off);
    off += pass_T(j);
  }
  for (int j = 0; j <= K; ++j) put(pass_T(j));
  for (int j = 0; j <= K; ++j) {
    const int Tp = pass_T(j);
    const long Nm = (long)(j == 0 ? K : j) * n;
    for (int t = 1; t <= Tp; ++t) {
      long R;
      if (kind == CIDER_SCHED_COSINE)
        R = (long)std::floor(0.5 * (1.0 - std::cos(M_PI * (double)t / (double)Tp)) * (double)Nm);
      else
        R = (long)t * Nm / Tp;
      put((int)R);
    }
  }
}

// Number of ints in the table of a K-row bin with T initial steps.
long schedule_ints(int K, int T) {
  long total = 2L * (K + 1);
  for (int j = 0; j <= K; ++j) total += (j == 0) ? T : std::max(1, (int)((long)T * j / K));
  return total;
}

std::vector<int> schedule_table(int K, int n, int T, int kind) {
  std::vector<int> out;
  out.reserve(schedule_ints(K, T));
  schedule_emit(K, n, T, kind, [&](int v) { out.push_back(v); });
  return out;
}

int get_sched(cider_weights* w, int K, int n, int T, int kind, int** out) {
  auto key = std::make_tuple(K, n, T, kind);
  auto it = w->sched.find(key);
  if (it != w->sched.end()) { *out = it->second; return CIDER_OK; }
  std::vector<int> tab = schedule_table(K, n, T, kind);
  int* d = nullptr;
  HIPCHK(hipMalloc(&d, tab.size() * sizeof(int)));
  HIPCHK(hipMemcpy(d, tab.data(), tab.size() * sizeof(int), hipMemcpyHostToDevice));
  w->sched[key] = d;
  *out = d;
  return CIDER_OK;
}

struct Layout {
  int num_bins = 0;
  int q = 2;              // symbols of the model (2: binary path)
  long total_tokens = 0;
  int total_slots = 0, total_rows = 0, max_n = 0, total_ugrp = 0;
  size_t off_ugrp = 0, off_ugrp32 = 0, off_tile = 0, off_R, off_E, off_ZE, off_H1, off_QKV, off_O, off_HID, off_lbar, off_logits, off_qw, off_p, off_S,
      off_bins, off_state, off_slot, off_row, off_X, off_XN, off_XN8, off_xscale, off_msg, off_rank, off_sym, total;
};

size_t esize(int prec) { return prec == kFP64 ? 8 : prec == CIDER_FP32 ? 4 : 2; }

// msg: GF(Q) check messages (sum over bins of K nnz), in units of Q floats.
Layout plan_layout(const cider_model_cfg& cfg, int num_bins, long T, int slots, int rows, int prec, long msg = 0) {
  Layout L;
  L.num_bins = num_bins;
  L.total_tokens = T;
  L.total_slots = slots;
  L.total_rows = rows;
  size_t d = cfg.d, F = (size_t)cfg.mlp_mult * cfg.d, es = esize(prec), o = 0;
  const size_t Q = cfg.q > 2 ? (size_t)cfg.q : 2;
  L.q = (int)Q;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes, 256); return at; };
  const size_t fs = prec == kFP64 ? 8 : 4;   // the FP32 buffers hold doubles in the FP64 mode
  L.off_R = take(T * d * fs);
  L.off_E = take(T * d * fs);
  L.off_ZE = take(T * 2 * d * es);
  L.off_H1 = take(T * d * es);
  L.off_XN = take(T * d * es);
  L.off_XN8 = take(prec == CIDER_FP8 ? T * d : 0);
  L.off_xscale = take(prec == CIDER_FP8 ? T * 4 : 0);
  L.off_QKV = take(T * 3 * d * es);
  L.off_O = take(T * d * es);
  L.off_HID = take(T * F * es);
  L.off_lbar = take(T * Q * fs);
  L.off_logits = take(T * Q * fs);
  L.off_qw = take(T * 4);
  L.off_p = take((size_t)slots * Q * fs);
  L.off_S = take((size_t)slots * Q * fs);
  L.off_msg = take(Q > 2 ? (size_t)msg * Q * 4 : 0);
  L.off_rank = take(Q > 2 ? T * 4 : 0);
  L.off_sym = take(Q > 2 ? T : 0);
  L.off_bins = take((size_t)num_bins * sizeof(DevBin));
  L.off_state = take((size_t)num_bins * sizeof(BinState));
  L.off_slot = take((size_t)slots * 4);
  L.off_row = take((size_t)rows * 4);
  L.off_ugrp = take(((size_t)slots + num_bins) * 2 * 4);   // user-attention groups, at most one per column
  L.off_tile = take(((size_t)T / 256 + 1) * 4);              // bin of the first token of each 256-token tile
  L.off_ugrp32 = take(((size_t)slots + num_bins) * 2 * 4);   // 32-slot user groups (at least two columns each)
  L.off_X = take(T);
  L.total = o;
  return L;
}

int ensure_ws(cider_weights* w, const cider_opts& o, size_t need, char** base) {
  if (o.workspace) {
    if (o.workspace_bytes < need)
      return fail(CIDER_EINVAL, "workspace too small: need " + std::to_string(need) + " bytes");
    *base = (char*)o.workspace;
    return CIDER_OK;
  }
  if (w->ws_bytes < need) {
    if (w->ws) {
      HIPCHK(hipDeviceSynchronize());
      HIPCHK(hipFree(w->ws));
      w->ws = nullptr;
      w->ws_bytes = 0;
    }
    size_t want = align_up(need + need / 8, 1 << 20);
    if (hipMalloc(&w->ws, want) != hipSuccess) return fail(CIDER_ENOMEM, "workspace hipMalloc failed");
    w->ws_bytes = want;
  }
  *base = (char*)w->ws;
  return CIDER_OK;
}

int ensure_pinned(cider_weights* w, size_t need) {
  if (!w->meta_done) HIPCHK(hipEventCreateWithFlags(&w->meta_done, hipEventDisableTiming));
  HIPCHK(hipEventSynchronize(w->meta_done));
  if (w->pinned_bytes < need) {
    if (w->pinned) HIPCHK(hipHostFree(w->pinned));
    w->pinned = nullptr;
    size_t want = align_up(need * 2, 1 << 16);
    HIPCHK(hipHostMalloc(&w->pinned, want, hipHostMallocDefault));
    w->pinned_bytes = want;
  }
  return CIDER_OK;
}

// Row-sublayer path a bin of n slots takes.  Bins are packed path by path,
// so the rows (and tokens) of one path are contiguous and each path runs as
// its own launches: a bin's kernels depend on its own shape only, never on
// the other bins it is batched with.
enum RowPath : int { kRowGeneral = 0, kRowBlockTr = 1, kRowAttnBlock = 2, kRowQkvAttn = 3, kRowPaths = 4 };

// FP8 at d = 256 runs the BF16 token-resident kernels, with the MLP up
// projection of the output projection + MLP kernel in e4m3: the precision
// the kernel choice follows.
bool fp8_tr_ok(const cider_model_cfg& m) {
  return m.q <= 2 && user_qkv_attn_ok(m.d, m.heads) && oproj_mlp3_ok(m.d, m.mlp_mult * m.d);
}
int choice_prec(const cider_model_cfg& m, int prec, bool use_blocks) {
  return (prec == kFP8 && use_blocks && fp8_tr_ok(m)) ? kBF16 : prec;
}

int row_path(const cider_model_cfg& m, int prec, bool use_blocks, int n) {
  prec = choice_prec(m, prec, use_blocks);
  if (prec != kBF16 || !use_blocks) return kRowGeneral;
  if (row_block_tr_ok(m.d, m.heads, n)) return kRowBlockTr;
  if (attn_block_ok(m.d, m.heads, n, false)) return kRowAttnBlock;
  if (row_qkv_attn_ok(m.d, m.heads, n)) return kRowQkvAttn;
  return kRowGeneral;
}

// The rows and tokens of one row path inside the packed batch.
struct RowSeg {
  int path, row0, rows, max_n;
  long tok0, toks;
};

struct Run {
  StepCtx ctx{};
  Work work{};
  int prec = 0;
  int forced_tile = -1;   // >= 0: every GEMM uses this tile (tests)
  bool use_blocks = true; // fused attention blocks where the shapes allow
  RowSeg seg[kRowPaths]{};
  int nseg = 0;
  int max_checks = 0;     // most checks of a bin's code (GF(Q) Module B grid)
  int max_K = kMaxK;      // most users of a bin (sizes the FP64 user-attention grid)
};

// Brackets a launch with events when profiling is on.
struct Timed {
  cider_weights* w;
  hipStream_t s;
  const char* name;
  hipEvent_t a = nullptr, b = nullptr;
  Timed(cider_weights* w_, hipStream_t s_, const char* n_) : w(w_), s(s_), name(n_) {
    if (w->prof_on) {
      hipEventCreate(&a);
      hipEventCreate(&b);
      hipEventRecord(a, s);
    }
  }
  ~Timed() {
    if (w->prof_on) {
      hipEventRecord(b, s);
      w->prof_pending.push_back(ProfRec{name, a, b});
    }
  }
};
#define TIMED(name, expr)            \
  do {                                \
    Timed t__(w, s, name);            \
    HIPCHK(expr);                     \
  } while (0)

constexpr int kMlpKey = 100;       // tuning-table keys: the fused MLP,
constexpr int kOprojMlpKey = 101;  // the d = 256 output projection + MLP,
constexpr int kUserMlpKey = 102;   // the d = 128 user sublayer + MLP

int bucket_of(long M) {
  int b = 0;
  while ((1L << (b + 1)) <= M) ++b;
  return b;
}

TuneKey tune_key(int epi, const GemmArgs& g) {
  const int ln = ((epi == kEpiResid || epi == kEpiGate) && g.ln_g) ? 1 : 0;
  return TuneKey{epi, ln, g.N, g.Kd, bucket_of(g.M)};
}

int tile_for(cider_weights* w, int epi, const GemmArgs& g) {
  const TuneKey key = tune_key(epi, g);
  auto it = w->tune.find(key);
  if (it != w->tune.end()) return it->second.tile;
  return epi == kMlpKey ? mlp_default_tile(g.N) : gemm_default_tile(epi, g.N, key.ln != 0);
}

// The variant of a token-resident kernel (key kOprojMlpKey / kUserMlpKey)
// for this batch: forced (tests), tuned earlier, or 0.
int variant_for(cider_weights* w, const Run& r, int key, int d, int F, long T, int count) {
  if (r.forced_tile >= 0) return r.forced_tile < count ? r.forced_tile : 0;
  auto it = w->tune.find(TuneKey{key, 0, d, F, bucket_of(T)});
  return it == w->tune.end() ? 0 : it->second.tile;
}

// Times each variant of a token-resident kernel on the live buffers (3
// launches each, best of them) and records the fastest.  The kernels rewrite
// R and XN in place, which the next forward recomputes from the embedding.
template <class Launch>
int tune_variants(cider_weights* w, const char* role, const TuneKey& key, int count, Launch launch, hipStream_t s) {
  if (w->tune.count(key)) return CIDER_OK;
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  double best = 1e30, dflt = 0;
  int best_t = 0;
  for (int t = 0; t < count; ++t) {
    if (launch(t) != hipSuccess) { (void)hipGetLastError(); continue; }
    double tmin = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
      HIPCHK(hipEventRecord(a, s));
      HIPCHK(launch(t));
      HIPCHK(hipEventRecord(b, s));
      HIPCHK(hipEventSynchronize(b));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, a, b));
      tmin = std::min(tmin, (double)ms);
    }
    if (t == 0) dflt = tmin;
    if (tmin < best) { best = tmin; best_t = t; }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  w->tune[key] = TuneVal{best_t, best, dflt, role};
  return CIDER_OK;
}

// Times every tile shape of one GEMM on the live buffers (3 launches each,
// best of them) and records the fastest.  Only transient buffers are written
// (the next forward recomputes them), never a grid or a bin state.
int tune_gemm(cider_weights* w, const char* role, int epi, const GemmArgs& g, const Mat& W, hipStream_t s) {
  TuneKey key = tune_key(epi, g);
  if (w->tune.count(key)) return CIDER_OK;
  const int cand = gemm_tile_count(epi, g.N, key.ln != 0);
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  double best = 1e30, dflt = 0;
  int best_t = 0;
  for (int t = 0; t < cand; ++t) {
    if (launch_gemm_bf16(epi, g, W, s, t) != hipSuccess) { (void)hipGetLastError(); continue; }
    double tmin = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
      HIPCHK(hipEventRecord(a, s));
      HIPCHK(launch_gemm_bf16(epi, g, W, s, t));
      HIPCHK(hipEventRecord(b, s));
      HIPCHK(hipEventSynchronize(b));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, a, b));
      tmin = std::min(tmin, (double)ms);
    }
    if (t == 0) dflt = tmin;
    if (tmin < best) { best = tmin; best_t = t; }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  w->tune[key] = TuneVal{best_t, best, dflt, role};
  return CIDER_OK;
}

// One denoiser forward over every bin of the batch, then Module B.
// GEMM operands are in the compute type (BF16 on the fast path), LayerNorms
// write a normalised copy XN, and the residual stream R stays FP32.
// The FP64 mode: the plain sequence of kernels in double (embedding and
// Module A, the gate GEMMs, per layer LayerNorm + QKV GEMM + attention +
// output GEMM twice and LayerNorm + MLP GEMMs, final projection, Module B).
int enqueue_forward64(cider_weights* w, const Run& r, hipStream_t s) {
  const DevModel64& M = w->dm64;
  const StepCtx& c = r.ctx;
  const Work& k = r.work;
  const long T = c.total_tokens;
  const int d = w->cfg.d, F = w->cfg.mlp_mult * w->cfg.d, h = w->cfg.heads;
  double* R = (double*)k.R;
  double* E = (double*)k.Ebuf;
  double* ZE = (double*)k.ZE;
  double* H1 = (double*)k.H1;
  double* XN = (double*)k.XN;
  double* QKV = (double*)k.QKV;
  double* O = (double*)k.O;
  double* HID = (double*)k.HID;
  auto gemm = [&](int epi, int N, int Kd, const double* A, const double* bias, double* out, const double* W) {
    Gemm64 g{T, N, Kd, A, bias, out, R, E};
    return launch_gemm64(epi, g, W, s);
  };
  TIMED("embed_demix", launch_embed_demix64(c, M, d, R, E, ZE, (const double*)k.p, s));
  TIMED("gemm_gate1", gemm(kEpiGelu, d, 2 * d, ZE, M.bg1, H1, M.Wg1));
  TIMED("gemm_gate2", gemm(kEpiGate, d, d, H1, M.bg2, nullptr, M.Wg2));
  for (int l = 0; l < w->cfg.n_layers; ++l) {
    const DevLayer64& L = M.layer[l];
    TIMED("layernorm", launch_layernorm64(T, d, R, L.ln1_g, L.ln1_b, XN, s));
    TIMED("gemm_qkv_row", gemm(kEpiStore, 3 * d, d, XN, L.bqkv_r, QKV, L.Wqkv_r));
    TIMED("attn_row", launch_row_attn64(c, QKV, O, d, h, c.max_n, s));
    TIMED("gemm_o_row", gemm(kEpiResid, d, d, O, L.bo_r, nullptr, L.Wo_r));
    TIMED("layernorm", launch_layernorm64(T, d, R, L.ln2_g, L.ln2_b, XN, s));
    TIMED("gemm_qkv_user", gemm(kEpiStore, 3 * d, d, XN, L.bqkv_u, QKV, L.Wqkv_u));
    TIMED("attn_user", launch_user_attn64(c, QKV, O, d, h, r.max_K, s));
    TIMED("gemm_o_user", gemm(kEpiResid, d, d, O, L.bo_u, nullptr, L.Wo_u));
    TIMED("layernorm", launch_layernorm64(T, d, R, L.ln3_g, L.ln3_b, XN, s));
    TIMED("gemm_mlp_up", gemm(kEpiGelu, F, d, XN, L.b1, HID, L.W1));
    TIMED("gemm_mlp_down", gemm(kEpiResid, d, F, HID, L.b2, nullptr, L.W2));
  }
  TIMED("final_proj", launch_final_proj64(T, d, M, R, (double*)k.lbar, s));
  TIMED("module_b", launch_module_b64(c, (const double*)k.lbar, (double*)k.logits, s));
  return CIDER_OK;
}

int enqueue_forward(cider_weights* w, const Run& r, hipStream_t s) {
  if (r.prec == kFP64) return enqueue_forward64(w, r, s);
  const DevModel& m = w->dm;
  const StepCtx& c = r.ctx;
  const Work& k = r.work;
  // FP8 on the d = 256 token-resident path: BF16 kernels, the MLP up
  // projection in e4m3
  const int prec = choice_prec(w->cfg, r.prec, r.use_blocks);
  const bool f8_up = prec != r.prec;
  const long T = c.total_tokens;
  const int d = m.d, F = m.mlp_mult * m.d;
  auto gemm = [&](int epi, const GemmArgs& g, const Mat& W) -> hipError_t {
    if (prec == kF32) return launch_gemm(prec, kProNone, epi, g, W, s);
    int tile = tile_for(w, epi, g);
    if (r.forced_tile >= 0) {
      const bool lnf = (epi == kEpiResid || epi == kEpiGate) && g.ln_g;
      tile = r.forced_tile < gemm_tile_count(epi, g.N, lnf) ? r.forced_tile : 0;
    }
    return launch_gemm_bf16(epi, g, W, s, tile);
  };
  auto ln = [&](const float* gg, const float* bb) { return launch_layernorm(prec, T, d, k.R, gg, bb, k.XN, s); };
  // BF16: the LayerNorm that follows a residual update runs in that GEMM's
  // epilogue (set ln_g / ln_b / out); FP32 runs it as its own kernel.
  const bool fused_ln = prec != kF32;
  const bool f8 = prec == kFP8;
  const size_t es = esize(prec);
  // LayerNorm epilogue into XN (or XN8 and its scales) for the tokens from tok0 on
  auto next_ln = [&](GemmArgs& g, const float* gg, const float* bb, long tok0 = 0) {
    if (!fused_ln) return;
    g.ln_g = gg;
    g.ln_b = bb;
    if (f8) { g.out = k.XN8 + tok0 * d; g.out_scale = k.xscale + tok0; }
    else g.out = (char*)k.XN + tok0 * d * es;
  };
  // the GEMMs fed by a LayerNorm (QKV, MLP up) read XN8 with its per-token
  // scale in FP8, the others stay BF16
  // BF16 at d in {128, 256}: token-resident projections (256 tokens per
  // workgroup, weights streamed through LDS once per tile)
  const bool p3 = prec == kBF16 && proj3_ok(d);
  auto oproj = [&](const GemmArgs& g, const Mat& W) -> hipError_t {
    return p3 ? launch_oproj3_bf16(g, W, s) : gemm(kEpiResid, g, W);
  };
  auto qkv = [&](GemmArgs& g, const Mat& W, long tok0 = 0) -> hipError_t {
    if (prec == kBF16 && qkv3_ok(d)) return launch_proj3_bf16(g, W, s);
    if (!f8) return gemm(kEpiStore, g, W);
    g.A = k.XN8 + tok0 * d;
    g.a_scale = k.xscale + tok0;
    return launch_gemm_fp8(g, W, s);
  };
  // BF16: fused attention blocks where the shapes allow (the row variant is a row path)
  const bool blk_user = prec == kBF16 && r.use_blocks && attn_block_ok(d, m.heads, c.max_n, true);
  const bool user_mlp = prec == kBF16 && r.use_blocks && user_mlp_tr_ok(d, m.heads, F);
  // d = 256: the user-attention output projection runs with the MLP (needs the fused
  // QKV + user attention, which leaves O in k.O)
  const bool oproj_mlp = prec == kBF16 && r.use_blocks && !user_mlp && user_qkv_attn_ok(d, m.heads) &&
                         oproj_mlp3_ok(d, F);
  // d = 256 with the unfused row sublayer (which leaves O in k.O): its output projection runs
  // with the user sublayer's QKV projection and attention
  // (only where no row can take a sublayer-complete row path, whatever its length)
  const bool oproj_user = prec == kBF16 && r.use_blocks && !row_block_tr_ok(d, m.heads, 1) &&
                          !attn_block_ok(d, m.heads, 1, false) && !user_mlp && !user_block_tr_ok(d, m.heads) &&
                          !blk_user && oproj_user_attn_ok(d, m.heads);
  GemmArgs g{};
  g.M = T;
  // BF16 at d = 128 and 256: embedding, Module A and the first LayerNorm in one kernel
  const bool qary = m.q > 2;
  const bool embed_gate = !qary && prec == kBF16 && r.use_blocks && fused_ln &&
                          (embed_gate3_ok(d) || embed_gate_z_ok(d));
  if (qary) TIMED("embed_demix", launch_embed_demix_q(c, w->ew, k, prec, s));
  else if (!embed_gate) TIMED("embed_demix", launch_embed_demix(c, w->ew, k, prec, s));
  // gate MLP: H1 = GELU([Z ; e] Wg1^T + bg1); R = g Z + (1 - g) e, g = sigmoid(H1 Wg2^T + bg2)
  if (embed_gate) {
    EmbedGateArgs ea{};
    ea.Wg1 = m.Wg1.b16; ea.bg1 = m.bg1; ea.Wg2 = m.Wg2.b16; ea.bg2 = m.bg2;
    ea.ln_g = m.layer[0].ln1_g; ea.ln_b = m.layer[0].ln1_b;
    ea.p = k.p; ea.R = k.R; ea.XN = (bf16*)k.XN; ea.ug = m.ug;
    if (embed_gate_z_ok(d)) TIMED("embed_gate", launch_embed_gate_z(c, w->ew, ea, s));
    else TIMED("embed_gate", launch_embed_gate3(c, w->ew, ea, s));
  } else if (prec == kBF16 && d == 256) {
    // d = 256 without the fused blocks: the gate MLP on [Z ; e] as two
    // token-resident kernels
    g.N = d; g.Kd = 2 * d; g.A = k.ZE; g.bias = m.bg1; g.out = k.H1;
    TIMED("gate1", launch_proj3_bf16(g, m.Wg1, s, true));
    g = GemmArgs{}; g.M = T;
    g.N = d; g.Kd = d; g.A = k.H1; g.bias = m.bg2; g.R = k.R; g.E = k.Ebuf;
    next_ln(g, m.layer[0].ln1_g, m.layer[0].ln1_b);
    TIMED("gate2", launch_oproj3_bf16(g, m.Wg2, s, true));
  } else if (fused_ln && gate_fusable(d)) {
    // BF16 / FP8: both gate layers, the blend and the first LayerNorm in one kernel
    g.N = d; g.Kd = 2 * d; g.A = k.ZE; g.bias = m.bg2; g.R = k.R; g.E = k.Ebuf;
    next_ln(g, m.layer[0].ln1_g, m.layer[0].ln1_b);
    TIMED("gate_fused", launch_gate_bf16(g, m.Wg1, m.bg1, m.Wg2, s));
  } else {
    g.N = d; g.Kd = 2 * d; g.A = k.ZE; g.bias = m.bg1; g.out = k.H1;
    TIMED("gemm_gate1", gemm(kEpiGelu, g, m.Wg1));
    g = GemmArgs{}; g.M = T;
    g.N = d; g.Kd = d; g.A = k.H1; g.bias = m.bg2; g.R = k.R; g.E = k.Ebuf;
    if (fused_ln) next_ln(g, m.layer[0].ln1_g, m.layer[0].ln1_b);
    TIMED("gemm_gate2", gemm(kEpiGate, g, m.Wg2));
  }
  for (int l = 0; l < m.n_layers; ++l) {
    const DevLayer& L = m.layer[l];
    if (!fused_ln) TIMED("layernorm", ln(L.ln1_g, L.ln1_b));
    // the row sublayer, one launch sequence per row path (rows and tokens of a path are contiguous)
    for (int si = 0; si < r.nseg; ++si) {
      const RowSeg& sg = r.seg[si];
      StepCtx sc = c;
      sc.row_first = sg.row0;
      sc.total_rows = sg.rows;
      sc.max_n = sg.max_n;
      if (sg.path == kRowBlockTr) {
        // BF16, head width 16, n <= 128: the row-attention sublayer token-resident (one row per workgroup)
        TIMED("row_block", launch_row_block_tr(sc, k.XN, L, L.ln2_g, L.ln2_b, k.R, d, m.heads, s));
        continue;
      }
      if (sg.path == kRowAttnBlock) {
        // BF16: QKV projection, row attention, output projection, residual and LN2 in one kernel
        TIMED("attn_block_row", launch_attn_block(sc, false, k.XN, L, L.ln2_g, L.ln2_b, k.R, d, m.heads, s));
        continue;
      }
      if (sg.path == kRowQkvAttn) {
        // BF16, head width 32, n <= 256: QKV projection and row attention in one kernel
        TIMED("qkv_attn_row", launch_row_qkv_attn(sc, k.XN, L.Wqkv_r, L.bqkv_r, k.O, d, m.heads, s));
      } else {
        // token-wise projections over the path's tokens; the attention indexes tokens absolutely
        g = GemmArgs{}; g.M = sg.toks;
        g.N = 3 * d; g.Kd = d; g.A = (char*)k.XN + sg.tok0 * d * es; g.bias = L.bqkv_r;
        g.out = (char*)k.QKV + sg.tok0 * 3 * d * es;
        TIMED("gemm_qkv_row", qkv(g, L.Wqkv_r, sg.tok0));
        if (prec == kF32) TIMED("attn_row", launch_row_attn(sc, prec, k.QKV, k.O, d, m.heads, sg.max_n, s));
        else TIMED("attn_row", launch_row_attn_mfma(sc, k.QKV, k.O, d, m.heads, sg.max_n, s));
      }
      if (!oproj_user) {
        g = GemmArgs{}; g.M = sg.toks;
        g.N = d; g.Kd = d; g.A = (char*)k.O + sg.tok0 * d * es; g.bias = L.bo_r; g.R = k.R + sg.tok0 * d;
        next_ln(g, L.ln2_g, L.ln2_b, sg.tok0);
        TIMED("gemm_o_row", oproj(g, L.Wo_r));
      }
    }
    if (!fused_ln) TIMED("layernorm", ln(L.ln2_g, L.ln2_b));
    if (user_mlp) {
      // the user-attention sublayer runs with the MLP below, in one kernel
    } else if (prec == kBF16 && r.use_blocks && user_block_tr_ok(d, m.heads)) {
      // BF16, head width 16: the user-attention sublayer token-resident (whole-column groups per wave)
      TIMED("user_block", launch_user_block_tr(c, k.XN, L, L.ln3_g, L.ln3_b, k.R, d, m.heads, s));
    } else if (blk_user) {
      TIMED("attn_block_user", launch_attn_block(c, true, k.XN, L, L.ln3_g, L.ln3_b, k.R, d, m.heads, s));
    } else {
      if (oproj_user) {
        // BF16, d = 256: the row sublayer's output projection (O in k.O, R updated) with the user
        // sublayer's QKV projection and attention, O_user back into k.O
        TIMED("oproj_user_attn", launch_oproj_user_attn(c, k.O, L.Wo_r, L.bo_r, L.ln2_g, L.ln2_b, k.R, L.Wqkv_u,
                                                         L.bqkv_u, k.O, d, m.heads, s));
      } else if (prec == kBF16 && r.use_blocks && user_qkv_attn_ok(d, m.heads)) {
        // BF16, head width 32: QKV projection and user attention in one kernel
        TIMED("qkv_attn_user", launch_user_qkv_attn(c, k.XN, L.Wqkv_u, L.bqkv_u, k.O, d, m.heads, s));
      } else {
        g = GemmArgs{}; g.M = T;
        g.N = 3 * d; g.Kd = d; g.A = k.XN; g.bias = L.bqkv_u; g.out = k.QKV;
        TIMED("gemm_qkv_user", qkv(g, L.Wqkv_u));
        if (prec == kF32) TIMED("attn_user", launch_user_attn(c, prec, k.QKV, k.O, d, m.heads, s));
        else TIMED("attn_user", launch_user_attn_mfma(c, k.QKV, k.O, d, m.heads, s));
      }
      if (!oproj_mlp) {
        g = GemmArgs{}; g.M = T;
        g.N = d; g.Kd = d; g.A = k.O; g.bias = L.bo_u; g.R = k.R;
        next_ln(g, L.ln3_g, L.ln3_b);
        TIMED("gemm_o_user", oproj(g, L.Wo_u));
      }
    }
    if (!fused_ln) TIMED("layernorm", ln(L.ln3_g, L.ln3_b));
    if (fused_ln) {
      // BF16: up, GELU and down in one kernel, hidden layer on chip
      g = GemmArgs{}; g.M = T;
      g.N = d; g.Kd = d; g.A = k.XN; g.bias = L.b2; g.R = k.R;
      if (l + 1 < m.n_layers) {
        next_ln(g, m.layer[l + 1].ln1_g, m.layer[l + 1].ln1_b);
      } else if (qary) {
        // GF(Q): the Q-way projection runs as its own kernel on R; the epilogue's
        // LayerNorm output is not read
        next_ln(g, m.lnf_g, m.lnf_b);
      } else {
        // last block: final LayerNorm and symbol projection in the epilogue
        g.ln_g = m.lnf_g; g.ln_b = m.lnf_b; g.proj_w = m.W; g.proj_out = k.lbar;
      }
      if (f8) {
        g.A = k.XN8;
        g.a_scale = k.xscale;
        TIMED("mlp_fused", launch_mlp_fp8(g, L.W1, L.b1, L.W2, F, s));
      } else if (user_mlp) {
        // BF16, d = 128, head width 16: user-attention sublayer + MLP, token-resident, one kernel
        const int v = variant_for(w, r, kUserMlpKey, d, F, T, user_mlp_tr_variants());
        TIMED("user_mlp", launch_user_mlp_tr(c, k.XN, L, g, d, m.heads, F, s, v));
      } else if (oproj_mlp) {
        // BF16, d = 256: the user sublayer's output projection + MLP in one kernel (O in, R and XN out)
        g.A = k.O;
        const int v = variant_for(w, r, kOprojMlpKey, d, F, T, oproj_mlp3_variants());
        TIMED("oproj_mlp", launch_oproj_mlp3_bf16(g, L.Wo_u, L.bo_u, L.ln3_g, L.ln3_b, L.W1, L.b1, L.W2, F, s, v, f8_up));
      } else if (mlp3_ok(d, F)) {
        // token-resident MLP: 256 tokens per workgroup, weights streamed once per tile
        TIMED("mlp_fused", launch_mlp3_bf16(g, L.W1, L.b1, L.W2, F, s));
      } else if (prec == kBF16 && mlp16_ok(d, F)) {
        // d = 384: token-resident MLP with 16 tokens per wave, 128 per workgroup
        TIMED("mlp_fused", launch_mlp16_bf16(g, L.W1, L.b1, L.W2, F, s));
      } else {
        int mt = tile_for(w, kMlpKey, g);
        if (r.forced_tile >= 0) mt = r.forced_tile < mlp_tile_count(d) ? r.forced_tile : 0;
        TIMED("mlp_fused", launch_mlp_bf16(g, L.W1, L.b1, L.W2, F, s, mt, k.HID));
      }
    } else {
      g = GemmArgs{}; g.M = T;
      g.N = F; g.Kd = d; g.A = k.XN; g.bias = L.b1; g.out = k.HID;
      TIMED("gemm_mlp_up", gemm(kEpiGelu, g, L.W1));
      g = GemmArgs{}; g.M = T;
      g.N = d; g.Kd = F; g.A = k.HID; g.bias = L.b2; g.R = k.R;
      TIMED("gemm_mlp_down", gemm(kEpiResid, g, L.W2));
    }
  }
  if (qary) {
    TIMED("final_proj", launch_final_proj_q(c, w->ew, k, s));
    TIMED("module_b", launch_module_b_q(c, k, r.max_checks, s));
    return CIDER_OK;
  }
  if (!fused_ln) TIMED("final_proj", launch_final_proj(c, w->ew, k, s));
  TIMED("module_b", launch_module_b(c, k, s));
  return CIDER_OK;
}

int tune_mlp(cider_weights* w, const GemmArgs& g, const DevLayer& L, int F, void* hid, hipStream_t s) {
  TuneKey key = tune_key(kMlpKey, g);
  if (w->tune.count(key)) return CIDER_OK;
  const int cand = mlp_tile_count(g.N);
  hipEvent_t a, b;
  HIPCHK(hipEventCreate(&a));
  HIPCHK(hipEventCreate(&b));
  double best = 1e30, dflt = 0;
  int best_t = 0;
  for (int t = 0; t < cand; ++t) {
    if (launch_mlp_bf16(g, L.W1, L.b1, L.W2, F, s, t, hid) != hipSuccess) { (void)hipGetLastError(); continue; }
    double tmin = 1e30;
    for (int rep = 0; rep < 3; ++rep) {
      HIPCHK(hipEventRecord(a, s));
      HIPCHK(launch_mlp_bf16(g, L.W1, L.b1, L.W2, F, s, t, hid));
      HIPCHK(hipEventRecord(b, s));
      HIPCHK(hipEventSynchronize(b));
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, a, b));
      tmin = std::min(tmin, (double)ms);
    }
    if (t == 0) dflt = tmin;
    if (tmin < best) { best = tmin; best_t = t; }
  }
  hipEventDestroy(a);
  hipEventDestroy(b);
  w->tune[key] = TuneVal{best_t, best, dflt, "mlp_fused"};
  return CIDER_OK;
}

// Tunes every GEMM shape of the forward for this batch size (BF16 only).
int autotune_forward(cider_weights* w, const Run& r, hipStream_t s) {
  if (r.prec == kF32 || r.prec == kFP64) return CIDER_OK;
  // FP8 at d = 256 takes the BF16 kernels (its up projection has no variants)
  const int prec = choice_prec(w->cfg, r.prec, r.use_blocks);
  const bool f8_up = prec != r.prec;
  const DevModel& m = w->dm;
  const Work& k = r.work;
  const long T = r.ctx.total_tokens;
  const int d = m.d, F = m.mlp_mult * m.d;
  const DevLayer& L = m.layer[0];
  int rc;
  GemmArgs g{};
  // the separate QKV / output-projection GEMMs run only where a fused
  // attention block does not
  const bool blocks = prec == kBF16 && r.use_blocks && attn_block_ok(d, m.heads, r.ctx.max_n, false) &&
                      attn_block_ok(d, m.heads, r.ctx.max_n, true);
  if (!blocks && !(prec == kBF16 && proj3_ok(d))) {
    if (!(prec == kBF16 && qkv3_ok(d))) {
      g = GemmArgs{}; g.M = T; g.N = 3 * d; g.Kd = d; g.A = k.XN; g.bias = L.bqkv_r; g.out = k.QKV;
      if ((rc = tune_gemm(w, "gemm_qkv", kEpiStore, g, L.Wqkv_r, s))) return rc;
    }
    g = GemmArgs{}; g.M = T; g.N = d; g.Kd = d; g.A = k.O; g.bias = L.bo_r; g.R = k.R;
    g.ln_g = L.ln2_g; g.ln_b = L.ln2_b; g.out = k.XN;
    if ((rc = tune_gemm(w, "gemm_o_ln", kEpiResid, g, L.Wo_r, s))) return rc;
  }
  if (prec == kBF16 && !mlp3_ok(d, F) && !mlp16_ok(d, F)) {
    g = GemmArgs{}; g.M = T; g.N = d; g.Kd = d; g.A = k.XN; g.bias = L.b2; g.R = k.R;
    g.ln_g = L.ln1_g; g.ln_b = L.ln1_b; g.out = k.XN;
    if ((rc = tune_mlp(w, g, L, F, k.HID, s))) return rc;
  }
  // the token-resident kernels with variants (the same choice as the forward's)
  const bool user_mlp = prec == kBF16 && r.use_blocks && user_mlp_tr_ok(d, m.heads, F);
  const bool oproj_mlp = prec == kBF16 && r.use_blocks && !user_mlp && user_qkv_attn_ok(d, m.heads) &&
                         oproj_mlp3_ok(d, F);
  g = GemmArgs{}; g.M = T; g.N = d; g.Kd = d; g.A = k.XN; g.bias = L.b2; g.R = k.R;
  g.ln_g = L.ln1_g; g.ln_b = L.ln1_b; g.out = k.XN;
  if (user_mlp) {
    const StepCtx& c = r.ctx;
    auto launch = [&](int v) { return launch_user_mlp_tr(c, k.XN, L, g, d, m.heads, F, s, v); };
    if ((rc = tune_variants(w, "user_mlp_tr", TuneKey{kUserMlpKey, 0, d, F, bucket_of(T)}, user_mlp_tr_variants(),
                            launch, s)))
      return rc;
  }
  if (oproj_mlp && !f8_up) {
    g.A = k.O;
    auto launch = [&](int v) {
      return launch_oproj_mlp3_bf16(g, L.Wo_u, L.bo_u, L.ln3_g, L.ln3_b, L.W1, L.b1, L.W2, F, s, v);
    };
    if ((rc = tune_variants(w, "oproj_mlp3", TuneKey{kOprojMlpKey, 0, d, F, bucket_of(T)}, oproj_mlp3_variants(),
                            launch, s)))
      return rc;
  }
  return CIDER_OK;
}

int enqueue_step(cider_weights* w, const Run& r, hipStream_t s) {
  int rc = enqueue_forward(w, r, s);
  if (rc) return rc;
  if (r.ctx.qhead) TIMED("quality_head", launch_quality_head(r.ctx, w->ew, r.work, s));
  if (r.ctx.q > 2) TIMED("site_key", launch_site_key_q(r.ctx, r.work, s));
  if (r.prec == kFP64) TIMED("step_tail", launch_step_tail64(r.ctx, (const double*)r.work.logits, s));
  else TIMED("step_tail", launch_step_tail(r.ctx, r.work, s));
  return CIDER_OK;
}

// Runs `iters` refinement steps, replaying a captured graph when allowed.
int run_steps(cider_weights* w, const Run& r, int iters, bool use_graph, hipStream_t s) {
  if (iters <= 0) return CIDER_OK;
  if (!use_graph || s == nullptr || w->prof_on) {
    for (int i = 0; i < iters; ++i) {
      int rc = enqueue_step(w, r, s);
      if (rc) return rc;
    }
    return CIDER_OK;
  }
  std::vector<char> key(sizeof(Run) + sizeof(hipStream_t));
  std::memcpy(key.data(), &r, sizeof(Run));
  std::memcpy(key.data() + sizeof(Run), &s, sizeof(hipStream_t));
  GraphSlot& gs = w->graph;
  if (!gs.exec || gs.key != key) {
    if (gs.exec) {
      HIPCHK(hipEventSynchronize(gs.done));
      HIPCHK(hipGraphExecDestroy(gs.exec));
      gs.exec = nullptr;
    }
    if (!gs.done) HIPCHK(hipEventCreateWithFlags(&gs.done, hipEventDisableTiming));
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
    int rc = enqueue_step(w, r, s);
    hipError_t e = hipStreamEndCapture(s, &graph);
    if (rc) { if (graph) hipGraphDestroy(graph); return rc; }
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    e = hipGraphInstantiate(&gs.exec, graph, nullptr, nullptr, 0);
    hipGraphDestroy(graph);
    if (e != hipSuccess) { gs.exec = nullptr; return hip_fail(e, "hipGraphInstantiate"); }
    gs.key = key;
  }
  for (int i = 0; i < iters; ++i) HIPCHK(hipGraphLaunch(gs.exec, s));
  HIPCHK(hipEventRecord(gs.done, s));
  return CIDER_OK;
}

struct BinIn {
  const float* y;
  float sigma2;
  const cider_code* code;
  int K, n;
  uint8_t* out_sym;
  float* out_logits;
  uint8_t* out_valid;
  int32_t* out_rounds = nullptr;
  uint8_t* X = nullptr;     // persistent grid (serving); null: workspace
  BinState* st = nullptr;   // persistent state (serving); null: workspace
  const float* S = nullptr; // GF(Q) path: device [n][Q] log evidence (y is null)
};

int check_opts(const cider_opts& o) {
  if (o.precision < 0 || o.precision > 3) return fail(CIDER_EINVAL, "precision must be 0..3");
  if (o.schedule != CIDER_SCHED_LINEAR && o.schedule != CIDER_SCHED_COSINE)
    return fail(CIDER_EINVAL, "unknown schedule");
  if (o.remask_max_rounds < 0 || o.remask_max_rounds > 16) return fail(CIDER_EINVAL, "remask_max_rounds 0..16");
  if (!(o.tau > 0.f) || !(o.lam_max > 0.f) || !(o.lam_min > 0.f) || !(o.eta >= 0.f))
    return fail(CIDER_EINVAL, "tau, lam_max, lam_min must be > 0 and eta >= 0");
  if (o.first_reveal < 0 || o.first_reveal > 2) return fail(CIDER_EINVAL, "first_reveal must be 0, 1 or 2");
  if (!(o.tau_max > 0.f) || !(o.tau_min > 0.f)) return fail(CIDER_EINVAL, "tau_max and tau_min must be > 0");
  if (o.qhead) {
    if (!o.remask) return fail(CIDER_EINVAL, "the quality head is a remask criterion: remask must be 1");
    if (o.qhead_hidden < 1 || o.qhead_hidden > 64) return fail(CIDER_EINVAL, "qhead_hidden must be 1..64");
    if (o.remask_stages < 1 || o.remask_stages > 4) return fail(CIDER_EINVAL, "remask_stages must be 1..4");
    for (int i = 0; i < o.remask_stages; ++i)
      if (!std::isfinite(o.remask_phi[i])) return fail(CIDER_EINVAL, "remask_phi must be finite");
  }
  return CIDER_OK;
}

int check_prec(const cider_weights* w, const cider_opts& o) {
  if (o.precision == kFP64 && (w->cfg.q > 2 || o.qhead))
    return fail(CIDER_EUNSUPPORTED, "the FP64 mode covers the binary path without the quality head");
  if (w->cfg.q > 2) {
    if (o.precision == CIDER_FP8) return fail(CIDER_EUNSUPPORTED, "GF(Q) decoding runs in FP32 or BF16");
    if (o.remask || o.qhead) return fail(CIDER_EUNSUPPORTED, "GF(Q) decoding has no remasking");
    if (o.final_argmax) return fail(CIDER_EUNSUPPORTED, "GF(Q) decoding outputs the held-fixed grid");
  }
  if (o.qhead && w->cfg.d > 1024) return fail(CIDER_EUNSUPPORTED, "the quality head needs d <= 1024");
  if (o.precision == CIDER_FP8 && (w->cfg.d % 128 != 0 || (w->cfg.mlp_mult * w->cfg.d) % 64 != 0))
    return fail(CIDER_EUNSUPPORTED, "FP8 needs d to be a multiple of 128");
  return CIDER_OK;
}

int check_bin(const cider_weights* w, const BinIn& b, int steps) {
  const bool qary = w->cfg.q > 2;
  if (!(qary ? b.S : b.y) || !b.code || !b.out_sym)
    return fail(CIDER_EINVAL, qary ? "null S, code or out_symbols" : "null y, code or out_symbols");
  if (qary != (b.S != nullptr))
    return fail(CIDER_EINVAL, qary ? "weights for GF(Q) codes need GF(Q) bins (cider_decode_q_batch)"
                                   : "binary weights need binary bins (cider_decode, cider_decode_batch)");
  if (qary ? (b.code->q_bits == 0 || (1 << b.code->q_bits) != w->cfg.q) : b.code->q_bits != 0)
    return fail(CIDER_EINVAL, "the code's field does not match the weights' symbol count");
  if (row_attn_mfma_lds(b.n, w->cfg.d / w->cfg.heads) > 160 * 1024)
    return fail(CIDER_EUNSUPPORTED, "n * d/heads too large for LDS-resident row attention (n*dh*4 <= 160 KB)");
  if (b.K < 1 || b.K > CIDER_MAX_K) return fail(CIDER_EINVAL, "K must be 1..16");
  if (b.n < 1 || b.n > std::min(w->cfg.n_max, CIDER_MAX_N)) return fail(CIDER_EINVAL, "n out of range for the model");
  if (b.code->n != b.n) return fail(CIDER_EINVAL, "code length != n");
  if (b.code->device != w->device) return fail(CIDER_EINVAL, "code and weights live on different devices");
  if (!qary && (!(b.sigma2 > 0.f) || !std::isfinite(b.sigma2))) return fail(CIDER_EINVAL, "sigma2 must be > 0");
  if (steps < 1 || (long)steps > (long)b.K * b.n) return fail(CIDER_EINVAL, "steps must be 1..K*n");
  return CIDER_OK;
}

// Points a Run's step context and work buffers at a laid-out workspace
// whose per-bin metadata (bins, slot / row / group / tile maps) is in place.
void fill_run(Run* r, const Layout& L, char* base, const cider_opts& o, int B, long T, int slots, int rows,
              int max_n, int ngrp, int ngrp32) {
  StepCtx& c = r->ctx;
  c = StepCtx{};
  c.num_bins = B;
  c.bins = (const DevBin*)(base + L.off_bins);
  c.slot_bin = (const int*)(base + L.off_slot);
  c.row_bin = (const int*)(base + L.off_row);
  c.ugrp = (const int*)(base + L.off_ugrp);
  c.tile_bin = (const int*)(base + L.off_tile);
  c.ugrp32 = (const int*)(base + L.off_ugrp32);
  c.total_ugrp32 = ngrp32;
  c.total_slots = slots;
  c.total_rows = rows;
  c.total_ugrp = ngrp;
  c.total_tokens = T;
  c.max_n = max_n;
  c.schedule = o.schedule;
  c.remask = o.remask;
  c.max_rounds = o.remask_max_rounds;
  c.final_argmax = o.final_argmax;
  c.remask_thr = o.remask_thr;
  c.first_verbatim = o.first_reveal == 2;
  c.q_inv_tau = 1.0f / o.tau_min;
  c.qhead = o.qhead;
  c.qh_hidden = o.qhead_hidden;
  for (int i = 0; i < 4; ++i) c.phi[i] = o.remask_phi[i];
  if (o.qhead) c.max_rounds = o.remask_stages;
  c.tau = o.tau;
  c.eta = o.eta;
  c.lam_max = o.lam_max;
  c.lam_min = o.lam_min;
  c.gamma_override = -1.f;
  c.reveal_override = -1;
  c.first_override = 0;
  c.q = L.q;
  c.mask = c.q > 2 ? c.q : kMask;
  c.tau_max = o.tau_max;
  c.tau_min = o.tau_min;
  c.msg = c.q > 2 ? (float*)(base + L.off_msg) : nullptr;
  c.rank = c.q > 2 ? (unsigned*)(base + L.off_rank) : nullptr;
  c.sym = c.q > 2 ? (uint8_t*)(base + L.off_sym) : nullptr;
  Work& k = r->work;
  k.R = (float*)(base + L.off_R);
  k.Ebuf = (float*)(base + L.off_E);
  k.ZE = base + L.off_ZE;
  k.H1 = base + L.off_H1;
  k.XN = base + L.off_XN;
  k.XN8 = (uint8_t*)(base + L.off_XN8);
  k.xscale = (float*)(base + L.off_xscale);
  k.QKV = base + L.off_QKV;
  k.O = base + L.off_O;
  k.HID = base + L.off_HID;
  k.ascale = nullptr;
  k.lbar = (float*)(base + L.off_lbar);
  k.logits = (float*)(base + L.off_logits);
  k.qw = (float*)(base + L.off_qw);
  c.qw = k.qw;
  k.p = (float*)(base + L.off_p);
  k.S = (float*)(base + L.off_S);
  r->prec = o.precision;
}

// Lays out a batch in the workspace and uploads its metadata; fills `r`.
int prepare(cider_weights* w, const std::vector<BinIn>& bins, int steps, const cider_opts& o,
            hipStream_t s, Run* r, Layout* Lout, bool init_grids) {
  const int B = (int)bins.size();
  long T = 0, msg = 0;
  int slots = 0, rows = 0, max_n = 0;
  r->max_checks = 0;
  r->max_K = 1;
  for (const BinIn& b : bins) {
    r->max_K = std::max(r->max_K, b.K);
    T += (long)b.K * b.n;
    slots += b.n;
    rows += b.K;
    max_n = std::max(max_n, b.n);
    msg += (long)b.K * b.code->nnz;
    r->max_checks = std::max(r->max_checks, b.code->m);
  }
  Layout L = plan_layout(w->cfg, B, T, slots, rows, o.precision, msg);
  L.max_n = max_n;
  char* base = nullptr;
  int rc = ensure_ws(w, o, L.total, &base);
  if (rc) return rc;
  int ngrp = 0, ngrp32 = 0;
  for (const BinIn& b : bins) {
    ngrp += (b.n + ugrp_cols(b.K) - 1) / ugrp_cols(b.K);
    ngrp32 += (b.n + 32 / b.K - 1) / (32 / b.K);
  }
  const int ntile = (int)((T + 255) / 256);
  size_t meta = B * sizeof(DevBin) + (size_t)(slots + rows) * 4 + (size_t)ngrp * 2 * 4 + (size_t)ntile * 4 +
                (size_t)ngrp32 * 2 * 4;
  rc = ensure_pinned(w, meta);
  if (rc) return rc;
  DevBin* hb = (DevBin*)w->pinned;
  int* hslot = (int*)((char*)w->pinned + B * sizeof(DevBin));
  int* hrow = hslot + slots;
  int* hgrp = hrow + rows;
  int* htile = hgrp + 2 * (size_t)ngrp;
  int* hgrp32 = htile + ntile;
  int go32 = 0;
  int go = 0;
  long tok = 0, mo = 0;
  int so = 0, ro = 0;
  // pack the bins path by path (stable within a path)
  std::vector<int> path_of(B), ord(B);
  for (int i = 0; i < B; ++i) {
    path_of[i] = row_path(w->cfg, o.precision, o.fused_blocks != 0, bins[i].n);
    ord[i] = i;
  }
  std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return path_of[x] < path_of[y]; });
  r->nseg = 0;
  for (int i = 0; i < B; ++i) {
    const BinIn& b = bins[ord[i]];
    const int pth = path_of[ord[i]];
    if (r->nseg == 0 || r->seg[r->nseg - 1].path != pth) {
      RowSeg& sg = r->seg[r->nseg++];
      sg = RowSeg{pth, ro, 0, 0, tok, 0};
    }
    RowSeg& sg = r->seg[r->nseg - 1];
    sg.rows += b.K;
    sg.toks += (long)b.K * b.n;
    sg.max_n = std::max(sg.max_n, b.n);
    int* sched = nullptr;
    rc = get_sched(w, b.K, b.n, steps, o.schedule, &sched);
    if (rc) return rc;
    DevBin db{};
    db.tok_off = (int)tok;
    db.K = b.K; db.n = b.n; db.m = b.code->m;
    db.slot_off = so; db.row_off = ro;
    db.row_ptr = b.code->d_row_ptr; db.col_idx = b.code->d_col_idx;
    db.var_ptr = b.code->d_var_ptr; db.var_edge = b.code->d_var_edge;
    db.sched = sched;
    db.y = b.y; db.sigma2 = b.sigma2;
    db.X = b.X ? b.X : (uint8_t*)(base + L.off_X) + tok;
    db.out_sym = b.out_sym; db.out_logits = b.out_logits; db.out_valid = b.out_valid; db.out_rounds = b.out_rounds;
    db.st = b.st ? b.st : (BinState*)(base + L.off_state) + i;
    db.S = b.S;
    db.coef = b.code->d_coef;
    db.q_bits = b.code->q_bits;
    db.msg_off = (int)mo;
    mo += (long)b.K * b.code->nnz;
    hb[i] = db;
    for (int l = 0; l < b.n; ++l) hslot[so + l] = i;
    for (int k = 0; k < b.K; ++k) hrow[ro + k] = i;
    for (int l0 = 0; l0 < b.n; l0 += ugrp_cols(b.K)) {
      hgrp[2 * go] = i;
      hgrp[2 * go + 1] = l0;
      ++go;
    }
    for (long t0 = (tok + 255) / 256 * 256; t0 < tok + (long)b.K * b.n; t0 += 256) htile[t0 / 256] = i;
    for (int l0 = 0; l0 < b.n; l0 += 32 / b.K) {
      hgrp32[2 * go32] = i;
      hgrp32[2 * go32 + 1] = l0;
      ++go32;
    }
    tok += (long)b.K * b.n;
    so += b.n;
    ro += b.K;
  }
  if (T > (long)INT32_MAX) return fail(CIDER_EINVAL, "batch too large");
  HIPCHK(hipMemcpyAsync(base + L.off_bins, hb, B * sizeof(DevBin), hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(base + L.off_slot, hslot, (size_t)slots * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(base + L.off_row, hrow, (size_t)rows * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipMemcpyAsync(base + L.off_ugrp, hgrp, (size_t)ngrp * 2 * 4, hipMemcpyHostToDevice, s));
  if (ntile) HIPCHK(hipMemcpyAsync(base + L.off_tile, htile, (size_t)ntile * 4, hipMemcpyHostToDevice, s));
  if (ngrp32) HIPCHK(hipMemcpyAsync(base + L.off_ugrp32, hgrp32, (size_t)ngrp32 * 2 * 4, hipMemcpyHostToDevice, s));
  HIPCHK(hipEventRecord(w->meta_done, s));

  fill_run(r, L, base, o, B, T, slots, rows, max_n, ngrp, ngrp32);
  const StepCtx& c = r->ctx;
  const Work& k = r->work;
  if (c.q > 2) HIPCHK(launch_evidence_q(c, k.p, s));
  else if (o.precision == kFP64) HIPCHK(launch_evidence64(c, (double*)k.p, s));
  else HIPCHK(launch_evidence(c, k.S, k.p, s));
  if (init_grids) {
    HIPCHK(launch_init_bins(c, steps, o.first_reveal, s));
  }
  *Lout = L;
  return CIDER_OK;
}

int decode_impl(cider_weights* w, const std::vector<BinIn>& bins, int steps, const cider_opts& o,
                hipStream_t s) {
  int rc = check_opts(o);
  if (rc) return rc;
  rc = check_prec(w, o);
  if (rc) return rc;
  if (bins.empty()) return CIDER_OK;
  for (const BinIn& b : bins) {
    rc = check_bin(w, b, steps);
    if (rc) return rc;
  }
  std::lock_guard<std::mutex> lock(w->mu);
  HIPCHK(hipSetDevice(w->device));
  w->prof_on = o.profile != 0;
  Run r;
  Layout L;
  rc = prepare(w, bins, steps, o, s, &r, &L, true);
  if (rc) return rc;
  if (o.autotune >= 2) r.forced_tile = o.autotune - 2;
  r.use_blocks = o.fused_blocks != 0;
  if (o.autotune == 1 && !w->prof_on) {
    rc = autotune_forward(w, r, s);
    if (rc) return rc;
  }
  const bool graph = o.use_graph != 0;
  // initial pass: steps reveal steps + the final pass
  rc = run_steps(w, r, steps + 1, graph, s);
  if (rc) return rc;
  // remask rounds: the quality head's stages, else remask_max_rounds
  const int rounds = o.qhead ? o.remask_stages : o.remask_max_rounds;
  if (o.remask && rounds > 0) {
    const BinState* dst = (const BinState*)((const char*)r.ctx.bins - L.off_bins + L.off_state);
    std::vector<BinState> hst(bins.size());
    for (int round = 0; round < rounds; ++round) {
      HIPCHK(hipMemcpyAsync(hst.data(), dst, hst.size() * sizeof(BinState), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      bool busy = false;
      for (const BinState& st : hst) busy |= st.phase != kDone;
      if (!busy) break;
      // a remask pass has at most `steps` reveal steps, then its final pass
      rc = run_steps(w, r, steps + 1, graph, s);
      if (rc) return rc;
    }
  }
  return CIDER_OK;
}

// ---- decoding without allocation ----------------------------------------
// For callers that cannot allocate (HIP graph capture, tight serving loops):
// a single-bin decode whose workspace, per-bin metadata and reveal-schedule
// table live in the file-scope device array `scratch` (one copy per GPU, held
// until the process ends) instead of memory the library allocates.  Metadata
// reaches the device through kernel arguments, never through host staging
// buffers, so nothing on the host is allocated either.  Every call on a GPU
// shares that GPU's array: calls that overlap on one GPU race.

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch_at[kMaxDevices] = {};

struct SingleBinMeta {
  DevBin db;
  int K, n, ngrp, cols, ngrp32, cols32, ntile;
};

// Writes the packed-batch maps of a batch that holds one bin: every slot,
// row and tile belongs to bin 0; user groups start every `cols` columns.
__global__ void k_single_bin_meta(SingleBinMeta a, DevBin* bins, int* slot, int* row, int* grp, int* tile,
                                  int* grp32) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) bins[0] = a.db;
  if (i < a.n) slot[i] = 0;
  if (i < a.K) row[i] = 0;
  if (i < a.ngrp) {
    grp[2 * i] = 0;
    grp[2 * i + 1] = i * a.cols;
  }
  if (i < a.ntile) tile[i] = 0;
  if (i < a.ngrp32) {
    grp32[2 * i] = 0;
    grp32[2 * i + 1] = i * a.cols32;
  }
}

constexpr int kChunkInts = 240;
struct IntChunk {
  int v[kChunkInts];
  int count;
};

__global__ void k_put_ints(IntChunk c, int* dst) {
  const int i = threadIdx.x;
  if (i < c.count) dst[i] = c.v[i];
}

// Streams ints to device memory in kernel-argument chunks.
struct ChunkWriter {
  IntChunk c{};
  int* dst;
  hipStream_t s;
  hipError_t err = hipSuccess;
  long written = 0;
  void put(int v) {
    c.v[c.count++] = v;
    if (c.count == kChunkInts) flush();
  }
  void flush() {
    if (c.count && err == hipSuccess) {
      hipLaunchKernelGGL(k_put_ints, dim3(1), dim3(256), 0, s, c, dst + written);
      err = hipGetLastError();
    }
    written += c.count;
    c.count = 0;
  }
};

}  // namespace

// The scratch array.  In host code its name stands for the host-side shadow,
// not a device address: kernels get the address looked up per device below.
static __device__ __align__(256) char scratch[CIDER_NOALLOC_SCRATCH_BYTES];

namespace {

// Device address of this device's copy of `scratch`; the device must be current.
int scratch_base(int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(CIDER_EUNSUPPORTED, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_at[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return hip_fail(e, "hipGetSymbolAddress(scratch)");
    g_scratch_at[dev] = (char*)p;
  }
  *out = g_scratch_at[dev];
  return CIDER_OK;
}

int decode_noalloc_impl(cider_weights* w, const BinIn& b, int steps, const cider_opts& o, hipStream_t s) {
  int rc = check_opts(o);
  if (rc) return rc;
  rc = check_prec(w, o);
  if (rc) return rc;
  rc = check_bin(w, b, steps);
  if (rc) return rc;
  if (o.profile) return fail(CIDER_EINVAL, "profile = 1 creates timing events: not available without allocation");
  if (o.workspace) return fail(CIDER_EINVAL, "the allocation-free decode uses its own scratch: workspace must be NULL");
  const long T = (long)b.K * b.n;
  Layout L = plan_layout(w->cfg, 1, T, b.n, b.K, o.precision);
  L.max_n = b.n;
  const size_t sched_at = L.total;
  const size_t need = align_up(sched_at + (size_t)schedule_ints(b.K, steps) * sizeof(int), 256);
  if (need > CIDER_NOALLOC_SCRATCH_BYTES) {
    char msg[160];
    std::snprintf(msg, sizeof(msg), "bin needs %zu bytes of scratch, the allocation-free decode has %zu", need,
                  (size_t)CIDER_NOALLOC_SCRATCH_BYTES);
    return fail(CIDER_EINVAL, msg);
  }
  std::lock_guard<std::mutex> lock(w->mu);
  HIPCHK(hipSetDevice(w->device));
  char* base = nullptr;
  rc = scratch_base(w->device, &base);
  if (rc) return rc;
  w->prof_on = false;

  SingleBinMeta a{};
  a.K = b.K;
  a.n = b.n;
  a.cols = ugrp_cols(b.K);
  a.ngrp = (b.n + a.cols - 1) / a.cols;
  a.cols32 = 32 / b.K;
  a.ngrp32 = (b.n + a.cols32 - 1) / a.cols32;
  a.ntile = (int)((T + 255) / 256);
  DevBin& db = a.db;
  db.tok_off = 0;
  db.K = b.K; db.n = b.n; db.m = b.code->m;
  db.slot_off = 0; db.row_off = 0;
  db.row_ptr = b.code->d_row_ptr; db.col_idx = b.code->d_col_idx;
  db.var_ptr = b.code->d_var_ptr; db.var_edge = b.code->d_var_edge;
  db.sched = (const int*)(base + sched_at);
  db.y = b.y; db.sigma2 = b.sigma2;
  db.X = (uint8_t*)(base + L.off_X);
  db.out_sym = b.out_sym; db.out_logits = b.out_logits; db.out_valid = b.out_valid; db.out_rounds = b.out_rounds;
  db.st = (BinState*)(base + L.off_state);
  const int span = std::max({a.n, a.K, a.ngrp, a.ntile, a.ngrp32, 1});
  hipLaunchKernelGGL(k_single_bin_meta, dim3((span + 255) / 256), dim3(256), 0, s, a, (DevBin*)(base + L.off_bins),
                     (int*)(base + L.off_slot), (int*)(base + L.off_row), (int*)(base + L.off_ugrp),
                     (int*)(base + L.off_tile), (int*)(base + L.off_ugrp32));
  HIPCHK(hipGetLastError());
  ChunkWriter cw;
  cw.dst = (int*)(base + sched_at);
  cw.s = s;
  schedule_emit(b.K, b.n, steps, o.schedule, [&](int v) { cw.put(v); });
  cw.flush();
  HIPCHK(cw.err);

  Run r;
  r.nseg = 1;
  r.seg[0] = RowSeg{row_path(w->cfg, o.precision, o.fused_blocks != 0, b.n), 0, b.K, b.n, 0, T};
  fill_run(&r, L, base, o, 1, T, b.n, b.K, b.n, a.ngrp, a.ngrp32);
  HIPCHK(launch_evidence(r.ctx, r.work.S, r.work.p, s));
  HIPCHK(launch_init_bins(r.ctx, steps, o.first_reveal, s));
  if (o.autotune >= 2) r.forced_tile = o.autotune - 2;
  r.use_blocks = o.fused_blocks != 0;
  // eager launches: instantiating a graph would allocate
  rc = run_steps(w, r, steps + 1, false, s);
  if (rc) return rc;
  const int rounds = o.qhead ? o.remask_stages : o.remask_max_rounds;
  if (o.remask && rounds > 0) {
    BinState st{};
    for (int round = 0; round < rounds; ++round) {
      HIPCHK(hipMemcpyAsync(&st, base + L.off_state, sizeof(BinState), hipMemcpyDeviceToHost, s));
      HIPCHK(hipStreamSynchronize(s));
      if (st.phase == kDone) break;
      rc = run_steps(w, r, steps + 1, false, s);
      if (rc) return rc;
    }
  }
  return CIDER_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

void cider_opts_default(cider_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->precision = CIDER_BF16;
  o->schedule = CIDER_SCHED_LINEAR;
  o->first_reveal = 1;
  o->remask = 0;
  o->remask_max_rounds = 2;
  o->final_argmax = 0;
  o->use_graph = 1;
  o->remask_thr = 0.9f;
  o->tau = 1.0f;
  o->eta = 1.0f;
  o->lam_max = 20.0f;
  o->lam_min = 1e-6f;
  o->tau_max = 1.0f;
  o->tau_min = 1.0f;
  o->qhead = nullptr;
  o->qhead_hidden = 0;
  o->remask_stages = 3;
  o->remask_phi[0] = 0.96f;
  o->remask_phi[1] = 0.90f;
  o->remask_phi[2] = 0.85f;
  o->remask_phi[3] = 0.0f;
  o->autotune = 1;
  o->profile = 0;
  o->fused_blocks = 1;
  o->workspace = nullptr;
  o->workspace_bytes = 0;
}

const char* cider_strerror(int st) {
  switch (st) {
    case CIDER_OK: return "ok";
    case CIDER_EINVAL: return "invalid argument";
    case CIDER_ENOMEM: return "out of memory";
    case CIDER_EDEVICE: return "HIP device error";
    case CIDER_EUNSUPPORTED: return "unsupported";
    case CIDER_EAGAIN: return "try again";
    default: return "unknown status";
  }
}

const char* cider_last_error(void) { return g_err; }

size_t cider_weights_blob_floats(const cider_model_cfg* cfg) {
  std::string why;
  if (!cfg_ok(cfg, &why)) return 0;
  return blob_floats(cfg);
}

int cider_weights_create(const cider_model_cfg* cfg, const float* blob, size_t n_floats, cider_weights** out) {
  std::string why;
  if (!out) return fail(CIDER_EINVAL, "null out");
  *out = nullptr;
  if (!cfg_ok(cfg, &why)) return fail(CIDER_EINVAL, why);
  if (!blob || n_floats != blob_floats(cfg)) return fail(CIDER_EINVAL, "blob size does not match cfg");
  for (size_t i = 0; i < n_floats; ++i)
    if (!std::isfinite(blob[i])) return fail(CIDER_EINVAL, "blob holds a non-finite value");
  cider_weights* w = new cider_weights();
  w->cfg = *cfg;
  HIPCHK(hipGetDevice(&w->device));
  float* dblob = nullptr;
  if (hipMalloc(&dblob, n_floats * 4) != hipSuccess) { delete w; return fail(CIDER_ENOMEM, "weights hipMalloc"); }
  w->allocs.push_back(dblob);
  HIPCHK(hipMemcpy(dblob, blob, n_floats * 4, hipMemcpyHostToDevice));
  const int d = cfg->d, F = cfg->mlp_mult * cfg->d;
  size_t off = 0;
  auto vec = [&](size_t cnt) { const float* p = dblob + off; off += cnt; return p; };
  auto mat = [&](int rows, int cols, Mat* M) -> int {
    size_t cnt = (size_t)rows * cols;
    M->f32 = dblob + off;
    M->rows = rows;
    M->cols = cols;
    std::vector<uint16_t> hb(cnt);
    for (size_t i = 0; i < cnt; ++i) hb[i] = f32_to_bf16_bits(blob[off + i]);
    void* db = nullptr;
    if (hipMalloc(&db, cnt * 2) != hipSuccess) return fail(CIDER_ENOMEM, "weights hipMalloc");
    w->allocs.push_back(db);
    HIPCHK(hipMemcpy(db, hb.data(), cnt * 2, hipMemcpyHostToDevice));
    M->b16 = (const bf16*)db;
    // OCP e4m3 copy with one per-tensor scale amax / 448
    float amax = 0.f;
    for (size_t i = 0; i < cnt; ++i) amax = std::max(amax, std::fabs(blob[off + i]));
    const float sc = amax > 0.f ? amax / 448.0f : 1.0f;
    std::vector<uint8_t> h8(cnt);
    for (size_t i = 0; i < cnt; ++i) h8[i] = f32_to_e4m3(blob[off + i] / sc);
    void* d8 = nullptr;
    if (hipMalloc(&d8, cnt) != hipSuccess) return fail(CIDER_ENOMEM, "weights hipMalloc");
    w->allocs.push_back(d8);
    HIPCHK(hipMemcpy(d8, h8.data(), cnt, hipMemcpyHostToDevice));
    M->f8 = (const uint8_t*)d8;
    M->f8_scale = sc;
    if (cols % 16 == 0) {
      // k-ordered BF16 copy (see Mat::b16k)
      static const int kperm[16] = {0, 1, 2, 3, 8, 9, 10, 11, 4, 5, 6, 7, 12, 13, 14, 15};
      std::vector<uint16_t> hk(cnt);
      for (int r = 0; r < rows; ++r)
        for (int c = 0; c < cols; ++c) hk[(size_t)r * cols + c] = hb[(size_t)r * cols + (c & ~15) + kperm[c & 15]];
      void* dk = nullptr;
      if (hipMalloc(&dk, cnt * 2) != hipSuccess) return fail(CIDER_ENOMEM, "weights hipMalloc");
      w->allocs.push_back(dk);
      HIPCHK(hipMemcpy(dk, hk.data(), cnt * 2, hipMemcpyHostToDevice));
      M->b16k = (const bf16*)dk;
    }
    off += cnt;
    return CIDER_OK;
  };
  DevModel& m = w->dm;
  size_t off_v = 0, off_wg1 = 0;
  m.n_layers = cfg->n_layers; m.d = d; m.heads = cfg->heads; m.mlp_mult = cfg->mlp_mult; m.n_max = cfg->n_max;
  m.q = cfg->q > 2 ? cfg->q : 2;
  int rc = 0;
  m.E = vec((size_t)(m.q + 1) * d);
  m.P = vec((size_t)cfg->n_max * d);
  m.u = vec(d);
  m.W = vec((size_t)m.q * d);
  off_v = off;
  m.v = vec((size_t)m.q * d);
  off_wg1 = off;
  if ((rc = mat(d, 2 * d, &m.Wg1))) goto bad;
  m.bg1 = vec(d);
  if ((rc = mat(d, d, &m.Wg2))) goto bad;
  m.bg2 = vec(d);
  for (int l = 0; l < cfg->n_layers; ++l) {
    DevLayer& L = m.layer[l];
    L.ln1_g = vec(d); L.ln1_b = vec(d);
    const size_t off_wqr = off;
    if ((rc = mat(3 * d, d, &L.Wqkv_r))) goto bad;
    L.bqkv_r = vec(3 * (size_t)d);
    const size_t off_wor = off;
    if ((rc = mat(d, d, &L.Wo_r))) goto bad;
    L.bo_r = vec(d);
    L.ln2_g = vec(d); L.ln2_b = vec(d);
    const size_t off_wqu = off;
    if ((rc = mat(3 * d, d, &L.Wqkv_u))) goto bad;
    L.bqkv_u = vec(3 * (size_t)d);
    const size_t off_wou = off;
    if ((rc = mat(d, d, &L.Wo_u))) goto bad;
    L.bo_u = vec(d);
    L.ln3_g = vec(d); L.ln3_b = vec(d);
    {
      const size_t off_w1 = off;
      if ((rc = mat(F, d, &L.W1))) goto bad;
      if (d % 64 == 0) {
        // e4m3 copy of W1 for the token-resident FP8 up projection: in each
        // 64-column block, position 32 h + 8 s + e holds column
        // 16 s + 8 (e / 4) + 4 h + e % 4 (the order of a lane's X1 bytes)
        std::vector<uint8_t> p8((size_t)F * d);
        for (int row = 0; row < F; ++row)
          for (int t = 0; t < d / 64; ++t)
            for (int h = 0; h < 2; ++h)
              for (int sb = 0; sb < 4; ++sb)
                for (int e = 0; e < 8; ++e) {
                  const int col = 64 * t + 16 * sb + 8 * (e >> 2) + 4 * h + (e & 3);
                  p8[(size_t)row * d + 64 * t + 32 * h + 8 * sb + e] =
                      f32_to_e4m3(blob[off_w1 + (size_t)row * d + col] / L.W1.f8_scale);
                }
        void* dp = nullptr;
        if (hipMalloc(&dp, p8.size()) != hipSuccess) { rc = fail(CIDER_ENOMEM, "weights hipMalloc"); goto bad; }
        w->allocs.push_back(dp);
        if (hipMemcpy(dp, p8.data(), p8.size(), hipMemcpyHostToDevice) != hipSuccess) {
          rc = fail(CIDER_EDEVICE, "weights upload");
          goto bad;
        }
        L.W1.f8p = (const uint8_t*)dp;
        if (oproj_mlp3_ok(d, F)) {
          std::vector<uint8_t> f8f(p8.size());
          om4_fragment_copy_f8(d, F, p8.data(), f8f.data());
          void* df = nullptr;
          if (hipMalloc(&df, f8f.size()) != hipSuccess) { rc = fail(CIDER_ENOMEM, "weights hipMalloc"); goto bad; }
          w->allocs.push_back(df);
          if (hipMemcpy(df, f8f.data(), f8f.size(), hipMemcpyHostToDevice) != hipSuccess) {
            rc = fail(CIDER_EDEVICE, "weights upload");
            goto bad;
          }
          L.W1.f8f = (const uint8_t*)df;
        }
      }
    }
    L.b1 = vec(F);
    {
      const size_t off_w1 = off - (size_t)F - (size_t)F * d, off_w2 = off;
      if ((rc = mat(d, F, &L.W2))) goto bad;
      // fragment-major copies for the four-wave kernels: W_o (user), W1 and
      // W2 for the output projection + MLP, W_o (row) and the user Wqkv for
      // the row output projection + user attention
      // (d = 256); at d = 128 the same for the user sublayer + MLP kernel
      const bool om4 = oproj_mlp3_ok(d, F), ou4 = oproj_user_attn_ok(d, cfg->heads);
      // and the row sublayer
      const bool umf = user_mlp_tr_ok(d, cfg->heads, F), rbf = row_block_tr_ok(d, cfg->heads, 1);
      Mat* dstm[11] = {&L.Wo_u,   &L.W1,    &L.W2, &L.Wo_r, &L.Wqkv_u, &L.Wqkv_u,
                       &L.Wo_u,   &L.W1,    &L.W2, &L.Wqkv_r, &L.Wo_r};
      const int roles[11] = {0, 1, 2, 0, 3, 5, 6, 1, 2, 5, 6};
      const size_t offs[11] = {off_wou, off_w1, off_w2, off_wor, off_wqu, off_wqu,
                               off_wou, off_w1, off_w2, off_wqr, off_wor};
      for (int k = 0; k < 11; ++k) {
        if (!(k < 3 ? om4 : k < 5 ? ou4 : k < 9 ? umf : rbf)) continue;
        const size_t cnt = (size_t)dstm[k]->rows * dstm[k]->cols;
        std::vector<uint16_t> hf(cnt);
        om4_fragment_copy(roles[k], d, F, blob + offs[k], hf.data(), f32_to_bf16_bits);
        void* df = nullptr;
        if (hipMalloc(&df, cnt * 2) != hipSuccess) { rc = fail(CIDER_ENOMEM, "weights hipMalloc"); goto bad; }
        w->allocs.push_back(df);
        if (hipMemcpy(df, hf.data(), cnt * 2, hipMemcpyHostToDevice) != hipSuccess) {
          rc = fail(CIDER_EDEVICE, "weights upload");
          goto bad;
        }
        dstm[k]->b16f = (const bf16*)df;
      }
    }
    L.b2 = vec(d);
  }
  m.lnf_g = vec(d);
  m.lnf_b = vec(d);
  if (off != n_floats) { rc = fail(CIDER_EINVAL, "internal layout mismatch"); goto bad; }
  if (m.q == 2) {
    // the gate's e input is a combination of the two rows v_a, so its share of
    // the first gate layer folds into ug[a] = Wg1[:, d:2d] v_a (FP64 sums)
    std::vector<float> hug(2 * (size_t)d);
    for (int a = 0; a < 2; ++a)
      for (int j = 0; j < d; ++j) {
        double acc = 0.0;
        for (int i = 0; i < d; ++i)
          acc += (double)blob[off_wg1 + (size_t)j * 2 * d + d + i] * (double)blob[off_v + (size_t)a * d + i];
        hug[(size_t)a * d + j] = (float)acc;
      }
    void* dug = nullptr;
    if (hipMalloc(&dug, hug.size() * 4) != hipSuccess) { rc = fail(CIDER_ENOMEM, "weights hipMalloc"); goto bad; }
    w->allocs.push_back(dug);
    if (hipMemcpy(dug, hug.data(), hug.size() * 4, hipMemcpyHostToDevice) != hipSuccess) {
      rc = fail(CIDER_EDEVICE, "weights copy");
      goto bad;
    }
    m.ug = (const float*)dug;
  }
  w->ew = EmbedW{d, m.E, m.P, m.u, m.W, m.v, m.lnf_g, m.lnf_b, m.q};
  {
    // double copies for the FP64 mode, at the FP32 blob's offsets
    std::vector<double> h64(blob, blob + n_floats);
    double* d64 = nullptr;
    if (hipMalloc(&d64, n_floats * 8) != hipSuccess) { rc = fail(CIDER_ENOMEM, "weights hipMalloc"); goto bad; }
    w->allocs.push_back(d64);
    if (hipMemcpy(d64, h64.data(), n_floats * 8, hipMemcpyHostToDevice) != hipSuccess) {
      rc = fail(CIDER_EDEVICE, "weights copy");
      goto bad;
    }
    auto to64 = [&](const float* p) { return (const double*)(d64 + (p - dblob)); };
    DevModel64& M = w->dm64;
    M.E = to64(m.E); M.P = to64(m.P); M.u = to64(m.u); M.W = to64(m.W); M.v = to64(m.v);
    M.Wg1 = to64(m.Wg1.f32); M.bg1 = to64(m.bg1); M.Wg2 = to64(m.Wg2.f32); M.bg2 = to64(m.bg2);
    M.lnf_g = to64(m.lnf_g); M.lnf_b = to64(m.lnf_b);
    for (int l = 0; l < cfg->n_layers; ++l) {
      const DevLayer& L = m.layer[l];
      DevLayer64& X = M.layer[l];
      X.ln1_g = to64(L.ln1_g); X.ln1_b = to64(L.ln1_b); X.Wqkv_r = to64(L.Wqkv_r.f32); X.bqkv_r = to64(L.bqkv_r);
      X.Wo_r = to64(L.Wo_r.f32); X.bo_r = to64(L.bo_r);
      X.ln2_g = to64(L.ln2_g); X.ln2_b = to64(L.ln2_b); X.Wqkv_u = to64(L.Wqkv_u.f32); X.bqkv_u = to64(L.bqkv_u);
      X.Wo_u = to64(L.Wo_u.f32); X.bo_u = to64(L.bo_u);
      X.ln3_g = to64(L.ln3_g); X.ln3_b = to64(L.ln3_b); X.W1 = to64(L.W1.f32); X.b1 = to64(L.b1);
      X.W2 = to64(L.W2.f32); X.b2 = to64(L.b2);
    }
  }
  *out = w;
  return CIDER_OK;
bad:
  for (void* p : w->allocs) hipFree(p);
  delete w;
  return rc;
}

void cider_weights_destroy(cider_weights* w) {
  if (!w) return;
  hipSetDevice(w->device);
  hipDeviceSynchronize();
  if (w->graph.exec) hipGraphExecDestroy(w->graph.exec);
  if (w->graph.done) hipEventDestroy(w->graph.done);
  if (w->meta_done) hipEventDestroy(w->meta_done);
  for (auto& kv : w->sched) hipFree(kv.second);
  for (void* p : w->allocs) hipFree(p);
  if (w->ws) hipFree(w->ws);
  if (w->pinned) hipHostFree(w->pinned);
  delete w;
}

int cider_code_create(int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* col_idx, cider_code** out) {
  if (!out) return fail(CIDER_EINVAL, "null out");
  *out = nullptr;
  if (n < 1 || n > CIDER_MAX_N || m < 1 || m > 4 * CIDER_MAX_N || !row_ptr || !col_idx)
    return fail(CIDER_EINVAL, "bad code sizes or null arrays");
  if (row_ptr[0] != 0) return fail(CIDER_EINVAL, "row_ptr[0] must be 0");
  for (int j = 0; j < m; ++j) {
    int deg = row_ptr[j + 1] - row_ptr[j];
    if (deg < 1 || deg > kMaxDeg) return fail(CIDER_EINVAL, "check degree must be 1..32");
  }
  const int nnz = row_ptr[m];
  if (nnz > 4096) return fail(CIDER_EINVAL, "at most 4096 edges");
  std::vector<int> vdeg(n, 0);
  for (int j = 0; j < m; ++j)
    for (int e = row_ptr[j]; e < row_ptr[j + 1]; ++e) {
      int v = col_idx[e];
      if (v < 0 || v >= n) return fail(CIDER_EINVAL, "column index out of range");
      if (e > row_ptr[j] && col_idx[e - 1] >= v) return fail(CIDER_EINVAL, "columns must ascend within a row");
      if (++vdeg[v] > kMaxDeg) return fail(CIDER_EINVAL, "slot degree must be <= 32");
    }
  std::vector<int> var_ptr(n + 1, 0), var_edge(nnz);
  for (int v = 0; v < n; ++v) var_ptr[v + 1] = var_ptr[v] + vdeg[v];
  std::vector<int> fill(var_ptr.begin(), var_ptr.end() - 1);
  for (int j = 0; j < m; ++j)
    for (int e = row_ptr[j]; e < row_ptr[j + 1]; ++e) var_edge[fill[col_idx[e]]++] = e;  // ascending j
  cider_code* c = new cider_code();
  c->n = n; c->m = m; c->nnz = nnz;
  c->row_ptr.assign(row_ptr, row_ptr + m + 1);
  c->col_idx.assign(col_idx, col_idx + nnz);
  hipError_t e = hipGetDevice(&c->device);
  if (e == hipSuccess) e = hipMalloc(&c->d_row_ptr, (m + 1) * 4);
  if (e == hipSuccess) e = hipMalloc(&c->d_col_idx, nnz * 4);
  if (e == hipSuccess) e = hipMalloc(&c->d_var_ptr, (n + 1) * 4);
  if (e == hipSuccess) e = hipMalloc(&c->d_var_edge, nnz * 4);
  if (e == hipSuccess) e = hipMemcpy(c->d_row_ptr, row_ptr, (m + 1) * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_col_idx, col_idx, nnz * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_var_ptr, var_ptr.data(), (n + 1) * 4, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(c->d_var_edge, var_edge.data(), nnz * 4, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    cider_code_destroy(c);
    return hip_fail(e, "cider_code_create");
  }
  *out = c;
  return CIDER_OK;
}

void cider_code_destroy(cider_code* c) {
  if (!c) return;
  hipFree(c->d_row_ptr);
  hipFree(c->d_col_idx);
  hipFree(c->d_var_ptr);
  hipFree(c->d_var_edge);
  hipFree(c->d_coef);
  delete c;
}

int cider_code_create_q(int32_t n, int32_t m, const int32_t* row_ptr, const int32_t* col_idx, const uint8_t* coef,
                        int32_t q_bits, cider_code** out) {
  if (!out) return fail(CIDER_EINVAL, "null out");
  *out = nullptr;
  if (q_bits < 2 || q_bits > 6 || !coef || !row_ptr) return fail(CIDER_EINVAL, "q_bits must be 2..6 with coefficients");
  if (m < 1 || m > 4 * CIDER_MAX_N || row_ptr[0] != 0) return fail(CIDER_EINVAL, "bad code sizes");
  for (int j = 0; j < m; ++j)
    if (row_ptr[j + 1] - row_ptr[j] > kQaryMaxDeg) return fail(CIDER_EINVAL, "GF(Q) check degree must be 1..16");
  const int nnz = row_ptr[m];
  for (int e = 0; e < nnz; ++e)
    if (coef[e] < 1 || coef[e] >= (1 << q_bits)) return fail(CIDER_EINVAL, "coefficients must be nonzero field elements");
  cider_code* c = nullptr;
  int rc = cider_code_create(n, m, row_ptr, col_idx, &c);
  if (rc) return rc;
  hipError_t e = hipMalloc(&c->d_coef, (size_t)nnz);
  if (e == hipSuccess) e = hipMemcpy(c->d_coef, coef, (size_t)nnz, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    cider_code_destroy(c);
    return hip_fail(e, "cider_code_create_q");
  }
  c->q_bits = q_bits;
  *out = c;
  return CIDER_OK;
}

int cider_workspace_size(const cider_weights* w, int32_t num_bins, int64_t total_tokens, int64_t total_slots,
                         const cider_opts* opts, size_t* bytes) {
  if (!w || !bytes || num_bins < 0 || total_tokens < 0 || total_slots < 0) return fail(CIDER_EINVAL, "bad args");
  cider_opts o;
  if (opts) o = *opts; else cider_opts_default(&o);
  long rows_bound = (long)num_bins * CIDER_MAX_K;
  if (total_tokens < rows_bound) rows_bound = total_tokens;
  Layout L = plan_layout(w->cfg, num_bins, total_tokens, (int)total_slots, (int)rows_bound, o.precision);
  *bytes = L.total;
  return CIDER_OK;
}

int cider_decode(const float* y, float sigma2, const cider_code* code, int32_t K, int32_t n, const cider_weights* w,
                 int32_t steps, uint8_t* out_symbols, const cider_opts* opts, void* stream) {
  if (!w) return fail(CIDER_EINVAL, "null weights");
  cider_opts o;
  if (opts) o = *opts; else cider_opts_default(&o);
  std::vector<BinIn> bins{BinIn{y, sigma2, code, K, n, out_symbols, nullptr, nullptr}};
  return decode_impl(const_cast<cider_weights*>(w), bins, steps, o, (hipStream_t)stream);
}

int cider_decode_noalloc(const float* y, float sigma2, const cider_code* code, int32_t K, int32_t n,
                         const cider_weights* w, int32_t steps, uint8_t* out_symbols, const cider_opts* opts,
                         void* stream) {
  if (!w) return fail(CIDER_EINVAL, "null weights");
  cider_opts o;
  if (opts) o = *opts; else cider_opts_default(&o);
  const BinIn b{y, sigma2, code, K, n, out_symbols, nullptr, nullptr};
  return decode_noalloc_impl(const_cast<cider_weights*>(w), b, steps, o, (hipStream_t)stream);
}

int cider_decode_batch(int32_t num_bins, const cider_bin* bins, const cider_weights* w, int32_t steps,
                       const cider_opts* opts, void* stream) {
  if (!w) return fail(CIDER_EINVAL, "null weights");
  if (num_bins < 0 || (num_bins > 0 && !bins)) return fail(CIDER_EINVAL, "bad bin list");
  cider_opts o;
  if (opts) o = *opts; else cider_opts_default(&o);
  std::vector<BinIn> v;
  v.reserve(num_bins);
  for (int i = 0; i < num_bins; ++i)
    v.push_back(BinIn{bins[i].y, bins[i].sigma2, bins[i].code, bins[i].K, bins[i].n, bins[i].out_symbols,
                      bins[i].out_logits, bins[i].out_row_valid, bins[i].out_rounds});
  return decode_impl(const_cast<cider_weights*>(w), v, steps, o, (hipStream_t)stream);
}

int cider_decode_q_batch(int32_t num_bins, const cider_qbin* bins, const cider_weights* w, int32_t steps,
                         const cider_opts* opts, void* stream) {
  if (!w) return fail(CIDER_EINVAL, "null weights");
  if (num_bins < 0 || (num_bins > 0 && !bins)) return fail(CIDER_EINVAL, "bad bin list");
  cider_opts o;
  if (opts) o = *opts; else cider_opts_default(&o);
  std::vector<BinIn> v;
  v.reserve(num_bins);
  for (int i = 0; i < num_bins; ++i) {
    BinIn b{nullptr, 1.0f, bins[i].code, bins[i].K, bins[i].n, bins[i].out_symbols, bins[i].out_logits,
            bins[i].out_row_valid};
    b.S = bins[i].S;
    v.push_back(b);
  }
  return decode_impl(const_cast<cider_weights*>(w), v, steps, o, (hipStream_t)stream);
}

int cider_step_debug_q(const uint8_t* X_in, uint8_t* X_out, const float* S, const cider_code* code, int32_t K,
                       int32_t n, const cider_weights* wc, float gamma, int32_t reveal_count, int32_t first,
                       const cider_opts* opts, float* out_lbar, float* out_logits, void* stream) {
  if (!wc || !X_in) return fail(CIDER_EINVAL, "null weights or X_in");
  cider_weights* w = const_cast<cider_weights*>(wc);
  cider_opts o;
  if (opts) o = *opts; else cider_opts_default(&o);
  int rc = check_opts(o);
  if (rc) return rc;
  rc = check_prec(w, o);
  if (rc) return rc;
  uint8_t dummy = 0;
  BinIn b{nullptr, 1.0f, code, K, n, &dummy, nullptr, nullptr};
  b.S = S;
  rc = check_bin(w, b, 1);
  if (rc) return rc;
  if (reveal_count < 0 || reveal_count > K * n) return fail(CIDER_EINVAL, "reveal_count out of range");
  if (!(gamma >= 0.f && gamma <= 1.f)) return fail(CIDER_EINVAL, "gamma must be in [0, 1]");
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(w->mu);
  HIPCHK(hipSetDevice(w->device));
  Run r;
  Layout L;
  std::vector<BinIn> bins{b};
  rc = prepare(w, bins, 1, o, s, &r, &L, true);
  if (rc) return rc;
  char* base = (char*)r.ctx.bins - L.off_bins;
  uint8_t* Xw = (uint8_t*)(base + L.off_X);
  HIPCHK(hipMemcpyAsync(Xw, X_in, (size_t)K * n, hipMemcpyDeviceToDevice, s));
  if (o.autotune >= 2) r.forced_tile = o.autotune - 2;
  r.use_blocks = o.fused_blocks != 0;
  r.ctx.gamma_override = gamma;
  r.ctx.reveal_override = reveal_count;
  r.ctx.first_override = first ? 1 : 0;
  rc = enqueue_forward(w, r, s);
  if (rc) return rc;
  const size_t T = (size_t)K * n, Q = (size_t)w->cfg.q;
  if (out_lbar) HIPCHK(hipMemcpyAsync(out_lbar, r.work.lbar, T * Q * 4, hipMemcpyDeviceToDevice, s));
  if (out_logits) HIPCHK(hipMemcpyAsync(out_logits, r.work.logits, T * Q * 4, hipMemcpyDeviceToDevice, s));
  if (X_out) {
    HIPCHK(launch_site_key_q(r.ctx, r.work, s));
    HIPCHK(launch_step_tail(r.ctx, r.work, s));
    HIPCHK(hipMemcpyAsync(X_out, Xw, T, hipMemcpyDeviceToDevice, s));
  }
  return CIDER_OK;
}

int cider_step_debug(const uint8_t* X_in, uint8_t* X_out, const float* y, float sigma2, const cider_code* code,
                     int32_t K, int32_t n, const cider_weights* wc, float gamma, int32_t reveal_count, int32_t first,
                     const cider_opts* opts, float* out_lbar, float* out_logits, float* out_z, void* stream) {
  if (!wc || !X_in) return fail(CIDER_EINVAL, "null weights or X_in");
  cider_weights* w = const_cast<cider_weights*>(wc);
  cider_opts o;
  if (opts) o = *opts; else cider_opts_default(&o);
  int rc = check_opts(o);
  if (rc) return rc;
  rc = check_prec(w, o);
  if (rc) return rc;
  uint8_t dummy = 0;
  BinIn b{y, sigma2, code, K, n, &dummy, nullptr, nullptr};
  rc = check_bin(w, b, 1);
  if (rc) return rc;
  if (reveal_count < 0 || reveal_count > K * n) return fail(CIDER_EINVAL, "reveal_count out of range");
  if (!(gamma >= 0.f && gamma <= 1.f)) return fail(CIDER_EINVAL, "gamma must be in [0, 1]");
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lock(w->mu);
  HIPCHK(hipSetDevice(w->device));
  Run r;
  Layout L;
  std::vector<BinIn> bins{b};
  rc = prepare(w, bins, 1, o, s, &r, &L, true);
  if (rc) return rc;
  char* base = (char*)r.ctx.bins - L.off_bins;
  uint8_t* Xw = (uint8_t*)(base + L.off_X);
  HIPCHK(hipMemcpyAsync(Xw, X_in, (size_t)K * n, hipMemcpyDeviceToDevice, s));
  if (o.autotune >= 2) r.forced_tile = o.autotune - 2;
  r.use_blocks = o.fused_blocks != 0;
  r.ctx.gamma_override = gamma;
  r.ctx.reveal_override = reveal_count;
  r.ctx.first_override = first ? 1 : 0;
  rc = enqueue_forward(w, r, s);
  if (rc) return rc;
  const size_t T = (size_t)K * n, fs = o.precision == kFP64 ? 8 : 4;
  if (out_lbar) HIPCHK(hipMemcpyAsync(out_lbar, r.work.lbar, T * 2 * fs, hipMemcpyDeviceToDevice, s));
  if (out_logits) HIPCHK(hipMemcpyAsync(out_logits, r.work.logits, T * 2 * fs, hipMemcpyDeviceToDevice, s));
  if (out_z) HIPCHK(hipMemcpyAsync(out_z, r.work.R, T * w->cfg.d * fs, hipMemcpyDeviceToDevice, s));
  if (X_out) {
    if (o.precision == kFP64) HIPCHK(launch_step_tail64(r.ctx, (const double*)r.work.logits, s));
    else HIPCHK(launch_step_tail(r.ctx, r.work, s));
    HIPCHK(hipMemcpyAsync(X_out, Xw, T, hipMemcpyDeviceToDevice, s));
  }
  return CIDER_OK;
}

int cider_amp_evidence(const float* y, const int32_t* rows, int64_t slots, int32_t n_s, int32_t Q, float rho,
                       float su2, int32_t iters, float* out_S, void* stream) {
  if (slots < 0 || slots >= ((int64_t)1 << 31) || n_s < 1 || n_s > 64 || Q < 2 || Q > 64 || iters < 0 ||
      iters > 10000 || !(rho > 0.f && rho < 1.f) || !(su2 > 0.f) || !std::isfinite(su2))
    return fail(CIDER_EINVAL, "bad AMP arguments");
  if (slots > 0 && (!y || !rows || !out_S)) return fail(CIDER_EINVAL, "null AMP buffer");
  AmpArgs g{};
  g.y = y; g.rows = rows; g.slots = (long)slots; g.ns = n_s; g.Q = Q;
  g.rho = rho; g.su2 = su2; g.iters = iters; g.S = out_S;
  const hipError_t err = launch_amp_evidence(g, (hipStream_t)stream);
  if (err != hipSuccess) return hip_fail(err, "cider_amp_evidence");
  return CIDER_OK;
}

int cider_gf64_check_update(const float* p_edge, const int32_t* row_ptr, const uint8_t* coef, int64_t checks,
                            int64_t edges, float* out_msg, void* stream) {
  if (checks < 0 || edges < 0 || checks >= ((int64_t)1 << 31) || edges >= ((int64_t)1 << 31))
    return fail(CIDER_EINVAL, "bad GF(64) check-update sizes");
  if (checks > 0 && (!p_edge || !row_ptr || !coef || !out_msg)) return fail(CIDER_EINVAL, "null GF(64) buffer");
  GfCheckArgs g{};
  g.p = p_edge; g.row_ptr = row_ptr; g.coef = coef; g.checks = (long)checks; g.edges = (long)edges; g.out = out_msg;
  const hipError_t err = launch_gf64_check(g, (hipStream_t)stream);
  if (err != hipSuccess) return hip_fail(err, "cider_gf64_check_update");
  return CIDER_OK;
}

int cider_evidence(const float* y, float sigma2, int32_t K, int32_t n, float* out_S, float* out_p, void* stream) {
  if (!y || K < 1 || K > CIDER_MAX_K || n < 1 || n > CIDER_MAX_N || !(sigma2 > 0.f))
    return fail(CIDER_EINVAL, "bad evidence arguments");
  hipStream_t s = (hipStream_t)stream;
  DevBin hb{};
  hb.K = K; hb.n = n; hb.y = y; hb.sigma2 = sigma2;
  std::vector<int> slot(n, 0);
  DevBin* db = nullptr;
  int* ds = nullptr;
  HIPCHK(hipMalloc(&db, sizeof(DevBin)));
  hipError_t e = hipMalloc(&ds, n * 4);
  if (e == hipSuccess) e = hipMemcpy(db, &hb, sizeof(DevBin), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(ds, slot.data(), n * 4, hipMemcpyHostToDevice);
  StepCtx c{};
  c.num_bins = 1; c.bins = db; c.slot_bin = ds; c.total_slots = n;
  if (e == hipSuccess) e = launch_evidence(c, out_S, out_p, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  hipFree(db);
  hipFree(ds);
  if (e != hipSuccess) return hip_fail(e, "cider_evidence");
  return CIDER_OK;
}

int cider_tuning_read(const cider_weights* wc, cider_tuning_entry* out, int32_t max, int32_t* n_out) {
  if (!wc || !n_out || max < 0 || (max > 0 && !out)) return fail(CIDER_EINVAL, "bad tuning arguments");
  cider_weights* w = const_cast<cider_weights*>(wc);
  std::lock_guard<std::mutex> lock(w->mu);
  int i = 0;
  for (auto& kv : w->tune) {
    if (i >= max) break;
    std::memset(out[i].role, 0, sizeof(out[i].role));
    std::strncpy(out[i].role, kv.second.role.c_str(), sizeof(out[i].role) - 1);
    out[i].n = kv.first.N;
    out[i].kd = kv.first.Kd;
    out[i].bucket = kv.first.bucket;
    out[i].tile = kv.second.tile;
    out[i].best_ms = kv.second.best_ms;
    out[i].default_ms = kv.second.default_ms;
    ++i;
  }
  *n_out = i;
  return CIDER_OK;
}

int cider_profile_read(const cider_weights* wc, cider_kernel_stat* out, int32_t max, int32_t* n_out,
                       int32_t reset) {
  if (!wc || !n_out || max < 0 || (max > 0 && !out)) return fail(CIDER_EINVAL, "bad profile arguments");
  cider_weights* w = const_cast<cider_weights*>(wc);
  std::lock_guard<std::mutex> lock(w->mu);
  HIPCHK(hipSetDevice(w->device));
  for (ProfRec& p : w->prof_pending) {
    float ms = 0.f;
    HIPCHK(hipEventSynchronize(p.b));
    HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
    auto& st = w->prof_stats[p.name];
    st.first += 1;
    st.second += ms;
    hipEventDestroy(p.a);
    hipEventDestroy(p.b);
  }
  w->prof_pending.clear();
  int i = 0;
  for (auto& kv : w->prof_stats) {
    if (i >= max) break;
    std::memset(out[i].name, 0, sizeof(out[i].name));
    std::strncpy(out[i].name, kv.first.c_str(), sizeof(out[i].name) - 1);
    out[i].launches = kv.second.first;
    out[i].total_ms = kv.second.second;
    ++i;
  }
  *n_out = i;
  if (reset) w->prof_stats.clear();
  return CIDER_OK;
}

}  // extern "C"

// ===========================================================================
// Serving: continuous batching of arriving bins.
//
// A worker thread owns a HIP stream and a set of device-resident slots.  A
// slot holds one admitted bin's received samples, grid, decoding state and
// output; the transient per-token buffers are shared and re-laid out only when
// the resident set changes.  Each iteration advances every resident bin by one
// refinement step (each at its own phase: reveal step, final pass, remask
// pass), reads back the bin states, hands finished bins to the completion list
// and admits waiting requests while slots, tokens and the HBM budget allow.
namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Request {
  uint64_t id;
  std::vector<float> y;
  float sigma2;
  const cider_code* code;
  int K, n;
  uint8_t* out_host;
  double t_submit;
};

struct Slot {
  bool used = false;
  Request req;
  double t_admit = 0;
  float* y = nullptr;
  uint8_t* X = nullptr;
  uint8_t* out = nullptr;
  BinState* st = nullptr;
};

}  // namespace

struct cider_server {
  cider_server_cfg cfg{};
  cider_weights* w = nullptr;
  int device = 0;
  hipStream_t stream = nullptr;
  std::thread worker;
  std::mutex mu;
  std::condition_variable cv, cv_done;
  bool stop = false;
  int status = CIDER_OK;
  std::string err;
  std::deque<Request> queue;
  std::vector<Slot> slots;
  std::vector<cider_result> done;
  uint64_t next_id = 1;
  long inflight = 0;  // queued + resident
  void* ws = nullptr;
  size_t ws_bytes = 0;
  char* dev_pool = nullptr;
  BinState* h_states = nullptr;
  // resident set, for admission: the step workspace it needs must fit ws_bytes
  long res_tokens = 0, res_msg = 0;
  int res_bins = 0, res_slots = 0, res_rows = 0;
  long admitted = 0, deferred_hbm = 0;   // admissions, and admissions that waited for HBM
};

namespace {

void server_loop(cider_server* S) {
  hipSetDevice(S->device);
  cider_weights* w = S->w;
  const int T = S->cfg.steps;
  cider_opts o = S->cfg.opts;
  o.workspace = S->ws;
  o.workspace_bytes = S->ws_bytes;
  o.profile = 0;
  long tokens_in_use = 0;
  bool changed = true;
  Run run;
  Layout L;
  std::vector<int> order;  // slot index of each packed bin
  auto fail_all = [&](int rc) {
    std::lock_guard<std::mutex> lk(S->mu);
    S->status = rc;
    S->err = g_err;
    S->stop = true;
    S->cv_done.notify_all();
  };
  while (true) {
    // ---- admit
    {
      std::unique_lock<std::mutex> lk(S->mu);
      if (S->stop) break;
      bool any = false;
      for (const Slot& sl : S->slots) any |= sl.used;
      if (!any && S->queue.empty()) {
        S->cv.wait_for(lk, std::chrono::milliseconds(2));
        continue;
      }
      while (!S->queue.empty()) {
        const Request& rq = S->queue.front();
        long tok = (long)rq.K * rq.n;
        if (tokens_in_use + tok > S->cfg.max_tokens) break;
        int free_i = -1;
        for (int i = 0; i < (int)S->slots.size(); ++i)
          if (!S->slots[i].used) { free_i = i; break; }
        if (free_i < 0) break;
        // HBM budget: the workspace of the resident set with this bin added,
        // laid out exactly as the next step will lay it out
        const Layout need = plan_layout(w->cfg, S->res_bins + 1, S->res_tokens + tok, S->res_slots + rq.n,
                                        S->res_rows + rq.K, o.precision, S->res_msg + (long)rq.K * rq.code->nnz);
        if (need.total > S->ws_bytes) {
          if (S->res_bins == 0) { fail_all(CIDER_ENOMEM); break; }   // cannot fit even alone
          S->deferred_hbm += 1;
          break;
        }
        S->res_bins += 1;
        S->res_tokens += tok;
        S->res_slots += rq.n;
        S->res_rows += rq.K;
        S->res_msg += (long)rq.K * rq.code->nnz;
        S->admitted += 1;
        Slot& sl = S->slots[free_i];
        sl.used = true;
        sl.req = std::move(S->queue.front());
        S->queue.pop_front();
        sl.t_admit = now_s();
        tokens_in_use += tok;
        // device state of the new bin: samples, all-mask grid, initial pass
        const int K = sl.req.K, n = sl.req.n;
        hipMemcpyAsync(sl.y, sl.req.y.data(), n * sizeof(float), hipMemcpyHostToDevice, S->stream);
        hipMemsetAsync(sl.X, kMask, (size_t)K * n, S->stream);
        BinState st{};
        st.phase = kReveal; st.t = 1; st.pass_T = T; st.n_masked = K * n; st.masked = K * n;
        st.first = (o.first_reveal && T > 1) ? 1 : 0;
        S->h_states[free_i] = st;
        hipMemcpyAsync(sl.st, &S->h_states[free_i], sizeof(BinState), hipMemcpyHostToDevice, S->stream);
        hipStreamSynchronize(S->stream);   // the host copies above are staged from pageable memory
        changed = true;
      }
    }
    // ---- (re)build the packed layout when the resident set changed
    if (changed) {
      std::vector<BinIn> bins;
      order.clear();
      for (int i = 0; i < (int)S->slots.size(); ++i) {
        Slot& sl = S->slots[i];
        if (!sl.used) continue;
        BinIn b{sl.y, sl.req.sigma2, sl.req.code, sl.req.K, sl.req.n, sl.out, nullptr, nullptr};
        b.X = sl.X;
        b.st = sl.st;
        bins.push_back(b);
        order.push_back(i);
      }
      if (bins.empty()) continue;
      std::lock_guard<std::mutex> lk(w->mu);
      int rc = prepare(w, bins, T, o, S->stream, &run, &L, false);
      if (rc) { fail_all(rc); break; }
      run.use_blocks = o.fused_blocks != 0;
      changed = false;
    }
    // ---- one refinement step for every resident bin
    {
      std::lock_guard<std::mutex> lk(w->mu);
      int rc = enqueue_step(w, run, S->stream);
      if (rc) { fail_all(rc); break; }
    }
    // ---- read back states; retire finished bins
    for (size_t j = 0; j < order.size(); ++j)
      hipMemcpyAsync(&S->h_states[order[j]], S->slots[order[j]].st, sizeof(BinState), hipMemcpyDeviceToHost,
                     S->stream);
    hipError_t e = hipStreamSynchronize(S->stream);
    if (e != hipSuccess) { set_err(hipGetErrorString(e)); fail_all(CIDER_EDEVICE); break; }
    for (size_t j = 0; j < order.size(); ++j) {
      Slot& sl = S->slots[order[j]];
      const BinState& st = S->h_states[order[j]];
      if (st.phase != kDone) continue;
      hipMemcpy(sl.req.out_host, sl.out, (size_t)sl.req.K * sl.req.n, hipMemcpyDeviceToHost);
      cider_result res{};
      res.id = sl.req.id; res.K = sl.req.K; res.n = sl.req.n; res.status = CIDER_OK; res.rounds = st.round;
      res.t_submit = sl.req.t_submit; res.t_admit = sl.t_admit; res.t_done = now_s();
      std::lock_guard<std::mutex> lk(S->mu);
      S->done.push_back(res);
      tokens_in_use -= (long)sl.req.K * sl.req.n;
      S->res_bins -= 1;
      S->res_tokens -= (long)sl.req.K * sl.req.n;
      S->res_slots -= sl.req.n;
      S->res_rows -= sl.req.K;
      S->res_msg -= (long)sl.req.K * sl.req.code->nnz;
      sl.used = false;
      sl.req.y.clear();
      S->inflight -= 1;
      changed = true;
      S->cv_done.notify_all();
    }
  }
}

}  // namespace

extern "C" {

// Device bytes a server needs at the least: the per-slot bin state of
// max_slots bins plus the step workspace of one largest bin (K = 16, n = n_max).
static size_t server_floor(const cider_server_cfg* cfg, size_t per_slot) {
  const cider_model_cfg& m = cfg->weights->cfg;
  const int n = std::min(m.n_max, CIDER_MAX_N);
  const Layout one = plan_layout(m, 1, (long)CIDER_MAX_K * n, n, CIDER_MAX_K, cfg->opts.precision, 0);
  return per_slot * (size_t)cfg->max_slots + one.total;
}

static size_t server_per_slot() {
  return align_up(CIDER_MAX_N * 4, 256) + 2 * align_up(CIDER_MAX_K * CIDER_MAX_N, 256) + align_up(sizeof(BinState), 256);
}

int cider_server_budget_floor(const cider_server_cfg* cfg, size_t* bytes) {
  if (!cfg || !cfg->weights || !bytes || cfg->max_slots < 1) return fail(CIDER_EINVAL, "null cfg, weights or bytes");
  *bytes = server_floor(cfg, server_per_slot());
  return CIDER_OK;
}

int cider_server_create(const cider_server_cfg* cfg, cider_server** out) {
  if (!out) return fail(CIDER_EINVAL, "null out");
  *out = nullptr;
  if (!cfg || !cfg->weights) return fail(CIDER_EINVAL, "null cfg or weights");
  if (cfg->steps < 1 || cfg->max_slots < 1 || cfg->max_slots > 65536 || cfg->max_queue < 1 || cfg->max_tokens < 1)
    return fail(CIDER_EINVAL, "steps, max_slots, max_queue and max_tokens must be positive");
  int rc = check_opts(cfg->opts);
  if (rc) return rc;
  rc = check_prec(cfg->weights, cfg->opts);
  if (rc) return rc;
  cider_server* S = new cider_server();
  S->cfg = *cfg;
  S->w = const_cast<cider_weights*>(cfg->weights);
  S->device = S->w->device;
  hipSetDevice(S->device);
  // step workspace for max_tokens spread over up to max_slots bins of n <= n_max
  long slots_bound = std::min<long>((long)cfg->max_slots * CIDER_MAX_N, cfg->max_tokens);
  Layout Lw = plan_layout(S->w->cfg, cfg->max_slots, cfg->max_tokens, (int)slots_bound,
                          (int)std::min<long>((long)cfg->max_slots * CIDER_MAX_K, cfg->max_tokens), cfg->opts.precision);
  const size_t per_slot = server_per_slot();
  // with an HBM budget the workspace takes what the slot state leaves of it, and
  // admission keeps the resident set's workspace within it; without one the
  // workspace is sized for max_tokens
  size_t ws_bytes = Lw.total;
  if (cfg->hbm_budget) {
    const size_t pool = per_slot * cfg->max_slots, floor = server_floor(cfg, per_slot);
    if (cfg->hbm_budget < floor) {
      delete S;
      return fail(CIDER_EINVAL, "hbm_budget below the slot state plus one largest bin's workspace: " +
                                    std::to_string(floor) + " bytes");
    }
    ws_bytes = cfg->hbm_budget - pool;
  }
  if (hipStreamCreateWithFlags(&S->stream, hipStreamNonBlocking) != hipSuccess ||
      hipMalloc(&S->ws, ws_bytes) != hipSuccess ||
      hipMalloc((void**)&S->dev_pool, per_slot * cfg->max_slots) != hipSuccess ||
      hipHostMalloc((void**)&S->h_states, sizeof(BinState) * cfg->max_slots, hipHostMallocDefault) != hipSuccess) {
    if (S->stream) hipStreamDestroy(S->stream);
    if (S->ws) hipFree(S->ws);
    if (S->dev_pool) hipFree(S->dev_pool);
    delete S;
    return fail(CIDER_ENOMEM, "server allocation failed");
  }
  S->ws_bytes = ws_bytes;
  S->slots.resize(cfg->max_slots);
  for (int i = 0; i < cfg->max_slots; ++i) {
    char* p = S->dev_pool + per_slot * i;
    Slot& sl = S->slots[i];
    sl.y = (float*)p;
    p += align_up(CIDER_MAX_N * 4, 256);
    sl.X = (uint8_t*)p;
    p += align_up(CIDER_MAX_K * CIDER_MAX_N, 256);
    sl.out = (uint8_t*)p;
    p += align_up(CIDER_MAX_K * CIDER_MAX_N, 256);
    sl.st = (BinState*)p;
  }
  S->worker = std::thread(server_loop, S);
  *out = S;
  return CIDER_OK;
}

int cider_server_submit(cider_server* S, const float* y_host, float sigma2, const cider_code* code, int32_t K,
                        int32_t n, uint8_t* out_host, uint64_t* id) {
  if (!S || !y_host || !out_host || !id) return fail(CIDER_EINVAL, "null argument");
  uint8_t dummy = 0;
  BinIn b{y_host, sigma2, code, K, n, &dummy, nullptr, nullptr};
  int rc = check_bin(S->w, b, S->cfg.steps);
  if (rc) return rc;
  if ((long)K * n > S->cfg.max_tokens) return fail(CIDER_EINVAL, "bin larger than max_tokens");
  std::lock_guard<std::mutex> lk(S->mu);
  if (S->status != CIDER_OK) return fail(S->status, "server stopped: " + S->err);
  if ((int)S->queue.size() >= S->cfg.max_queue) return fail(CIDER_EAGAIN, "queue full");
  Request rq;
  rq.id = S->next_id++;
  rq.y.assign(y_host, y_host + n);
  rq.sigma2 = sigma2;
  rq.code = code;
  rq.K = K;
  rq.n = n;
  rq.out_host = out_host;
  rq.t_submit = now_s();
  *id = rq.id;
  S->queue.push_back(std::move(rq));
  S->inflight += 1;
  S->cv.notify_one();
  return CIDER_OK;
}

int cider_server_poll(cider_server* S, cider_result* out, int32_t max, int32_t* n_done) {
  if (!S || !n_done || max < 0 || (max > 0 && !out)) return fail(CIDER_EINVAL, "bad poll arguments");
  std::lock_guard<std::mutex> lk(S->mu);
  int k = std::min<int>(max, (int)S->done.size());
  for (int i = 0; i < k; ++i) out[i] = S->done[i];
  S->done.erase(S->done.begin(), S->done.begin() + k);
  *n_done = k;
  if (S->status != CIDER_OK) return fail(S->status, "server stopped: " + S->err);
  return CIDER_OK;
}

int cider_server_drain(cider_server* S) {
  if (!S) return fail(CIDER_EINVAL, "null server");
  std::unique_lock<std::mutex> lk(S->mu);
  S->cv_done.wait(lk, [&] { return S->inflight == 0 || S->status != CIDER_OK; });
  if (S->status != CIDER_OK) return fail(S->status, "server stopped: " + S->err);
  return CIDER_OK;
}

void cider_server_destroy(cider_server* S) {
  if (!S) return;
  {
    std::lock_guard<std::mutex> lk(S->mu);
    S->stop = true;
    S->cv.notify_all();
  }
  if (S->worker.joinable()) S->worker.join();
  hipSetDevice(S->device);
  hipStreamSynchronize(S->stream);
  hipStreamDestroy(S->stream);
  hipFree(S->ws);
  hipFree(S->dev_pool);
  hipHostFree(S->h_states);
  delete S;
}

}  // extern "C"
