// The FP64 precision mode: the plain path's kernels with every value in
// double, from the evidence to the reveal keys.  Where the float paths round
// the residual stream, the softmaxes and the margins to FP32, these keep the
// FP64 oracle's precision, so that the integer decisions of a decode (reveal
// cut, argmax, first-reveal row) come out as the oracle's whenever they are
// farther from a tie than double rounding (~1e-15 relative).  The GEMMs are
// LDS-tiled FMA (64 x 64 output tile, 4 x 4 per thread); the attention,
// LayerNorm, embedding and Module B kernels mirror their FP32 counterparts;
// the reveal selects on the 64-bit bits of the double margins and breaks
// ties between equal margins by the smaller flat index with a second select.
#include "cider_internal.h"

namespace cider {
namespace {

__device__ __forceinline__ double wsum64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double gelu64(double x) { return 0.5 * x * (1.0 + erf(x * 0.70710678118654752440)); }

// ---------------------------------------------------------------------------
// Evidence (as k_evidence), beliefs in double.
__global__ void k_evidence64(StepCtx c, double* p) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= c.total_slots) return;
  const DevBin& b = c.bins[c.slot_bin[s]];
  const int l = s - b.slot_off, K = b.K;
  const double y = (double)b.y[l];
  const double inv2s = 1.0 / (2.0 * (double)b.sigma2);
  double lw[kMaxK + 1];
  double lc = 0.0, mx = -1e300;
  for (int m = 0; m <= K; ++m) {
    if (m > 0) lc += log((double)(K - m + 1)) - log((double)m);
    const double dm = y - (double)(K - 2 * m);
    lw[m] = lc - dm * dm * inv2s;
    mx = fmax(mx, lw[m]);
  }
  double tot = 0.0, t0 = 0.0, t1 = 0.0;
  for (int m = 0; m <= K; ++m) {
    const double e = exp(lw[m] - mx);
    tot += e;
    if (m < K) t0 += e;
    if (m > 0) t1 += e;
  }
  const double s0 = log(t0) - log(tot), s1 = log(t1) - log(tot);
  const double mm = fmax(s0, s1);
  const double e0 = exp(s0 - mm), e1 = exp(s1 - mm);
  p[2 * s] = e0 / (e0 + e1);
  p[2 * s + 1] = e1 / (e0 + e1);
}

// ---------------------------------------------------------------------------
// Embedding + Module A (as k_embed_demix), one wave per slot.
__global__ __launch_bounds__(256) void k_embed_demix64(StepCtx c, DevModel64 m, int d, double* R, double* Ebuf,
                                                       double* ZE, const double* pbuf) {
  __shared__ double s_lb[4][kMaxK][2];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + wave;
  bool active = s < c.total_slots;
  const DevBin* bp = active ? &c.bins[c.slot_bin[s]] : nullptr;
  BinState st = {};
  if (active) {
    st = *bp->st;
    active = st.phase != kDone;
  }
  int K = 0, n = 1, l = 0;
  double gamma = 0.0;
  if (active) {
    K = bp->K; n = bp->n; l = s - bp->slot_off;
    gamma = c.gamma_override >= 0.f ? (double)c.gamma_override : (double)st.masked / (double)(K * n);
  }
  for (int k = 0; k < K; ++k) {
    const int x = min((int)bp->X[k * n + l], kMask);
    double a0 = 0.0, a1 = 0.0;
    for (int col = lane; col < d; col += 64) {
      const double z = (m.E[(size_t)x * d + col] + m.P[(size_t)l * d + col]) + gamma * m.u[col];
      a0 = fma(z, m.W[col], a0);
      a1 = fma(z, m.W[d + col], a1);
    }
    a0 = wsum64(a0);
    a1 = wsum64(a1);
    if (lane == 0) { s_lb[wave][k][0] = a0 / (double)c.tau; s_lb[wave][k][1] = a1 / (double)c.tau; }
  }
  __syncthreads();
  if (!active) return;
  const double p0 = pbuf[2 * s], p1 = pbuf[2 * s + 1];
  double mx0 = -INFINITY, mx1 = -INFINITY;
  for (int k = 0; k < K; ++k) { mx0 = fmax(mx0, s_lb[wave][k][0]); mx1 = fmax(mx1, s_lb[wave][k][1]); }
  double den0 = 0.0, den1 = 0.0;
  for (int k = 0; k < K; ++k) { den0 += exp(s_lb[wave][k][0] - mx0); den1 += exp(s_lb[wave][k][1] - mx1); }
  for (int k = 0; k < K; ++k) {
    const double c0 = exp(s_lb[wave][k][0] - mx0) / den0 * p0, c1 = exp(s_lb[wave][k][1] - mx1) / den1 * p1;
    const int x = min((int)bp->X[k * n + l], kMask);
    const size_t tok = (size_t)bp->tok_off + (size_t)k * n + l;
    for (int col = lane; col < d; col += 64) {
      const double z = (m.E[(size_t)x * d + col] + m.P[(size_t)l * d + col]) + gamma * m.u[col];
      const double e = c0 * m.v[col] + c1 * m.v[d + col];
      R[tok * d + col] = z;
      Ebuf[tok * d + col] = e;
      ZE[tok * 2 * d + col] = z;
      ZE[tok * 2 * d + d + col] = e;
    }
  }
}

// ---------------------------------------------------------------------------
// GEMM out = epi(A W^T + bias): 64 x 64 tile per 256-thread workgroup, each
// thread a 4 x 4 block (rows ty + 16 i, columns tx + 16 j), k in slices of 16
// staged in LDS; every element sums its k terms in ascending order.
constexpr int GB = 64, GK = 16;
constexpr bool kGemm64Mfma = true;   // the matrix-core GEMM below; false: the FMA tile

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm64(Gemm64 g, const double* __restrict__ W) {
  __shared__ double As[GK][GB + 1];
  __shared__ double Bs[GK][GB + 1];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const long m0 = (long)blockIdx.x * GB;
  const int n0 = blockIdx.y * GB;
  double acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
  for (int k0 = 0; k0 < g.Kd; k0 += GK) {
    for (int idx = tid; idx < GB * GK; idx += 256) {
      const int r = idx / GK, kk = idx - r * GK;
      const long gm = m0 + r;
      As[kk][r] = gm < g.M ? g.A[gm * g.Kd + k0 + kk] : 0.0;
      Bs[kk][r] = W[(long)(n0 + r) * g.Kd + k0 + kk];
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      double a[4], bb[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty + 16 * i];
#pragma unroll
      for (int j = 0; j < 4; ++j) bb[j] = Bs[kk][tx + 16 * j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], bb[j], acc[i][j]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const long row = m0 + ty + 16 * i;
    if (row >= g.M) continue;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int col = n0 + tx + 16 * j;
      const double v = acc[i][j] + (g.bias ? g.bias[col] : 0.0);
      const long o = row * g.N + col;
      if (EPI == kEpiStore) g.out[o] = v;
      else if (EPI == kEpiGelu) g.out[o] = gelu64(v);
      else if (EPI == kEpiResid) g.R[o] = g.R[o] + v;
      else {
        const double gt = 1.0 / (1.0 + exp(-v));
        g.R[o] = gt * g.R[o] + (1.0 - gt) * g.E[o];
      }
    }
  }
}

// The same GEMM on the matrix cores: four waves in a 2 x 2 arrangement, a
// wave a 32 x 32 sub-tile of 2 x 2 v_mfma_f64_16x16x4 blocks (lane l supplies
// A[l % 16][k0 + l / 16] and B[k0 + l / 16][l % 16] and holds rows
// l / 16 + 4 r, column l % 16 of a block's result: the double-precision
// instruction interleaves its result rows); k in slices of 16 in LDS.
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <int EPI>
__global__ __launch_bounds__(256) void k_gemm64_mfma(Gemm64 g, const double* __restrict__ W) {
  __shared__ double As[GB][GK + 1];
  __shared__ double Bs[GB][GK + 1];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int wr = wave >> 1, wc = wave & 1;
  const long m0 = (long)blockIdx.x * GB;
  const int n0 = blockIdx.y * GB;
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = 0; k0 < g.Kd; k0 += GK) {
    for (int idx = tid; idx < GB * GK; idx += 256) {
      const int r = idx / GK, kk = idx - r * GK;
      const long gm = m0 + r;
      As[r][kk] = gm < g.M ? g.A[gm * g.Kd + k0 + kk] : 0.0;
      Bs[r][kk] = W[(long)(n0 + r) * g.Kd + k0 + kk];
    }
    __syncthreads();
#pragma unroll
    for (int st = 0; st < GK / 4; ++st)
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const double a = As[wr * 32 + i * 16 + (lane & 15)][st * 4 + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const double bv = Bs[wc * 32 + j * 16 + (lane & 15)][st * 4 + (lane >> 4)];
          acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, bv, acc[i][j], 0, 0, 0);
        }
      }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wc * 32 + j * 16 + (lane & 15);
      const double bias = g.bias ? g.bias[col] : 0.0;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long row = m0 + wr * 32 + i * 16 + (lane >> 4) + 4 * r;
        if (row >= g.M) continue;
        const double v = acc[i][j][r] + bias;
        const long o = row * g.N + col;
        if (EPI == kEpiStore) g.out[o] = v;
        else if (EPI == kEpiGelu) g.out[o] = gelu64(v);
        else if (EPI == kEpiResid) g.R[o] = g.R[o] + v;
        else {
          const double gt = 1.0 / (1.0 + exp(-v));
          g.R[o] = gt * g.R[o] + (1.0 - gt) * g.E[o];
        }
      }
    }
}

// ---------------------------------------------------------------------------
// LayerNorm over d of each token (eps 1e-5), one wave per token.
__global__ __launch_bounds__(256) void k_layernorm64(long T, int d, const double* __restrict__ R,
                                                     const double* __restrict__ g, const double* __restrict__ b,
                                                     double* __restrict__ out) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long t = (long)blockIdx.x * 4 + wave;
  if (t >= T) return;
  double s = 0.0;
  for (int col = lane; col < d; col += 64) s += R[t * d + col];
  const double mean = wsum64(s) / (double)d;
  double q = 0.0;
  for (int col = lane; col < d; col += 64) {
    const double dv = R[t * d + col] - mean;
    q = fma(dv, dv, q);
  }
  const double rstd = 1.0 / sqrt(wsum64(q) / (double)d + 1e-5);
  for (int col = lane; col < d; col += 64) out[t * d + col] = (R[t * d + col] - mean) * rstd * g[col] + b[col];
}

// ---------------------------------------------------------------------------
// Row attention (as k_row_attn): one workgroup per (row, head, 256 queries),
// keys and values through LDS 32 at a time, online softmax in double.
constexpr int kQ64 = 256;

template <int DH>
__global__ __launch_bounds__(kQ64) void k_row_attn64(StepCtx c, const double* __restrict__ QKV,
                                                     double* __restrict__ O, int d, int heads) {
  constexpr int kKC64 = DH >= 64 ? 8 : (DH >= 32 ? 16 : 32);   // scores of a chunk stay in registers
  __shared__ double s_k[kKC64][DH + 1];
  __shared__ double s_v[kKC64][DH + 1];
  const int item = blockIdx.x;
  const int r = c.row_first + item / heads, h = item % heads;
  const DevBin& b = c.bins[c.row_bin[r]];
  if (b.st->phase == kDone) return;
  const int n = b.n, k = r - b.row_off;
  const int q0 = blockIdx.y * kQ64;
  if (q0 >= n) return;
  const long tok0 = (long)b.tok_off + (long)k * n;
  const int l = q0 + threadIdx.x;
  const bool valid = l < n;
  const double scale = 1.0 / sqrt((double)DH);
  double q[DH], o[DH];
#pragma unroll
  for (int i = 0; i < DH; ++i) {
    q[i] = valid ? QKV[(tok0 + l) * 3 * d + h * DH + i] : 0.0;
    o[i] = 0.0;
  }
  double mrun = -INFINITY, lsum = 0.0;
  for (int j0 = 0; j0 < n; j0 += kKC64) {
    const int nk = min(kKC64, n - j0);
    for (int idx = threadIdx.x; idx < kKC64 * DH; idx += kQ64) {
      const int jj = idx / DH, ii = idx - jj * DH;
      double kv = 0.0, vv = 0.0;
      if (jj < nk) {
        const double* base = QKV + (tok0 + j0 + jj) * 3 * d + h * DH + ii;
        kv = base[d];
        vv = base[2 * d];
      }
      s_k[jj][ii] = kv;
      s_v[jj][ii] = vv;
    }
    __syncthreads();
    double sc[kKC64];
    double cmax = -INFINITY;
#pragma unroll
    for (int jj = 0; jj < kKC64; ++jj) {
      double a = 0.0;
#pragma unroll
      for (int i = 0; i < DH; ++i) a = fma(q[i], s_k[jj][i], a);
      sc[jj] = jj < nk ? a * scale : -INFINITY;
      cmax = fmax(cmax, sc[jj]);
    }
    const double mnew = fmax(mrun, cmax);
    const double corr = exp(mrun - mnew);
    lsum *= corr;
#pragma unroll
    for (int i = 0; i < DH; ++i) o[i] *= corr;
#pragma unroll
    for (int jj = 0; jj < kKC64; ++jj) {
      const double pj = exp(sc[jj] - mnew);
      lsum += pj;
#pragma unroll
      for (int i = 0; i < DH; ++i) o[i] = fma(pj, s_v[jj][i], o[i]);
    }
    mrun = mnew;
    __syncthreads();
  }
  if (valid) {
#pragma unroll
    for (int i = 0; i < DH; ++i) O[(tok0 + l) * d + h * DH + i] = o[i] / lsum;
  }
}

// Row attention on the matrix cores: one wave per 16 queries of a (row,
// head), four waves per workgroup.  Per tile of 16 keys the wave forms
// S^T = K Q^T with v_mfma_f64_16x16x4 (lane l then holds the scores of
// keys l / 16 + 4 r for query l % 16), keeps an online softmax per query
// (maximum across the four lane groups of a column), and accumulates
// O^T = V^T P^T, whose B operand for k-step s is exactly the lane's
// probability r = s.  Keys and values pass through LDS 32 at a time.
constexpr bool kRowAttn64Mfma = true;

template <int DH>
__global__ __launch_bounds__(256) void k_row_attn64_mfma(StepCtx c, const double* __restrict__ QKV,
                                                         double* __restrict__ O, int d, int heads) {
  constexpr int KT = 32, NS = DH / 4, NT = DH / 16;
  __shared__ double sK[KT][DH + 1];
  __shared__ double sV[KT][DH + 1];
  const int item = blockIdx.x;
  const int r = c.row_first + item / heads, h = item % heads;
  const DevBin& b = c.bins[c.row_bin[r]];
  if (b.st->phase == kDone) return;
  const int n = b.n, k = r - b.row_off;
  const int qb = blockIdx.y * 64;
  if (qb >= n) return;
  const long tok0 = (long)b.tok_off + (long)k * n;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, qi = lane & 15, g = lane >> 4;
  const int q = qb + wave * 16 + qi;
  const bool qv = q < n;
  const double scale = 1.0 / sqrt((double)DH);
  double qf[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) qf[s] = qv ? QKV[(tok0 + q) * 3 * d + h * DH + 4 * s + g] : 0.0;
  f64x4 acc[NT];
#pragma unroll
  for (int t = 0; t < NT; ++t) acc[t] = f64x4{0.0, 0.0, 0.0, 0.0};
  double mrun = -INFINITY, lpart = 0.0;
  for (int j0 = 0; j0 < n; j0 += KT) {
    const int nk = min(KT, n - j0);
    for (int idx = tid; idx < KT * DH; idx += 256) {
      const int jj = idx / DH, ii = idx - jj * DH;
      double kv = 0.0, vv = 0.0;
      if (jj < nk) {
        const double* base = QKV + (tok0 + j0 + jj) * 3 * d + h * DH + ii;
        kv = base[d];
        vv = base[2 * d];
      }
      sK[jj][ii] = kv;
      sV[jj][ii] = vv;
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < KT / 16; ++t) {
      if (t * 16 >= nk) break;                          // uniform over the workgroup
      f64x4 st = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int s = 0; s < NS; ++s)
        st = __builtin_amdgcn_mfma_f64_16x16x4f64(sK[t * 16 + qi][4 * s + g], qf[s], st, 0, 0, 0);
      double p[4], tmax = -INFINITY;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        const int key = j0 + t * 16 + g + 4 * rr;
        p[rr] = key < n ? st[rr] * scale : -INFINITY;
        tmax = fmax(tmax, p[rr]);
      }
      tmax = fmax(tmax, __shfl_xor(tmax, 16));
      tmax = fmax(tmax, __shfl_xor(tmax, 32));
      const double mnew = fmax(mrun, tmax);
      const double corr = exp(mrun - mnew);             // 0 on the first tile
      lpart *= corr;
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) acc[u][rr] *= corr;
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) {
        p[rr] = exp(p[rr] - mnew);
        lpart += p[rr];
      }
      mrun = mnew;
#pragma unroll
      for (int u = 0; u < NT; ++u)
#pragma unroll
        for (int s = 0; s < 4; ++s)
          acc[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(sV[t * 16 + 4 * s + g][u * 16 + qi], p[s], acc[u], 0, 0, 0);
    }
    __syncthreads();
  }
  double lsum = lpart + __shfl_xor(lpart, 16);
  lsum += __shfl_xor(lsum, 32);
  if (qv) {
#pragma unroll
    for (int u = 0; u < NT; ++u)
#pragma unroll
      for (int rr = 0; rr < 4; ++rr) O[(tok0 + q) * d + h * DH + u * 16 + g + 4 * rr] = acc[u][rr] / lsum;
  }
}

// User attention (as k_user_attn): DH consecutive lanes per (slot, head,
// query row), lane i holding feature i, max_K query rows per (slot, head).
// Scores are summed across the group's lanes and broadcast from its first
// lane, so every lane applies the same softmax; loads and stores are whole
// head rows.  DH divides 64, so a group never straddles a wave.
template <int DH>
__global__ __launch_bounds__(256) void k_user_attn64(StepCtx c, const double* __restrict__ QKV,
                                                     double* __restrict__ O, int d, int heads, int max_K) {
  const long item = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const int i = (int)(item % DH);
  const long grp = item / DH;
  const long per_slot = (long)heads * max_K;
  const long s = grp / per_slot;
  bool live = s < c.total_slots;
  int h = 0, kq = 0, n = 1, K = 1;
  long tok_l = 0;                                    // token of user 0 at this slot
  if (live) {
    const int rem = (int)(grp - s * per_slot);
    h = rem / max_K;
    kq = rem - h * max_K;
    const DevBin& b = c.bins[c.slot_bin[s]];
    live = kq < b.K && b.st->phase != kDone;
    n = b.n;
    K = b.K;
    tok_l = (long)b.tok_off + (s - b.slot_off);
  }
  if (!live) K = 0;                                  // uniform per group: no score, no store
  const int lead = (int)(threadIdx.x & 63) & ~(DH - 1);
  const double scale = 1.0 / sqrt((double)DH);
  const double qv = live ? QKV[(tok_l + (long)kq * n) * 3 * d + h * DH + i] : 0.0;
  double sc[kMaxK];
  double mx = -INFINITY;
#pragma unroll
  for (int j = 0; j < kMaxK; ++j) {
    if (j < K) {
      double a = qv * QKV[(tok_l + (long)j * n) * 3 * d + d + h * DH + i];
#pragma unroll
      for (int off = DH / 2; off >= 1; off >>= 1) a += __shfl_xor(a, off);
      a = __shfl(a, lead);
      sc[j] = a * scale;
      mx = fmax(mx, sc[j]);
    }
  }
  double lsum = 0.0, o = 0.0;
#pragma unroll
  for (int j = 0; j < kMaxK; ++j) {
    if (j < K) {
      sc[j] = exp(sc[j] - mx);
      lsum += sc[j];
      o = fma(sc[j], QKV[(tok_l + (long)j * n) * 3 * d + 2 * d + h * DH + i], o);
    }
  }
  if (live) O[(tok_l + (long)kq * n) * d + h * DH + i] = o / lsum;
}

// ---------------------------------------------------------------------------
// Final LayerNorm and the symbol projection, one wave per token.
__global__ __launch_bounds__(256) void k_final_proj64(long T, int d, DevModel64 m, const double* __restrict__ R,
                                                      double* __restrict__ lbar) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long t = (long)blockIdx.x * 4 + wave;
  if (t >= T) return;
  double s = 0.0;
  for (int col = lane; col < d; col += 64) s += R[t * d + col];
  const double mean = wsum64(s) / (double)d;
  double q = 0.0;
  for (int col = lane; col < d; col += 64) {
    const double dv = R[t * d + col] - mean;
    q = fma(dv, dv, q);
  }
  const double rstd = 1.0 / sqrt(wsum64(q) / (double)d + 1e-5);
  double a0 = 0.0, a1 = 0.0;
  for (int col = lane; col < d; col += 64) {
    const double hv = (R[t * d + col] - mean) * rstd * m.lnf_g[col] + m.lnf_b[col];
    a0 = fma(hv, m.W[col], a0);
    a1 = fma(hv, m.W[d + col], a1);
  }
  a0 = wsum64(a0);
  a1 = wsum64(a1);
  if (lane == 0) { lbar[2 * t] = a0; lbar[2 * t + 1] = a1; }
}

// ---------------------------------------------------------------------------
// Module B (as k_module_b) in double, one workgroup per row; each slot forms
// the extrinsic messages of its checks (ascending) itself.
__device__ __forceinline__ double phi64(double x) { return log1p(2.0 / expm1(x)); }

constexpr int kMaxEdges64 = 4096;

__global__ __launch_bounds__(256) void k_module_b64(StepCtx c, const double* lbar, double* logits) {
  __shared__ double s_lam[kMaxN];
  __shared__ double s_ph[kMaxEdges64];
  __shared__ uint8_t s_neg[kMaxEdges64];
  const int r = blockIdx.x;
  const DevBin& b = c.bins[c.row_bin[r]];
  if (b.st->phase == kDone) return;
  const int k = r - b.row_off, n = b.n, m = b.m, nnz = b.row_ptr[m];
  const size_t tok0 = (size_t)b.tok_off + (size_t)k * n;
  const uint8_t* X = b.X + k * n;
  const double lmax = (double)c.lam_max, lmin = (double)c.lam_min;
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    const int x = X[l];
    double lam;
    if (x == 0) lam = lmax;
    else if (x == 1) lam = -lmax;
    else lam = fmin(fmax(lbar[2 * (tok0 + l)] - lbar[2 * (tok0 + l) + 1], -lmax), lmax);
    s_lam[l] = lam;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nnz; e += blockDim.x) {
    const double lam = s_lam[b.col_idx[e]];
    s_ph[e] = phi64(fmax(fabs(lam), lmin));
    s_neg[e] = lam >= 0.0 ? 0 : 1;
  }
  __syncthreads();
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    double bias = 0.0;
    for (int i = b.var_ptr[l]; i < b.var_ptr[l + 1]; ++i) {
      const int e = b.var_edge[i];
      int j = 0;
      while (b.row_ptr[j + 1] <= e) ++j;                 // the edge's check
      double acc = 0.0;
      int neg = 0;
      for (int f = b.row_ptr[j]; f < b.row_ptr[j + 1]; ++f) {
        if (f == e) continue;
        acc += s_ph[f];
        neg ^= s_neg[f];
      }
      const double mg = phi64(acc);
      bias += neg ? -mg : mg;
    }
    const double hb = 0.5 * (double)c.eta * bias;
    logits[2 * (tok0 + l)] = lbar[2 * (tok0 + l)] + hb;
    logits[2 * (tok0 + l) + 1] = lbar[2 * (tok0 + l) + 1] - hb;
  }
}

// ---------------------------------------------------------------------------
// Step tail (reveal / final pass / remask / outputs) with double margins, one
// workgroup of 1024 threads per bin.  Reveal: a most-significant-digit radix
// select over the 64-bit margin bits (top bit set on candidates) finds the
// take-th largest margin v and how many candidates equal to v to take; a
// second select over the complemented flat index of those equal to v keeps
// the smallest indexes.
constexpr int kTail64 = 1024;
constexpr int kKeys64 = (kMaxK * kMaxN) / kTail64;
constexpr unsigned long long kCand = 1ull << 63;

// take-th largest among keys (nonzero, filtered by keep(i)), bits [lo, 64):
// returns the key value and, in *need, how many keys equal to it to take
template <int NK, class Keep>
__device__ unsigned long long radix_select(const unsigned long long (&keys)[NK], Keep keep, int take, int lo,
                                           int* need_out, unsigned* s_hist, int* s_wsum, unsigned long long* s_prefix,
                                           int* s_need) {
  const int tid = threadIdx.x;
  unsigned long long prefix = 0ull, pmask = 0ull;
  int need = take;
  for (int shift = 56; shift >= lo; shift -= 8) {
    if (tid < 256) s_hist[tid] = 0u;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NK; ++i) {
      const unsigned long long kk = keys[i];
      if (kk != 0ull && keep(i) && (kk & pmask) == prefix) atomicAdd(&s_hist[(kk >> shift) & 0xFFu], 1u);
    }
    __syncthreads();
    int v = 0, incl = 0;
    if (tid < 256) {
      v = (int)s_hist[255 - tid];
      incl = v;
#pragma unroll
      for (int o = 1; o < 64; o <<= 1) {
        const int t = __shfl_up(incl, o, 64);
        if ((tid & 63) >= o) incl += t;
      }
      if ((tid & 63) == 63) s_wsum[tid >> 6] = incl;
    }
    __syncthreads();
    if (tid < 256) {
      for (int w = 0; w < (tid >> 6); ++w) incl += s_wsum[w];
      const int excl = incl - v;
      if (excl < need && incl >= need) {
        *s_prefix = prefix | ((unsigned long long)(255 - tid) << shift);
        *s_need = need - excl;
      }
    }
    __syncthreads();
    prefix = *s_prefix;
    need = *s_need;
    pmask |= 0xFFull << shift;
    __syncthreads();
  }
  *need_out = need;
  return prefix;
}

__global__ __launch_bounds__(kTail64) void k_step_tail64(StepCtx c, const double* logits) {
  __shared__ unsigned s_hist[256];
  __shared__ int s_wsum[4];
  __shared__ unsigned long long s_prefix;
  __shared__ int s_need;
  __shared__ int s_cnt, s_eq;
  __shared__ int s_syn[kMaxK];
  __shared__ double s_q[kMaxK];
  __shared__ int s_low;
  const DevBin& b = c.bins[blockIdx.x];
  BinState st = *b.st;
  if (st.phase == kDone) return;
  const int K = b.K, n = b.n, tot = K * n, tid = threadIdx.x;
  const double* lg = logits + 2 * (size_t)b.tok_off;
  auto margin_key = [&](int site) -> unsigned long long {
    return kCand | (unsigned long long)__double_as_longlong(fabs(lg[2 * site] - lg[2 * site + 1]));
  };

  if (st.phase == kReveal) {
    const int* hdr = b.sched;
    const int off = hdr[st.sched_j];
    int r;
    bool first;
    if (c.reveal_override >= 0) {
      int masked = 0;
      for (int site = tid; site < tot; site += kTail64) masked += b.X[site] == c.mask;
      if (tid == 0) s_cnt = 0;
      __syncthreads();
      if (masked) atomicAdd(&s_cnt, masked);
      __syncthreads();
      st.masked = s_cnt;
      __syncthreads();
      r = min(c.reveal_override, st.masked);
      first = c.first_override != 0;
    } else {
      r = hdr[2 * (K + 1) + off + st.t - 1] - st.revealed;
      if (c.schedule == 1) r = max(1, r);
      if (st.t == st.pass_T) r = st.n_masked - st.revealed;
      r = max(0, min(r, st.masked));
      first = st.first && st.t == 1;
    }
    unsigned long long keys[kKeys64], tie[kKeys64];
    int site_of[kKeys64];
#pragma unroll
    for (int i = 0; i < kKeys64; ++i) { keys[i] = 0ull; tie[i] = 0ull; site_of[i] = -1; }
    if (first) {
      if (tid < n) {
        unsigned long long best = 0ull;
        int bs = -1;
        for (int k = 0; k < K; ++k) {
          const int site = k * n + tid;
          if (b.X[site] == c.mask) {
            const unsigned long long kk = margin_key(site);
            if (kk > best) { best = kk; bs = site; }             // ties keep the smaller k
          }
        }
        keys[0] = best;
        site_of[0] = bs;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kKeys64; ++i) {
        const int site = tid + i * kTail64;
        if (site < tot && b.X[site] == c.mask) { keys[i] = margin_key(site); site_of[i] = site; }
      }
    }
#pragma unroll
    for (int i = 0; i < kKeys64; ++i)
      if (keys[i]) tie[i] = kCand | (unsigned long long)(0xFFFFFFFFu - (unsigned)site_of[i]);
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    int mine = 0;
#pragma unroll
    for (int i = 0; i < kKeys64; ++i) mine += keys[i] != 0ull;
    if (mine) atomicAdd(&s_cnt, mine);
    __syncthreads();
    const int ncand = s_cnt;
    const int take = (first && c.first_verbatim && c.reveal_override < 0) ? ncand : min(r, ncand);
    unsigned long long vthr = ~0ull, tthr = ~0ull;
    if (take > 0 && take == ncand) {
      vthr = 1ull;
      tthr = 0ull;
    } else if (take > 0) {
      int need = 0;
      vthr = radix_select<kKeys64>(keys, [](int) { return true; }, take, 0, &need, s_hist, s_wsum, &s_prefix, &s_need);
      // how many candidates equal the threshold: all of them taken, or the smallest flat indexes
      if (tid == 0) s_eq = 0;
      __syncthreads();
      int eq = 0;
#pragma unroll
      for (int i = 0; i < kKeys64; ++i) eq += keys[i] == vthr;
      if (eq) atomicAdd(&s_eq, eq);
      __syncthreads();
      if (need >= s_eq) {
        tthr = 0ull;
      } else {
        int need2 = 0;
        tthr = radix_select<kKeys64>(tie, [&](int i) { return keys[i] == vthr; }, need, 0, &need2, s_hist, s_wsum,
                                     &s_prefix, &s_need);
      }
    }
#pragma unroll
    for (int i = 0; i < kKeys64; ++i) {
      const unsigned long long kk = keys[i];
      if (kk != 0ull && (kk > vthr || (kk == vthr && tie[i] >= tthr))) {
        const int site = site_of[i];
        b.X[site] = (lg[2 * site] >= lg[2 * site + 1]) ? 0 : 1;
      }
    }
    __syncthreads();
    if (tid == 0) {
      st.revealed += take;
      st.masked -= take;
      st.t += 1;
      if (st.t > st.pass_T) st.phase = kFinal;
      *b.st = st;
    }
    return;
  }

  // ---- final pass: row status, remask decision, outputs -------------------
  const int wave = tid >> 6, lane = tid & 63;
  if (tid < kMaxK) s_syn[tid] = 0;
  __syncthreads();
  for (int idx = tid; idx < K * b.m; idx += kTail64) {
    const int k = idx / b.m, j = idx - k * b.m;
    int par = 0;
    for (int e = b.row_ptr[j]; e < b.row_ptr[j + 1]; ++e) par ^= b.X[k * n + b.col_idx[e]];
    if (par & 1) atomicOr(&s_syn[k], 1);
  }
  if (wave < K) {
    double acc = 0.0;
    for (int l = lane; l < n; l += 64) {
      const int site = wave * n + l;
      acc += 1.0 / (1.0 + exp(-fabs(lg[2 * site] - lg[2 * site + 1]) * (double)c.q_inv_tau));
    }
    acc = wsum64(acc);
    if (lane == 0) s_q[wave] = acc / (double)n;
  }
  __syncthreads();
  if (tid == 0) {
    int low = 0;
    for (int k = 0; k < K; ++k)
      if (s_syn[k] || s_q[k] < (double)c.remask_thr) low |= 1 << k;
    s_low = low;
  }
  __syncthreads();
  const int low = s_low;
  if (c.remask && st.round < c.max_rounds && low != 0) {
    for (int site = tid; site < tot; site += kTail64)
      if ((low >> (site / n)) & 1) b.X[site] = (uint8_t)c.mask;
    if (tid == 0) {
      const int j = __popc(low);
      st.phase = kReveal;
      st.t = 1;
      st.pass_T = b.sched[K + 1 + j];
      st.n_masked = j * n;
      st.revealed = 0;
      st.masked = j * n;
      st.first = 0;
      st.round += 1;
      st.sched_j = j;
      st.low_rows = low;
      *b.st = st;
    }
    return;
  }
  for (int site = tid; site < tot; site += kTail64) {
    const uint8_t x = c.final_argmax ? (uint8_t)((lg[2 * site] >= lg[2 * site + 1]) ? 0 : 1) : b.X[site];
    b.out_sym[site] = x;
    if (c.final_argmax) b.X[site] = x;
    if (b.out_logits) {
      b.out_logits[2 * site] = (float)lg[2 * site];
      b.out_logits[2 * site + 1] = (float)lg[2 * site + 1];
    }
  }
  __syncthreads();
  if (c.final_argmax) {
    if (tid < kMaxK) s_syn[tid] = 0;
    __syncthreads();
    for (int idx = tid; idx < K * b.m; idx += kTail64) {
      const int k = idx / b.m, j = idx - k * b.m;
      int par = 0;
      for (int e = b.row_ptr[j]; e < b.row_ptr[j + 1]; ++e) par ^= b.X[k * n + b.col_idx[e]];
      if (par & 1) atomicOr(&s_syn[k], 1);
    }
    __syncthreads();
  }
  if (tid < K && b.out_valid) b.out_valid[tid] = s_syn[tid] ? 0 : 1;
  if (tid == 0) {
    int valid = 0;
    for (int k = 0; k < K; ++k)
      if (!s_syn[k]) valid |= 1 << k;
    st.valid_rows = valid;
    st.phase = kDone;
    *b.st = st;
    if (b.out_rounds) *b.out_rounds = st.round;
  }
}

}  // namespace

hipError_t launch_evidence64(const StepCtx& c, double* p, hipStream_t s) {
  if (c.total_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_evidence64, dim3((c.total_slots + 255) / 256), dim3(256), 0, s, c, p);
  return hipGetLastError();
}

hipError_t launch_embed_demix64(const StepCtx& c, const DevModel64& m, int d, double* R, double* E, double* ZE,
                                const double* p, hipStream_t s) {
  if (c.total_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_embed_demix64, dim3((c.total_slots + 3) / 4), dim3(256), 0, s, c, m, d, R, E, ZE, p);
  return hipGetLastError();
}

hipError_t launch_gemm64(int epi, const Gemm64& g, const double* W, hipStream_t s) {
  if (g.M == 0) return hipSuccess;
  if (g.N % GB != 0 || g.Kd % GK != 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)((g.M + GB - 1) / GB), (unsigned)(g.N / GB)), block(256);
  if (kGemm64Mfma) {
    if (epi == kEpiStore) hipLaunchKernelGGL(k_gemm64_mfma<kEpiStore>, grid, block, 0, s, g, W);
    else if (epi == kEpiGelu) hipLaunchKernelGGL(k_gemm64_mfma<kEpiGelu>, grid, block, 0, s, g, W);
    else if (epi == kEpiResid) hipLaunchKernelGGL(k_gemm64_mfma<kEpiResid>, grid, block, 0, s, g, W);
    else hipLaunchKernelGGL(k_gemm64_mfma<kEpiGate>, grid, block, 0, s, g, W);
  } else {
    if (epi == kEpiStore) hipLaunchKernelGGL(k_gemm64<kEpiStore>, grid, block, 0, s, g, W);
    else if (epi == kEpiGelu) hipLaunchKernelGGL(k_gemm64<kEpiGelu>, grid, block, 0, s, g, W);
    else if (epi == kEpiResid) hipLaunchKernelGGL(k_gemm64<kEpiResid>, grid, block, 0, s, g, W);
    else hipLaunchKernelGGL(k_gemm64<kEpiGate>, grid, block, 0, s, g, W);
  }
  return hipGetLastError();
}

hipError_t launch_layernorm64(long T, int d, const double* R, const double* g, const double* b, double* out,
                              hipStream_t s) {
  if (T == 0) return hipSuccess;
  hipLaunchKernelGGL(k_layernorm64, dim3((unsigned)((T + 3) / 4)), dim3(256), 0, s, T, d, R, g, b, out);
  return hipGetLastError();
}

hipError_t launch_row_attn64(const StepCtx& c, const double* QKV, double* O, int d, int heads, int max_n,
                             hipStream_t s) {
  if (c.total_rows == 0) return hipSuccess;
  const int dh = d / heads;
  if (kRowAttn64Mfma) {
    dim3 grid((unsigned)(c.total_rows * heads), (unsigned)((max_n + 63) / 64)), block(256);
    if (dh == 16) hipLaunchKernelGGL(k_row_attn64_mfma<16>, grid, block, 0, s, c, QKV, O, d, heads);
    else if (dh == 32) hipLaunchKernelGGL(k_row_attn64_mfma<32>, grid, block, 0, s, c, QKV, O, d, heads);
    else if (dh == 64) hipLaunchKernelGGL(k_row_attn64_mfma<64>, grid, block, 0, s, c, QKV, O, d, heads);
    else return hipErrorInvalidValue;
    return hipGetLastError();
  }
  dim3 grid((unsigned)(c.total_rows * heads), (unsigned)((max_n + kQ64 - 1) / kQ64)), block(kQ64);
  if (dh == 16) hipLaunchKernelGGL(k_row_attn64<16>, grid, block, 0, s, c, QKV, O, d, heads);
  else if (dh == 32) hipLaunchKernelGGL(k_row_attn64<32>, grid, block, 0, s, c, QKV, O, d, heads);
  else if (dh == 64) hipLaunchKernelGGL(k_row_attn64<64>, grid, block, 0, s, c, QKV, O, d, heads);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_user_attn64(const StepCtx& c, const double* QKV, double* O, int d, int heads, int max_K,
                              hipStream_t s) {
  if (c.total_slots == 0) return hipSuccess;
  if (max_K < 1 || max_K > kMaxK) return hipErrorInvalidValue;
  const int dh = d / heads;
  const long items = (long)c.total_slots * heads * max_K * dh;
  dim3 grid((unsigned)((items + 255) / 256)), block(256);
  if (dh == 16) hipLaunchKernelGGL(k_user_attn64<16>, grid, block, 0, s, c, QKV, O, d, heads, max_K);
  else if (dh == 32) hipLaunchKernelGGL(k_user_attn64<32>, grid, block, 0, s, c, QKV, O, d, heads, max_K);
  else if (dh == 64) hipLaunchKernelGGL(k_user_attn64<64>, grid, block, 0, s, c, QKV, O, d, heads, max_K);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_final_proj64(long T, int d, const DevModel64& m, const double* R, double* lbar, hipStream_t s) {
  if (T == 0) return hipSuccess;
  hipLaunchKernelGGL(k_final_proj64, dim3((unsigned)((T + 3) / 4)), dim3(256), 0, s, T, d, m, R, lbar);
  return hipGetLastError();
}

hipError_t launch_module_b64(const StepCtx& c, const double* lbar, double* logits, hipStream_t s) {
  if (c.total_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_module_b64, dim3((unsigned)c.total_rows), dim3(256), 0, s, c, lbar, logits);
  return hipGetLastError();
}

hipError_t launch_step_tail64(const StepCtx& c, const double* logits, hipStream_t s) {
  hipLaunchKernelGGL(k_step_tail64, dim3((unsigned)c.num_bins), dim3(kTail64), 0, s, c, logits);
  return hipGetLastError();
}

}  // namespace cider
