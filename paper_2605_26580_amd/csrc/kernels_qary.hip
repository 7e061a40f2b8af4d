// The GF(Q) pieces of the refinement step (Q = 2^m symbols, the paper's main
// setting of Q-ary LDPC codes): evidence beliefs, embedding and Module A over
// Q symbols, the final Q-way projection, Module B's exact check messages over
// GF(Q), and the reveal keys.  The denoiser blocks in between are the binary
// path's kernels unchanged.  FP32 throughout; small per-slot / per-token
// work, one wavefront per unit, lane a = symbol a.
#include "cider_internal.h"

namespace cider {
namespace {

__device__ __forceinline__ float wsum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ float wmax(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

// Product in GF(2^m), polynomial basis (x^2+x+1, x^3+x+1, x^4+x+1,
// x^5+x^2+1, x^6+x+1).
__device__ __forceinline__ int gfm(int a, int b, int m) {
  const int poly = m == 2 ? 0x7 : m == 3 ? 0xB : m == 4 ? 0x13 : m == 5 ? 0x25 : 0x43;
  int r = 0;
  for (int i = 0; i < m; ++i) {
    if (b & 1) r ^= a;
    b >>= 1;
    a <<= 1;
    if (a >> m) a ^= poly;
  }
  return r;
}

template <typename T> __device__ __forceinline__ void put(T* p, float v);
template <> __device__ __forceinline__ void put<float>(float* p, float v) { *p = v; }
template <> __device__ __forceinline__ void put<bf16>(bf16* p, float v) { *p = (bf16)v; }

// ---------------------------------------------------------------------------
// p[s][a] = softmax_a S[l][a] (the normalised per-slot belief), one wave per slot.
__global__ __launch_bounds__(256) void k_evidence_q(StepCtx c, float* p) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + wave;
  if (s >= c.total_slots) return;
  const DevBin& b = c.bins[c.slot_bin[s]];
  const int Q = c.q, l = s - b.slot_off;
  const float v = lane < Q ? b.S[(size_t)l * Q + lane] : -INFINITY;
  const float mx = wmax(v);
  const float e = lane < Q ? expf(v - mx) : 0.f;
  const float tot = wsum(e);
  if (lane < Q) p[(size_t)s * Q + lane] = e / tot;
}

// ---------------------------------------------------------------------------
// Embedding + Module A over Q symbols, one workgroup per slot (all K rows):
//   Z[k]    = E[X[k,l]] + P[l] + gamma u
//   lb[k,a] = <Z[k], w_a>;  r[., a] = softmax over k of lb[., a] / tau
//   e[k]    = sum_a r[k,a] p[l,a] v_a
// Writes R = Z, Ebuf = e (FP32) and ZE = [Z ; e] in the compute type.
constexpr int kEmbMaxD = 512;
constexpr int kQaryMaxQ = 64;

template <typename TC>
__global__ __launch_bounds__(256) void k_embed_demix_q(StepCtx c, EmbedW m, float* R, float* Ebuf, TC* ZE,
                                                       const float* pbuf) {
  __shared__ float sZ[kMaxK][kEmbMaxD];
  __shared__ float sR[kMaxK][kQaryMaxQ];
  __shared__ float sP[kQaryMaxQ];
  const int s = blockIdx.x, tid = threadIdx.x;
  const DevBin& b = c.bins[c.slot_bin[s]];
  const BinState st = *b.st;
  if (st.phase == kDone) return;                 // whole workgroup
  const int K = b.K, n = b.n, l = s - b.slot_off, d = m.d, Q = c.q;
  const float gamma = c.gamma_override >= 0.f ? c.gamma_override : (float)st.masked / (float)(K * n);
  for (int i = tid; i < K * d; i += blockDim.x) {
    const int k = i / d, col = i - k * d;
    const int x = min((int)b.X[k * n + l], Q);
    sZ[k][col] = (m.E[(size_t)x * d + col] + m.P[(size_t)l * d + col]) + gamma * m.u[col];
  }
  if (tid < Q) sP[tid] = pbuf[(size_t)s * Q + tid];
  __syncthreads();
  for (int i = tid; i < K * Q; i += blockDim.x) {
    const int k = i / Q, a = i - k * Q;
    const float* wa = m.W + (size_t)a * d;
    float acc = 0.f;
    for (int col = 0; col < d; ++col) acc = fmaf(sZ[k][col], wa[col], acc);
    sR[k][a] = acc / c.tau;
  }
  __syncthreads();
  if (tid < Q) {
    float mx = -INFINITY;
    for (int k = 0; k < K; ++k) mx = fmaxf(mx, sR[k][tid]);
    float den = 0.f;
    for (int k = 0; k < K; ++k) den += expf(sR[k][tid] - mx);
    for (int k = 0; k < K; ++k) sR[k][tid] = expf(sR[k][tid] - mx) / den * sP[tid];   // r[k,a] p[a]
  }
  __syncthreads();
  for (int i = tid; i < K * d; i += blockDim.x) {
    const int k = i / d, col = i - k * d;
    float e = 0.f;
    for (int a = 0; a < Q; ++a) e = fmaf(sR[k][a], m.v[(size_t)a * d + col], e);
    const size_t tok = (size_t)b.tok_off + (size_t)k * n + l;
    const float z = sZ[k][col];
    R[tok * d + col] = z;
    Ebuf[tok * d + col] = e;
    put<TC>(ZE + tok * 2 * d + col, z);
    put<TC>(ZE + tok * 2 * d + d + col, e);
  }
}

// ---------------------------------------------------------------------------
// lbar[t][a] = <LN_f(R[t]), w_a>, one single-wave workgroup per token: the
// normalised row in LDS, lane a takes the dot product with w_a in column order.
__global__ __launch_bounds__(64) void k_final_proj_q(long T, EmbedW m, const float* R, float* lbar) {
  __shared__ float sH[kEmbMaxD];
  const int lane = threadIdx.x;
  const long t = blockIdx.x;
  const int d = m.d, Q = m.q;
  float sum = 0.f;
  for (int col = lane; col < d; col += 64) sum += R[t * d + col];
  const float mean = wsum(sum) / (float)d;
  float var = 0.f;
  for (int col = lane; col < d; col += 64) {
    const float dv = R[t * d + col] - mean;
    var = fmaf(dv, dv, var);
  }
  const float rstd = 1.0f / sqrtf(wsum(var) / (float)d + 1e-5f);
  for (int col = lane; col < d; col += 64) sH[col] = (R[t * d + col] - mean) * rstd * m.lnf_g[col] + m.lnf_b[col];
  __syncthreads();
  if (lane < Q) {
    const float* wa = m.W + (size_t)lane * d;
    float acc = 0.f;
    for (int col = 0; col < d; ++col) acc = fmaf(sH[col], wa[col], acc);
    lbar[t * Q + lane] = acc;
  }
}

// ---------------------------------------------------------------------------
// Module B over GF(Q), messages: one wave per (row, check).  Each edge i of
// the check brings its site's distribution q_i -- softmax of the projected
// logits clipped lam_max below their maximum on a masked site, exp(lam_max
// [a = x]) normalised on a site revealed as x -- permuted by its coefficient
// (y_i(alpha_i a) = q_i(a)).  The message to edge o is the distribution of the
// other edges' sum, F_o (x) B_o with F_o the XOR convolution of the edges
// before o and B_o of those after it, read at alpha_o a; its logarithm,
// centred over a, is stored per row and edge.
__device__ __forceinline__ float xor_conv_lane(const float* A, const float* B, int c, int Q) {
  float acc = 0.f;
  for (int x = 0; x < Q; ++x) acc = fmaf(A[x], B[x ^ c], acc);
  return acc;
}

// one single-wave workgroup per (row, check): grid (rows, checks)
__global__ __launch_bounds__(64) void k_module_b_q_msgs(StepCtx c, const float* lbar) {
  __shared__ float sY[kQaryMaxDeg][kQaryMaxQ];
  __shared__ float sF[kQaryMaxDeg + 1][kQaryMaxQ];
  __shared__ float sB[kQaryMaxDeg + 1][kQaryMaxQ];
  const int lane = threadIdx.x;
  const int r = blockIdx.x, j = blockIdx.y;
  const DevBin& b = c.bins[c.row_bin[r]];
  if (b.st->phase == kDone || j >= b.m) return;   // whole workgroup
  const int Q = c.q, qm = b.q_bits, k = r - b.row_off, n = b.n;
  const int e0 = b.row_ptr[j], dc = b.row_ptr[j + 1] - e0;
  if (dc < 1 || dc > kQaryMaxDeg) return;
  const float lmax = c.lam_max;
  const bool act = lane < Q;
  for (int i = 0; i < dc; ++i) {
    const int l = b.col_idx[e0 + i];
    const size_t tok = (size_t)b.tok_off + (size_t)k * n + l;
    const int x = b.X[k * n + l];
    float q;
    if (x < Q) {
      const float big = expf(lmax);
      q = (lane == x ? big : 1.0f) / (big + (float)(Q - 1));
    } else {
      const float v = act ? lbar[tok * Q + lane] : -INFINITY;
      const float mx = wmax(v);
      const float e = act ? expf(fmaxf(v - mx, -lmax)) : 0.f;
      q = e / wsum(e);
    }
    if (act) sY[i][gfm(b.coef[e0 + i], lane, qm)] = q;
  }
  if (act) {
    sF[0][lane] = lane == 0 ? 1.f : 0.f;
    sB[dc - 1][lane] = lane == 0 ? 1.f : 0.f;
  }
  __syncthreads();
  for (int i = 0; i + 1 < dc; ++i) {
    const float f = act ? xor_conv_lane(sF[i], sY[i], lane, Q) : 0.f;
    const float bb = act ? xor_conv_lane(sB[dc - 1 - i], sY[dc - 1 - i], lane, Q) : 0.f;
    if (act) {
      sF[i + 1][lane] = f;
      sB[dc - 2 - i][lane] = bb;
    }
    __syncthreads();
  }
  const size_t base = (size_t)b.msg_off + (size_t)k * b.row_ptr[b.m] + e0;
  for (int o = 0; o < dc; ++o) {
    // distribution of the other edges' sum, read at alpha_o a
    float v = 0.f;
    if (act) v = xor_conv_lane(sF[o], sB[o], gfm(b.coef[e0 + o], lane, qm), Q);
    const float tot = wsum(v);
    const float lg = act ? logf(fmaxf(v / tot, 1e-37f)) : 0.f;
    const float mean = wsum(lg) / (float)Q;
    if (act) c.msg[(base + o) * Q + lane] = lg - mean;
  }
}

// logits = lbar + eta * sum over the slot's checks (ascending) of the message,
// one wave per token of a row.
__global__ __launch_bounds__(256) void k_module_b_q_sum(StepCtx c, const float* lbar, float* logits) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x;
  const DevBin& b = c.bins[c.row_bin[r]];
  if (b.st->phase == kDone) return;
  const int Q = c.q, k = r - b.row_off, n = b.n, nnz = b.row_ptr[b.m];
  if (lane >= Q) return;
  for (int l = wave; l < n; l += 4) {
    const size_t tok = (size_t)b.tok_off + (size_t)k * n + l;
    float acc = 0.f;
    for (int i = b.var_ptr[l]; i < b.var_ptr[l + 1]; ++i)
      acc += c.msg[((size_t)b.msg_off + (size_t)k * nnz + b.var_edge[i]) * Q + lane];
    logits[tok * Q + lane] = lbar[tok * Q + lane] + c.eta * acc;
  }
}

// ---------------------------------------------------------------------------
// Reveal keys, one wave per token of a row in its reveal phase: the argmax
// symbol a* (first maximum) and the uncertainty u = log(1 + sum_{a != a*}
// exp((L_a - L_a*) / tau_t)) = -log max_a softmax(L / tau_t)_a at the pass's
// annealed temperature tau_t = tau_max w + tau_min (1 - w),
// w = (1 + cos(pi (t - 1) / (T - 1))) / 2; rank = bits(+inf) - bits(u), so a
// larger rank is a more confident site.
__global__ __launch_bounds__(256) void k_site_key_q(StepCtx c, const float* logits) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int r = blockIdx.x;
  const DevBin& b = c.bins[c.row_bin[r]];
  const BinState st = *b.st;
  if (st.phase != kReveal) return;
  const int Q = c.q, k = r - b.row_off, n = b.n;
  const float w = st.pass_T <= 1 ? 1.0f
                                 : 0.5f * (1.0f + cosf(3.14159265358979f * (float)(st.t - 1) / (float)(st.pass_T - 1)));
  const float inv_tau = 1.0f / (c.tau_max * w + c.tau_min * (1.0f - w));
  for (int l = wave; l < n; l += 4) {
    const size_t tok = (size_t)b.tok_off + (size_t)k * n + l;
    const float v = lane < Q ? logits[tok * Q + lane] : -INFINITY;
    const float mx = wmax(v);
    // first maximum: the smallest lane holding it
    const unsigned long long ball = __ballot(lane < Q && v == mx);
    const int am = ball ? __ffsll((long long)ball) - 1 : 0;
    const float e = (lane < Q && lane != am) ? expf((v - mx) * inv_tau) : 0.f;
    const float u = log1pf(wsum(e));
    if (lane == 0) {
      c.rank[tok] = 0x7F800000u - __float_as_uint(u);
      c.sym[tok] = (uint8_t)am;
    }
  }
}

}  // namespace

hipError_t launch_evidence_q(const StepCtx& c, float* p, hipStream_t s) {
  if (c.total_slots == 0) return hipSuccess;
  hipLaunchKernelGGL(k_evidence_q, dim3((c.total_slots + 3) / 4), dim3(256), 0, s, c, p);
  return hipGetLastError();
}

hipError_t launch_embed_demix_q(const StepCtx& c, const EmbedW& m, const Work& w, int prec, hipStream_t s) {
  if (c.total_slots == 0) return hipSuccess;
  if (m.d > kEmbMaxD || c.q > kQaryMaxQ) return hipErrorInvalidValue;
  if (prec == kF32)
    hipLaunchKernelGGL(k_embed_demix_q<float>, dim3(c.total_slots), dim3(256), 0, s, c, m, w.R, w.Ebuf,
                       (float*)w.ZE, (const float*)w.p);
  else
    hipLaunchKernelGGL(k_embed_demix_q<bf16>, dim3(c.total_slots), dim3(256), 0, s, c, m, w.R, w.Ebuf,
                       (bf16*)w.ZE, (const float*)w.p);
  return hipGetLastError();
}

hipError_t launch_final_proj_q(const StepCtx& c, const EmbedW& m, const Work& w, hipStream_t s) {
  const long T = c.total_tokens;
  if (T == 0) return hipSuccess;
  if (m.d > kEmbMaxD || m.q > kQaryMaxQ) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_final_proj_q, dim3((unsigned)T), dim3(64), 0, s, T, m, w.R, w.lbar);
  return hipGetLastError();
}

hipError_t launch_module_b_q(const StepCtx& c, const Work& w, int max_checks, hipStream_t s) {
  if (c.total_rows == 0) return hipSuccess;
  if (c.q > kQaryMaxQ || !c.msg) return hipErrorInvalidValue;
  if (max_checks > 0) {
    dim3 grid((unsigned)c.total_rows, (unsigned)max_checks);
    hipLaunchKernelGGL(k_module_b_q_msgs, grid, dim3(64), 0, s, c, w.lbar);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_module_b_q_sum, dim3((unsigned)c.total_rows), dim3(256), 0, s, c, w.lbar, w.logits);
  return hipGetLastError();
}

hipError_t launch_site_key_q(const StepCtx& c, const Work& w, hipStream_t s) {
  if (c.total_rows == 0) return hipSuccess;
  if (c.q > kQaryMaxQ || !c.rank || !c.sym) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_site_key_q, dim3((unsigned)c.total_rows), dim3(256), 0, s, c, w.logits);
  return hipGetLastError();
}

}  // namespace cider
