// Per-slot, per-row and per-bin kernels of the refinement step: evidence,
// embedding + Module A, final projection, Module B and the step tail
// (confidence-ranked reveal, final-pass row status and remasking).
#include "cider_internal.h"

namespace cider {

namespace {

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ float wave_max(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  return v;
}

template <typename T>
__device__ __forceinline__ void store_c(T* p, float v);
template <>
__device__ __forceinline__ void store_c<float>(float* p, float v) { *p = v; }
template <>
__device__ __forceinline__ void store_c<bf16>(bf16* p, float v) { *p = (bf16)v; }

// phi(x) = log((e^x + 1) / (e^x - 1)), the self-inverse map of the binary
// check rule in log-magnitude form.
__device__ __forceinline__ float phi_f(float x) { return log1pf(2.0f / expm1f(x)); }

}  // namespace

// ---------------------------------------------------------------------------
// Evidence: exact posterior over m = number of users sending bit 1 at a slot,
// P(m | y) ~ C(K, m) exp(-(y - (K - 2m))^2 / (2 sigma2)); bit 0 is present iff
// m < K and bit 1 iff m > 0.  Computed in FP64 with log-sum-exp.
__global__ void k_evidence(StepCtx c, float* S, float* p) {
  int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= c.total_slots) return;
  const DevBin& b = c.bins[c.slot_bin[s]];
  int l = s - b.slot_off;
  int K = b.K;
  double y = (double)b.y[l];
  double inv2s = 1.0 / (2.0 * (double)b.sigma2);
  double lw[kMaxK + 1];
  double lc = 0.0;  // log C(K, m), built up incrementally
  double mx = -1e300;
  for (int m = 0; m <= K; ++m) {
    if (m > 0) lc += log((double)(K - m + 1)) - log((double)m);
    double dm = y - (double)(K - 2 * m);
    lw[m] = lc - dm * dm * inv2s;
    mx = fmax(mx, lw[m]);
  }
  double tot = 0.0, t0 = 0.0, t1 = 0.0;
  for (int m = 0; m <= K; ++m) {
    double e = exp(lw[m] - mx);
    tot += e;
    if (m < K) t0 += e;
    if (m > 0) t1 += e;
  }
  double s0 = log(t0) - log(tot), s1 = log(t1) - log(tot);
  double mm = fmax(s0, s1);
  double e0 = exp(s0 - mm), e1 = exp(s1 - mm);
  if (S) { S[2 * s] = (float)s0; S[2 * s + 1] = (float)s1; }
  if (p) { p[2 * s] = (float)(e0 / (e0 + e1)); p[2 * s + 1] = (float)(e1 / (e0 + e1)); }
}

hipError_t launch_evidence(const StepCtx& c, float* S, float* p, hipStream_t s) {
  if (c.total_slots == 0) return hipSuccess;
  int th = 256, bl = (c.total_slots + th - 1) / th;
  hipLaunchKernelGGL(k_evidence, dim3(bl), dim3(th), 0, s, c, S, p);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Fresh decoding state: all-mask grid, initial pass of T steps.
__global__ void k_init_bins(StepCtx c, int T, int first_reveal) {
  const DevBin& b = c.bins[blockIdx.x];
  int tot = b.K * b.n;
  for (int i = threadIdx.x; i < tot; i += blockDim.x) b.X[i] = (uint8_t)c.mask;
  if (threadIdx.x == 0) {
    BinState st = {};
    st.phase = kReveal;
    st.t = 1;
    st.pass_T = T;
    st.n_masked = tot;
    st.revealed = 0;
    st.masked = tot;
    st.first = (first_reveal && T > 1) ? 1 : 0;
    st.round = 0;
    st.sched_j = 0;
    *b.st = st;
  }
}

hipError_t launch_init_bins(const StepCtx& c, int T, int first_reveal, hipStream_t s) {
  hipLaunchKernelGGL(k_init_bins, dim3(c.num_bins), dim3(256), 0, s, c, T, first_reveal);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Embedding + Module A, one wavefront per slot (all K rows of the slot):
//   Z[k]  = E[X[k,l]] + P[l] + gamma u
//   lb[k,a] = <Z[k], w_a>,  r[., a] = softmax over k of lb[., a] / tau
//   e[k]  = sum_a r[k,a] p[l,a] v_a
// Writes R = Z (FP32), Ebuf = e (FP32) and ZE = [Z ; e] in the compute type;
// the gate MLP GEMMs then form Z~ = g Z + (1 - g) e in place in R.
template <typename TC, int NC>
__global__ __launch_bounds__(256) void k_embed_demix(StepCtx c, EmbedW m, float* R, float* Ebuf,
                                                     TC* ZE, const float* pbuf) {
  __shared__ float s_lb[4][kMaxK][2];
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int s = blockIdx.x * 4 + wave;
  bool active = s < c.total_slots;
  const DevBin* bp = active ? &c.bins[c.slot_bin[s]] : nullptr;
  BinState st = {};
  if (active) {
    st = *bp->st;
    active = st.phase != kDone;
  }
  const int d = m.d;
  int K = 0, n = 1, l = 0;
  float gamma = 0.f, p0 = 0.f, p1 = 0.f;
  float pe[NC], uu[NC], w0[NC], w1[NC];
  if (active) {
    K = bp->K; n = bp->n; l = s - bp->slot_off;
    gamma = c.gamma_override >= 0.f ? c.gamma_override : (float)st.masked / (float)(K * n);
    p0 = pbuf[2 * s]; p1 = pbuf[2 * s + 1];
  }
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    int col = lane + 64 * i;
    bool ok = active && col < d;
    pe[i] = ok ? m.P[(size_t)l * d + col] : 0.f;
    uu[i] = ok ? m.u[col] : 0.f;
    w0[i] = ok ? m.W[col] : 0.f;
    w1[i] = ok ? m.W[d + col] : 0.f;
  }
  for (int k = 0; k < K; ++k) {
    int x = min((int)bp->X[k * n + l], kMask);  // any value above 1 is a mask
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      int col = lane + 64 * i;
      float z = (col < d) ? (m.E[(size_t)x * d + col] + pe[i]) + gamma * uu[i] : 0.f;
      a0 = fmaf(z, w0[i], a0);
      a1 = fmaf(z, w1[i], a1);
    }
    a0 = wave_sum(a0);
    a1 = wave_sum(a1);
    if (lane == 0) { s_lb[wave][k][0] = a0; s_lb[wave][k][1] = a1; }
  }
  __syncthreads();
  if (!active) return;
  // softmax over the K rows, for each symbol a
  float mx0 = -INFINITY, mx1 = -INFINITY;
  for (int k = 0; k < K; ++k) {
    mx0 = fmaxf(mx0, s_lb[wave][k][0] / c.tau);
    mx1 = fmaxf(mx1, s_lb[wave][k][1] / c.tau);
  }
  float den0 = 0.f, den1 = 0.f;
  for (int k = 0; k < K; ++k) {
    den0 += expf(s_lb[wave][k][0] / c.tau - mx0);
    den1 += expf(s_lb[wave][k][1] / c.tau - mx1);
  }
  float v0[NC], v1[NC];
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    int col = lane + 64 * i;
    v0[i] = (col < d) ? m.v[col] : 0.f;
    v1[i] = (col < d) ? m.v[d + col] : 0.f;
  }
  for (int k = 0; k < K; ++k) {
    float r0 = expf(s_lb[wave][k][0] / c.tau - mx0) / den0;
    float r1 = expf(s_lb[wave][k][1] / c.tau - mx1) / den1;
    float c0 = r0 * p0, c1 = r1 * p1;
    int x = min((int)bp->X[k * n + l], kMask);  // any value above 1 is a mask
    size_t tok = (size_t)bp->tok_off + (size_t)k * n + l;
#pragma unroll
    for (int i = 0; i < NC; ++i) {
      int col = lane + 64 * i;
      if (col < d) {
        float z = (m.E[(size_t)x * d + col] + pe[i]) + gamma * uu[i];
        float e = c0 * v0[i] + c1 * v1[i];
        R[tok * d + col] = z;
        Ebuf[tok * d + col] = e;
        store_c<TC>(ZE + tok * 2 * d + col, z);
        store_c<TC>(ZE + tok * 2 * d + d + col, e);
      }
    }
  }
}

hipError_t launch_embed_demix(const StepCtx& c, const EmbedW& m, const Work& w, int prec,
                              hipStream_t s) {
  if (c.total_slots == 0) return hipSuccess;
  dim3 grid((c.total_slots + 3) / 4), block(256);
  int nc = (m.d + 63) / 64;
#define EMB_CASE(TC, NCV)                                                                      \
  hipLaunchKernelGGL((k_embed_demix<TC, NCV>), grid, block, 0, s, c, m, w.R, w.Ebuf, (TC*)w.ZE, \
                     (const float*)w.p)
  if (prec == kF32) {
    if (nc <= 2) EMB_CASE(float, 2); else if (nc <= 4) EMB_CASE(float, 4); else EMB_CASE(float, 8);
  } else {
    if (nc <= 2) EMB_CASE(bf16, 2); else if (nc <= 4) EMB_CASE(bf16, 4); else EMB_CASE(bf16, 8);
  }
#undef EMB_CASE
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Final LayerNorm and the symbol projection: lbar[t, a] = <LN_f(R[t]), w_a>,
// one wavefront per token, FP32.
template <int NC>
__global__ __launch_bounds__(256) void k_final_proj(long T, EmbedW m, const float* R, float* lbar) {
  int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  long t = (long)blockIdx.x * 4 + wave;
  if (t >= T) return;
  const int d = m.d;
  float x[NC];
  float sum = 0.f;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    int col = lane + 64 * i;
    x[i] = (col < d) ? R[t * d + col] : 0.f;
    sum += x[i];
  }
  float mean = wave_sum(sum) / (float)d;
  float var = 0.f;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    int col = lane + 64 * i;
    float dv = (col < d) ? x[i] - mean : 0.f;
    var = fmaf(dv, dv, var);
  }
  var = wave_sum(var) / (float)d;
  float rstd = 1.0f / sqrtf(var + 1e-5f);
  float a0 = 0.f, a1 = 0.f;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    int col = lane + 64 * i;
    if (col < d) {
      float h = (x[i] - mean) * rstd * m.lnf_g[col] + m.lnf_b[col];
      a0 = fmaf(h, m.W[col], a0);
      a1 = fmaf(h, m.W[d + col], a1);
    }
  }
  a0 = wave_sum(a0);
  a1 = wave_sum(a1);
  if (lane == 0) { lbar[2 * t] = a0; lbar[2 * t + 1] = a1; }
}

hipError_t launch_final_proj(const StepCtx& c, const EmbedW& m, const Work& w, hipStream_t s) {
  long T = c.total_tokens;
  if (T == 0) return hipSuccess;
  dim3 grid((unsigned)((T + 3) / 4)), block(256);
  int nc = (m.d + 63) / 64;
  if (nc <= 2) hipLaunchKernelGGL(k_final_proj<2>, grid, block, 0, s, T, m, w.R, w.lbar);
  else if (nc <= 4) hipLaunchKernelGGL(k_final_proj<4>, grid, block, 0, s, T, m, w.R, w.lbar);
  else hipLaunchKernelGGL(k_final_proj<8>, grid, block, 0, s, T, m, w.R, w.lbar);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Module B, binary logit-bias form, one workgroup per row of a bin.
// lambda[l] = clip(lbar0 - lbar1, +-lam_max) on masked sites, +-lam_max on
// revealed ones.  Check j sends slot l the extrinsic message
//   m = prod_{l' != l} sgn(lambda[l']) * phi(sum_{l' != l} phi(max(|lambda[l']|, lam_min)))
// summed over l' in ascending order with the target left out explicitly; the
// bias b[l] sums the messages of l's checks in ascending check order and the
// logits become lbar0 + eta b / 2, lbar1 - eta b / 2.
constexpr int kMaxEdges = 4096;

__global__ __launch_bounds__(256) void k_module_b(StepCtx c, const float* lbar, float* logits) {
  __shared__ float s_lam[kMaxN];
  __shared__ float s_ph[kMaxEdges];
  __shared__ uint8_t s_neg[kMaxEdges];
  __shared__ float s_msg[kMaxEdges];
  int r = blockIdx.x;
  const DevBin& b = c.bins[c.row_bin[r]];
  if (b.st->phase == kDone) return;
  const int k = r - b.row_off, n = b.n, m = b.m, nnz = b.row_ptr[m];
  const size_t tok0 = (size_t)b.tok_off + (size_t)k * n;
  const uint8_t* X = b.X + k * n;
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    int x = X[l];
    float lam;
    if (x == 0) lam = c.lam_max;
    else if (x == 1) lam = -c.lam_max;
    else lam = fminf(fmaxf(lbar[2 * (tok0 + l)] - lbar[2 * (tok0 + l) + 1], -c.lam_max), c.lam_max);
    s_lam[l] = lam;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < nnz; e += blockDim.x) {
    float lam = s_lam[b.col_idx[e]];
    s_ph[e] = phi_f(fmaxf(fabsf(lam), c.lam_min));
    s_neg[e] = lam >= 0.f ? 0 : 1;
  }
  __syncthreads();
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    const int e0 = b.row_ptr[j], e1 = b.row_ptr[j + 1];
    for (int e = e0; e < e1; ++e) {
      float acc = 0.f;
      int neg = 0;
      for (int f = e0; f < e1; ++f) {
        if (f == e) continue;
        acc += s_ph[f];
        neg ^= s_neg[f];
      }
      float mg = phi_f(acc);
      s_msg[e] = neg ? -mg : mg;
    }
  }
  __syncthreads();
  for (int l = threadIdx.x; l < n; l += blockDim.x) {
    float bias = 0.f;
    for (int i = b.var_ptr[l]; i < b.var_ptr[l + 1]; ++i) bias += s_msg[b.var_edge[i]];
    float h = 0.5f * c.eta * bias;
    logits[2 * (tok0 + l)] = lbar[2 * (tok0 + l)] + h;
    logits[2 * (tok0 + l) + 1] = lbar[2 * (tok0 + l) + 1] - h;
  }
}

hipError_t launch_module_b(const StepCtx& c, const Work& w, hipStream_t s) {
  if (c.total_rows == 0) return hipSuccess;
  hipLaunchKernelGGL(k_module_b, dim3(c.total_rows), dim3(256), 0, s, c, w.lbar, w.logits);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Step tail, one workgroup of 1024 threads per bin.
//
// Reveal phase: candidates are the masked sites (or, on the first step of a
// pass with first-reveal, each slot's best masked row, ties to the smaller k;
// the verbatim mode reveals all of those, the hybrid mode r of them).
// Each candidate gets the 64-bit key (bits of |L0 - L1|) << 32 | ~(k n + l),
// which orders by margin and then by smaller flat index; a most-significant-
// digit radix select finds the r-th largest key and every candidate at or
// above it takes its argmax symbol (ties to bit 0).
//
// Final phase: per row, syndrome H x and q = mean over slots of the max
// probability sigmoid(|L0 - L1| / tau_min) (the annealed inference
// temperature's end value); rows with nonzero syndrome or q < thr are
// remasked for T_rm steps while rounds remain, otherwise the bin is done and
// its outputs are written.
constexpr int kTailThreads = 1024;
constexpr int kKeysPerThread = (kMaxK * kMaxN) / kTailThreads;

// Product in GF(2^m), polynomial basis, primitive polynomial of degree m
// (x^2+x+1, x^3+x+1, x^4+x+1, x^5+x^2+1, x^6+x+1).
__device__ __forceinline__ int gf_mul_q(int a, int b, int m) {
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

__device__ __forceinline__ unsigned long long site_key(float margin, int flat) {
  return ((unsigned long long)__float_as_uint(margin) << 32) |
         (unsigned long long)(0xFFFFFFFFu - (unsigned)flat);
}

template <bool QARY>
__global__ __launch_bounds__(kTailThreads) void k_step_tail(StepCtx c, const float* logits) {
  __shared__ unsigned s_hist[256];
  __shared__ int s_wsum[4];
  __shared__ unsigned long long s_prefix;
  __shared__ int s_need;
  __shared__ int s_cnt;
  __shared__ int s_syn[kMaxK];
  __shared__ float s_q[kMaxK];
  __shared__ int s_low;
  const DevBin& b = c.bins[blockIdx.x];
  BinState st = *b.st;
  if (st.phase == kDone) return;
  const int K = b.K, n = b.n, tot = K * n, tid = threadIdx.x;
  const int Q = QARY ? c.q : 2;
  const float* lg = logits + (size_t)Q * b.tok_off;
  // reveal key: confidence (margin bits, or the GF(Q) rank) over the complemented flat index
  auto key_of = [&](int site) -> unsigned long long {
    if constexpr (QARY)
      return ((unsigned long long)c.rank[(size_t)b.tok_off + site] << 32) |
             (unsigned long long)(0xFFFFFFFFu - (unsigned)site);
    else
      return site_key(fabsf(lg[2 * site] - lg[2 * site + 1]), site);
  };

  if (st.phase == kReveal) {
    const int* hdr = b.sched;
    const int off = hdr[st.sched_j], len = hdr[K + 1 + st.sched_j];
    (void)len;
    int r;
    bool first;
    if (c.reveal_override >= 0) {
      int masked = 0;
      for (int site = tid; site < tot; site += kTailThreads) masked += b.X[site] == c.mask;
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

    unsigned long long keys[kKeysPerThread];
#pragma unroll
    for (int i = 0; i < kKeysPerThread; ++i) keys[i] = 0ull;
    if (first) {
      if (tid < n) {
        unsigned long long best = 0ull;
        for (int k = 0; k < K; ++k) {
          int site = k * n + tid;
          if (b.X[site] == c.mask) {
            unsigned long long kk = key_of(site);
            if (kk > best) best = kk;
          }
        }
        keys[0] = best;
      }
    } else {
#pragma unroll
      for (int i = 0; i < kKeysPerThread; ++i) {
        int site = tid + i * kTailThreads;
        if (site < tot && b.X[site] == c.mask)
          keys[i] = key_of(site);
      }
    }
    if (tid == 0) s_cnt = 0;
    __syncthreads();
    int mine = 0;
#pragma unroll
    for (int i = 0; i < kKeysPerThread; ++i) mine += keys[i] != 0ull;
    if (mine) atomicAdd(&s_cnt, mine);
    __syncthreads();
    const int ncand = s_cnt;
    // verbatim first-reveal: every slot's selected site; the schedule's
    // cumulative targets take over from the next step
    const int take = (first && c.first_verbatim && c.reveal_override < 0) ? ncand : min(r, ncand);
    unsigned long long thr = ~0ull;  // select nothing
    if (take > 0 && take == ncand) {
      thr = 1ull;  // every candidate
    } else if (take > 0) {
      unsigned long long prefix = 0ull, pmask = 0ull;
      int need = take;
      for (int shift = 56; shift >= 0; shift -= 8) {
        if (tid < 256) s_hist[tid] = 0u;
        __syncthreads();
#pragma unroll
        for (int i = 0; i < kKeysPerThread; ++i) {
          unsigned long long kk = keys[i];
          if (kk != 0ull && (kk & pmask) == prefix) atomicAdd(&s_hist[(kk >> shift) & 0xFFu], 1u);
        }
        __syncthreads();
        // suffix scan over the 256 buckets (highest first) on four waves: the
        // bucket where the running count first reaches `need` holds the r-th key
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
            s_prefix = prefix | ((unsigned long long)(255 - tid) << shift);
            s_need = need - excl;
          }
        }
        __syncthreads();
        prefix = s_prefix;
        need = s_need;
        pmask |= 0xFFull << shift;
        __syncthreads();
      }
      thr = prefix;
    }
#pragma unroll
    for (int i = 0; i < kKeysPerThread; ++i) {
      unsigned long long kk = keys[i];
      if (kk != 0ull && kk >= thr) {
        int site = (int)(0xFFFFFFFFu - (unsigned)(kk & 0xFFFFFFFFull));
        if constexpr (QARY)
          b.X[site] = c.sym[(size_t)b.tok_off + site];
        else
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
  for (int idx = tid; idx < K * b.m; idx += kTailThreads) {
    int k = idx / b.m, j = idx - k * b.m;
    int par = 0;
    for (int e = b.row_ptr[j]; e < b.row_ptr[j + 1]; ++e) {
      if constexpr (QARY)
        par ^= gf_mul_q(b.coef[e], b.X[k * n + b.col_idx[e]], b.q_bits);
      else
        par ^= b.X[k * n + b.col_idx[e]];
    }
    if (QARY ? par != 0 : (par & 1)) atomicOr(&s_syn[k], 1);
  }
  if (!QARY && wave < K) {
    float acc = 0.f;
    if (c.qhead) {
      // quality head: the row's mean omega
      const float* qrow = c.qw + (size_t)b.tok_off + (size_t)wave * n;
      for (int l = lane; l < n; l += 64) acc += qrow[l];
    } else {
      for (int l = lane; l < n; l += 64) {
        int site = wave * n + l;
        float mg = fabsf(lg[2 * site] - lg[2 * site + 1]);
        acc += 1.0f / (1.0f + expf(-mg * c.q_inv_tau));
      }
    }
    acc = wave_sum(acc);
    if (lane == 0) s_q[wave] = acc / (float)n;
  }
  if (QARY && tid < kMaxK) s_q[tid] = 1.0f;
  __syncthreads();
  if (tid == 0) {
    int low = 0;
    if (c.qhead) {
      // after final pass s (s = rounds already run) the threshold is phi_s
      const float thr = c.phi[min(st.round, 3)];
      for (int k = 0; k < K; ++k)
        if (s_q[k] < thr) low |= 1 << k;
    } else {
      for (int k = 0; k < K; ++k)
        if (s_syn[k] || s_q[k] < c.remask_thr) low |= 1 << k;
    }
    s_low = low;
  }
  __syncthreads();
  const int low = s_low;
  if (c.remask && st.round < c.max_rounds && low != 0) {
    for (int site = tid; site < tot; site += kTailThreads)
      if ((low >> (site / n)) & 1) b.X[site] = (uint8_t)c.mask;
    if (tid == 0) {
      int j = __popc(low);
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
  // done: output grid, logits and row validity
  for (int site = tid; site < tot; site += kTailThreads) {
    uint8_t x = (!QARY && c.final_argmax) ? (uint8_t)((lg[2 * site] >= lg[2 * site + 1]) ? 0 : 1) : b.X[site];
    b.out_sym[site] = x;
    if (!QARY && c.final_argmax) b.X[site] = x;
    if (b.out_logits)
      for (int a = 0; a < Q; ++a) b.out_logits[(size_t)Q * site + a] = lg[(size_t)Q * site + a];
  }
  __syncthreads();
  if (!QARY && c.final_argmax) {
    if (tid < kMaxK) s_syn[tid] = 0;
    __syncthreads();
    for (int idx = tid; idx < K * b.m; idx += kTailThreads) {
      int k = idx / b.m, j = idx - k * b.m;
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

// PRISM-style quality head (Appendix, PRISM-style quality head and remasking
// plug-in), for the tokens of every bin in its final pass: from the final
// residual Z, Zhat = LN_f(Z), h = W1 Zhat + b1 (H hidden units), and
// omega = sigmoid(w2 . GELU(LN_H(h)) + b2), LN_H with its own gain and bias.
// One wave per token, FP32: the token's d features sit d / 64 per lane, each
// hidden unit is a wave reduction and then lives in lane j < H.  With STAGE
// the workgroup copies W1 (H d floats, at most 64 KB) into LDS once and its
// waves read it from there for every token they take; otherwise W1 is read
// from L2 per token.  It is a plug-in that runs once per final pass, beside
// the L layers of the forward pass.
// psi = [W1 (H x d, row-major) | b1 | gain | bias | w2 | b2].
constexpr int kQhWaves = 4;
constexpr int kQhMaxNC = 16;   // d <= 1024

template <bool STAGE>
__global__ __launch_bounds__(64 * kQhWaves) void k_quality_head(StepCtx c, EmbedW m, const float* __restrict__ R,
                                                               float* __restrict__ qw) {
  extern __shared__ float sW1[];        // STAGE: W1 [H][d]
  const DevBin& b = c.bins[blockIdx.x];
  if (b.st->phase != kFinal) return;    // the same for every wave of the workgroup
  const int d = m.d, H = c.qh_hidden;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int tot = b.K * b.n;
  const float* W1g = c.qhead;
  if (STAGE) {
    const int nw = H * d;               // a multiple of 64 (d is)
    for (int i = 4 * (int)threadIdx.x; i < nw; i += 4 * 64 * kQhWaves)
      *(float4*)&sW1[i] = *(const float4*)&W1g[i];
    __syncthreads();
  }
  const float* W1 = STAGE ? sW1 : W1g;
  const float* b1 = W1g + (size_t)H * d;
  const float* hg = b1 + H;
  const float* hb = hg + H;
  const float* w2 = hb + H;
  const float b2 = w2[H];
  const bool act = lane < H;
  const float b1j = act ? b1[lane] : 0.f, hgj = act ? hg[lane] : 0.f, hbj = act ? hb[lane] : 0.f;
  const float w2j = act ? w2[lane] : 0.f;
  for (int i = blockIdx.y * kQhWaves + wave; i < tot; i += gridDim.y * kQhWaves) {
    const size_t tok = (size_t)b.tok_off + i;
    const float* z = R + tok * d;
    float zh[kQhMaxNC];
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < kQhMaxNC; ++q) {
      const int col = lane + 64 * q;
      zh[q] = col < d ? z[col] : 0.f;
      s += zh[q];
    }
    const float mean = wave_sum(s) / (float)d;
    float v = 0.f;
#pragma unroll
    for (int q = 0; q < kQhMaxNC; ++q) {
      const int col = lane + 64 * q;
      const float t = col < d ? zh[q] - mean : 0.f;
      v = fmaf(t, t, v);
    }
    const float rstd = rsqrtf(wave_sum(v) / (float)d + 1e-5f);
#pragma unroll
    for (int q = 0; q < kQhMaxNC; ++q) {
      const int col = lane + 64 * q;
      zh[q] = col < d ? (zh[q] - mean) * rstd * m.lnf_g[col] + m.lnf_b[col] : 0.f;
    }
    float hj = 0.f;
    for (int j = 0; j < H; ++j) {
      const float* wr = W1 + (size_t)j * d;
      float a = 0.f;
#pragma unroll
      for (int q = 0; q < kQhMaxNC; ++q) {
        const int col = lane + 64 * q;
        if (col < d) a = fmaf(wr[col], zh[q], a);
      }
      a = wave_sum(a);
      if (lane == j) hj = a + b1j;
    }
    const float hm = wave_sum(act ? hj : 0.f) / (float)H;
    const float dv = act ? hj - hm : 0.f;
    const float hr = rsqrtf(wave_sum(dv * dv) / (float)H + 1e-5f);
    float o = 0.f;
    if (act) {
      const float x = dv * hr * hgj + hbj;
      o = w2j * (0.5f * x * (1.0f + erff(x * 0.70710678118654752f)));
    }
    o = wave_sum(o) + b2;
    if (lane == 0) qw[tok] = 1.0f / (1.0f + expf(-o));
  }
}

hipError_t launch_quality_head(const StepCtx& c, const EmbedW& m, const Work& w, hipStream_t s) {
  if (!c.qhead || c.qh_hidden < 1 || c.qh_hidden > 64 || m.d < 1 || m.d > 64 * kQhMaxNC) return hipErrorInvalidValue;
  // one workgroup row per bin (grid x); along y enough workgroups for the largest grid
  // (kMaxK rows of max_n slots), at most 32
  const int need = (kMaxK * c.max_n + kQhWaves - 1) / kQhWaves;
  const int gx = need < 32 ? need : 32;
  const size_t wbytes = (size_t)c.qh_hidden * m.d * sizeof(float);
  if (wbytes <= 65536 && (m.d % 64) == 0 && ((uintptr_t)c.qhead % 16) == 0)
    hipLaunchKernelGGL(k_quality_head<true>, dim3(c.num_bins, gx), dim3(64 * kQhWaves), wbytes, s, c, m, w.R, w.qw);
  else
    hipLaunchKernelGGL(k_quality_head<false>, dim3(c.num_bins, gx), dim3(64 * kQhWaves), 0, s, c, m, w.R, w.qw);
  return hipGetLastError();
}

hipError_t launch_step_tail(const StepCtx& c, const Work& w, hipStream_t s) {
  if (c.q > 2)
    hipLaunchKernelGGL(k_step_tail<true>, dim3(c.num_bins), dim3(kTailThreads), 0, s, c, w.logits);
  else
    hipLaunchKernelGGL(k_step_tail<false>, dim3(c.num_bins), dim3(kTailThreads), 0, s, c, w.logits);
  return hipGetLastError();
}

}  // namespace cider
