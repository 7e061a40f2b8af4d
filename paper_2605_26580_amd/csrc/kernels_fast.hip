// BF16 hot-path kernels for gfx950: LayerNorm to the compute type, a
// double-buffered MFMA GEMM, and MFMA row attention.
//
// MFMA conventions used below (16x16 output blocks, 64-lane wave):
//   output   lane l, register r  ->  row 4*(l/16) + r, column l % 16
//   operands lane l holds row (A) / column (B) l % 16 and the k-group l / 16;
// both operands of one instruction always use the same k-group assignment,
// so the sum over k is the full dot product whatever order the hardware
// walks the k elements of a group in.
#include "cider_internal.h"
#include "device_math.h"

namespace cider {

namespace {

typedef __bf16 bf16x2 __attribute__((__vector_size__(2 * sizeof(__bf16))));
typedef float f32x2 __attribute__((__vector_size__(2 * sizeof(float))));

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// The dispatcher sends workgroup b to XCD b % 8, and each XCD has its own L2.
// xcd_logical maps b to a logical id so that XCD x runs one contiguous range
// of logical ids; workgroups adjacent in logical order (the heads of one row,
// the column tiles of one token tile) then share an L2 and read their common
// inputs from HBM once.  A bijection on [0, nb) for any nb.
__device__ __forceinline__ int xcd_logical(int b, int nb) {
  const int x = b & 7, i = b >> 3, q = nb >> 3, rem = nb & 7;
  return x * q + min(x, rem) + i;
}

}  // namespace

// ---------------------------------------------------------------------------
// LayerNorm over d of the FP32 residual, written in the compute type.  One
// wavefront per token; lane i owns the NC consecutive columns i*NC.. so loads
// and stores are vectorised.  Two-pass mean / variance in FP32.
template <typename TC, int NC>
__global__ __launch_bounds__(256) void k_layernorm(long T, int d, const float* __restrict__ R,
                                                   const float* __restrict__ g, const float* __restrict__ b,
                                                   TC* __restrict__ out) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const long t = (long)blockIdx.x * 4 + wave;
  if (t >= T) return;
  const int c0 = lane * NC;
  const bool on = c0 < d;
  float x[NC];
  float s = 0.f;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    x[i] = on ? R[t * d + c0 + i] : 0.f;
    s += x[i];
  }
  const float mean = wave_sum(s) / (float)d;
  float q = 0.f;
#pragma unroll
  for (int i = 0; i < NC; ++i) {
    float dv = on ? x[i] - mean : 0.f;
    q = fmaf(dv, dv, q);
  }
  const float rstd = 1.0f / sqrtf(wave_sum(q) / (float)d + 1e-5f);
  if (on) {
#pragma unroll
    for (int i = 0; i < NC; ++i) out[t * d + c0 + i] = (TC)((x[i] - mean) * rstd * g[c0 + i] + b[c0 + i]);
  }
}

hipError_t launch_layernorm(int prec, long T, int d, const float* R, const float* g, const float* b, void* out,
                            hipStream_t s) {
  if (T == 0) return hipSuccess;
  dim3 grid((unsigned)((T + 3) / 4)), block(256);
  const int nc = d / 64;  // d is a multiple of 64, at most 512
#define LN_CASE(TC, NCV) hipLaunchKernelGGL((k_layernorm<TC, NCV>), grid, block, 0, s, T, d, R, g, b, (TC*)out)
  if (prec == kF32) {
    if (nc == 1) LN_CASE(float, 1); else if (nc == 2) LN_CASE(float, 2); else if (nc <= 4) LN_CASE(float, 4);
    else LN_CASE(float, 8);
  } else {
    if (nc == 1) LN_CASE(bf16, 1); else if (nc == 2) LN_CASE(bf16, 2); else if (nc <= 4) LN_CASE(bf16, 4);
    else LN_CASE(bf16, 8);
  }
#undef LN_CASE
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// BF16 GEMM  out = epi(A W^T + bias), A [M][Kd] tokens, W [N][Kd].
//
// Workgroup tile BM tokens x BN columns, K in slices of BK staged through two
// LDS buffers (the next slice is fetched into registers while the current one
// is multiplied).  Four waves in a 2 x 2 arrangement; a wave computes BN/2
// columns x BM/2 tokens as (BN/32) x (BM/32) MFMA 16x16x32 blocks.  The FP32
// results are then staged in LDS (reusing the slice buffers) and a row pass
// writes whole token rows with coalesced accesses:
//   Store / Gelu     out (BF16) = v or GELU(v)
//   Resid            R += v
//   Gate             R = g R + (1 - g) E,  g = sigmoid(v)      (Module A blend)
//   ResidLN, GateLN  as Resid / Gate, then XN = LayerNorm(R) with the next
//                    block's gain and bias; needs BN == N so a workgroup owns
//                    complete rows.
// Each output is accumulated over k in the same order in every tile, so a
// token's result does not depend on the other tokens of its batch.
namespace {

constexpr int GPAD = 8;

enum : int { kEpiResidLN = 4, kEpiGateLN = 5, kEpiResidLN8 = 6, kEpiGateLN8 = 7, kEpiResidProj = 8,
             kEpiGeluB0 = 9 };   // GELU with the accumulators started at the bias (the fused MLP's up order)

typedef int i32x8 __attribute__((__vector_size__(8 * sizeof(int))));
typedef int i32x4 __attribute__((__vector_size__(4 * sizeof(int))));

template <int BM, int BN, int BK>
struct GemmSmem {
  static constexpr size_t loop = (size_t)2 * (BM + BN) * (BK + GPAD) * sizeof(bf16);
  static constexpr size_t stage = (size_t)BM * (BN + 4) * sizeof(float);
  static constexpr size_t bytes = loop > stage ? loop : stage;
};

// Row pass of the GEMM epilogues: sC holds the BM x BN FP32 tile (bias
// added, row stride BN + 4).  A lane group of LPR lanes owns one token row per
// pass and covers its BN columns in 4-column groups; all loads of a chunk of
// passes are issued before any of them is used, so global-memory latency
// overlaps.
template <int BM, int BN, int EPI>
__device__ __forceinline__ void row_pass(const float* sC, long m0, int n0, const GemmArgs& g, int wave, int lane) {
  constexpr int LDC = BN + 4;
  constexpr int CG = BN / 4;                     // 4-column groups per row
  constexpr int LPR = CG <= 16 ? 16 : (CG <= 32 ? 32 : 64);   // lanes per row, a power of two
  constexpr int RPI = 64 / LPR;                  // rows per wave pass
  constexpr int GPL = (CG + LPR - 1) / LPR;      // column groups per lane
  constexpr int NIT = BM / (4 * RPI);            // passes per wave
  constexpr int CH = (NIT * GPL <= 16) ? NIT : (16 / GPL > 0 ? 16 / GPL : 1);
  constexpr bool RES = EPI != kEpiStore && EPI != kEpiGelu && EPI != kEpiGeluB0;
  constexpr bool GATE = EPI == kEpiGate || EPI == kEpiGateLN || EPI == kEpiGateLN8;
  constexpr bool F8OUT = EPI == kEpiResidLN8 || EPI == kEpiGateLN8;
  constexpr bool PROJ = EPI == kEpiResidProj;   // final LayerNorm + symbol projection
  constexpr bool LNX = EPI == kEpiResidLN || EPI == kEpiGateLN || F8OUT || PROJ;
  const int grp = lane / LPR, cl = lane % LPR;
  float* __restrict__ Rg = g.R;
  const float* __restrict__ Eg = g.E;
  bf16* __restrict__ Og = (bf16*)g.out;
#pragma unroll
  for (int it0 = 0; it0 < NIT; it0 += CH) {
    f32x4 vv[CH][GPL], rr[CH][GPL], ee[GATE ? CH : 1][GPL];
#pragma unroll
    for (int it = 0; it < CH; ++it) {
      const int ml = ((it0 + it) * 4 + wave) * RPI + grp;
      const long m = m0 + ml;
#pragma unroll
      for (int u = 0; u < GPL; ++u) {
        const int cg = cl + u * LPR;
        if (cg < CG) {
          vv[it][u] = *(const f32x4*)&sC[ml * LDC + cg * 4];
          if (RES && m < g.M) {
            const long o = m * g.N + n0 + cg * 4;
            rr[it][u] = *(const f32x4*)(Rg + o);
            if (GATE) ee[GATE ? it : 0][u] = *(const f32x4*)(Eg + o);
          }
        }
      }
    }
#pragma unroll
    for (int it = 0; it < CH; ++it) {
      const int ml = ((it0 + it) * 4 + wave) * RPI + grp;
      const long m = m0 + ml;
      const bool mv = m < g.M;
      float sum = 0.f;
#pragma unroll
      for (int u = 0; u < GPL; ++u) {
        const int cg = cl + u * LPR;
        if (cg >= CG || !mv) continue;
        f32x4 v = vv[it][u];
        if (!RES) {
          if (EPI == kEpiGelu || EPI == kEpiGeluB0) {
#pragma unroll
            for (int r = 0; r < 4; ++r) v[r] = gelu_f(v[r]);
          }
          bf16x4 h = {(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
          *(bf16x4*)(Og + m * g.N + n0 + cg * 4) = h;
        } else {
          f32x4 res;
          if (!GATE) {
            res = rr[it][u] + v;
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const float gt = sigmoid_f(v[r]);
              res[r] = gt * rr[it][u][r] + (1.0f - gt) * ee[GATE ? it : 0][u][r];
            }
          }
          *(f32x4*)(Rg + m * g.N + n0 + cg * 4) = res;
          vv[it][u] = res;
          sum += (res[0] + res[1]) + (res[2] + res[3]);
        }
      }
      if (LNX) {
        // reduce over the LPR lanes of this row's group (a power of two)
#pragma unroll
        for (int o = LPR / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
        const float mean = sum / (float)BN;
        float q = 0.f;
#pragma unroll
        for (int u = 0; u < GPL; ++u) {
          const int cg = cl + u * LPR;
          if (cg >= CG || !mv) continue;
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float dv = vv[it][u][r] - mean;
            q = fmaf(dv, dv, q);
          }
        }
#pragma unroll
        for (int o = LPR / 2; o > 0; o >>= 1) q += __shfl_xor(q, o, 64);
        const float rstd = 1.0f / sqrtf(q / (float)BN + 1e-5f);
        if (PROJ) {
          float a0 = 0.f, a1 = 0.f;
#pragma unroll
          for (int u = 0; u < GPL; ++u) {
            const int cg = cl + u * LPR;
            if (cg >= CG || !mv) continue;
            const int c = cg * 4;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const float hv = (vv[it][u][r] - mean) * rstd * g.ln_g[c + r] + g.ln_b[c + r];
              a0 = fmaf(hv, g.proj_w[c + r], a0);
              a1 = fmaf(hv, g.proj_w[BN + c + r], a1);
            }
          }
#pragma unroll
          for (int o = LPR / 2; o > 0; o >>= 1) {
            a0 += __shfl_xor(a0, o, 64);
            a1 += __shfl_xor(a1, o, 64);
          }
          if (cl == 0 && mv) {
            g.proj_out[2 * m] = a0;
            g.proj_out[2 * m + 1] = a1;
          }
        } else if (!F8OUT) {
#pragma unroll
          for (int u = 0; u < GPL; ++u) {
            const int cg = cl + u * LPR;
            if (cg >= CG || !mv) continue;
            const int c = cg * 4;
            bf16x4 h;
#pragma unroll
            for (int r = 0; r < 4; ++r) h[r] = (bf16)((vv[it][u][r] - mean) * rstd * g.ln_g[c + r] + g.ln_b[c + r]);
            *(bf16x4*)(Og + m * BN + c) = h;
          }
        } else {
          // OCP e4m3 copy with a per-token scale amax / 448
          float amax = 0.f;
#pragma unroll
          for (int u = 0; u < GPL; ++u) {
            const int cg = cl + u * LPR;
            if (cg >= CG || !mv) continue;
            const int c = cg * 4;
#pragma unroll
            for (int r = 0; r < 4; ++r)
              amax = fmaxf(amax, fabsf((vv[it][u][r] - mean) * rstd * g.ln_g[c + r] + g.ln_b[c + r]));
          }
#pragma unroll
          for (int o = LPR / 2; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
          const float sc = amax > 0.f ? amax / 448.0f : 1.0f;
          const float inv = 1.0f / sc;
          uint8_t* O8 = (uint8_t*)g.out;
#pragma unroll
          for (int u = 0; u < GPL; ++u) {
            const int cg = cl + u * LPR;
            if (cg >= CG || !mv) continue;
            const int c = cg * 4;
            float hq[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
              hq[r] = fminf(fmaxf(((vv[it][u][r] - mean) * rstd * g.ln_g[c + r] + g.ln_b[c + r]) * inv, -448.f), 448.f);
            int pk = __builtin_amdgcn_cvt_pk_fp8_f32(hq[0], hq[1], 0, false);
            pk = __builtin_amdgcn_cvt_pk_fp8_f32(hq[2], hq[3], pk, true);
            *(int*)(O8 + m * BN + c) = pk;
          }
          if (cl == 0 && mv) g.out_scale[m] = sc;
        }
      }
    }
  }
}

// The LayerNorm of the residual row pass as a kernel of its own, over R as
// the plain residual GEMM left it: the same lanes per row, the same column
// groups per lane and the same order of every sum and shuffle as row_pass
// (EPI = ResidLN, BN = N), so XN is bit-identical to the fused epilogue's.
// Lets a LayerNorm-fed residual GEMM run with the plain tiles, whose weight
// traffic per token is far lower than a full-row tile's when N is large.
template <int BN, bool PROJ>
__global__ __launch_bounds__(256) void k_ln_rows(GemmArgs g) {
  constexpr int CG = BN / 4;
  constexpr int LPR = CG <= 16 ? 16 : (CG <= 32 ? 32 : 64);
  constexpr int RPI = 64 / LPR;
  constexpr int GPL = (CG + LPR - 1) / LPR;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, grp = lane / LPR, cl = lane % LPR;
  const long m = ((long)blockIdx.x * 4 + wave) * RPI + grp;
  const bool mv = m < g.M;
  f32x4 vv[GPL];
  float sum = 0.f;
#pragma unroll
  for (int u = 0; u < GPL; ++u) {
    const int cg = cl + u * LPR;
    if (cg >= CG || !mv) continue;
    vv[u] = *(const f32x4*)(g.R + m * BN + cg * 4);
    sum += (vv[u][0] + vv[u][1]) + (vv[u][2] + vv[u][3]);
  }
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  const float mean = sum / (float)BN;
  float q = 0.f;
#pragma unroll
  for (int u = 0; u < GPL; ++u) {
    const int cg = cl + u * LPR;
    if (cg >= CG || !mv) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float dv = vv[u][r] - mean;
      q = fmaf(dv, dv, q);
    }
  }
#pragma unroll
  for (int o = LPR / 2; o > 0; o >>= 1) q += __shfl_xor(q, o, 64);
  const float rstd = 1.0f / sqrtf(q / (float)BN + 1e-5f);
  if (PROJ) {
    // the final LayerNorm and the two-way symbol projection (row_pass's PROJ)
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int u = 0; u < GPL; ++u) {
      const int cg = cl + u * LPR;
      if (cg >= CG || !mv) continue;
      const int c = cg * 4;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float hv = (vv[u][r] - mean) * rstd * g.ln_g[c + r] + g.ln_b[c + r];
        a0 = fmaf(hv, g.proj_w[c + r], a0);
        a1 = fmaf(hv, g.proj_w[BN + c + r], a1);
      }
    }
#pragma unroll
    for (int o = LPR / 2; o > 0; o >>= 1) {
      a0 += __shfl_xor(a0, o, 64);
      a1 += __shfl_xor(a1, o, 64);
    }
    if (cl == 0 && mv) {
      g.proj_out[2 * m] = a0;
      g.proj_out[2 * m + 1] = a1;
    }
    return;
  }
  bf16* __restrict__ Og = (bf16*)g.out;
#pragma unroll
  for (int u = 0; u < GPL; ++u) {
    const int cg = cl + u * LPR;
    if (cg >= CG || !mv) continue;
    const int c = cg * 4;
    bf16x4 h;
#pragma unroll
    for (int r = 0; r < 4; ++r) h[r] = (bf16)((vv[u][r] - mean) * rstd * g.ln_g[c + r] + g.ln_b[c + r]);
    *(bf16x4*)(Og + m * BN + c) = h;
  }
}

hipError_t launch_ln_rows(const GemmArgs& g, hipStream_t s) {
  const int rpb = 4 * (64 / ((g.N / 4) <= 16 ? 16 : ((g.N / 4) <= 32 ? 32 : 64)));   // rows per workgroup
  dim3 grid((unsigned)((g.M + rpb - 1) / rpb)), block(256);
  const bool pj = g.proj_out != nullptr;
#define CIDER_LNR(N)                                                               \
  case N:                                                                          \
    if (pj) hipLaunchKernelGGL((k_ln_rows<N, true>), grid, block, 0, s, g);        \
    else hipLaunchKernelGGL((k_ln_rows<N, false>), grid, block, 0, s, g);          \
    break;
  switch (g.N) {
    CIDER_LNR(64) CIDER_LNR(128) CIDER_LNR(192) CIDER_LNR(256)
    CIDER_LNR(320) CIDER_LNR(384) CIDER_LNR(448) CIDER_LNR(512)
    default: return hipErrorInvalidValue;
  }
#undef CIDER_LNR
  return hipGetLastError();
}

// Workgroups of 4 waves that LDS lets share a CU: the register budget the
// compiler may use without lowering occupancy below what LDS already sets.
constexpr int lds_waves(size_t bytes) {
  return (int)(163840 / bytes) < 1 ? 1 : ((int)(163840 / bytes) > 8 ? 8 : (int)(163840 / bytes));
}

template <int BM, int BN, int BK, int EPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(lds_waves(GemmSmem<BM, BN, BK>::bytes))))
void k_gemm_bf16(GemmArgs g, const bf16* __restrict__ W) {
  constexpr int TI = BN / 32;  // column blocks per wave
  constexpr int TJ = BM / 32;  // token blocks per wave
  constexpr int LDK = BK + GPAD;
  __shared__ __attribute__((aligned(16))) char smem[GemmSmem<BM, BN, BK>::bytes];
  bf16* sA = (bf16*)smem;                       // [2][BM][LDK]
  bf16* sW = sA + 2 * BM * LDK;                 // [2][BN][LDK]
  float* sC = (float*)smem;                     // [BM][BN + 4] after the K loop
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nN = g.N / BN;
  const int lb = xcd_logical((int)blockIdx.x, (int)gridDim.x);
  const long m0 = (long)(lb / nN) * BM;
  const int n0 = (lb - (lb / nN) * nN) * BN;
  const int Kd = g.Kd;
  const bf16* A = (const bf16*)g.A;
  const int wn = (wave >> 1) * (BN / 2), wm = (wave & 1) * (BM / 2);

  constexpr int CPR = BK / 8;                    // 16-byte chunks per row of a slice
  constexpr int ACH = (BM * CPR + 255) / 256;
  constexpr int WCH = (BN * CPR + 255) / 256;
  bf16x8 ra[ACH], rw[WCH];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int c = 0; c < ACH; ++c) {
      const int idx = tid + c * 256, row = idx / CPR, kc = (idx % CPR) * 8;
      const long gm = m0 + row;
      if (row < BM && gm < g.M) ra[c] = *(const bf16x8*)(A + gm * Kd + k0 + kc);
      else ra[c] = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
    }
#pragma unroll
    for (int c = 0; c < WCH; ++c) {
      const int idx = tid + c * 256, row = idx / CPR, kc = (idx % CPR) * 8;
      if (row < BN) rw[c] = *(const bf16x8*)(W + (long)(n0 + row) * Kd + k0 + kc);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int c = 0; c < ACH; ++c) {
      const int idx = tid + c * 256, row = idx / CPR, kc = (idx % CPR) * 8;
      if (row < BM) *(bf16x8*)&sA[(buf * BM + row) * LDK + kc] = ra[c];
    }
#pragma unroll
    for (int c = 0; c < WCH; ++c) {
      const int idx = tid + c * 256, row = idx / CPR, kc = (idx % CPR) * 8;
      if (row < BN) *(bf16x8*)&sW[(buf * BN + row) * LDK + kc] = rw[c];
    }
  };

  // B0: the accumulators start at the bias (columns wn + 16 i + 4 (lane/16) + r)
  constexpr bool B0 = EPI == kEpiGeluB0;
  f32x4 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    f32x4 a0 = f32x4{0.f, 0.f, 0.f, 0.f};
    if (B0 && g.bias) {
      const int nl = n0 + wn + i * 16 + (lane >> 4) * 4;
      a0 = f32x4{g.bias[nl], g.bias[nl + 1], g.bias[nl + 2], g.bias[nl + 3]};
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = a0;
  }

  const int nk = Kd / BK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) fetch((kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 32) {
      bf16x8 fw[TI], fa[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i)
        fw[i] = *(const bf16x8*)&sW[(buf * BN + wn + i * 16 + (lane & 15)) * LDK + ks + (lane >> 4) * 8];
#pragma unroll
      for (int j = 0; j < TJ; ++j)
        fa[j] = *(const bf16x8*)&sA[(buf * BM + wm + j * 16 + (lane & 15)) * LDK + ks + (lane >> 4) * 8];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[i], fa[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) stash(buf ^ 1);
    __syncthreads();
  }

  // stage v = acc + bias: lane holds columns wn + 16 i + 4 (lane/16) + r of token wm + 16 j + lane%16
  constexpr int LDC = BN + 4;
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    const int nl = wn + i * 16 + (lane >> 4) * 4;
    f32x4 bias = f32x4{0.f, 0.f, 0.f, 0.f};
    if (g.bias && !B0) {
#pragma unroll
      for (int r = 0; r < 4; ++r) bias[r] = g.bias[n0 + nl + r];
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int ml = wm + j * 16 + (lane & 15);
      *(f32x4*)&sC[ml * LDC + nl] = acc[i][j] + bias;
    }
  }
  __syncthreads();

  row_pass<BM, BN, EPI>(sC, m0, n0, g, wave, lane);
}

template <int BM, int BN, int BK>
hipError_t gemm_bf16_t(int epi, const GemmArgs& g, const bf16* W, hipStream_t s) {
  dim3 grid((unsigned)(((g.M + BM - 1) / BM) * (g.N / BN))), block(256);
  switch (epi) {
    case kEpiStore: hipLaunchKernelGGL((k_gemm_bf16<BM, BN, BK, kEpiStore>), grid, block, 0, s, g, W); break;
    case kEpiGelu: hipLaunchKernelGGL((k_gemm_bf16<BM, BN, BK, kEpiGelu>), grid, block, 0, s, g, W); break;
    case kEpiGeluB0: hipLaunchKernelGGL((k_gemm_bf16<BM, BN, BK, kEpiGeluB0>), grid, block, 0, s, g, W); break;
    case kEpiResid: hipLaunchKernelGGL((k_gemm_bf16<BM, BN, BK, kEpiResid>), grid, block, 0, s, g, W); break;
    case kEpiGate: hipLaunchKernelGGL((k_gemm_bf16<BM, BN, BK, kEpiGate>), grid, block, 0, s, g, W); break;
    case kEpiResidLN: hipLaunchKernelGGL((k_gemm_bf16<BM, BN, BK, kEpiResidLN>), grid, block, 0, s, g, W); break;
    case kEpiGateLN: hipLaunchKernelGGL((k_gemm_bf16<BM, BN, BK, kEpiGateLN>), grid, block, 0, s, g, W); break;
    case kEpiResidLN8: hipLaunchKernelGGL((k_gemm_bf16<BM, BN, BK, kEpiResidLN8>), grid, block, 0, s, g, W); break;
    case kEpiGateLN8: hipLaunchKernelGGL((k_gemm_bf16<BM, BN, BK, kEpiGateLN8>), grid, block, 0, s, g, W); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

// Tile shapes the GEMM can run with.  Every shape accumulates each output over
// k in the same order (32-wide MFMA steps from k = 0 up), and the fused
// LayerNorm always spans the full row, so the choice never changes a result;
// the autotuner picks among them by measured time.
//   plain epilogues : 0 = 128x128, 1 = 64x128, 2 = 128x64, 3 = 64x64 (BM x BN)
//   LayerNorm fused : BN = N, 0 = BM 128 (N <= 128) or 64, 1 = BM 64, 2 = BM 32;
//                     for a residual GEMM with a BF16 LayerNorm output, then
//                     the plain tiles followed by k_ln_rows (same result)
static int ln_fused_tiles(int N) { return N <= 128 ? 3 : 2; }
static int plain_tiles(int N) { return (N % 128 == 0) ? 4 : 2; }
int gemm_tile_count(int epi, int N, bool ln) {
  if (ln) return ln_fused_tiles(N) + ((epi == kEpiResid || epi == kEpiGate) ? plain_tiles(N) : 0);
  return plain_tiles(N);
}

// The tile used before (or without) tuning: a full-row tile re-streams the
// whole weight matrix for every 32-64 tokens, which at N >= 320 costs more
// than the split form's extra pass over R (measured at d = 384: 0.38 against
// 0.75 ms per output projection).
int gemm_default_tile(int epi, int N, bool ln) {
  return (ln && (epi == kEpiResid || epi == kEpiGate) && N >= 320 && N % 64 == 0 && N <= 512) ? ln_fused_tiles(N) : 0;
}

// epi: Store, Gelu, Resid, Gate; with ln_g set (Resid / Gate) the next
// LayerNorm is applied in the epilogue and written to g.out.
hipError_t launch_gemm_bf16(int epi, const GemmArgs& g, const Mat& W, hipStream_t s, int tile) {
  if (g.M == 0) return hipSuccess;
  if (g.Kd % 64 != 0) return hipErrorInvalidValue;
  const bool ln = (epi == kEpiResid || epi == kEpiGate) && g.ln_g != nullptr;
  if (ln && tile >= ln_fused_tiles(g.N)) {
    if ((epi != kEpiResid && epi != kEpiGate) || g.out_scale || g.proj_out || g.N % 64 != 0 || g.N > 512) {
      tile = 0;                                   // no split form: the default fused tile
    } else {
      // residual (or gate-blend) GEMM with a plain tile, then the row LayerNorm over R
      GemmArgs gr = g;
      gr.ln_g = gr.ln_b = nullptr;
      gr.out = nullptr;
      const hipError_t e = launch_gemm_bf16(epi, gr, W, s, tile - ln_fused_tiles(g.N));
      if (e != hipSuccess) return e;
      return launch_ln_rows(g, s);
    }
  }
  if (ln) {
    const bool f8 = g.out_scale != nullptr;
    const int e = epi == kEpiResid ? (f8 ? kEpiResidLN8 : kEpiResidLN) : (f8 ? kEpiGateLN8 : kEpiGateLN);
    const int bm = (tile == 0) ? (g.N <= 128 ? 128 : 64) : (tile == 1 ? 64 : 32);
#define LNT(BNV, BKV)                                                    \
  if (bm == 128) return gemm_bf16_t<128, BNV, BKV>(e, g, W.b16, s);      \
  if (bm == 64) return gemm_bf16_t<64, BNV, BKV>(e, g, W.b16, s);        \
  return gemm_bf16_t<32, BNV, BKV>(e, g, W.b16, s);
#define LNT_SMALL(BNV, BKV)                                              \
  if (bm == 128) return hipErrorInvalidValue;                            \
  if (bm == 64) return gemm_bf16_t<64, BNV, BKV>(e, g, W.b16, s);        \
  return gemm_bf16_t<32, BNV, BKV>(e, g, W.b16, s);
    switch (g.N) {
      case 64: { LNT(64, 64) }
      case 128: { LNT(128, 64) }
      case 192: { LNT_SMALL(192, 64) }
      case 256: { LNT_SMALL(256, 64) }
      case 320: { LNT_SMALL(320, 32) }
      case 384: { LNT_SMALL(384, 32) }
      case 448: { LNT_SMALL(448, 32) }
      case 512: { LNT_SMALL(512, 32) }
      default: return hipErrorInvalidValue;
    }
#undef LNT_SMALL
#undef LNT
  }
  if (g.N % 128 == 0) {
    switch (tile) {
      case 0: return gemm_bf16_t<128, 128, 64>(epi, g, W.b16, s);
      case 1: return gemm_bf16_t<64, 128, 64>(epi, g, W.b16, s);
      case 2: return gemm_bf16_t<128, 64, 64>(epi, g, W.b16, s);
      default: return gemm_bf16_t<64, 64, 64>(epi, g, W.b16, s);
    }
  }
  if (g.N % 64 == 0) {
    if (tile == 0 || tile == 2) return gemm_bf16_t<128, 64, 64>(epi, g, W.b16, s);
    return gemm_bf16_t<64, 64, 64>(epi, g, W.b16, s);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Fused MLP block: R += W2 GELU(W1 XN + b1) + b2 for a tile of BM tokens, with
// the 4d-wide hidden layer kept on chip.  The XN tile sits in LDS; the hidden
// layer is produced FCH columns at a time (up GEMM, GELU, BF16 into LDS) and
// consumed at once by the down GEMM, whose BM x D accumulators stay in
// registers across chunks.  The weight chunks W1[c:c+FCH][:] and
// W2[:][c:c+FCH] are staged in LDS with 16-byte loads, and the next chunk is
// fetched into registers while the current one is multiplied.  The epilogue is
// the GEMM row pass: residual add and, with ln_g set, the next LayerNorm.
namespace {

template <int BM, int DIN, int D, int FCH>
struct MlpSmem {
  static constexpr size_t a = (size_t)BM * (DIN + GPAD) * sizeof(bf16);
  static constexpr size_t h = (size_t)BM * (FCH + GPAD) * sizeof(bf16);
  static constexpr size_t w1 = (size_t)FCH * (DIN + GPAD) * sizeof(bf16);
  static constexpr size_t w2 = (size_t)D * (FCH + GPAD) * sizeof(bf16);
  static constexpr size_t c = (size_t)BM * (D + 4) * sizeof(float);
  static constexpr size_t loop = a + h + w1 + w2;
  static constexpr size_t bytes = loop > c ? loop : c;
};

template <int BM, int DIN, int D, int FCH, int EPI>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(lds_waves(MlpSmem<BM, DIN, D, FCH>::bytes))))
void k_mlp_bf16(GemmArgs g, const bf16* __restrict__ W1, const float* __restrict__ b1, const bf16* __restrict__ W2,
                int F) {
  constexpr int LDA = DIN + GPAD, LDH = FCH + GPAD, LDW1 = DIN + GPAD, LDW2 = FCH + GPAD;
  constexpr int TI1 = FCH / 32, TJ1 = BM / 32;   // up GEMM: (FCH/2) hidden x (BM/2) tokens per wave
  constexpr int TI2 = D / 32, TJ2 = BM / 32;     // down GEMM: (D/2) outputs x (BM/2) tokens per wave
  constexpr int PW1 = FCH * DIN / 8 / 256;       // 16-byte chunks per thread of a W1 chunk
  constexpr int PW2 = D * FCH / 8 / 256;
  static_assert(PW1 * 256 * 8 == FCH * DIN && PW2 * 256 * 8 == D * FCH, "weight chunks must split over 256 threads");
  static_assert(BM % 32 == 0 && FCH % 32 == 0 && D % 32 == 0 && DIN % 32 == 0, "MFMA tiling");
  __shared__ __attribute__((aligned(16))) char smem[MlpSmem<BM, DIN, D, FCH>::bytes];
  bf16* sA = (bf16*)smem;
  bf16* sH = sA + BM * LDA;
  bf16* sW1 = sH + BM * LDH;
  bf16* sW2 = sW1 + FCH * LDW1;
  float* sC = (float*)smem;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const long m0 = (long)blockIdx.x * BM;
  const bf16* A = (const bf16*)g.A;

  bf16x8 pw1[PW1], pw2[PW2];
  auto fetchW = [&](int c0) {
#pragma unroll
    for (int i = 0; i < PW1; ++i) {
      const int idx = tid + i * 256, row = idx / (DIN / 8), kc = (idx - row * (DIN / 8)) * 8;
      pw1[i] = *(const bf16x8*)(W1 + (long)(c0 + row) * DIN + kc);
    }
#pragma unroll
    for (int i = 0; i < PW2; ++i) {
      const int idx = tid + i * 256, row = idx / (FCH / 8), kc = (idx - row * (FCH / 8)) * 8;
      pw2[i] = *(const bf16x8*)(W2 + (long)row * F + c0 + kc);
    }
  };
  auto stashW = [&]() {
#pragma unroll
    for (int i = 0; i < PW1; ++i) {
      const int idx = tid + i * 256, row = idx / (DIN / 8), kc = (idx - row * (DIN / 8)) * 8;
      *(bf16x8*)&sW1[row * LDW1 + kc] = pw1[i];
    }
#pragma unroll
    for (int i = 0; i < PW2; ++i) {
      const int idx = tid + i * 256, row = idx / (FCH / 8), kc = (idx - row * (FCH / 8)) * 8;
      *(bf16x8*)&sW2[row * LDW2 + kc] = pw2[i];
    }
  };

  fetchW(0);
  constexpr int CPR = DIN / 8;
  for (int idx = tid; idx < BM * CPR; idx += 256) {
    const int row = idx / CPR, kc = (idx - row * CPR) * 8;
    const long gm = m0 + row;
    bf16x8 v = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
    if (gm < g.M) v = *(const bf16x8*)(A + gm * DIN + kc);
    *(bf16x8*)&sA[row * LDA + kc] = v;
  }
  stashW();
  __syncthreads();

  f32x4 acc2[TI2][TJ2];
#pragma unroll
  for (int i = 0; i < TI2; ++i)
#pragma unroll
    for (int j = 0; j < TJ2; ++j) acc2[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int wn1 = (wave >> 1) * (FCH / 2), wm = (wave & 1) * (BM / 2), wn2 = (wave >> 1) * (D / 2);

  for (int c0 = 0; c0 < F; c0 += FCH) {
    const bool more = c0 + FCH < F;
    if (more) fetchW(c0 + FCH);
    // up: H[token][j] = GELU(b1[c0 + j] + sum_k XN[token][k] W1[c0 + j][k]),
    // the accumulators starting from the bias
    f32x4 acc1[TI1][TJ1];
#pragma unroll
    for (int i = 0; i < TI1; ++i) {
      const int hn = wn1 + i * 16 + (lane >> 4) * 4;
      const f32x4 bb = f32x4{b1[c0 + hn], b1[c0 + hn + 1], b1[c0 + hn + 2], b1[c0 + hn + 3]};
#pragma unroll
      for (int j = 0; j < TJ1; ++j) acc1[i][j] = bb;
    }
#pragma unroll
    for (int ks = 0; ks < DIN; ks += 32) {
      bf16x8 fw[TI1], fa[TJ1];
#pragma unroll
      for (int i = 0; i < TI1; ++i) fw[i] = *(const bf16x8*)&sW1[(wn1 + i * 16 + (lane & 15)) * LDW1 + ks + (lane >> 4) * 8];
#pragma unroll
      for (int j = 0; j < TJ1; ++j) fa[j] = *(const bf16x8*)&sA[(wm + j * 16 + (lane & 15)) * LDA + ks + (lane >> 4) * 8];
#pragma unroll
      for (int i = 0; i < TI1; ++i)
#pragma unroll
        for (int j = 0; j < TJ1; ++j) acc1[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[i], fa[j], acc1[i][j], 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < TI1; ++i) {
      const int hn = wn1 + i * 16 + (lane >> 4) * 4;
#pragma unroll
      for (int j = 0; j < TJ1; ++j) {
        const int ml = wm + j * 16 + (lane & 15);
        const f32x4 v = acc1[i][j];
        bf16x4 hv = {(bf16)gelu_f(v[0]), (bf16)gelu_f(v[1]), (bf16)gelu_f(v[2]), (bf16)gelu_f(v[3])};
        *(bf16x4*)&sH[ml * LDH + hn] = hv;
      }
    }
    __syncthreads();
    // down: acc2[token][o] += sum_j H[token][j] W2[o][c0 + j]
#pragma unroll
    for (int ks = 0; ks < FCH; ks += 32) {
      bf16x8 fw[TI2], fh[TJ2];
#pragma unroll
      for (int i = 0; i < TI2; ++i) fw[i] = *(const bf16x8*)&sW2[(wn2 + i * 16 + (lane & 15)) * LDW2 + ks + (lane >> 4) * 8];
#pragma unroll
      for (int j = 0; j < TJ2; ++j) fh[j] = *(const bf16x8*)&sH[(wm + j * 16 + (lane & 15)) * LDH + ks + (lane >> 4) * 8];
#pragma unroll
      for (int i = 0; i < TI2; ++i)
#pragma unroll
        for (int j = 0; j < TJ2; ++j) acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[i], fh[j], acc2[i][j], 0, 0, 0);
    }
    __syncthreads();
    if (more) {
      stashW();
      __syncthreads();
    }
  }

  // stage out = acc2 + b2 (sC overlaps the loop buffers, no longer read)
  constexpr int LDC = D + 4;
#pragma unroll
  for (int i = 0; i < TI2; ++i) {
    const int nl = wn2 + i * 16 + (lane >> 4) * 4;
    f32x4 bias;
#pragma unroll
    for (int r = 0; r < 4; ++r) bias[r] = g.bias[nl + r];
#pragma unroll
    for (int j = 0; j < TJ2; ++j) {
      const int ml = wm + j * 16 + (lane & 15);
      *(f32x4*)&sC[ml * LDC + nl] = acc2[i][j] + bias;
    }
  }
  __syncthreads();
  row_pass<BM, D, EPI>(sC, m0, 0, g, wave, lane);
}

template <int BM, int D, int FCH>
hipError_t mlp_t(bool ln, const GemmArgs& g, const bf16* W1, const float* b1, const bf16* W2, int F, hipStream_t s) {
  if (F % FCH != 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)((g.M + BM - 1) / BM)), block(256);
  if (g.proj_out) hipLaunchKernelGGL((k_mlp_bf16<BM, D, D, FCH, kEpiResidProj>), grid, block, 0, s, g, W1, b1, W2, F);
  else if (ln && g.out_scale) hipLaunchKernelGGL((k_mlp_bf16<BM, D, D, FCH, kEpiResidLN8>), grid, block, 0, s, g, W1, b1, W2, F);
  else if (ln) hipLaunchKernelGGL((k_mlp_bf16<BM, D, D, FCH, kEpiResidLN>), grid, block, 0, s, g, W1, b1, W2, F);
  else hipLaunchKernelGGL((k_mlp_bf16<BM, D, D, FCH, kEpiResid>), grid, block, 0, s, g, W1, b1, W2, F);
  return hipGetLastError();
}

// Module A gate MLP: R = g R + (1 - g) E with g = sigmoid(W_g2 GELU(W_g1 [Z ; e] + b1) + b2),
// then the first block's LayerNorm into XN (or XN8 with its scales).
template <int BM, int D, int FCH>
hipError_t gate_t(const GemmArgs& g, const bf16* W1, const float* b1, const bf16* W2, hipStream_t s) {
  if (D % FCH != 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)((g.M + BM - 1) / BM)), block(256);
  if (g.out_scale) hipLaunchKernelGGL((k_mlp_bf16<BM, 2 * D, D, FCH, kEpiGateLN8>), grid, block, 0, s, g, W1, b1, W2, D);
  else hipLaunchKernelGGL((k_mlp_bf16<BM, 2 * D, D, FCH, kEpiGateLN>), grid, block, 0, s, g, W1, b1, W2, D);
  return hipGetLastError();
}

}  // namespace

// Fused-MLP tile shapes (BM tokens, FCH hidden columns per chunk).  The
// hidden dimension is always consumed in 32-wide MFMA steps from 0 up, so every
// shape gives the same result; the autotuner picks by time.
// Fused tiles per width, then two split forms: the up projection as a GEMM
// whose accumulators start at b1 (the fused kernel's order) with GELU into
// the hidden buffer, the down projection as a plain residual GEMM (128- or
// 64-token tiles) and the row LayerNorm (or final LayerNorm and projection)
// after it -- bit-identical to the fused kernel, with the weights streamed
// per 128 tokens instead of per 32-64.
static int mlp_fused_tiles(int D) { return D == 128 ? 4 : (D == 64 || D == 256 ? 2 : 1); }
int mlp_tile_count(int D) { return mlp_fused_tiles(D) + 2; }
// Widths whose fused kernel runs 32-token tiles start on the split form
// (measured at d = 384: 1.39 against 2.86 ms per MLP).
int mlp_default_tile(int D) { return D >= 320 ? mlp_fused_tiles(D) : 0; }

// R += W2 GELU(W1 XN + b1) + b2 (g.A = XN, g.bias = b2, g.R = R, and with
// g.ln_g set the next LayerNorm into g.out).
hipError_t launch_mlp_bf16(const GemmArgs& g, const Mat& W1, const float* b1, const Mat& W2, int F, hipStream_t s,
                           int tile, void* hid) {
  if (g.M == 0) return hipSuccess;
  const bool ln = g.ln_g != nullptr;
  if (tile >= mlp_fused_tiles(g.N)) {
    const int sp = tile - mlp_fused_tiles(g.N);
    if (!hid || !ln || g.out_scale || F % 128 != 0 || g.N % 64 != 0 || g.N > 512 || g.Kd != g.N) {
      tile = 0;                                   // no split form: the default fused tile
    } else {
      GemmArgs gu{};
      gu.M = g.M; gu.N = F; gu.Kd = g.N; gu.A = g.A; gu.bias = b1; gu.out = hid;
      hipError_t e = gemm_bf16_t<128, 128, 64>(kEpiGeluB0, gu, W1.b16, s);
      if (e != hipSuccess) return e;
      GemmArgs gd = g;
      gd.A = hid; gd.Kd = F;
      gd.ln_g = gd.ln_b = nullptr; gd.out = nullptr; gd.proj_w = nullptr; gd.proj_out = nullptr;
      if (g.N % 128 == 0) e = sp == 0 ? gemm_bf16_t<128, 128, 64>(kEpiResid, gd, W2.b16, s)
                                      : gemm_bf16_t<64, 128, 64>(kEpiResid, gd, W2.b16, s);
      else e = sp == 0 ? gemm_bf16_t<128, 64, 64>(kEpiResid, gd, W2.b16, s)
                       : gemm_bf16_t<64, 64, 64>(kEpiResid, gd, W2.b16, s);
      if (e != hipSuccess) return e;
      return launch_ln_rows(g, s);
    }
  }
  switch (g.N) {
    case 64:
      if (tile == 1) return mlp_t<32, 64, 64>(ln, g, W1.b16, b1, W2.b16, F, s);
      return mlp_t<64, 64, 64>(ln, g, W1.b16, b1, W2.b16, F, s);
    case 128:
      if (tile == 1) return mlp_t<128, 128, 64>(ln, g, W1.b16, b1, W2.b16, F, s);
      if (tile == 2) return mlp_t<32, 128, 64>(ln, g, W1.b16, b1, W2.b16, F, s);
      if (tile == 3) return mlp_t<64, 128, 128>(ln, g, W1.b16, b1, W2.b16, F, s);
      return mlp_t<64, 128, 64>(ln, g, W1.b16, b1, W2.b16, F, s);
    case 192: return mlp_t<64, 192, 64>(ln, g, W1.b16, b1, W2.b16, F, s);
    case 256:
      if (tile == 1) return mlp_t<32, 256, 64>(ln, g, W1.b16, b1, W2.b16, F, s);
      return mlp_t<64, 256, 64>(ln, g, W1.b16, b1, W2.b16, F, s);
    case 320: return mlp_t<32, 320, 64>(ln, g, W1.b16, b1, W2.b16, F, s);
    case 384: return mlp_t<32, 384, 64>(ln, g, W1.b16, b1, W2.b16, F, s);
    case 448: return mlp_t<32, 448, 32>(ln, g, W1.b16, b1, W2.b16, F, s);
    case 512: return mlp_t<32, 512, 32>(ln, g, W1.b16, b1, W2.b16, F, s);
    default: return hipErrorInvalidValue;
  }
}

// Module A gate MLP fused (g.A = [Z ; e] of width 2d, g.bias = b_g2, g.R = R,
// g.E = e, g.ln_g / ln_b / out = the first block's LayerNorm output).
hipError_t launch_gate_bf16(const GemmArgs& g, const Mat& Wg1, const float* bg1, const Mat& Wg2, hipStream_t s) {
  if (g.M == 0) return hipSuccess;
  switch (g.N) {
    case 64: return gate_t<32, 64, 32>(g, Wg1.b16, bg1, Wg2.b16, s);
    case 128: return gate_t<32, 128, 32>(g, Wg1.b16, bg1, Wg2.b16, s);
    case 192: return gate_t<32, 192, 32>(g, Wg1.b16, bg1, Wg2.b16, s);
    case 256: return gate_t<32, 256, 32>(g, Wg1.b16, bg1, Wg2.b16, s);
    case 320: return gate_t<32, 320, 32>(g, Wg1.b16, bg1, Wg2.b16, s);
    case 384: return gate_t<32, 384, 32>(g, Wg1.b16, bg1, Wg2.b16, s);
    case 448: return gate_t<32, 448, 32>(g, Wg1.b16, bg1, Wg2.b16, s);
    default: return hipErrorInvalidValue;
  }
}

// d = 512 would need 172 KB of LDS for the [Z ; e] tile and one W_g1 chunk.
// At d >= 320 the fused gate's 32-token tiles re-stream both gate matrices
// per tile; the two GEMMs (with the split LayerNorm) stream them per 128.
bool gate_fusable(int d) { return d <= 256 && d % 64 == 0; }

// ---------------------------------------------------------------------------
// FP8 (OCP e4m3) token GEMMs fed by a LayerNorm: out = A W^T with A = XN8
// (per-token scale a_scale[m]) and W in e4m3 with one per-tensor scale.  Uses
// v_mfma_scale_f32_16x16x128_f8f6f4 with unit block scales (E8M0 127), a lane
// holding 32 consecutive k of its row; the FP32 result is scaled by
// a_scale[m] * w_scale, the bias added, and the row pass writes BF16.
namespace {

template <int BM, int BN>
__global__ __launch_bounds__(256) void k_gemm_fp8(GemmArgs g, const uint8_t* __restrict__ W, float w_scale) {
  constexpr int BK = 128, LDK = BK + 16;
  constexpr int TI = BN / 32, TJ = BM / 32;
  constexpr size_t loop = (size_t)2 * (BM + BN) * LDK;
  constexpr size_t stage = (size_t)BM * (BN + 4) * sizeof(float);
  __shared__ __attribute__((aligned(16))) char smem[loop > stage ? loop : stage];
  uint8_t* sA = (uint8_t*)smem;              // [2][BM][LDK]
  uint8_t* sW = sA + 2 * BM * LDK;           // [2][BN][LDK]
  float* sC = (float*)smem;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int nN = g.N / BN;
  const int lb = xcd_logical((int)blockIdx.x, (int)gridDim.x);
  const long m0 = (long)(lb / nN) * BM;
  const int n0 = (lb - (lb / nN) * nN) * BN;
  const int Kd = g.Kd;
  const uint8_t* A = (const uint8_t*)g.A;
  const int wn = (wave >> 1) * (BN / 2), wm = (wave & 1) * (BM / 2);
  constexpr int CPR = BK / 16;
  constexpr int ACH = (BM * CPR + 255) / 256, WCH = (BN * CPR + 255) / 256;
  i32x4 ra[ACH], rw[WCH];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int c = 0; c < ACH; ++c) {
      const int idx = tid + c * 256, row = idx / CPR, kc = (idx % CPR) * 16;
      const long gm = m0 + row;
      if (row < BM && gm < g.M) ra[c] = *(const i32x4*)(A + gm * Kd + k0 + kc);
      else ra[c] = i32x4{0, 0, 0, 0};
    }
#pragma unroll
    for (int c = 0; c < WCH; ++c) {
      const int idx = tid + c * 256, row = idx / CPR, kc = (idx % CPR) * 16;
      if (row < BN) rw[c] = *(const i32x4*)(W + (long)(n0 + row) * Kd + k0 + kc);
    }
  };
  auto stash = [&](int buf) {
#pragma unroll
    for (int c = 0; c < ACH; ++c) {
      const int idx = tid + c * 256, row = idx / CPR, kc = (idx % CPR) * 16;
      if (row < BM) *(i32x4*)&sA[(buf * BM + row) * LDK + kc] = ra[c];
    }
#pragma unroll
    for (int c = 0; c < WCH; ++c) {
      const int idx = tid + c * 256, row = idx / CPR, kc = (idx % CPR) * 16;
      if (row < BN) *(i32x4*)&sW[(buf * BN + row) * LDK + kc] = rw[c];
    }
  };
  auto frag = [&](const uint8_t* p) {
    const i32x4 lo = *(const i32x4*)p, hi = *(const i32x4*)(p + 16);
    return i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  };
  f32x4 acc[TI][TJ];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int nk = Kd / BK;
  fetch(0);
  stash(0);
  __syncthreads();
  for (int kt = 0; kt < nk; ++kt) {
    const int buf = kt & 1;
    if (kt + 1 < nk) fetch((kt + 1) * BK);
    i32x8 fw[TI], fa[TJ];
#pragma unroll
    for (int i = 0; i < TI; ++i) fw[i] = frag(&sW[(buf * BN + wn + i * 16 + (lane & 15)) * LDK + (lane >> 4) * 32]);
#pragma unroll
    for (int j = 0; j < TJ; ++j) fa[j] = frag(&sA[(buf * BM + wm + j * 16 + (lane & 15)) * LDK + (lane >> 4) * 32]);
#pragma unroll
    for (int i = 0; i < TI; ++i)
#pragma unroll
      for (int j = 0; j < TJ; ++j)
        acc[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(fw[i], fa[j], acc[i][j], 0, 0, 0, 127, 0, 127);
    if (kt + 1 < nk) stash(buf ^ 1);
    __syncthreads();
  }
  constexpr int LDC = BN + 4;
#pragma unroll
  for (int i = 0; i < TI; ++i) {
    const int nl = wn + i * 16 + (lane >> 4) * 4;
    f32x4 bias = f32x4{0.f, 0.f, 0.f, 0.f};
    if (g.bias) {
#pragma unroll
      for (int r = 0; r < 4; ++r) bias[r] = g.bias[n0 + nl + r];
    }
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      const int ml = wm + j * 16 + (lane & 15);
      const long m = m0 + ml;
      const float sc = (m < g.M ? g.a_scale[m] : 0.f) * w_scale;
      *(f32x4*)&sC[ml * LDC + nl] = acc[i][j] * sc + bias;
    }
  }
  __syncthreads();
  row_pass<BM, BN, kEpiStore>(sC, m0, n0, g, wave, lane);
}

// The fused MLP with its up-projection in FP8: the XN8 tile and the W1 chunks
// are e4m3 in LDS, GELU(acc * a_scale[token] * w1_scale + b1) goes to LDS in
// BF16 and the down-projection runs in BF16 as in k_mlp_bf16.
template <int BM, int D, int FCH, int EPI>
__global__ __launch_bounds__(256) void k_mlp_fp8(GemmArgs g, const uint8_t* __restrict__ W1, float w1_scale,
                                                 const float* __restrict__ b1, const bf16* __restrict__ W2, int F) {
  constexpr int LDA = D + 16, LDH = FCH + GPAD, LDW1 = D + 16, LDW2 = FCH + GPAD;
  constexpr int TI1 = FCH / 32, TJ1 = BM / 32;
  constexpr int TI2 = D / 32, TJ2 = BM / 32;
  constexpr int PW1 = FCH * D / 16 / 256;        // 16-byte chunks per thread of a W1 chunk (e4m3)
  constexpr int PW2 = D * FCH / 8 / 256;
  constexpr size_t a = (size_t)BM * LDA, h = (size_t)BM * LDH * 2, w1 = (size_t)FCH * LDW1,
                   w2 = (size_t)D * LDW2 * 2, cst = (size_t)BM * (D + 4) * 4;
  constexpr size_t loop = a + h + w1 + w2;
  __shared__ __attribute__((aligned(16))) char smem[loop > cst ? loop : cst];
  uint8_t* sA = (uint8_t*)smem;
  bf16* sH = (bf16*)(smem + a);
  uint8_t* sW1 = (uint8_t*)(smem + a + h);
  bf16* sW2 = (bf16*)(smem + a + h + w1);
  float* sC = (float*)smem;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const long m0 = (long)blockIdx.x * BM;
  const uint8_t* A = (const uint8_t*)g.A;
  i32x4 pw1[PW1];
  bf16x8 pw2[PW2];
  auto fetchW = [&](int c0) {
#pragma unroll
    for (int i = 0; i < PW1; ++i) {
      const int idx = tid + i * 256, row = idx / (D / 16), kc = (idx - row * (D / 16)) * 16;
      pw1[i] = *(const i32x4*)(W1 + (long)(c0 + row) * D + kc);
    }
#pragma unroll
    for (int i = 0; i < PW2; ++i) {
      const int idx = tid + i * 256, row = idx / (FCH / 8), kc = (idx - row * (FCH / 8)) * 8;
      pw2[i] = *(const bf16x8*)(W2 + (long)row * F + c0 + kc);
    }
  };
  auto stashW = [&]() {
#pragma unroll
    for (int i = 0; i < PW1; ++i) {
      const int idx = tid + i * 256, row = idx / (D / 16), kc = (idx - row * (D / 16)) * 16;
      *(i32x4*)&sW1[row * LDW1 + kc] = pw1[i];
    }
#pragma unroll
    for (int i = 0; i < PW2; ++i) {
      const int idx = tid + i * 256, row = idx / (FCH / 8), kc = (idx - row * (FCH / 8)) * 8;
      *(bf16x8*)&sW2[row * LDW2 + kc] = pw2[i];
    }
  };
  auto frag8 = [&](const uint8_t* p) {
    const i32x4 lo = *(const i32x4*)p, hi = *(const i32x4*)(p + 16);
    return i32x8{lo[0], lo[1], lo[2], lo[3], hi[0], hi[1], hi[2], hi[3]};
  };
  fetchW(0);
  constexpr int CPR = D / 16;
  for (int idx = tid; idx < BM * CPR; idx += 256) {
    const int row = idx / CPR, kc = (idx - row * CPR) * 16;
    const long gm = m0 + row;
    i32x4 v = i32x4{0, 0, 0, 0};
    if (gm < g.M) v = *(const i32x4*)(A + gm * D + kc);
    *(i32x4*)&sA[row * LDA + kc] = v;
  }
  stashW();
  __syncthreads();
  f32x4 acc2[TI2][TJ2];
#pragma unroll
  for (int i = 0; i < TI2; ++i)
#pragma unroll
    for (int j = 0; j < TJ2; ++j) acc2[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int wn1 = (wave >> 1) * (FCH / 2), wm = (wave & 1) * (BM / 2), wn2 = (wave >> 1) * (D / 2);
  float tsc[TJ1];
#pragma unroll
  for (int j = 0; j < TJ1; ++j) {
    const long m = m0 + wm + j * 16 + (lane & 15);
    tsc[j] = (m < g.M ? g.a_scale[m] : 0.f) * w1_scale;
  }
  for (int c0 = 0; c0 < F; c0 += FCH) {
    const bool more = c0 + FCH < F;
    if (more) fetchW(c0 + FCH);
    f32x4 acc1[TI1][TJ1];
#pragma unroll
    for (int i = 0; i < TI1; ++i)
#pragma unroll
      for (int j = 0; j < TJ1; ++j) acc1[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int ks = 0; ks < D; ks += 128) {
      i32x8 fw[TI1], fa[TJ1];
#pragma unroll
      for (int i = 0; i < TI1; ++i) fw[i] = frag8(&sW1[(wn1 + i * 16 + (lane & 15)) * LDW1 + ks + (lane >> 4) * 32]);
#pragma unroll
      for (int j = 0; j < TJ1; ++j) fa[j] = frag8(&sA[(wm + j * 16 + (lane & 15)) * LDA + ks + (lane >> 4) * 32]);
#pragma unroll
      for (int i = 0; i < TI1; ++i)
#pragma unroll
        for (int j = 0; j < TJ1; ++j)
          acc1[i][j] = __builtin_amdgcn_mfma_scale_f32_16x16x128_f8f6f4(fw[i], fa[j], acc1[i][j], 0, 0, 0, 127, 0, 127);
    }
#pragma unroll
    for (int i = 0; i < TI1; ++i) {
      const int hn = wn1 + i * 16 + (lane >> 4) * 4;
      f32x4 bb;
#pragma unroll
      for (int r = 0; r < 4; ++r) bb[r] = b1[c0 + hn + r];
#pragma unroll
      for (int j = 0; j < TJ1; ++j) {
        const int ml = wm + j * 16 + (lane & 15);
        const f32x4 v = acc1[i][j] * tsc[j] + bb;
        bf16x4 hv = {(bf16)gelu_f(v[0]), (bf16)gelu_f(v[1]), (bf16)gelu_f(v[2]), (bf16)gelu_f(v[3])};
        *(bf16x4*)&sH[ml * LDH + hn] = hv;
      }
    }
    __syncthreads();
#pragma unroll
    for (int ks = 0; ks < FCH; ks += 32) {
      bf16x8 fw[TI2], fh[TJ2];
#pragma unroll
      for (int i = 0; i < TI2; ++i) fw[i] = *(const bf16x8*)&sW2[(wn2 + i * 16 + (lane & 15)) * LDW2 + ks + (lane >> 4) * 8];
#pragma unroll
      for (int j = 0; j < TJ2; ++j) fh[j] = *(const bf16x8*)&sH[(wm + j * 16 + (lane & 15)) * LDH + ks + (lane >> 4) * 8];
#pragma unroll
      for (int i = 0; i < TI2; ++i)
#pragma unroll
        for (int j = 0; j < TJ2; ++j) acc2[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[i], fh[j], acc2[i][j], 0, 0, 0);
    }
    __syncthreads();
    if (more) {
      stashW();
      __syncthreads();
    }
  }
  constexpr int LDC = D + 4;
#pragma unroll
  for (int i = 0; i < TI2; ++i) {
    const int nl = wn2 + i * 16 + (lane >> 4) * 4;
    f32x4 bias;
#pragma unroll
    for (int r = 0; r < 4; ++r) bias[r] = g.bias[nl + r];
#pragma unroll
    for (int j = 0; j < TJ2; ++j) {
      const int ml = wm + j * 16 + (lane & 15);
      *(f32x4*)&sC[ml * LDC + nl] = acc2[i][j] + bias;
    }
  }
  __syncthreads();
  row_pass<BM, D, EPI>(sC, m0, 0, g, wave, lane);
}

template <int BM, int D, int FCH>
hipError_t mlp8_t(const GemmArgs& g, const Mat& W1, const float* b1, const Mat& W2, int F, hipStream_t s) {
  if (F % FCH != 0) return hipErrorInvalidValue;
  dim3 grid((unsigned)((g.M + BM - 1) / BM)), block(256);
  if (g.proj_out)
    hipLaunchKernelGGL((k_mlp_fp8<BM, D, FCH, kEpiResidProj>), grid, block, 0, s, g, W1.f8, W1.f8_scale, b1, W2.b16, F);
  else if (g.ln_g && g.out_scale)
    hipLaunchKernelGGL((k_mlp_fp8<BM, D, FCH, kEpiResidLN8>), grid, block, 0, s, g, W1.f8, W1.f8_scale, b1, W2.b16, F);
  else
    hipLaunchKernelGGL((k_mlp_fp8<BM, D, FCH, kEpiResid>), grid, block, 0, s, g, W1.f8, W1.f8_scale, b1, W2.b16, F);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_gemm_fp8(const GemmArgs& g, const Mat& W, hipStream_t s) {
  if (g.M == 0) return hipSuccess;
  if (g.Kd % 128 != 0 || g.N % 128 != 0 || !W.f8 || !g.a_scale) return hipErrorInvalidValue;
  dim3 grid((unsigned)(((g.M + 127) / 128) * (g.N / 128))), block(256);
  hipLaunchKernelGGL((k_gemm_fp8<128, 128>), grid, block, 0, s, g, W.f8, W.f8_scale);
  return hipGetLastError();
}

hipError_t launch_mlp_fp8(const GemmArgs& g, const Mat& W1, const float* b1, const Mat& W2, int F, hipStream_t s) {
  if (g.M == 0) return hipSuccess;
  if (!W1.f8 || !g.a_scale) return hipErrorInvalidValue;
  switch (g.N) {
    case 128: return mlp8_t<64, 128, 64>(g, W1, b1, W2, F, s);
    case 256: return mlp8_t<64, 256, 64>(g, W1, b1, W2, F, s);
    case 384: return mlp8_t<32, 384, 64>(g, W1, b1, W2, F, s);
    case 512: return mlp8_t<32, 512, 32>(g, W1, b1, W2, F, s);
    default: return hipErrorInvalidValue;
  }
}

// ---------------------------------------------------------------------------
// Row attention on MFMA, streaming the keys.  One workgroup per (row, head,
// block of 64 QT queries); each wave owns QT tiles of 16 queries.  The row's
// keys and values pass through LDS 64 at a time (K [key][dh] and V^T
// [dh][key] of the chunk; the next chunk is read into registers while the
// current one is used), and for each of its query tiles a wave forms
//   S^T = K Q^T       (A = keys from LDS, B = the tile's queries)
//   O^T += V^T P^T    (A = values from LDS, B = probabilities)
// so a lane keeps one query (lane % 16): its running max, its sum and its
// output columns; the online-softmax rescale is applied in FP32.  LDS does
// not grow with n, so several workgroups share a CU at any row length; each
// query sees the keys in the same 64-key blocks from 0 up.
namespace {

constexpr int AKB = 64;   // keys per MFMA block (and per LDS chunk)
constexpr int AQT = 2;    // query tiles of 16 per wave

template <int DH>
__global__ __launch_bounds__(256) void k_row_attn_mfma(StepCtx c, const bf16* __restrict__ QKV, bf16* __restrict__ O,
                                                       int d, int heads) {
  constexpr int DT = DH / 16;                    // output column blocks
  constexpr int QE = (DH == 16) ? 4 : 8;         // dh elements per lane per MFMA
  constexpr int QS = (DH == 64) ? 2 : 1;         // MFMA k-steps over dh
  constexpr int LDK = DH + 8, LDV = AKB + 8;
  constexpr int NPC = AKB * DH / 8;              // 8-element pieces of K (and of V) per chunk
  constexpr int CPT = (NPC + 255) / 256;         // per thread
  typedef __bf16 qv_t __attribute__((__vector_size__(QE * sizeof(__bf16))));
  __shared__ __attribute__((aligned(16))) bf16 sK[AKB * LDK];
  __shared__ __attribute__((aligned(16))) bf16 sVt[DH * LDV];
  const int lb = xcd_logical((int)blockIdx.x, (int)gridDim.x);
  const int r = c.row_first + lb / heads, h = lb - (lb / heads) * heads;
  const DevBin& b = c.bins[c.row_bin[r]];
  if (b.st->phase == kDone) return;
  const int n = b.n, k = r - b.row_off;
  const int qb = blockIdx.y * (64 * AQT);
  if (qb >= n) return;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const long tok0 = (long)b.tok_off + (long)k * n;
  const long ld = 3L * d;
  // scores are scaled by log2(e)/sqrt(dh) so the softmax uses exp2 (one v_exp_f32)
  const float scale = 1.4426950408889634f / sqrtf((float)DH);

  bf16x8 pk[CPT], pv[CPT];
  auto fetch = [&](int j0) {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int idx = tid + i * 256, key = idx / (DH / 8), c8 = (idx - key * (DH / 8)) * 8;
      pk[i] = pv[i] = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
      if (idx < NPC && j0 + key < n) {
        const bf16* base = QKV + (tok0 + j0 + key) * ld + h * DH + c8;
        pk[i] = *(const bf16x8*)(base + d);
        pv[i] = *(const bf16x8*)(base + 2 * d);
      }
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int i = 0; i < CPT; ++i) {
      const int idx = tid + i * 256, key = idx / (DH / 8), c8 = (idx - key * (DH / 8)) * 8;
      if (idx >= NPC) continue;
      *(bf16x8*)&sK[key * LDK + c8] = pk[i];
#pragma unroll
      for (int e = 0; e < 8; ++e) sVt[(c8 + e) * LDV + key] = pv[i][e];
    }
  };

  qv_t fq[AQT][QS];
  float mrun[AQT], lsum[AQT];
  f32x4 oacc[AQT][DT];
#pragma unroll
  for (int a = 0; a < AQT; ++a) {
    const int q = qb + (wave * AQT + a) * 16 + (lane & 15);
#pragma unroll
    for (int s = 0; s < QS; ++s) {
      if (q < n) {
        fq[a][s] = *(const qv_t*)(QKV + (tok0 + q) * ld + h * DH + s * 32 + (lane >> 4) * QE);
      } else {
#pragma unroll
        for (int e = 0; e < QE; ++e) fq[a][s][e] = (bf16)0.f;
      }
    }
    mrun[a] = -INFINITY;
    lsum[a] = 0.f;
#pragma unroll
    for (int t = 0; t < DT; ++t) oacc[a][t] = f32x4{0.f, 0.f, 0.f, 0.f};
  }

  fetch(0);
  for (int j0 = 0; j0 < n; j0 += AKB) {
    stash();
    __syncthreads();
    if (j0 + AKB < n) fetch(j0 + AKB);
#pragma unroll
    for (int a = 0; a < AQT; ++a) {
      if (qb + (wave * AQT + a) * 16 >= n) continue;   // the tile holds no query (uniform per wave)
      // scores of 64 keys: lane holds keys j0 + 16 t + 4 (lane/16) + rr of its query
      f32x4 st[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        f32x4 acc = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < QS; ++s) {
          const qv_t fk = *(const qv_t*)&sK[(t * 16 + (lane & 15)) * LDK + s * 32 + (lane >> 4) * QE];
          if constexpr (DH == 16) acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fk, fq[a][s], acc, 0, 0, 0);
          else acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fk, fq[a][s], acc, 0, 0, 0);
        }
        st[t] = acc;
      }
      // raw scores; keys past n (only in the last block) get -inf
      if (j0 + AKB > n) {
#pragma unroll
        for (int t = 0; t < 4; ++t)
#pragma unroll
          for (int rr = 0; rr < 4; ++rr)
            if (j0 + t * 16 + (lane >> 4) * 4 + rr >= n) st[t][rr] = -INFINITY;
      }
      float bmax = -INFINITY;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) bmax = fmaxf(bmax, st[t][rr]);
      bmax = fmaxf(bmax, __shfl_xor(bmax, 16, 64));
      bmax = xhalf_max(bmax);
      // running max kept in scaled units: p = 2^(scale s - m), one FMA and one v_exp_f32
      const float mnew = fmaxf(mrun[a], bmax * scale);
      const float corr = __builtin_amdgcn_exp2f(mrun[a] - mnew);
      float psum = 0.f;
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          const float p = __builtin_amdgcn_exp2f(fmaf(st[t][rr], scale, -mnew));
          st[t][rr] = p;
          psum += p;
        }
      psum += __shfl_xor(psum, 16, 64);
      psum = xhalf_sum(psum);
      lsum[a] = lsum[a] * corr + psum;
      mrun[a] = mnew;
#pragma unroll
      for (int t = 0; t < DT; ++t) oacc[a][t] = oacc[a][t] * corr;
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        bf16x8 fp;
#pragma unroll
        for (int rr = 0; rr < 4; ++rr) {
          fp[rr] = (bf16)st[2 * u][rr];
          fp[4 + rr] = (bf16)st[2 * u + 1][rr];
        }
#pragma unroll
        for (int t = 0; t < DT; ++t) {
          const bf16* vrow = &sVt[(t * 16 + (lane & 15)) * LDV];
          const bf16x4 v0 = *(const bf16x4*)(vrow + (2 * u) * 16 + (lane >> 4) * 4);
          const bf16x4 v1 = *(const bf16x4*)(vrow + (2 * u + 1) * 16 + (lane >> 4) * 4);
          bf16x8 fv = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
          oacc[a][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fv, fp, oacc[a][t], 0, 0, 0);
        }
      }
    }
    __syncthreads();                              // every wave is done with this chunk
  }
#pragma unroll
  for (int a = 0; a < AQT; ++a) {
    const int q = qb + (wave * AQT + a) * 16 + (lane & 15);
    if (q < n) {
      const float inv = 1.0f / lsum[a];
#pragma unroll
      for (int t = 0; t < DT; ++t) {
        const f32x4 v = oacc[a][t] * inv;
        bf16x4 hv = {(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
        *(bf16x4*)(O + (tok0 + q) * d + h * DH + t * 16 + (lane >> 4) * 4) = hv;
      }
    }
  }
}

}  // namespace

// LDS of the row attention: one 64-key chunk of K and V^T, whatever n is.
size_t row_attn_mfma_lds(int max_n, int dh) {
  (void)max_n;
  return (size_t)AKB * (dh + 8) * 2 + (size_t)dh * (AKB + 8) * 2;
}

hipError_t launch_row_attn_mfma(const StepCtx& c, const void* QKV, void* O, int d, int heads, int max_n,
                                hipStream_t s) {
  if (c.total_rows == 0) return hipSuccess;
  const int dh = d / heads;
  dim3 grid((unsigned)(c.total_rows * heads), (unsigned)((max_n + 64 * AQT - 1) / (64 * AQT))), block(256);
  if (dh == 16) hipLaunchKernelGGL((k_row_attn_mfma<16>), grid, block, 0, s, c, (const bf16*)QKV, (bf16*)O, d, heads);
  else if (dh == 32) hipLaunchKernelGGL((k_row_attn_mfma<32>), grid, block, 0, s, c, (const bf16*)QKV, (bf16*)O, d, heads);
  else if (dh == 64) hipLaunchKernelGGL((k_row_attn_mfma<64>), grid, block, 0, s, c, (const bf16*)QKV, (bf16*)O, d, heads);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace cider
