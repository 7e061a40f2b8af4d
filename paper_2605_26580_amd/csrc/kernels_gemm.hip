// Token-wise GEMMs of the denoiser on the gfx950 matrix cores.
//
//   out[m, n] = epi( sum_k pro(A)[m, k] W[n, k] + bias[n] )
//
// A is the packed token matrix (rows = tokens of every bin), W a weight
// matrix in PyTorch layout [N][Kd].  Prologue: none, or LayerNorm over the
// Kd columns of an FP32 A (statistics computed by the workgroup for its own
// rows).  Epilogues: store, GELU + store, residual add into the FP32 stream
// R, or the Module A gate blend R = g R + (1 - g) E with g = sigmoid(.).
//
// Tiling: 64 x 64 output tile per workgroup of four wavefronts, each wave a
// 32 x 32 sub-tile of 2 x 2 MFMA 16x16 blocks; K in slices of 32 staged in
// LDS.  BF16 uses v_mfma_f32_16x16x32_bf16 (one instruction per slice),
// FP32 v_mfma_f32_16x16x4_f32 (eight per slice).  Every output element is
// accumulated in the same order whatever tile it falls in, so a token's
// result does not depend on which other tokens share its batch.
#include "cider_internal.h"

namespace cider {

namespace {

constexpr int BM = 64, BN = 64, BK = 32;

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ float gelu_f(float x) { return 0.5f * x * (1.0f + erff(x * 0.70710678118654752f)); }

template <typename TC> struct Tr;
template <> struct Tr<float> { static constexpr int PAD = 4; };
template <> struct Tr<bf16> { static constexpr int PAD = 8; };

template <typename TC>
__device__ __forceinline__ TC to_c(float v) { return (TC)v; }

template <typename TC, int PRO, int EPI>
__global__ __launch_bounds__(256) void k_gemm(GemmArgs g, const TC* __restrict__ W) {
  constexpr int PAD = Tr<TC>::PAD;
  __shared__ __attribute__((aligned(16))) TC As[BM][BK + PAD];
  __shared__ __attribute__((aligned(16))) TC Bs[BN][BK + PAD];
  __shared__ float s_mean[BM], s_rstd[BM];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const long m0 = (long)blockIdx.x * BM;
  const int n0 = blockIdx.y * BN;
  const int Kd = g.Kd;

  if (PRO == kProLN) {
    const float* A = (const float*)g.A;
    for (int rr = 0; rr < BM / 4; ++rr) {
      const int row = wave * (BM / 4) + rr;
      const long gm = m0 + row;
      float sum = 0.f;
      if (gm < g.M)
        for (int c = lane; c < Kd; c += 64) sum += A[gm * Kd + c];
      const float mean = wave_sum(sum) / (float)Kd;
      float sq = 0.f;
      if (gm < g.M)
        for (int c = lane; c < Kd; c += 64) {
          float dx = A[gm * Kd + c] - mean;
          sq = fmaf(dx, dx, sq);
        }
      const float var = wave_sum(sq) / (float)Kd;
      if (lane == 0) {
        s_mean[row] = mean;
        s_rstd[row] = 1.0f / sqrtf(var + 1e-5f);
      }
    }
    __syncthreads();
  }

  f32x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};
  const int wr = wave >> 1, wc = wave & 1;
  const int lrow = tid >> 2, lk = (tid & 3) * 8;

  for (int k0 = 0; k0 < Kd; k0 += BK) {
    {  // A slice: thread loads 8 consecutive k of one row
      const long gm = m0 + lrow;
      TC vals[8];
      if (gm < g.M) {
        if (PRO == kProLN) {
          const float* src = (const float*)g.A + gm * Kd + k0 + lk;
          const float mean = s_mean[lrow], rstd = s_rstd[lrow];
#pragma unroll
          for (int i = 0; i < 8; ++i)
            vals[i] = to_c<TC>((src[i] - mean) * rstd * g.ln_g[k0 + lk + i] + g.ln_b[k0 + lk + i]);
        } else {
          const TC* src = (const TC*)g.A + gm * Kd + k0 + lk;
#pragma unroll
          for (int i = 0; i < 8; ++i) vals[i] = src[i];
        }
      } else {
#pragma unroll
        for (int i = 0; i < 8; ++i) vals[i] = to_c<TC>(0.f);
      }
#pragma unroll
      for (int i = 0; i < 8; ++i) As[lrow][lk + i] = vals[i];
    }
    {  // W slice
      const TC* src = W + (long)(n0 + lrow) * Kd + k0 + lk;
#pragma unroll
      for (int i = 0; i < 8; ++i) Bs[lrow][lk + i] = src[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      const int ar = wr * 32 + i * 16 + (lane & 15);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        const int bc = wc * 32 + j * 16 + (lane & 15);
        if constexpr (sizeof(TC) == 2) {
          bf16x8 a = *(const bf16x8*)&As[ar][(lane >> 4) * 8];
          bf16x8 b = *(const bf16x8*)&Bs[bc][(lane >> 4) * 8];
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
        } else {
#pragma unroll
          for (int s = 0; s < BK / 4; ++s) {
            float a = As[ar][s * 4 + (lane >> 4)];
            float b = Bs[bc][s * 4 + (lane >> 4)];
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[i][j], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }

  // epilogue: lane holds rows 4*(lane/16)+r, column lane%16 of each 16x16 block
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int col = n0 + wc * 32 + j * 16 + (lane & 15);
      const float bias = g.bias ? g.bias[col] : 0.f;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const long row = m0 + wr * 32 + i * 16 + (lane >> 4) * 4 + r;
        if (row >= g.M) continue;
        const float v = acc[i][j][r] + bias;
        const long o = row * g.N + col;
        if (EPI == kEpiStore) {
          ((TC*)g.out)[o] = to_c<TC>(v);
        } else if (EPI == kEpiGelu) {
          ((TC*)g.out)[o] = to_c<TC>(gelu_f(v));
        } else if (EPI == kEpiResid) {
          g.R[o] = g.R[o] + v;
        } else {
          const float gt = 1.0f / (1.0f + expf(-v));
          g.R[o] = gt * g.R[o] + (1.0f - gt) * g.E[o];
        }
      }
    }
}

template <typename TC>
hipError_t gemm_t(int pro, int epi, const GemmArgs& g, const TC* W, hipStream_t s) {
  dim3 grid((unsigned)((g.M + BM - 1) / BM), (unsigned)(g.N / BN)), block(256);
#define GEMM_CASE(P, E) \
  if (pro == P && epi == E) { hipLaunchKernelGGL((k_gemm<TC, P, E>), grid, block, 0, s, g, W); return hipGetLastError(); }
  GEMM_CASE(kProNone, kEpiStore)
  GEMM_CASE(kProNone, kEpiGelu)
  GEMM_CASE(kProNone, kEpiResid)
  GEMM_CASE(kProNone, kEpiGate)
  GEMM_CASE(kProLN, kEpiStore)
  GEMM_CASE(kProLN, kEpiGelu)
#undef GEMM_CASE
  return hipErrorInvalidValue;
}

}  // namespace

hipError_t launch_gemm(int prec, int pro, int epi, const GemmArgs& g, const Mat& W, hipStream_t s) {
  if (g.M == 0) return hipSuccess;
  if (g.N % BN != 0 || g.Kd % BK != 0) return hipErrorInvalidValue;
  if (prec == kF32) return gemm_t<float>(pro, epi, g, W.f32, s);
  return gemm_t<bf16>(pro, epi, g, W.b16, s);
}

}  // namespace cider
