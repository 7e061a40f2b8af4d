// Check-node update of the GF(64) parity layer (Q-ary LDPC code over
// GF(64); FFT-BP's check update in the Walsh-Hadamard domain).
//
// For a check sum_i alpha_i x_i = 0 and each of its edges o, the message to
// variable o is m_o(a) proportional to the probability that the other
// variables' weighted sum equals alpha_o a.  In characteristic 2 the sum is
// a XOR, so the distribution of a sum is the XOR-convolution of the
// summands' distributions, a pointwise product after a Walsh-Hadamard
// transform.  One wave per check, lane a = symbol a: each incoming edge
// distribution is permuted by its coefficient (lane b reads symbol
// alpha^-1 b), transformed in-wave with six xor-lane butterflies and kept
// in LDS; each outgoing message is the product of the other edges'
// transforms, transformed back, read at lane alpha_o a and normalised.
// FP32.  Field: polynomial basis, primitive polynomial x^6 + x + 1.
#include "cider_internal.h"

namespace cider {
namespace {

constexpr int kGfWaves = 4;
constexpr int kGfMaxDeg = 32;

__device__ __forceinline__ int gf64_mul(int a, int b) {
  int r = 0;
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    if (b & 1) r ^= a;
    b >>= 1;
    a <<= 1;
    if (a & 64) a ^= 0x43;    // x^6 = x + 1
  }
  return r;
}

// alpha^-1 = alpha^62 (the multiplicative group has order 63); 0 maps to 0
__device__ __forceinline__ int gf64_inv(int a) {
  int r = 1, p = a;
#pragma unroll
  for (int e = 62, i = 0; i < 6; ++i, e >>= 1) {
    if (e & 1) r = gf64_mul(r, p);
    p = gf64_mul(p, p);
  }
  return r;
}

// unnormalised Walsh-Hadamard transform across the wave (lane = index)
__device__ __forceinline__ float wht64(float v, int lane) {
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const float o = __shfl_xor(v, d, 64);
    v = (lane & d) ? o - v : v + o;
  }
  return v;
}

__device__ __forceinline__ float wave_sum_gf(float v) {
#pragma unroll
  for (int d = 32; d > 0; d >>= 1) v += __shfl_xor(v, d, 64);
  return v;
}

__global__ __launch_bounds__(64 * kGfWaves) void k_gf64_check(GfCheckArgs g) {
  __shared__ float sT[kGfWaves][kGfMaxDeg][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long j = (long)blockIdx.x * kGfWaves + wave;
  if (j >= g.checks) return;
  const long e0 = g.row_ptr[j], e1 = g.row_ptr[j + 1];
  const int dc = (int)(e1 - e0);
  if (e0 < 0 || e1 > g.edges || dc < 1 || dc > kGfMaxDeg) return;   // malformed row: left unwritten
  for (int i = 0; i < dc; ++i) {
    const int al = g.coef[e0 + i] & 63;
    const float q = g.p[(e0 + i) * 64 + gf64_mul(gf64_inv(al), lane)];   // q(b) = p(alpha^-1 b)
    sT[wave][i][lane] = wht64(q, lane);
  }
  for (int o = 0; o < dc; ++o) {
    float prod = 1.0f;
    for (int i = 0; i < dc; ++i)
      if (i != o) prod *= sT[wave][i][lane];
    const float s = wht64(prod, lane) * (1.0f / 64.0f);    // distribution of the others' sum
    const int al = g.coef[e0 + o] & 63;
    const float v = __shfl(s, gf64_mul(al, lane), 64);      // m_o(a) = s(alpha_o a)
    const float tot = wave_sum_gf(v);
    g.out[(e0 + o) * 64 + lane] = v / tot;
  }
}

}  // namespace

hipError_t launch_gf64_check(const GfCheckArgs& g, hipStream_t s) {
  if (g.checks <= 0) return hipSuccess;
  const long blocks = (g.checks + kGfWaves - 1) / kGfWaves;
  hipLaunchKernelGGL(k_gf64_check, dim3((unsigned)blocks), dim3(64 * kGfWaves), 0, s, g);
  return hipGetLastError();
}

}  // namespace cider
