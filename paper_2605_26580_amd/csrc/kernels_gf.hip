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
// The butterflies and sums exchange lanes through DPP and the row and
// half-wave swaps; only the two coefficient gathers go through the LDS
// crossbar.
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

// Lane exchange at xor distance D without the LDS crossbar: DPP moves
// within 16-lane rows (quad_perm [1,0,3,2] = xor 1, [2,3,0,1] = xor 2,
// [3,2,1,0] = xor 3; row_half_mirror = xor 7 within 8 lanes; row_mirror =
// xor 15 within 16), so xor 4 = (xor 3) then (xor 7) and xor 8 = (xor 7)
// then (xor 15); the row swap (permlane16) gives xor 16, the half-wave swap
// (permlane32) xor 32.
template <int CTRL>
__device__ __forceinline__ float gf_dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}

template <int D>
__device__ __forceinline__ float xor_lane_gf(float v, int lane) {
  if constexpr (D == 1) {
    return gf_dpp<0xb1>(v);
  } else if constexpr (D == 2) {
    return gf_dpp<0x4e>(v);
  } else if constexpr (D == 4) {
    return gf_dpp<0x141>(gf_dpp<0x1b>(v));
  } else if constexpr (D == 8) {
    return gf_dpp<0x140>(gf_dpp<0x141>(v));
  } else {
    static_assert(D == 16 || D == 32, "lane distance");
    const unsigned a = __float_as_uint(v);
    if constexpr (D == 16) {
      const auto r = __builtin_amdgcn_permlane16_swap(a, a, false, false);
      return __uint_as_float((lane & 16) ? r[0] : r[1]);
    } else {
      const auto r = __builtin_amdgcn_permlane32_swap(a, a, false, false);
      return __uint_as_float((lane & 32) ? r[0] : r[1]);
    }
  }
}

template <int D>
__device__ __forceinline__ float wht_stage(float v, int lane) {
  const float o = xor_lane_gf<D>(v, lane);
  return (lane & D) ? o - v : v + o;
}

// unnormalised Walsh-Hadamard transform across the wave (lane = index)
__device__ __forceinline__ float wht64(float v, int lane) {
  v = wht_stage<1>(v, lane);
  v = wht_stage<2>(v, lane);
  v = wht_stage<4>(v, lane);
  v = wht_stage<8>(v, lane);
  v = wht_stage<16>(v, lane);
  return wht_stage<32>(v, lane);
}

__device__ __forceinline__ float wave_sum_gf(float v, int lane) {
  v += xor_lane_gf<1>(v, lane);
  v += xor_lane_gf<2>(v, lane);
  v += xor_lane_gf<4>(v, lane);
  v += xor_lane_gf<8>(v, lane);
  v += xor_lane_gf<16>(v, lane);
  return v + xor_lane_gf<32>(v, lane);
}

__global__ __launch_bounds__(64 * kGfWaves) void k_gf64_check(GfCheckArgs g) {
  __shared__ float sT[kGfWaves][kGfMaxDeg][64];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const long j = (long)blockIdx.x * kGfWaves + wave;
  if (j >= g.checks) return;
  const long e0 = g.row_ptr[j], e1 = g.row_ptr[j + 1];
  const int dc = (int)(e1 - e0);
  if (e0 < 0 || e1 > g.edges || dc < 1 || dc > kGfMaxDeg) return;   // malformed row: left unwritten
  // lane i < dc holds edge i's coefficient and its inverse; the input
  // gathers of eight edges are issued together before their transforms
  const int myal = lane < dc ? (g.coef[e0 + lane] & 63) : 1;
  const int myinv = gf64_inv(myal);
  for (int i0 = 0; i0 < dc; i0 += 8) {
    float q[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int i = i0 + u;
      q[u] = 0.f;
      if (i < dc) q[u] = g.p[(e0 + i) * 64 + gf64_mul(__shfl(myinv, i, 64), lane)];   // q(b) = p(alpha^-1 b)
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (i0 + u < dc) sT[wave][i0 + u][lane] = wht64(q[u], lane);
  }
  for (int o = 0; o < dc; ++o) {
    float prod = 1.0f;
    for (int i = 0; i < dc; ++i)
      if (i != o) prod *= sT[wave][i][lane];
    const float s = wht64(prod, lane) * (1.0f / 64.0f);    // distribution of the others' sum
    const int al = __shfl(myal, o, 64);
    const float v = __shfl(s, gf64_mul(al, lane), 64);      // m_o(a) = s(alpha_o a)
    const float tot = wave_sum_gf(v, lane);
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
