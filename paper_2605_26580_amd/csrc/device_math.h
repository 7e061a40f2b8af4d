// Device math shared by the BF16 / FP8 kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace cider {

// GELU(x) = x Phi(x), written as max(x, 0) - |x| Q(|x|) with Q(u) = 1 - Phi(u)
// the Gaussian upper tail.  log2 Q(u) is smooth on [0, 6], so Q is taken as
// 2^h(u) with h a degree-4 polynomial fitted here to minimise the largest
// error of the GELU itself (the fit weights the error in h by u Q(u)), and u
// is clamped at 6, beyond which |x| Q(|x|) is below 1e-8.  The largest
// |error| over [-60, 60] in FP32 is 6.4e-6, far below the BF16 / FP8
// rounding of the hidden values it feeds.  It costs seven VALU operations and
// one hardware transcendental (2^x); the FP32 plain path keeps the erf form.
// Finite inputs only: +inf gives NaN.
__device__ __forceinline__ float gelu_f(float x) {
  const float u = __builtin_amdgcn_fmed3f(__builtin_fabsf(x), 0.0f, 6.0f);   // min(|x|, 6)
  const float h = fmaf(fmaf(fmaf(fmaf(0.0038685805f, u, -0.044090267f), u, -0.46799760f), u,
                            -1.1473827f), u, -1.0004778f);
  const float relu = __builtin_amdgcn_fmed3f(x, 0.0f, 3.4028235e38f);     // max(x, 0)
  return fmaf(-__builtin_fabsf(x), __builtin_amdgcn_exp2f(h), relu);
}

// Logistic 1 / (1 + e^-v) from the hardware 2^x and 1/x (relative error a few
// FP32 ulps; e^-v overflowing to +inf gives 0).
__device__ __forceinline__ float sigmoid_f(float v) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-v * 1.4426950408889634f));
}

// Reductions across the two halves of a wave (lanes l and l ^ 32) without a
// trip through LDS: v_permlane32_swap, applied to x in both operands, returns
// in every lane the low half's x (first result) and the high half's x (second
// result) of that lane's position, so both halves get the same value.
__device__ __forceinline__ float xhalf_max(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return fmaxf(__uint_as_float(r[0]), __uint_as_float(r[1]));
}
__device__ __forceinline__ float xhalf_sum(float x) {
  const auto r = __builtin_amdgcn_permlane32_swap(__float_as_uint(x), __float_as_uint(x), false, false);
  return __uint_as_float(r[0]) + __uint_as_float(r[1]);
}

}  // namespace cider
