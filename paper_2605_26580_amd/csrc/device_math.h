// Device math shared by the BF16 / FP8 kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>

namespace cider {

// GELU(x) = x Phi(x) with Phi(x) written as a logistic of an odd polynomial,
// Phi(x) ~ 1 / (1 + 2^f(x)), f(x) = c x (a0 + a2 x^2 + a4 x^4), c = -log2 e,
// coefficients fitted here for the least maximum error against x Phi(x) with
// the polynomial's argument clamped to [-10, 10] (beyond it Phi is 0 or 1 to
// FP32 precision).  The largest |error| over [-40, 40] in FP32 is 2.6e-5, far
// below the BF16 / FP8 rounding of the hidden values it feeds.  It costs seven
// VALU operations and the two hardware transcendentals (2^x, 1/x); the FP32
// plain path keeps the erf form.
__device__ __forceinline__ float gelu_f(float x) {
  const float xc = __builtin_amdgcn_fmed3f(x, -10.0f, 10.0f);   // clamp, one v_med3_f32
  const float s = xc * xc;
  const float f = xc * fmaf(fmaf(0.0010142630f, s, -0.10677572f), s, -2.3011212f);
  return x * __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(f));
}

// Logistic 1 / (1 + e^-v) from the hardware 2^x and 1/x (relative error a few
// FP32 ulps; e^-v overflowing to +inf gives 0).
__device__ __forceinline__ float sigmoid_f(float v) {
  return __builtin_amdgcn_rcpf(1.0f + __builtin_amdgcn_exp2f(-v * 1.4426950408889634f));
}

}  // namespace cider
