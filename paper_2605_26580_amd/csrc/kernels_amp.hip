// Slot-wise AMP-MMSE detector (Appendix, slot-wise AMP-MMSE detector;
// sensing-matrix construction) for gfx950, FP32.
//
// For each slot: Y = A U + eps in C^{n_s}, A[j][a] = w^{(R_j a) mod Q} / sqrt(n_s)
// with w = exp(-2 pi i / Q) (n_s rows R of the Q-point DFT), and the
// Bernoulli-Gaussian prior (1 - rho) delta_0 + rho CN(0, su2) on each U_a.
// AMP from U_hat = 0, Y_res = Y, for i < iters:
//   nu = ||Y_res||^2 / n_s,  R = U_hat + A^H Y_res,
//   U_hat' = eta(R),  Y_res' = Y - A U_hat' + Y_res / n_s * sum_a eta'(R_a),
// with eta(r) = p(r) su2 / (nu + su2) r, p the posterior activity, eta' the
// complex divergence c + t c' of eta(r) = c(t) r, t = |r|^2; then R and nu once
// more and S_a = log p(R_a; nu).
//
// One wave per slot: lane a holds coordinate a (R_a, U_hat_a; Q <= 64) and
// lane j holds measurement j (Y_j, Y_res_j, R_j; n_s <= 64).  The two
// matrix-vector products read the other side's vector from the wave's LDS
// row (a broadcast per step) and A's entries from a table of the Q roots of
// unity, indexed by (R_j a) mod Q: A is never stored.  The work per slot is
// 2 Q n_s complex multiply-adds per iteration, ALU-bound; slots are
// independent, four per workgroup.
#include "cider_internal.h"
#include "device_math.h"

namespace cider {

namespace {

constexpr int kAmpWaves = 4;


// x mod Q for 0 <= x < 2^22: the quotient from a float reciprocal with half a
// unit of headroom, so that no rounding of x / Q lands on the wrong integer.
__device__ __forceinline__ int mod_q(int x, int Q, float invQ) {
  return x - Q * (int)(((float)x + 0.5f) * invQ);
}

// log of the posterior activity for |r|^2 = t, and the activity itself:
// L = log(rho / (1 - rho)) + log(nu / (nu + su2)) + t (1/nu - 1/(nu + su2)),
// p = 1 / (1 + e^-L), log p = min(L, 0) - log1p(e^-|L|).
struct Activity {
  float logp, p;
};
__device__ __forceinline__ Activity activity(float t, float lodds0, float delta) {
  const float L = lodds0 + t * delta;
  const float e = expf(-fabsf(L));
  Activity a;
  a.logp = fminf(L, 0.f) - log1pf(e);
  a.p = L >= 0.f ? 1.0f / (1.0f + e) : e / (1.0f + e);
  return a;
}

// DPP lane moves within 16-lane rows (gfx9 encodings): quad_perm [1,0,3,2]
// = xor 1, [2,3,0,1] = xor 2, [3,2,1,0] = xor 3; row_half_mirror = xor 7
// within 8 lanes; row_mirror = xor 15 within 16.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ float2 dpp2(float2 v) {
  return make_float2(dpp<CTRL>(v.x), dpp<CTRL>(v.y));
}

// Sum over the wave, every lane ending with the same value: butterflies at
// distances 1, 2, 4, 8 (DPP; each step adds a lane and its partner, so both
// compute the same sum), then the row and half-wave swaps.
__device__ __forceinline__ float wave_sum64(float v) {
  v += dpp<0xb1>(v);
  v += dpp<0x4e>(v);
  v += dpp<0x141>(dpp<0x1b>(v));
  v += dpp<0x140>(dpp<0x141>(v));
  const unsigned a = __float_as_uint(v);
  const auto r = __builtin_amdgcn_permlane16_swap(a, a, false, false);
  v = __uint_as_float(r[0]) + __uint_as_float(r[1]);
  return xhalf_sum(v);
}

// The value of lane l ^ D, without LDS: DPP below 16, the row and half-wave
// swaps (v_permlane16_swap / v_permlane32_swap: applied to a value in both
// operands they return, in every lane, the value of the even and of the odd
// row / half at that position) at 16 and 32.
template <int D>
__device__ __forceinline__ float2 xor_lane(float2 v, int lane) {
  if constexpr (D == 1) {
    return dpp2<0xb1>(v);
  } else if constexpr (D == 2) {
    return dpp2<0x4e>(v);
  } else if constexpr (D == 4) {
    return dpp2<0x141>(dpp2<0x1b>(v));            // (x ^ 3) ^ 7
  } else if constexpr (D == 8) {
    return dpp2<0x140>(dpp2<0x141>(v));           // (x ^ 7) ^ 15
  } else {
    static_assert(D == 16 || D == 32, "lane distance");
    unsigned ax = __float_as_uint(v.x), ay = __float_as_uint(v.y);
    if constexpr (D == 16) {
      const auto rx = __builtin_amdgcn_permlane16_swap(ax, ax, false, false);
      const auto ry = __builtin_amdgcn_permlane16_swap(ay, ay, false, false);
      const bool odd = lane & 16;
      return make_float2(__uint_as_float(odd ? rx[0] : rx[1]), __uint_as_float(odd ? ry[0] : ry[1]));
    } else {
      const auto rx = __builtin_amdgcn_permlane32_swap(ax, ax, false, false);
      const auto ry = __builtin_amdgcn_permlane32_swap(ay, ay, false, false);
      const bool hi = lane & 32;
      return make_float2(__uint_as_float(hi ? rx[0] : rx[1]), __uint_as_float(hi ? ry[0] : ry[1]));
    }
  }
}

template <int S>
__device__ __forceinline__ float2 butterfly(float2 x, int lane, float2 w) {
  constexpr int d = 32 >> S;
  const float2 y = xor_lane<d>(x, lane);
  if (lane & d) {                                 // (a - b) w, this lane holding b
    const float tx = y.x - x.x, ty = y.y - x.y;
    return make_float2(tx * w.x - ty * w.y, tx * w.y + ty * w.x);
  }
  return make_float2(x.x + y.x, x.y + y.y);      // a + b
}

// 64-point DFT across the wave, one value per lane, radix-2 decimation in
// frequency: X[k] = sum_n x[n] w^(+-nk), w = exp(-2 pi i / 64), the sign
// negative for the forward transform.  Lane n ends with X[bitrev6(n)].
// twd[s]: this lane's twiddle w^e of the stage of span d = 32 >> s, e =
// (lane mod d) * 32 / d.
__device__ __forceinline__ float2 fft64(float2 x, int lane, const float2 (&twd)[6], bool inverse) {
  auto tw_s = [&](int s) { return make_float2(twd[s].x, inverse ? -twd[s].y : twd[s].y); };
  x = butterfly<0>(x, lane, tw_s(0));
  x = butterfly<1>(x, lane, tw_s(1));
  x = butterfly<2>(x, lane, tw_s(2));
  x = butterfly<3>(x, lane, tw_s(3));
  x = butterfly<4>(x, lane, tw_s(4));
  x = butterfly<5>(x, lane, tw_s(5));
  return x;
}

__global__ __launch_bounds__(64 * kAmpWaves) void k_amp_evidence(AmpArgs g) {
  __shared__ float2 tw[64];                       // w^k = exp(-2 pi i k / Q)
  __shared__ float2 vec[kAmpWaves][64];           // the wave's broadcast vector
  __shared__ int srow[kAmpWaves][64];             // the slot's DFT rows
  __shared__ float sx[kAmpWaves][64], sy[kAmpWaves][64];   // Q = 64: the scattered residual
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int Q = g.Q, ns = g.ns;
  if (tid < Q) {
    float sn, cs;
    sincospif(2.0f * (float)tid / (float)Q, &sn, &cs);
    tw[tid] = make_float2(cs, -sn);
  }
  __syncthreads();                                // the only workgroup barrier
  const long slot = (long)blockIdx.x * kAmpWaves + wave;
  if (slot >= g.slots) return;                    // whole wave
  const float inv_sqrt_ns = 1.0f / sqrtf((float)ns), invQ = 1.0f / (float)Q;
  const bool mj = lane < ns, ma = lane < Q;
  float2 y = make_float2(0.f, 0.f);
  int rj = 0;
  if (mj) {
    y = ((const float2*)g.y)[slot * ns + lane];
    rj = g.rows[slot * ns + lane] % Q;
    rj += rj < 0 ? Q : 0;
  }
  srow[wave][lane] = rj;
  const float lrho = logf(g.rho) - log1pf(-g.rho), su2 = g.su2;
  // Q = 64: both products as 64-point FFTs across the wave (the partial DFT is
  // rows R of the full one): A U_hat = FFT(U_hat) at rows R, A^H Y_res = the
  // inverse FFT of Y_res scattered to rows R (repeated rows add up)
  const bool fft = Q == 64;
  const int brev = (int)(__builtin_bitreverse32((unsigned)lane) >> 26);
  float2 twd[6];
#pragma unroll
  for (int s6 = 0; s6 < 6; ++s6) {
    const int d = 32 >> s6;
    twd[s6] = fft ? tw[(lane & (d - 1)) * (32 / d)] : make_float2(1.f, 0.f);
  }
  float2 res = y, uh = make_float2(0.f, 0.f), R = make_float2(0.f, 0.f);
  float nu = 1.f;
  for (int it = 0;; ++it) {
    // nu and R = U_hat + A^H Y_res (lane a; conj(A[j][a]) = conj(w^{(R_j a) mod Q}) / sqrt(n_s))
    nu = wave_sum64(res.x * res.x + res.y * res.y) / (float)ns;
    float2 acc = make_float2(0.f, 0.f);
    if (fft) {
      sx[wave][lane] = 0.f;
      sy[wave][lane] = 0.f;
      __builtin_amdgcn_wave_barrier();
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      if (mj) {
        atomicAdd(&sx[wave][rj], res.x);
        atomicAdd(&sy[wave][rj], res.y);
      }
      __builtin_amdgcn_wave_barrier();
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      const float2 V = fft64(make_float2(sx[wave][lane], sy[wave][lane]), lane, twd, true);
      vec[wave][brev] = V;                        // natural order
      __builtin_amdgcn_wave_barrier();
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      acc = vec[wave][lane];
      __builtin_amdgcn_wave_barrier();            // read before the next write of vec
      asm volatile("" ::: "memory");
    } else {
    vec[wave][lane] = res;
    __builtin_amdgcn_wave_barrier();
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    if (ma) {
      for (int j = 0; j < ns; ++j) {
        const float2 v = vec[wave][j];
        const float2 w = tw[mod_q(srow[wave][j] * lane, Q, invQ)];   // conj(w) v
        acc.x = fmaf(w.x, v.x, fmaf(w.y, v.y, acc.x));
        acc.y = fmaf(w.x, v.y, fmaf(-w.y, v.x, acc.y));
      }
    }
    }
    R = make_float2(uh.x + acc.x * inv_sqrt_ns, uh.y + acc.y * inv_sqrt_ns);
    if (it == g.iters) break;
    // denoiser and its divergence
    const float lodds0 = lrho + logf(nu / (nu + su2));
    const float delta = 1.0f / nu - 1.0f / (nu + su2), s = su2 / (nu + su2);
    const float t = R.x * R.x + R.y * R.y;
    const Activity act = activity(t, lodds0, delta);
    const float2 un = ma ? make_float2(act.p * s * R.x, act.p * s * R.y) : make_float2(0.f, 0.f);
    const float dv = ma ? s * act.p * (1.0f + t * (1.0f - act.p) * delta) : 0.f;
    const float D = wave_sum64(dv);
    // Y_res' = Y - A U_hat' + Y_res D / n_s (lane j; A[j][a] = w^{(R_j a) mod Q} / sqrt(n_s))
    __builtin_amdgcn_wave_barrier();              // every lane has read the residual row
    asm volatile("" ::: "memory");
    float2 au = make_float2(0.f, 0.f);
    if (fft) {
      const float2 X = fft64(un, lane, twd, false);
      vec[wave][brev] = X;                        // natural order
      __builtin_amdgcn_wave_barrier();
      asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
      if (mj) au = vec[wave][rj];
    } else {
    vec[wave][lane] = un;
    __builtin_amdgcn_wave_barrier();
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    if (mj) {
      for (int a = 0; a < Q; ++a) {
        const float2 v = vec[wave][a];
        const float2 w = tw[mod_q(rj * a, Q, invQ)];   // w v
        au.x = fmaf(w.x, v.x, fmaf(-w.y, v.y, au.x));
        au.y = fmaf(w.x, v.y, fmaf(w.y, v.x, au.y));
      }
    }
    }
    const float c = D / (float)ns;
    res = mj ? make_float2(y.x - au.x * inv_sqrt_ns + res.x * c, y.y - au.y * inv_sqrt_ns + res.y * c)
             : make_float2(0.f, 0.f);
    uh = un;
    __builtin_amdgcn_wave_barrier();              // every lane has read U_hat' before the next write
    asm volatile("" ::: "memory");
  }
  if (ma) {
    const float lodds0 = lrho + logf(nu / (nu + su2));
    const float delta = 1.0f / nu - 1.0f / (nu + su2);
    g.S[slot * Q + lane] = activity(R.x * R.x + R.y * R.y, lodds0, delta).logp;
  }
}

}  // namespace

hipError_t launch_amp_evidence(const AmpArgs& g, hipStream_t s) {
  if (g.slots == 0) return hipSuccess;
  if (g.ns < 1 || g.ns > 64 || g.Q < 2 || g.Q > 64 || g.iters < 0 || !g.y || !g.rows || !g.S)
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)((g.slots + kAmpWaves - 1) / kAmpWaves)), block(64 * kAmpWaves);
  hipLaunchKernelGGL(k_amp_evidence, grid, block, 0, s, g);
  return hipGetLastError();
}

}  // namespace cider
