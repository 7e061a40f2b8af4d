// The two attentions of a denoiser block.
//
// Row attention: every row k of a bin is a sequence over its n slots; h heads
// of width DH = d / h, scores scaled by 1/sqrt(DH), no mask.  One workgroup
// per (row, head, block of 256 queries); keys and values are streamed through
// LDS 64 at a time with an online softmax in FP32.
//
// User attention: every slot l of a bin is a sequence over its K rows (the
// cross-user demixing attention).  One thread per (slot, head, query row);
// K <= 16 keys, FP32 softmax.
//
// QKV holds per token [q (d) | k (d) | v (d)], head h at columns h*DH.. of
// each block; O receives the concatenated heads.
#include "cider_internal.h"

namespace cider {

namespace {

template <typename TC>
__device__ __forceinline__ float ld(const TC* p) { return (float)*p; }

constexpr int kQ = 256;   // queries per workgroup
constexpr int kKC = 64;   // keys per LDS chunk

template <typename TC, int DH>
__global__ __launch_bounds__(kQ) void k_row_attn(StepCtx c, const TC* __restrict__ QKV, TC* __restrict__ O,
                                                 int d, int heads) {
  __shared__ float s_k[kKC][DH + 1];
  __shared__ float s_v[kKC][DH + 1];
  const int item = blockIdx.x;
  const int r = item / heads, h = item - r * heads;
  const DevBin& b = c.bins[c.row_bin[r]];
  if (b.st->phase == kDone) return;
  const int n = b.n, k = r - b.row_off;
  const int q0 = blockIdx.y * kQ;
  if (q0 >= n) return;
  const long tok0 = (long)b.tok_off + (long)k * n;
  const int l = q0 + threadIdx.x;
  const bool valid = l < n;
  const float scale = 1.0f / sqrtf((float)DH);
  float q[DH], o[DH];
#pragma unroll
  for (int i = 0; i < DH; ++i) {
    q[i] = valid ? ld(QKV + (tok0 + l) * 3 * d + h * DH + i) * scale : 0.f;
    o[i] = 0.f;
  }
  float mrun = -INFINITY, lsum = 0.f;
  for (int j0 = 0; j0 < n; j0 += kKC) {
    const int nk = min(kKC, n - j0);
    for (int idx = threadIdx.x; idx < kKC * DH; idx += kQ) {
      int jj = idx / DH, ii = idx - jj * DH;
      float kv = 0.f, vv = 0.f;
      if (jj < nk) {
        const TC* base = QKV + (tok0 + j0 + jj) * 3 * d + h * DH + ii;
        kv = ld(base + d);
        vv = ld(base + 2 * d);
      }
      s_k[jj][ii] = kv;
      s_v[jj][ii] = vv;
    }
    __syncthreads();
    float sc[kKC];
    float cmax = -INFINITY;
#pragma unroll 8
    for (int jj = 0; jj < kKC; ++jj) {
      float a = 0.f;
#pragma unroll
      for (int i = 0; i < DH; ++i) a = fmaf(q[i], s_k[jj][i], a);
      sc[jj] = jj < nk ? a : -INFINITY;
      cmax = fmaxf(cmax, sc[jj]);
    }
    const float mnew = fmaxf(mrun, cmax);
    const float corr = expf(mrun - mnew);
    lsum *= corr;
#pragma unroll
    for (int i = 0; i < DH; ++i) o[i] *= corr;
#pragma unroll 8
    for (int jj = 0; jj < kKC; ++jj) {
      const float pj = expf(sc[jj] - mnew);
      lsum += pj;
#pragma unroll
      for (int i = 0; i < DH; ++i) o[i] = fmaf(pj, s_v[jj][i], o[i]);
    }
    mrun = mnew;
    __syncthreads();
  }
  if (valid) {
    const float inv = 1.0f / lsum;
#pragma unroll
    for (int i = 0; i < DH; ++i) O[(tok0 + l) * d + h * DH + i] = (TC)(o[i] * inv);
  }
}

template <typename TC, int DH>
__global__ __launch_bounds__(256) void k_user_attn(StepCtx c, const TC* __restrict__ QKV, TC* __restrict__ O,
                                                   int d, int heads) {
  // item = (slot, head, query row); rows beyond the bin's K exit
  const long item = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long per_slot = (long)heads * kMaxK;
  const long s = item / per_slot;
  if (s >= c.total_slots) return;
  const int rem = (int)(item - s * per_slot);
  const int h = rem / kMaxK, kq = rem - h * kMaxK;
  const DevBin& b = c.bins[c.slot_bin[s]];
  if (kq >= b.K || b.st->phase == kDone) return;
  const int n = b.n, l = (int)(s - b.slot_off), K = b.K;
  const long tq = (long)b.tok_off + (long)kq * n + l;
  const float scale = 1.0f / sqrtf((float)DH);
  float q[DH];
#pragma unroll
  for (int i = 0; i < DH; ++i) q[i] = ld(QKV + tq * 3 * d + h * DH + i) * scale;
  float sc[kMaxK];
  float mx = -INFINITY;
  for (int j = 0; j < K; ++j) {
    const long tk = (long)b.tok_off + (long)j * n + l;
    float a = 0.f;
#pragma unroll
    for (int i = 0; i < DH; ++i) a = fmaf(q[i], ld(QKV + tk * 3 * d + d + h * DH + i), a);
    sc[j] = a;
    mx = fmaxf(mx, a);
  }
  float o[DH];
#pragma unroll
  for (int i = 0; i < DH; ++i) o[i] = 0.f;
  float lsum = 0.f;
  for (int j = 0; j < K; ++j) {
    const long tk = (long)b.tok_off + (long)j * n + l;
    const float pj = expf(sc[j] - mx);
    lsum += pj;
#pragma unroll
    for (int i = 0; i < DH; ++i) o[i] = fmaf(pj, ld(QKV + tk * 3 * d + 2 * d + h * DH + i), o[i]);
  }
  const float inv = 1.0f / lsum;
#pragma unroll
  for (int i = 0; i < DH; ++i) O[tq * d + h * DH + i] = (TC)(o[i] * inv);
}

template <typename TC>
hipError_t row_t(const StepCtx& c, const void* QKV, void* O, int d, int heads, int max_n, hipStream_t s) {
  dim3 grid((unsigned)(c.total_rows * heads), (unsigned)((max_n + kQ - 1) / kQ)), block(kQ);
  const int dh = d / heads;
  if (dh == 16) hipLaunchKernelGGL((k_row_attn<TC, 16>), grid, block, 0, s, c, (const TC*)QKV, (TC*)O, d, heads);
  else if (dh == 32) hipLaunchKernelGGL((k_row_attn<TC, 32>), grid, block, 0, s, c, (const TC*)QKV, (TC*)O, d, heads);
  else if (dh == 64) hipLaunchKernelGGL((k_row_attn<TC, 64>), grid, block, 0, s, c, (const TC*)QKV, (TC*)O, d, heads);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename TC>
hipError_t user_t(const StepCtx& c, const void* QKV, void* O, int d, int heads, hipStream_t s) {
  const long items = (long)c.total_slots * heads * kMaxK;
  dim3 grid((unsigned)((items + 255) / 256)), block(256);
  const int dh = d / heads;
  if (dh == 16) hipLaunchKernelGGL((k_user_attn<TC, 16>), grid, block, 0, s, c, (const TC*)QKV, (TC*)O, d, heads);
  else if (dh == 32) hipLaunchKernelGGL((k_user_attn<TC, 32>), grid, block, 0, s, c, (const TC*)QKV, (TC*)O, d, heads);
  else if (dh == 64) hipLaunchKernelGGL((k_user_attn<TC, 64>), grid, block, 0, s, c, (const TC*)QKV, (TC*)O, d, heads);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace

hipError_t launch_row_attn(const StepCtx& c, int prec, const void* QKV, void* O, int d, int heads,
                           int max_n, hipStream_t s) {
  if (c.total_rows == 0) return hipSuccess;
  if (prec == kF32) return row_t<float>(c, QKV, O, d, heads, max_n, s);
  return row_t<bf16>(c, QKV, O, d, heads, max_n, s);
}

hipError_t launch_user_attn(const StepCtx& c, int prec, const void* QKV, void* O, int d, int heads,
                            hipStream_t s) {
  if (c.total_slots == 0) return hipSuccess;
  if (prec == kF32) return user_t<float>(c, QKV, O, d, heads, s);
  return user_t<bf16>(c, QKV, O, d, heads, s);
}

}  // namespace cider
