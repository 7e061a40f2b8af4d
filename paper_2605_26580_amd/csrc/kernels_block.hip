// Fused attention blocks for the BF16 path (gfx950).
//
// One pre-LN attention sublayer of the denoiser (QKV projection, softmax
// attention over one axis of the K x n grid, output projection, residual
// update, and the LayerNorm that feeds the next sublayer) runs as ONE kernel.
// A workgroup owns a set of token slots whose attention stays inside the set:
//   row attention  - the n <= 128 tokens of one row of one bin (128 slots);
//   user attention - whole columns of one bin (64 slots in 16-slot tiles,
//                    each tile holding floor(16/K) columns of K tokens).
// Phase 1 projects every slot to Q, K, V with the slot tile in LDS and the
// weights fed straight from L2 into the MFMA A operand; K and V^T stay in
// LDS and Q replaces the input tile.  Phase 2 gives each wave one 16-slot
// query tile: scores, exp2 softmax and P V for every head, with the O tile
// kept in registers.  Phase 3 stages W_o in LDS (over the dead Q/K/V
// buffers); each wave applies the output projection, bias, residual and
// LayerNorm to its tile in registers and writes R and the next XN.  Q, K, V
// and O never reach HBM: per token the sublayer reads XN and R and writes R
// and XN, the same bytes as the output-projection GEMM alone.
//
// MFMA conventions (16x16 blocks, 64-lane wave): output lane l, register r
// holds row 4(l/16) + r, column l%16; operand lane l holds row (A) / column (B)
// l%16 and k-group l/16.  Where a fragment built from MFMA outputs feeds the
// k side of another MFMA, k-slot 8g + j of lane group g stands for element
// 4g + j of the first 16-block (j < 4) or 4g + j - 4 of the second, and the
// other operand is read with the same assignment, so each MFMA still forms
// the full dot product.
#include "cider_internal.h"
#include "device_math.h"

namespace cider {

namespace {

template <int NT, int D>
struct BlkSmem {
  static constexpr int LDX = D + 8, LDV = NT + 8, LDW = D + 8;
  static constexpr size_t tok = 128 * sizeof(int);
  static constexpr size_t x = (size_t)NT * LDX * 2;     // XN tile, then Q
  static constexpr size_t k = (size_t)NT * LDX * 2;     // K, all heads
  static constexpr size_t vt = (size_t)D * LDV * 2;     // V^T, all heads
  static constexpr size_t w = (size_t)D * LDW * 2;      // W_o (phase 3, over x|k|vt)
  static constexpr size_t bytes = tok + x + k + vt;
  static_assert(w <= x + k + vt, "W_o staging must fit in the Q/K/V buffers");
  static_assert(bytes <= 160 * 1024, "LDS");
};

__device__ __forceinline__ bf16x4 to_bf16x4(const f32x4 v) {
  return bf16x4{(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
}

// Row attention: one 512-thread workgroup per CU (105 KB of LDS at d = 128).
// User attention: 54 KB, so three 256-thread workgroups share a CU when each
// wave keeps to 168 registers.
template <int NT, int D, int DH, bool USER>
__global__ __launch_bounds__(NT * 4) __attribute__((amdgpu_waves_per_eu(USER && D <= 128 ? 3 : 2))) void k_attn_block(StepCtx c, bf16* XN, const bf16* __restrict__ Wqkv,
                                                       const float* __restrict__ bqkv, const bf16* __restrict__ Wo,
                                                       const float* __restrict__ bo, float* __restrict__ R,
                                                       const float* __restrict__ ln_g, const float* __restrict__ ln_b) {
  using S = BlkSmem<NT, D>;
  constexpr int NTHR = NT * 4, NW = NT / 16;     // threads, waves (= 16-slot tiles)
  constexpr int LDX = S::LDX, LDV = S::LDV, LDW = S::LDW;
  constexpr int HEADS = D / DH;
  constexpr int NB = 3 * D / 16;                 // 16-feature blocks of Q | K | V
  constexpr int FBW = (NB + NW - 1) / NW;        // blocks per wave in phase 1
  constexpr int QBW = (D / 16 + NW - 1) / NW;    // of those, ones that can be Q blocks
  constexpr int DT = DH / 16;                    // 16-blocks per head
  constexpr int OB = D / 16;
  constexpr int QE = DH == 16 ? 4 : 8;           // k elements per lane of a QK^T MFMA
  constexpr int QS = DH == 64 ? 2 : 1;           // QK^T k-steps
  typedef __bf16 qv_t __attribute__((__vector_size__(QE * sizeof(__bf16))));
  static_assert(D % 32 == 0 && DH % 16 == 0 && DH <= 64, "shape");
  __shared__ __attribute__((aligned(16))) char smem[S::bytes];
  int* sTok = (int*)smem;
  bf16* sX = (bf16*)(smem + S::tok);
  bf16* sK = sX + NT * LDX;
  bf16* sVt = sK + NT * LDX;
  bf16* sW = sX;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g4 = lane >> 4, l16 = lane & 15;

  int bi, l0 = 0;
  if (USER) {
    bi = c.ugrp[2 * blockIdx.x];
    l0 = c.ugrp[2 * blockIdx.x + 1];
  } else {
    bi = c.row_bin[c.row_first + blockIdx.x];
  }
  const DevBin& b = c.bins[bi];
  if (b.st->phase == kDone) return;            // whole workgroup, before any barrier
  const int n = b.n, K = b.K;
  const int cpt = USER ? 16 / K : 1;             // columns per tile (user attention)
  const int ntv = USER ? min(NW, (n - l0 + cpt - 1) / cpt) : (n + 15) / 16;   // tiles with valid slots
  if (tid < NT) {
    int tok = -1;
    if (USER) {
      const int t = tid >> 4, j = tid & 15, col = l0 + t * cpt + j / K;
      if (j < cpt * K && col < n) tok = b.tok_off + (j % K) * n + col;
    } else if (tid < n) {
      tok = b.tok_off + (c.row_first + (int)blockIdx.x - b.row_off) * n + tid;
    }
    sTok[tid] = tok;
  }
  __syncthreads();
  for (int idx = tid; idx < NT * (D / 8); idx += NTHR) {
    const int slot = idx / (D / 8), c8 = (idx - slot * (D / 8)) * 8;
    const int tok = sTok[slot];
    bf16x8 v = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
    if (tok >= 0) v = *(const bf16x8*)(XN + (long)tok * D + c8);
    *(bf16x8*)&sX[slot * LDX + c8] = v;
  }
  __syncthreads();

  // ---- phase 1: [Q | K | V] = X Wqkv^T + b for every slot ----
  // Passes of FP feature blocks bound the accumulators.  The inner loop is
  // branch-free: every tile is computed (slots past the valid ones hold zeros
  // and get the bias alone, finite and masked out as keys), and a block index
  // past NB recomputes block NB - 1 and is discarded.
  {
    constexpr int FP = 3;
    bf16x4 qkeep[QBW][NW];
#pragma unroll
    for (int i0 = 0; i0 < FBW; i0 += FP) {
      f32x4 acc[FP][NW];
      const bf16* wbase[FP];
#pragma unroll
      for (int j = 0; j < FP; ++j) {
        wbase[j] = Wqkv + (long)(min(wave + NW * (i0 + j), NB - 1) * 16 + l16) * D + g4 * 8;
#pragma unroll
        for (int t = 0; t < NW; ++t) acc[j][t] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
#pragma unroll
      for (int ks = 0; ks < D; ks += 32) {
        bf16x8 fw[FP], fx[NW];
#pragma unroll
        for (int j = 0; j < FP; ++j) fw[j] = *(const bf16x8*)(wbase[j] + ks);
#pragma unroll
        for (int t = 0; t < NW; ++t) fx[t] = *(const bf16x8*)&sX[(t * 16 + l16) * LDX + ks + g4 * 8];
#pragma unroll
        for (int j = 0; j < FP; ++j)
#pragma unroll
          for (int t = 0; t < NW; ++t) acc[j][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw[j], fx[t], acc[j][t], 0, 0, 0);
      }
      // lane holds features fb*16 + 4 g4 + r of slot 16 t + l16
#pragma unroll
      for (int j = 0; j < FP; ++j) {
        const int i = i0 + j;
        const int fb = wave + NW * i;
        if (i >= FBW || fb >= NB) continue;
        const int f = fb * 16 + g4 * 4;
        const f32x4 bias = f32x4{bqkv[f], bqkv[f + 1], bqkv[f + 2], bqkv[f + 3]};
#pragma unroll
        for (int t = 0; t < NW; ++t) {
          const bf16x4 hv = to_bf16x4(acc[j][t] + bias);
          const int slot = t * 16 + l16;
          if (f < D) {
            if (i < QBW) qkeep[i < QBW ? i : 0][t] = hv;
          } else if (f < 2 * D) {
            *(bf16x4*)&sK[slot * LDX + f - D] = hv;
          } else {
#pragma unroll
            for (int r = 0; r < 4; ++r) sVt[(f - 2 * D + r) * LDV + slot] = hv[r];
          }
        }
      }
    }
    __syncthreads();                             // every read of the X tile is done
#pragma unroll
    for (int i = 0; i < QBW; ++i) {
      const int f = (wave + NW * i) * 16 + g4 * 4;
      if (f >= D) continue;
#pragma unroll
      for (int t = 0; t < NW; ++t) *(bf16x4*)&sX[(t * 16 + l16) * LDX + f] = qkeep[i][t];
    }
    __syncthreads();
  }

  // ---- phase 2: attention for this wave's 16-slot query tile, all heads ----
  const bool live = wave < ntv;
  const int qslot = wave * 16 + l16;
  // W_o and this tile's residual rows are fetched now; their latency hides
  // behind the attention math
  constexpr int PWO = D * D / 8 / NTHR;          // 16-byte W_o chunks per thread
  static_assert(PWO * NTHR * 8 == D * D, "W_o chunks must split over the workgroup");
  bf16x8 pwo[PWO];
#pragma unroll
  for (int i = 0; i < PWO; ++i) pwo[i] = *(const bf16x8*)(Wo + (long)(tid + i * NTHR) * 8);
  constexpr bool PRE_R = D <= 128;
  const int tok = sTok[qslot];
  const bool tv = tok >= 0;
  float* Rrow = R + (long)(tv ? tok : 0) * D;
  f32x4 rpre[PRE_R ? OB : 1];
  if (PRE_R) {
#pragma unroll
    for (int ob = 0; ob < OB; ++ob)
      rpre[PRE_R ? ob : 0] = tv ? *(const f32x4*)(Rrow + ob * 16 + g4 * 4) : f32x4{0.f, 0.f, 0.f, 0.f};
  }
  bf16x4 ofr[OB];                                // O[16 b + 4 g4 + r][query slot]
  if (live) {
    // exp2 of scale * (s - max s), scale = log2(e)/sqrt(dh): one FMA and one
    // v_exp_f32 per score
    const float scale = 1.4426950408889634f / sqrtf((float)DH);
    float kbias[4] = {0.f, 0.f, 0.f, 0.f};       // user attention: -inf off the query's column
    if (USER) {
      const int col_lo = (l16 / K) * K;          // key slots of this lane's column
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jk = g4 * 4 + r;
        const bool ok = sTok[wave * 16 + jk] >= 0 && (unsigned)(jk - col_lo) < (unsigned)K;
        kbias[r] = ok ? 0.f : -INFINITY;
      }
    }
    const bool full = USER || n >= NT;           // row attention: no key past n
#pragma unroll
    for (int h = 0; h < HEADS; ++h) {
      qv_t fq[QS];
#pragma unroll
      for (int s = 0; s < QS; ++s) fq[s] = *(const qv_t*)&sX[qslot * LDX + h * DH + s * 32 + g4 * QE];
      f32x4 oacc[DT];
#pragma unroll
      for (int t = 0; t < DT; ++t) oacc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
      float lsum;
      if (!USER) {
        f32x4 st[NW];
#pragma unroll
        for (int kt = 0; kt < NW; ++kt) {
          f32x4 a = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
          for (int s = 0; s < QS; ++s) {
            const qv_t fk = *(const qv_t*)&sK[(kt * 16 + l16) * LDX + h * DH + s * 32 + g4 * QE];
            if constexpr (DH == 16) a = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fk, fq[s], a, 0, 0, 0);
            else a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fk, fq[s], a, 0, 0, 0);
          }
          st[kt] = a;
        }
        if (!full) {
#pragma unroll
          for (int kt = 0; kt < NW; ++kt)
#pragma unroll
            for (int r = 0; r < 4; ++r)
              if (kt * 16 + g4 * 4 + r >= n) st[kt][r] = -INFINITY;
        }
        float mx = -INFINITY;
#pragma unroll
        for (int kt = 0; kt < NW; ++kt)
#pragma unroll
          for (int r = 0; r < 4; ++r) mx = fmaxf(mx, st[kt][r]);
        mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
        mx = xhalf_max(mx);
        const float mxs = -mx * scale;
        float ps = 0.f;
#pragma unroll
        for (int kt = 0; kt < NW; ++kt)
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const float p = __builtin_amdgcn_exp2f(fmaf(st[kt][r], scale, mxs));
            st[kt][r] = p;
            ps += p;
          }
        ps += __shfl_xor(ps, 16, 64);
        ps = xhalf_sum(ps);
        lsum = ps;
#pragma unroll
        for (int u = 0; u < NW / 2; ++u) {
          const bf16x8 fp = {(bf16)st[2 * u][0],     (bf16)st[2 * u][1],     (bf16)st[2 * u][2],
                             (bf16)st[2 * u][3],     (bf16)st[2 * u + 1][0], (bf16)st[2 * u + 1][1],
                             (bf16)st[2 * u + 1][2], (bf16)st[2 * u + 1][3]};
#pragma unroll
          for (int t = 0; t < DT; ++t) {
            const bf16* vrow = &sVt[(h * DH + t * 16 + l16) * LDV + 32 * u + g4 * 4];
            const bf16x4 v0 = *(const bf16x4*)vrow;
            const bf16x4 v1 = *(const bf16x4*)(vrow + 16);
            const bf16x8 fv = {v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
            oacc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fv, fp, oacc[t], 0, 0, 0);
          }
        }
      } else {
        f32x4 a = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int s = 0; s < QS; ++s) {
          const qv_t fk = *(const qv_t*)&sK[(wave * 16 + l16) * LDX + h * DH + s * 32 + g4 * QE];
          if constexpr (DH == 16) a = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fk, fq[s], a, 0, 0, 0);
          else a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fk, fq[s], a, 0, 0, 0);
        }
        float mx = -INFINITY;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          a[r] = a[r] + kbias[r];
          mx = fmaxf(mx, a[r]);
        }
        mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
        mx = xhalf_max(mx);
        // a padding query slot has no valid key (mx = -inf): p = 0 for it
        const float mxs = mx == -INFINITY ? 0.f : -mx * scale;
        float ps = 0.f;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const float p = __builtin_amdgcn_exp2f(fmaf(a[r], scale, mxs));
          a[r] = p;
          ps += p;
        }
        ps += __shfl_xor(ps, 16, 64);
        ps = xhalf_sum(ps);
        lsum = ps;
        const bf16x4 fp = to_bf16x4(a);
#pragma unroll
        for (int t = 0; t < DT; ++t) {
          const bf16x4 fv = *(const bf16x4*)&sVt[(h * DH + t * 16 + l16) * LDV + wave * 16 + g4 * 4];
          oacc[t] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fv, fp, oacc[t], 0, 0, 0);
        }
      }
      const float inv = lsum > 0.f ? 1.0f / lsum : 0.f;
#pragma unroll
      for (int t = 0; t < DT; ++t) ofr[h * DT + t] = to_bf16x4(oacc[t] * inv);
    }
  }

  // ---- phase 3: W_o into LDS, then projection + residual + LayerNorm ----
  __syncthreads();                               // Q, K, V^T are dead
#pragma unroll
  for (int i = 0; i < PWO; ++i) {
    const int idx = tid + i * NTHR, row = idx / (D / 8), c8 = (idx - row * (D / 8)) * 8;
    *(bf16x8*)&sW[row * LDW + c8] = pwo[i];
  }
  __syncthreads();
  if (!live) return;                             // after the last barrier
  f32x4 acc2[OB];
#pragma unroll
  for (int ob = 0; ob < OB; ++ob) acc2[ob] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < D / 32; ++s) {
    const bf16x8 fo = {ofr[2 * s][0],     ofr[2 * s][1],     ofr[2 * s][2],     ofr[2 * s][3],
                       ofr[2 * s + 1][0], ofr[2 * s + 1][1], ofr[2 * s + 1][2], ofr[2 * s + 1][3]};
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      const bf16* wrow = &sW[(ob * 16 + l16) * LDW + 32 * s + g4 * 4];
      const bf16x4 w0 = *(const bf16x4*)wrow;
      const bf16x4 w1 = *(const bf16x4*)(wrow + 16);
      const bf16x8 fw = {w0[0], w0[1], w0[2], w0[3], w1[0], w1[1], w1[2], w1[3]};
      acc2[ob] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fw, fo, acc2[ob], 0, 0, 0);
    }
  }
  // lane: features 16 ob + 4 g4 + r of the token in query slot `qslot`; the
  // four lanes l16, l16+16, l16+32, l16+48 together hold the whole row
  float sum = 0.f;
#pragma unroll
  for (int ob = 0; ob < OB; ++ob) {
    const int f = ob * 16 + g4 * 4;
    const f32x4 bias = f32x4{bo[f], bo[f + 1], bo[f + 2], bo[f + 3]};
    f32x4 rr;
    if (PRE_R) rr = rpre[PRE_R ? ob : 0];
    else rr = tv ? *(const f32x4*)(Rrow + f) : f32x4{0.f, 0.f, 0.f, 0.f};
    const f32x4 res = rr + (acc2[ob] + bias);
    acc2[ob] = res;
    if (tv) *(f32x4*)(Rrow + f) = res;
    sum += (res[0] + res[1]) + (res[2] + res[3]);
  }
  sum += __shfl_xor(sum, 16, 64);
  sum = xhalf_sum(sum);
  const float mean = sum / (float)D;
  float q = 0.f;
#pragma unroll
  for (int ob = 0; ob < OB; ++ob)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float dv = acc2[ob][r] - mean;
      q = fmaf(dv, dv, q);
    }
  q += __shfl_xor(q, 16, 64);
  q = xhalf_sum(q);
  const float rstd = 1.0f / sqrtf(q / (float)D + 1e-5f);
  if (tv) {
    bf16* xrow = XN + (long)tok * D;
#pragma unroll
    for (int ob = 0; ob < OB; ++ob) {
      const int f = ob * 16 + g4 * 4;
      bf16x4 hv;
#pragma unroll
      for (int r = 0; r < 4; ++r) hv[r] = (bf16)((acc2[ob][r] - mean) * rstd * ln_g[f + r] + ln_b[f + r]);
      *(bf16x4*)(xrow + f) = hv;
    }
  }
}

template <int NT, int D, int DH, bool USER>
hipError_t blk_t(const StepCtx& c, int grid, bf16* XN, const DevLayer& L, const float* ln_g, const float* ln_b,
                 float* R, hipStream_t s) {
  const bf16* Wqkv = USER ? L.Wqkv_u.b16 : L.Wqkv_r.b16;
  const float* bqkv = USER ? L.bqkv_u : L.bqkv_r;
  const bf16* Wo = USER ? L.Wo_u.b16 : L.Wo_r.b16;
  const float* bo = USER ? L.bo_u : L.bo_r;
  hipLaunchKernelGGL((k_attn_block<NT, D, DH, USER>), dim3((unsigned)grid), dim3(NT * 4), 0, s, c, XN, Wqkv, bqkv,
                     Wo, bo, R, ln_g, ln_b);
  return hipGetLastError();
}

template <int NT, bool USER>
hipError_t blk_dispatch(const StepCtx& c, int grid, int d, int dh, bf16* XN, const DevLayer& L,
                        const float* ln_g, const float* ln_b, float* R, hipStream_t s) {
#define CIDER_BLK(DD, HH) \
  if (d == DD && dh == HH) return blk_t<NT, DD, HH, USER>(c, grid, XN, L, ln_g, ln_b, R, s);
  CIDER_BLK(64, 16) CIDER_BLK(64, 32) CIDER_BLK(64, 64)
  CIDER_BLK(128, 16) CIDER_BLK(128, 32) CIDER_BLK(128, 64)
  CIDER_BLK(192, 16) CIDER_BLK(192, 32) CIDER_BLK(192, 64)
#undef CIDER_BLK
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Attention across the K rows of a slot, from a QKV buffer (the unfused
// path: d = 256 / 384, FP8).  One wave per 16-slot tile of floor(16/K)
// columns x K rows (the fused user block's tiling, groups of four tiles from
// the same (bin, first column) table).  Per head: S^T = K Q^T is one MFMA
// with Q and K fragments read straight from QKV, keys off the query's column
// are masked, the exp2 softmax runs over the lane's four keys and its three
// partner lanes, and O^T = V^T P^T is one 16x16x16 MFMA per 16 features with
// V^T staged in LDS (d x 16 values, this wave's only LDS).
template <int DH>
__global__ __launch_bounds__(64) void k_user_attn_mfma(StepCtx c, const bf16* __restrict__ QKV, bf16* __restrict__ O,
                                                       int d, int heads) {
  constexpr int QE = DH == 16 ? 4 : 8;           // k elements per lane of a QK^T MFMA
  constexpr int QS = DH == 64 ? 2 : 1;           // QK^T k-steps
  constexpr int DT = DH / 16;
  constexpr int LDV = 16 + 8;
  typedef __bf16 qv_t __attribute__((__vector_size__(QE * sizeof(__bf16))));
  extern __shared__ __attribute__((aligned(16))) char smem_ua[];
  bf16* sVt = (bf16*)smem_ua;                     // [d][LDV]
  const int gi = blockIdx.x >> 2, sub = blockIdx.x & 3;
  const DevBin& b = c.bins[c.ugrp[2 * gi]];
  if (b.st->phase == kDone) return;
  const int K = b.K, n = b.n, cpt = 16 / K;
  const int col0 = c.ugrp[2 * gi + 1] + sub * cpt;
  if (col0 >= n) return;                          // whole wave
  const int lane = threadIdx.x, g4 = lane >> 4, l16 = lane & 15;
  const long ld = 3L * d;
  auto slot_tok = [&](int j) -> long {
    const int col = col0 + j / K;
    return (j < cpt * K && col < n) ? (long)b.tok_off + (long)(j % K) * n + col : -1L;
  };
  // V^T of the tile's 16 slots
  for (int e = lane; e < 16 * (d / 8); e += 64) {
    const int j = e / (d / 8), c8 = (e - j * (d / 8)) * 8;
    const long t = slot_tok(j);
    bf16x8 v = bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
    if (t >= 0) v = *(const bf16x8*)(QKV + t * ld + 2 * d + c8);
#pragma unroll
    for (int i = 0; i < 8; ++i) sVt[(c8 + i) * LDV + j] = v[i];
  }
  __syncthreads();
  const long tq = slot_tok(l16);                  // this lane's query row and key row
  const bool qv = tq >= 0;
  float kbias[4];
  const int col_lo = (l16 / K) * K;               // key slots of this lane's column
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int jk = g4 * 4 + r;
    kbias[r] = (slot_tok(jk) >= 0 && (unsigned)(jk - col_lo) < (unsigned)K) ? 0.f : -INFINITY;
  }
  const float scale = 1.4426950408889634f / sqrtf((float)DH);
  const bf16* qrow = QKV + (qv ? tq : 0) * ld;
  for (int h = 0; h < heads; ++h) {
    f32x4 a = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < QS; ++s) {
      qv_t fq, fk;
      if (qv) {
        fq = *(const qv_t*)(qrow + h * DH + s * 32 + g4 * QE);
        fk = *(const qv_t*)(qrow + d + h * DH + s * 32 + g4 * QE);
      } else {
#pragma unroll
        for (int e = 0; e < QE; ++e) fq[e] = fk[e] = (bf16)0.f;
      }
      if constexpr (DH == 16) a = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fk, fq, a, 0, 0, 0);
      else a = __builtin_amdgcn_mfma_f32_16x16x32_bf16(fk, fq, a, 0, 0, 0);
    }
    // a[r]: score of key slot 4 g4 + r for query slot l16
    float mx = -INFINITY;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] += kbias[r];
      mx = fmaxf(mx, a[r]);
    }
    mx = fmaxf(mx, __shfl_xor(mx, 16, 64));
    mx = xhalf_max(mx);
    const float mxs = mx == -INFINITY ? 0.f : -mx * scale;
    float ps = 0.f;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a[r] = __builtin_amdgcn_exp2f(fmaf(a[r], scale, mxs));
      ps += a[r];
    }
    ps += __shfl_xor(ps, 16, 64);
    ps = xhalf_sum(ps);
    const float inv = ps > 0.f ? 1.0f / ps : 0.f;
    const bf16x4 fp = to_bf16x4(a);
#pragma unroll
    for (int t = 0; t < DT; ++t) {
      const bf16x4 fv = *(const bf16x4*)&sVt[(h * DH + t * 16 + l16) * LDV + g4 * 4];
      f32x4 oacc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(fv, fp, f32x4{0.f, 0.f, 0.f, 0.f}, 0, 0, 0);
      // oacc[r]: feature h DH + 16 t + 4 g4 + r of query slot l16
      if (qv) *(bf16x4*)(O + tq * d + h * DH + t * 16 + g4 * 4) = to_bf16x4(oacc * inv);
    }
  }
}

}  // namespace

// Cross-user attention from QKV into O (BF16): four tiles per (bin, first
// column) group, one wave each.
hipError_t launch_user_attn_mfma(const StepCtx& c, const void* QKV, void* O, int d, int heads, hipStream_t s) {
  if (c.total_ugrp == 0) return hipSuccess;
  if (heads <= 0 || d % heads || d % 16) return hipErrorInvalidValue;
  const int dh = d / heads;
  const size_t lds = (size_t)d * (16 + 8) * sizeof(bf16);
  dim3 grid((unsigned)(4 * c.total_ugrp)), block(64);
  if (dh == 16) hipLaunchKernelGGL((k_user_attn_mfma<16>), grid, block, lds, s, c, (const bf16*)QKV, (bf16*)O, d, heads);
  else if (dh == 32) hipLaunchKernelGGL((k_user_attn_mfma<32>), grid, block, lds, s, c, (const bf16*)QKV, (bf16*)O, d, heads);
  else if (dh == 64) hipLaunchKernelGGL((k_user_attn_mfma<64>), grid, block, lds, s, c, (const bf16*)QKV, (bf16*)O, d, heads);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

bool attn_block_ok(int d, int heads, int max_n, bool user) {
  if (heads <= 0 || d % heads) return false;
  const int dh = d / heads;
  if (!(d == 64 || d == 128 || d == 192)) return false;
  if (!(dh == 16 || dh == 32 || dh == 64)) return false;
  return user || max_n <= kBlkRowSlots;
}

// Row attention: grid = one workgroup per row.  User attention: grid = the
// host-built (bin, first column) groups in c.ugrp.
hipError_t launch_attn_block(const StepCtx& c, bool user, void* XN, const DevLayer& L, const float* ln_g,
                             const float* ln_b, float* R, int d, int heads, hipStream_t s) {
  const int grid = user ? c.total_ugrp : c.total_rows;
  if (grid == 0) return hipSuccess;
  if (!attn_block_ok(d, heads, c.max_n, user)) return hipErrorInvalidValue;
  const int dh = d / heads;
  if (user) return blk_dispatch<kBlkUserSlots, true>(c, grid, d, dh, (bf16*)XN, L, ln_g, ln_b, R, s);
  return blk_dispatch<kBlkRowSlots, false>(c, grid, d, dh, (bf16*)XN, L, ln_g, ln_b, R, s);
}

}  // namespace cider
