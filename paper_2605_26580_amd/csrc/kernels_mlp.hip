// Token-resident fused MLP for the BF16 path (gfx950).
//
//   R += W2 GELU(W1 XN + b1) + b2, then the next LayerNorm of R into XN
//   (or, after the last block, the final LayerNorm and the 2-way symbol
//   projection into lbar).
//
// A workgroup owns 256 tokens: NW waves of TB 32-token blocks each (at
// d = 128 and 256: 8 waves x 1 block, two waves per SIMD; TB = 2 halves the
// LDS reads per MFMA but leaves one wave per SIMD, which measured slower).
// Each wave keeps its XN rows in registers
// for the whole kernel as the B operand of v_mfma_f32_32x32x16_bf16 (lane l:
// token l%32 of a block, k-group l/32) and walks the hidden dimension in
// chunks of 32.  The chunk's W1 rows and W2 columns go
// from global memory straight into LDS (global_load_lds_dwordx4, no register
// staging), double-buffered, and every wave reads them as A operands:
//   up:    H[32 hidden][32 tokens]  = W1c[32][D] XN^T, D/16 MFMAs
//   GELU on the 16 values a lane holds, rounded to BF16;
//   down:  OUT[D][32 tokens] += W2c[D][32] H, 2 MFMAs per 32 output rows.
// The H block never leaves registers.  Output register r of lane l holds row
// 8(r/4) + 4(l/32) + r%4 of the up product; the W1 chunk is stored with its
// rows permuted (row j holds hidden unit sigma(j)) so that registers
// 8s..8s+7 of lane group l/32 hold hidden units 16s + 8(l/32) + 0..7 -- the
// k-values that group supplies to k-step s of the down MFMA, with W2 in its
// natural column order.
// Each DMA instruction fills 1 KB of LDS contiguously, 16 bytes per lane;
// rows are padded by 16 bytes (W1: D + 8 elements, W2: 40) so that the
// A-operand reads, lane base + a constant per k-step, are free of bank
// conflicts with 32 or 64 banks.  Lanes that land on a pad write a harmless
// copy; lanes past the end of a region are masked off.
#include "cider_internal.h"
#include "device_math.h"

namespace cider {

namespace {

typedef float f32x16 __attribute__((__vector_size__(16 * sizeof(float))));
typedef int i32x8 __attribute__((__vector_size__(8 * sizeof(int))));

constexpr int kM3BM = 256;                        // tokens per workgroup
constexpr int kM3FCH = 32;                        // hidden units per chunk

constexpr int kM3MaxF = 2048;                     // hidden width the b1 staging holds

template <int D, int NBUF = 2, int MAXF = kM3MaxF>
struct M3Smem {
  static constexpr int RB1 = D * 2 + 16;          // bytes per stored W1 chunk row (16 of them pad)
  static constexpr int RB2 = kM3FCH * 2 + 16;     // bytes per stored W2 chunk row
  static constexpr size_t w1 = (size_t)kM3FCH * RB1;
  static constexpr size_t w2 = (size_t)D * RB2;
  // regions on 16-byte boundaries (the DMA's LDS alignment); a region's last
  // DMA block masks the lanes past its end
  static constexpr size_t w1a = (w1 + 15) / 16 * 16;
  static constexpr size_t w2a = (w2 + 15) / 16 * 16;
  static constexpr size_t buf = w1a + w2a;
  static constexpr size_t vec = (size_t)5 * D * 4;           // epilogue vectors
  static constexpr size_t bytes = NBUF * buf + MAXF * 4 + vec;   // + all of b1
  static_assert(bytes <= 160 * 1024, "LDS");
};

// Waits until at most n of this wave's vector-memory operations (here: LDS
// DMA blocks of later weight chunks) are outstanding, then joins the
// workgroup barrier.  The count is an instruction immediate, so the
// uniform n selects one of a few fixed forms.
template <int N>
__device__ __forceinline__ void m3_wait_barrier_n() {
  asm volatile("s_waitcnt vmcnt(%0)" ::"n"(N) : "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}
__device__ __forceinline__ void m3_wait_barrier(int n) {
  switch (n) {
    case 0: m3_wait_barrier_n<0>(); break;
    case 1: m3_wait_barrier_n<1>(); break;
    case 2: m3_wait_barrier_n<2>(); break;
    case 3: m3_wait_barrier_n<3>(); break;
    case 4: m3_wait_barrier_n<4>(); break;
    case 5: m3_wait_barrier_n<5>(); break;
    case 6: m3_wait_barrier_n<6>(); break;
    case 7: m3_wait_barrier_n<7>(); break;
    case 8: m3_wait_barrier_n<8>(); break;
    case 9: m3_wait_barrier_n<9>(); break;
    case 10: m3_wait_barrier_n<10>(); break;
    case 11: m3_wait_barrier_n<11>(); break;
    case 12: m3_wait_barrier_n<12>(); break;
    default: m3_wait_barrier_n<0>(); break;
  }
}

// A run of N MFMAs whose A operands come from LDS, with each fragment read
// PF MFMAs ahead of its use (the scheduling barrier keeps that order, so each
// MFMA waits only for its own fragment, not for a read issued just before
// it).  ld(i) returns fragment i; op(i, w) issues MFMA i.
template <int N, int PF, class Ld, class Op>
__device__ __forceinline__ void mfma_pipe(Ld ld, Op op) {
  bf16x8 w[PF];
#pragma unroll
  for (int i = 0; i < PF; ++i)
    if (i < N) w[i] = ld(i);
#pragma unroll
  for (int i = 0; i < N; ++i) {
    op(i, w[i % PF]);
    if (i + PF < N) w[i % PF] = ld(i + PF);
    __builtin_amdgcn_sched_barrier(0);
  }
}

// Row j of the stored W1 chunk holds hidden unit sigma(j) of the chunk.
__device__ __forceinline__ int m3_sigma(int j) {
  const int q = j >> 3, g = (j >> 2) & 1, i = j & 3;
  return 16 * (q >> 1) + 8 * g + 4 * (q & 1) + i;
}

// One wave's share of the LDS DMA of an MLP weight chunk: rows sigma(0..31)
// of the chunk of W1 (row stride ld1) and the chunk's 32 columns of W2 (row
// stride ld2), as 1 KB blocks of 16 bytes per lane (rows padded to RB1 / RB2
// bytes; a pad lane copies something in bounds).  The per-lane source
// offsets relative to the chunk's first hidden unit are formed once (-1: the
// lane's bytes lie past its region), so a chunk costs one address add per
// block instead of a division by the row pitch.
template <int NW, int N1, int N2, int RB1, int RB2, int W1B, int W2B, int W1A, bool CACHE = true, int ES1 = 2>
struct M3ChunkDma {
  static constexpr int KM = (N1 + N2 + NW - 1) / NW;
  int off[CACHE ? KM : 1];
  int ld1_, ld2_, wave_, lane_;
  // offset of block k's lane within its chunk (constant divisors: the region
  // test is uniform across the wave)
  __device__ __forceinline__ int offset(int k) const {
    const int u = wave_ + NW * k;
    if (u < N1) {
      const int pos = u * 1024 + lane_ * 16, j = pos / RB1, o = pos - j * RB1;
      const bool data = o < RB1 - 16;
      return pos < W1B ? m3_sigma(data ? j : 0) * ld1_ + (data ? o / ES1 : 0) : -1;
    }
    const int pos = (u - N1) * 1024 + lane_ * 16, j = pos / RB2, o = pos - j * RB2;
    const bool data = o < RB2 - 16;
    return pos < W2B ? (data ? j : 0) * ld2_ + (data ? o / 2 : 0) : -1;
  }
  __device__ __forceinline__ void init(int wave, int lane, int ld1, int ld2) {
    ld1_ = ld1;
    ld2_ = ld2;
    wave_ = wave;
    lane_ = lane;
    if (CACHE) {
#pragma unroll
      for (int k = 0; k < KM; ++k) off[CACHE ? k : 0] = (wave + NW * k < N1 + N2) ? offset(k) : -1;
    }
  }
  // W1 holds ES1-byte elements (BF16, or e4m3 for the FP8 up projection)
  __device__ __forceinline__ void issue(const void* W1, const bf16* W2, int c0, char* base) const {
#pragma unroll
    for (int k = 0; k < KM; ++k) {
      const int u = wave_ + NW * k;
      if (u >= N1 + N2) break;
      const bool first = u < N1;
      const int o = CACHE ? off[CACHE ? k : 0] : offset(k);
      const void* src = first ? (const void*)((const char*)W1 + ((long)c0 * ld1_ + o) * ES1) : (const void*)(W2 + c0 + o);
      char* dst = base + (first ? u * 1024 : W1A + (u - N1) * 1024);
      if (o >= 0) __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
  }
};

// Per-feature vectors of the residual epilogue, staged in LDS at kernel
// start: bias [D], LayerNorm gain [D] and bias [D], and with the final
// projection its two rows [2][D].  Reading them from LDS keeps the
// epilogue's global traffic to the residual rows, whose loads can then all
// be issued ahead of the stores (nothing the stores write can alias them).
template <int D>
__device__ __forceinline__ void m3_stage_vectors(float* sv, const GemmArgs& g, bool proj, int tid, int nthr) {
  for (int i = tid; i < D; i += nthr) {
    sv[i] = g.bias[i];
    sv[D + i] = g.ln_g[i];
    sv[2 * D + i] = g.ln_b[i];
    if (proj) {
      sv[3 * D + i] = g.proj_w[i];
      sv[4 * D + i] = g.proj_w[D + i];
    }
  }
}

// Residual epilogue shared by the token-resident kernels: acc2[b][t] holds,
// for token tok0 + 32 t, output rows 32 b + 8 q + 4 g2 + i in register 4q + i
// (the two lanes l and l + 32 together hold the row).  R += acc2 + bias, then
// the next LayerNorm into g.out (BF16) or, with PROJ, the final LayerNorm and
// the 2-way projection into g.proj_out.  With GATE (Module A) the update is
// the gated blend R = s R + (1 - s) E, s = sigmoid(acc2 + bias), instead of
// R += acc2 + bias.  sv: the staged vectors.  Residual rows are loaded in
// batches of up to four output blocks, all loads of a batch issued before
// its stores.
template <int D, int TB, bool PROJ, bool GATE = false>
__device__ __forceinline__ void m3_residual_epilogue(f32x16 (&acc2)[D / 32][TB], long tok0, const GemmArgs& g,
                                                     int g2, const float* sv) {
  constexpr int OBK = D / 32;
  constexpr int HB = (GATE ? 2 : 4) < OBK ? (GATE ? 2 : 4) : OBK;   // output blocks per load batch
  const float* sbias = sv;
  const float* slg = sv + D;
  const float* slb = sv + 2 * D;
#pragma unroll
  for (int t = 0; t < TB; ++t) {
    const long tok = tok0 + 32 * t;
    const bool tv = tok < g.M;
    float* Rrow = g.R + (tv ? tok : 0) * D;
    const float* Erow = GATE ? g.E + (tv ? tok : 0) * D : nullptr;
    float sum = 0.f;
#pragma unroll
    for (int b0 = 0; b0 < OBK; b0 += HB) {
      f32x4 rr[HB][4], ee[GATE ? HB : 1][4];
#pragma unroll
      for (int bb = 0; bb < HB; ++bb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int f = 32 * (b0 + bb) + 8 * q + 4 * g2;
          rr[bb][q] = tv ? *(const f32x4*)(Rrow + f) : f32x4{0.f, 0.f, 0.f, 0.f};
          if (GATE) ee[GATE ? bb : 0][q] = tv ? *(const f32x4*)(Erow + f) : f32x4{0.f, 0.f, 0.f, 0.f};
        }
#pragma unroll
      for (int bb = 0; bb < HB; ++bb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int f = 32 * (b0 + bb) + 8 * q + 4 * g2;
          const f32x4 bias = *(const f32x4*)&sbias[f];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            float res;
            if (GATE) {
              const float gt = sigmoid_f(acc2[b0 + bb][t][4 * q + i] + bias[i]);
              res = gt * rr[bb][q][i] + (1.0f - gt) * ee[GATE ? bb : 0][q][i];
            } else {
              res = rr[bb][q][i] + (acc2[b0 + bb][t][4 * q + i] + bias[i]);
            }
            acc2[b0 + bb][t][4 * q + i] = res;
            sum += res;
          }
        }
      if (tv) {
#pragma unroll
        for (int bb = 0; bb < HB; ++bb)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int f = 32 * (b0 + bb) + 8 * q + 4 * g2;
            *(f32x4*)(Rrow + f) = f32x4{acc2[b0 + bb][t][4 * q], acc2[b0 + bb][t][4 * q + 1],
                                        acc2[b0 + bb][t][4 * q + 2], acc2[b0 + bb][t][4 * q + 3]};
          }
      }
    }
    sum = xhalf_sum(sum);
    const float mean = sum / (float)D;
    float qv = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float dv = acc2[b][t][r] - mean;
        qv = fmaf(dv, dv, qv);
      }
    qv = xhalf_sum(qv);
    const float rstd = 1.0f / sqrtf(qv / (float)D + 1e-5f);
    if (!PROJ) {
      if (tv) {
        bf16* xo = (bf16*)g.out + tok * D;
#pragma unroll
        for (int b = 0; b < OBK; ++b)
#pragma unroll
          for (int q = 0; q < 4; ++q) {
            const int f = 32 * b + 8 * q + 4 * g2;
            const f32x4 lg = *(const f32x4*)&slg[f];
            const f32x4 lb = *(const f32x4*)&slb[f];
            bf16x4 h;
#pragma unroll
            for (int i = 0; i < 4; ++i) h[i] = (bf16)((acc2[b][t][4 * q + i] - mean) * rstd * lg[i] + lb[i]);
            *(bf16x4*)(xo + f) = h;
          }
      }
    } else {
      const float* sp0 = sv + 3 * D;
      const float* sp1 = sv + 4 * D;
      float a0 = 0.f, a1 = 0.f;
#pragma unroll
      for (int b = 0; b < OBK; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int f = 32 * b + 8 * q + 4 * g2;
          const f32x4 lg = *(const f32x4*)&slg[f];
          const f32x4 lb = *(const f32x4*)&slb[f];
          const f32x4 w0 = *(const f32x4*)&sp0[f];
          const f32x4 w1 = *(const f32x4*)&sp1[f];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const float hv = (acc2[b][t][4 * q + i] - mean) * rstd * lg[i] + lb[i];
            a0 = fmaf(hv, w0[i], a0);
            a1 = fmaf(hv, w1[i], a1);
          }
        }
      a0 = xhalf_sum(a0);
      a1 = xhalf_sum(a1);
      if (tv && g2 == 0) {
        g.proj_out[2 * tok] = a0;
        g.proj_out[2 * tok + 1] = a1;
      }
    }
  }
}

// Row stores of a wave's 32 tokens held in the accumulator layout (lane
// (l32, g2) holds features 32 b + 8 q + 4 g2 + i of the wave's row l32 as
// value (b, q, i)) as whole 256-byte row segments, instead of 32- or 16-byte
// pieces of 32 rows per store instruction (a quarter of the cache lines per
// store).  The values pass through an 8 KB LDS slice of the wave: 32 rows of
// 256 bytes, the 16-byte pieces of row r stored at piece index XOR (r mod
// 16), so that the accumulator-layout writes (32 rows, one piece each) and
// the row-order reads (4 rows of 16 pieces) both spread over all banks.
// val(b, q) returns the lane's four values of block b, step q; rowtok(r) is
// the token of the wave's row r (lane r's token) or -1 (no store).  FP32 rows
// go out in D / 64 rounds of 64 columns, BF16 rows in D / 128 rounds of 128
// (pairs of steps exchanged between the wave's halves first, so that the
// BF16 slice is also written in whole 16-byte pieces: 8-byte writes to
// 16-byte slots would meet on the banks).
// RB = 128 gives 4 KB slices: 32 rows of 128 bytes (32 columns per round,
// pieces at index XOR (r mod 8), 8 rows per read instruction).
template <int D, int RB = 256, class Val, class RowTok>
__device__ __forceinline__ void rows_store_f32(Val val, float* dst, char* lds, int lane, RowTok rowtok) {
  static_assert(RB == 128 || RB == 256, "row segments of 128 or 256 bytes");
  constexpr int NP = RB / 16, CPR = RB / 4, BPR = RB / 128, RPI = 64 / NP;   // pieces/row, columns, blocks, rows
  static_assert(D % CPR == 0, "whole rounds");
  const int l32 = lane & 31, g2 = lane >> 5, sw = l32 & (NP - 1), rr = lane / NP, pp = lane % NP;
#pragma unroll
  for (int j = 0; j < D / CPR; ++j) {
#pragma unroll
    for (int bb = 0; bb < BPR; ++bb)
#pragma unroll
      for (int q = 0; q < 4; ++q) *(f32x4*)(lds + l32 * RB + 16 * ((8 * bb + 2 * q + g2) ^ sw)) = val(BPR * j + bb, q);
#pragma unroll
    for (int t = 0; t < 32 / RPI; ++t) {
      const int r = RPI * t + rr;
      const f32x4 v = *(const f32x4*)(lds + r * RB + 16 * (pp ^ (r & (NP - 1))));
      const long tr = rowtok(r);
      if (tr >= 0) *(f32x4*)(dst + tr * D + CPR * j + 4 * pp) = v;
    }
  }
}

template <int D, class Val, class RowTok>
__device__ __forceinline__ void rows_store_bf16(Val val, bf16* dst, char* lds, int lane, RowTok rowtok) {
  static_assert(D % 128 == 0, "whole 128-column rounds");
  const int l32 = lane & 31, g2 = lane >> 5, sw = l32 & 15, rr = lane >> 4, pp = lane & 15;
#pragma unroll
  for (int j = 0; j < D / 128; ++j) {
#pragma unroll
    for (int bb = 0; bb < 4; ++bb)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        // steps 2k and 2k + 1: this lane holds half g2 of pieces 4 bb + 2k and
        // 4 bb + 2k + 1, lane l ^ 32 the other halves; one exchange leaves
        // piece 4 bb + 2k + g2 whole in this lane (low half, then high half)
        typedef unsigned u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned))));
        typedef unsigned u32x4 __attribute__((__vector_size__(4 * sizeof(unsigned))));
        const u32x2 h0 = __builtin_bit_cast(u32x2, val(4 * j + bb, 2 * k));
        const u32x2 h1 = __builtin_bit_cast(u32x2, val(4 * j + bb, 2 * k + 1));
        const auto s0 = __builtin_amdgcn_permlane32_swap(h0[0], h1[0], false, false);
        const auto s1 = __builtin_amdgcn_permlane32_swap(h0[1], h1[1], false, false);
        *(u32x4*)(lds + l32 * 256 + 16 * ((4 * bb + 2 * k + g2) ^ sw)) = u32x4{s0[0], s1[0], s0[1], s1[1]};
      }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int r = 4 * t + rr;
      const bf16x8 v = *(const bf16x8*)(lds + r * 256 + 16 * (pp ^ (r & 15)));
      const long tr = rowtok(r);
      if (tr >= 0) *(bf16x8*)(dst + tr * D + 128 * j + 8 * pp) = v;
    }
  }
}

// m3_residual_epilogue for one 32-token block without projection or gate
// (R += acc2 + bias, then the next LayerNorm into g.out), with R and XN
// stored as whole 256-byte row segments through the wave's 8 KB LDS slice
// (rows_store_f32 / rows_store_bf16); the residual rows are loaded as in
// m3_residual_epilogue.
template <int D, class RowTok>
__device__ __forceinline__ void m3_residual_rows(f32x16 (&acc2)[D / 32][1], long tok, const GemmArgs& g, int g2,
                                                 const float* sv, char* lds, int lane, RowTok rowtok) {
  constexpr int OBK = D / 32, HB = 4 < OBK ? 4 : OBK;
  const float* sbias = sv;
  const float* slg = sv + D;
  const float* slb = sv + 2 * D;
  const bool tv = tok < g.M;
  const float* Rrow = g.R + (tv ? tok : 0) * D;
  float sum = 0.f;
#pragma unroll
  for (int b0 = 0; b0 < OBK; b0 += HB) {
    f32x4 rr[HB][4];
#pragma unroll
    for (int bb = 0; bb < HB; ++bb)
#pragma unroll
      for (int q = 0; q < 4; ++q)
        rr[bb][q] = tv ? *(const f32x4*)(Rrow + 32 * (b0 + bb) + 8 * q + 4 * g2) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int bb = 0; bb < HB; ++bb)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 bias = *(const f32x4*)&sbias[32 * (b0 + bb) + 8 * q + 4 * g2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float res = rr[bb][q][i] + (acc2[b0 + bb][0][4 * q + i] + bias[i]);
          acc2[b0 + bb][0][4 * q + i] = res;
          sum += res;
        }
      }
  }
  sum = xhalf_sum(sum);
  const float mean = sum / (float)D;
  float qv = 0.f;
#pragma unroll
  for (int b = 0; b < OBK; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float dv = acc2[b][0][r] - mean;
      qv = fmaf(dv, dv, qv);
    }
  qv = xhalf_sum(qv);
  const float rstd = 1.0f / sqrtf(qv / (float)D + 1e-5f);
  float mean2 = mean, rstd2 = rstd;
  asm volatile("" : "+v"(mean2), "+v"(rstd2));   // no (acc2 - mean) kept from the variance loop
  rows_store_bf16<D>(
      [&](int b, int q) {
        const int f = 32 * b + 8 * q + 4 * g2;
        const f32x4 lg = *(const f32x4*)&slg[f];
        const f32x4 lb = *(const f32x4*)&slb[f];
        bf16x4 h;
#pragma unroll
        for (int i = 0; i < 4; ++i) h[i] = (bf16)((acc2[b][0][4 * q + i] - mean2) * rstd2 * lg[i] + lb[i]);
        return h;
      },
      (bf16*)g.out, lds, lane, rowtok);
  rows_store_f32<D>(
      [&](int b, int q) {
        return f32x4{acc2[b][0][4 * q], acc2[b][0][4 * q + 1], acc2[b][0][4 * q + 2], acc2[b][0][4 * q + 3]};
      },
      g.R, lds, lane, rowtok);
}

template <int D, int TB, int NW, int WPE, int NBUF, bool PIPE, int SCHED, int MAXF, bool PROJ>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void k_mlp3(GemmArgs g, const bf16* __restrict__ W1, const float* __restrict__ b1, const bf16* __restrict__ W2,
            int F) {
  using S = M3Smem<D, NBUF, MAXF>;
  constexpr int BM = NW * TB * 32;                // tokens per workgroup
  constexpr int NTHR = NW * 64;
  constexpr int RB1 = S::RB1, RB2 = S::RB2;
  constexpr int KS1 = D / 16;                     // up-projection k-steps
  constexpr int OBK = D / 32;                     // 32-row output blocks
  constexpr int N1 = (int)((S::w1 + 1023) / 1024), N2 = (int)((S::w2 + 1023) / 1024);   // DMA blocks per chunk
  constexpr int NPW = (N1 + N2 + NW - 1) / NW;                        // per wave
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;
  const long tok0 = (long)blockIdx.x * BM + wave * (32 * TB) + l32;   // token of block t: tok0 + 32 t
  const int nch = F / kM3FCH;
  const bf16* __restrict__ A = (const bf16*)g.A;
  float* sb1 = (float*)(smem + NBUF * S::buf);
  float* sv = sb1 + MAXF;
  // DMA blocks this wave issues per chunk (uniform over the wave)
  const int nw = (N1 + N2) / NW + (wave < (N1 + N2) % NW ? 1 : 0);

  // ---- weight chunk c -> LDS buffer c % NBUF: 1 KB DMA blocks spread over
  // the waves; lane i of block u writes bytes [1024 u + 16 i, + 16) of its
  // region.  NBUF - 1 chunks are in flight ahead of the one being used.
  auto dma = [&](int c, int buf) {
    const int c0 = c * kM3FCH;
    char* base = smem + buf * S::buf;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
      const int u = wave + k * NW;                  // uniform over the wave
      if (u >= N1 + N2) break;
      const bool first = u < N1;
      const int pos = (first ? u : u - N1) * 1024 + lane * 16;
      const int rb = first ? RB1 : RB2;
      const int j = pos / rb, o = pos - j * rb;
      const bool data = o < rb - 16;                 // else a pad (copy something in bounds)
      const bf16* src;
      if (first) src = W1 + (long)(c0 + m3_sigma(data ? j : 0)) * D + (data ? o / 2 : 0);
      else src = W2 + (long)(data ? j : 0) * F + c0 + (data ? o / 2 : 0);
      char* dst = base + (first ? 0 : (int)S::w1a) + (pos - lane * 16);
      if (pos < (first ? (int)S::w1 : (int)S::w2))
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
  };
  for (int i = tid; i < F; i += NTHR) sb1[i] = b1[i];
  m3_stage_vectors<D>(sv, g, PROJ, tid, NTHR);

  // ---- this wave's XN rows, resident for the whole kernel
  bf16x8 xf[TB][KS1];
#pragma unroll
  for (int t = 0; t < TB; ++t) {
    const long tok = tok0 + 32 * t;
#pragma unroll
    for (int s = 0; s < KS1; ++s)
      xf[t][s] = tok < g.M ? *(const bf16x8*)(A + tok * D + 16 * s + 8 * g2) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  }

  f32x16 acc2[OBK][TB];
#pragma unroll
  for (int b = 0; b < OBK; ++b)
#pragma unroll
    for (int t = 0; t < TB; ++t)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc2[b][t][r] = 0.f;

  // up: acc[t][r] = b1[c0 + h] + sum_k W1[c0 + h][k] XN[token][k] for the
  // hidden unit h = sigma(8(r/4) + 4 g2 + r%4) = 16(q/2) + 8 g2 + 4(q%2) + i,
  // r = 4q + i (the accumulators start at the bias)
  auto up = [&](int c, f32x16 (&acc)[TB]) {
    const char* s1 = smem + (c % NBUF) * S::buf;
    const float* sb = sb1 + c * kM3FCH;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 bq = *(const f32x4*)&sb[16 * (q >> 1) + 8 * g2 + 4 * (q & 1)];
#pragma unroll
      for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) acc[t][4 * q + i] = bq[i];
    }
#pragma unroll
    for (int s = 0; s < KS1; ++s) {
      const bf16x8 a = *(const bf16x8*)(s1 + l32 * RB1 + (2 * s + g2) * 16);
#pragma unroll
      for (int t = 0; t < TB; ++t) acc[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, xf[t][s], acc[t], 0, 0, 0);
    }
  };
  // GELU of an up product, rounded to BF16: register 4q + i of token block t
  // becomes element 4(q%2) + i of k-fragment q/2, the k-values this lane
  // supplies to the down MFMAs
  auto gelu = [&](const f32x16 (&acc)[TB], bf16x8 (&h)[TB][2]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int t = 0; t < TB; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) h[t][q >> 1][4 * (q & 1) + i] = (bf16)gelu_f(acc[t][4 * q + i]);
  };
  // down: acc2[b] += W2[32 b + row][c0 + 16 s + 8 g2 + e] H[16 s + 8 g2 + e]
  auto down = [&](int c, const bf16x8 (&h)[TB][2]) {
    const char* s2 = smem + (c % NBUF) * S::buf + S::w1a;
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16x8 w = *(const bf16x8*)(s2 + (32 * b + l32) * RB2 + (2 * s + g2) * 16);
#pragma unroll
        for (int t = 0; t < TB; ++t) acc2[b][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, h[t][s], acc2[b][t], 0, 0, 0);
      }
  };

  const int pre = min(NBUF - 1, nch);            // chunks in flight before the loop
  for (int c = 0; c < pre; ++c) dma(c, c);
  __syncthreads();                                // b1 staged, and this wave's DMA of chunks < pre done
  f32x16 acc1[TB];
  bf16x8 hf[TB][2];
  if constexpr (!PIPE) {
    // One chunk at a time: up, GELU, down.
    for (int c = 0; c < nch; ++c) {
      // buffer (c + NBUF - 1) % NBUF was last read in iteration c - 1, before its closing barrier
      if (c + NBUF - 1 < nch) dma(c + NBUF - 1, (c + NBUF - 1) % NBUF);
      up(c, acc1);
      gelu(acc1, hf);
      down(c, hf);
      // chunk c + 1 complete in every wave: this wave may still have the DMA
      // of the chunks after it (at most NBUF - 2) outstanding
      if (c + 1 < nch) m3_wait_barrier(nw * (min(c + NBUF - 1, nch - 1) - (c + 1)));
    }
  } else {
    // Two-deep software pipeline: iteration c issues chunk c's down
    // projection, the GELU of chunk c + 1 and chunk c + 2's up projection,
    // three independent streams of MFMA and VALU work that the wave can
    // interleave.  It reads W2 of chunk c and W1 of chunk c + 2 and DMAs
    // chunk c + NBUF - 1 into the buffer of chunk c - 1, so NBUF >= 4.
    static_assert(NBUF >= 4, "four weight buffers");
    up(0, acc1);
    gelu(acc1, hf);
    if (nch > 1) up(1, acc1);
    int c = 0;
    for (; c + 2 < nch; ++c) {
      // buffer (c + NBUF - 1) % NBUF = (c - 1) % NBUF was last read in
      // iteration c - 1 (W2 of chunk c - 1), before its closing barrier
      if (c + NBUF - 1 < nch) dma(c + NBUF - 1, (c + NBUF - 1) % NBUF);
      bf16x8 hn[TB][2];
      if constexpr (SCHED == 0) {
        gelu(acc1, hn);
        up(c + 2, acc1);
        down(c, hf);
      } else {
        // The same three streams in a fixed order: every A fragment read
        // up front, then each MFMA followed by its share of the GELU pairs
        // (scheduling fences keep the order).
        const char* s1 = smem + ((c + 2) % NBUF) * S::buf;
        const char* s2 = smem + (c % NBUF) * S::buf + S::w1a;
        const float* sb = sb1 + (c + 2) * kM3FCH;
        bf16x8 a1[KS1], a2[2 * OBK];
#pragma unroll
        for (int k = 0; k < KS1; ++k) a1[k] = *(const bf16x8*)(s1 + l32 * RB1 + (2 * k + g2) * 16);
#pragma unroll
        for (int j = 0; j < 2 * OBK; ++j) a2[j] = *(const bf16x8*)(s2 + (32 * (j >> 1) + l32) * RB2 + (2 * (j & 1) + g2) * 16);
        f32x16 an[TB];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const f32x4 bq = *(const f32x4*)&sb[16 * (q >> 1) + 8 * g2 + 4 * (q & 1)];
#pragma unroll
          for (int t = 0; t < TB; ++t)
#pragma unroll
            for (int i = 0; i < 4; ++i) an[t][4 * q + i] = bq[i];
        }
        constexpr int NM = (KS1 + 2 * OBK) * TB;   // MFMAs of this iteration
        constexpr int NP = 8 * TB;                  // GELU pairs
#pragma unroll
        for (int m = 0; m < NM; ++m) {
          if (m < KS1 * TB) {
            const int k = m / TB, t = m % TB;
            an[t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a1[k], xf[t][k], an[t], 0, 0, 0);
          } else {
            const int j = (m - KS1 * TB) / TB, t = (m - KS1 * TB) % TB;
            acc2[j >> 1][t] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a2[j], hf[t][j & 1], acc2[j >> 1][t], 0, 0, 0);
          }
#pragma unroll
          for (int pr = (m * NP + NM - 1) / NM; pr < ((m + 1) * NP + NM - 1) / NM; ++pr) {
            const int t = pr / 8, r = 2 * (pr % 8), q = r >> 2, i = r & 3;
            hn[t][q >> 1][4 * (q & 1) + i] = (bf16)gelu_f(acc1[t][r]);
            hn[t][q >> 1][4 * (q & 1) + i + 1] = (bf16)gelu_f(acc1[t][r + 1]);
          }
          __builtin_amdgcn_sched_barrier(0);
        }
#pragma unroll
        for (int t = 0; t < TB; ++t) acc1[t] = an[t];
      }
#pragma unroll
      for (int t = 0; t < TB; ++t) {
        hf[t][0] = hn[t][0];
        hf[t][1] = hn[t][1];
      }
      // chunk c + 3 complete in every wave (the next iteration's up
      // projection reads it); later chunks may still be in flight
      m3_wait_barrier(nw * max(0, min(c + NBUF - 1, nch - 1) - (c + 3)));
    }
    // the last one or two chunks: their weights are complete and no DMA follows
    if (c + 1 < nch) {
      bf16x8 hn[TB][2];
      gelu(acc1, hn);
      down(c, hf);
      down(c + 1, hn);
    } else {
      down(c, hf);
    }
  }

  m3_residual_epilogue<D, TB, PROJ>(acc2, tok0, g, g2, sv);
}

template <int D, int TB, int NW, int WPE, int NBUF, bool PIPE, int SCHED = 0, int MAXF = kM3MaxF>
hipError_t mlp3_t(const GemmArgs& g, const bf16* W1, const float* b1, const bf16* W2, int F, hipStream_t s) {
  if (F > MAXF) return hipErrorInvalidValue;
  constexpr int BM = NW * TB * 32;
  dim3 grid((unsigned)((g.M + BM - 1) / BM)), block(NW * 64);
  if (g.proj_out) hipLaunchKernelGGL((k_mlp3<D, TB, NW, WPE, NBUF, PIPE, SCHED, MAXF, true>), grid, block, 0, s, g, W1, b1, W2, F);
  else hipLaunchKernelGGL((k_mlp3<D, TB, NW, WPE, NBUF, PIPE, SCHED, MAXF, false>), grid, block, 0, s, g, W1, b1, W2, F);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Token-resident projections with the same machinery (BF16, d in {128, 256}).
//
// k_proj3: out[M][N] = XN W^T + b in BF16 (the QKV projection, N = 3d).  A
// workgroup of 8 waves owns 256 tokens; each wave keeps its 32 XN rows in
// registers and walks the N outputs in chunks of 32 rows of W, DMA'd into
// LDS (rows padded by 16 bytes), double-buffered.  Lane l ends a chunk with
// outputs 8q + 4(l/32) + i of token l%32 and stores them as BF16.
template <int D, int CHB>
struct P3Smem {
  static constexpr int RB = D * 2 + 16;
  static constexpr size_t w = (size_t)32 * CHB * RB;          // one chunk: 32 CHB rows of W
  static constexpr size_t wa = (w + 1023) / 1024 * 1024;
  static constexpr size_t buf = wa;
  static constexpr size_t bytes = 2 * buf + 3 * 512 * 4;      // + the whole bias (N <= 1536)
  static_assert(bytes <= 160 * 1024, "LDS");
};

// Chunks of CHB 32-row blocks of W (128 rows at d <= 256, 64 at input width
// 512), so that a chunk's 16 CHB d / 256 MFMAs per wave cover the L2 round
// trip of the next chunk's DMA.
template <int D, int CHB, int WPE, bool GELU>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(WPE, WPE)))
void k_proj3(GemmArgs g, const bf16* __restrict__ W) {
  using S = P3Smem<D, CHB>;
  constexpr int NW = 8, RB = S::RB, KS = D / 16;
  constexpr int NB = (int)(S::wa / 1024), NPW = (NB + NW - 1) / NW;
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  float* sbias = (float*)(smem + 2 * S::buf);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;
  const long tok = (long)blockIdx.x * kM3BM + wave * 32 + l32;
  const bool tv = tok < g.M;
  const int N = g.N, nch = N / (32 * CHB);
  const bf16* __restrict__ A = (const bf16*)g.A;
  bf16* __restrict__ out = (bf16*)g.out;

  auto dma = [&](int c, int buf) {
    char* base = smem + buf * S::buf;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
      const int u = wave + k * NW;
      if (u >= NB) break;
      const int pos = u * 1024 + lane * 16, j = pos / RB, o = pos - j * RB;
      const bool data = o < RB - 16;
      const bf16* src = W + (long)(c * 32 * CHB + (data ? j : 0)) * D + (data ? o / 2 : 0);
      if (pos < (int)S::w)
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(base + u * 1024), 16, 0, 0);
    }
  };
  for (int i = tid; i < N; i += 512) sbias[i] = g.bias[i];

  bf16x8 xf[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s)
    xf[s] = tv ? *(const bf16x8*)(A + tok * D + 16 * s + 8 * g2) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};

  dma(0, 0);
  __syncthreads();
  for (int c = 0; c < nch; ++c) {
    const int buf = c & 1;
    if (c + 1 < nch) dma(c + 1, buf ^ 1);       // its last readers finished before the previous barrier
    const char* sw = smem + buf * S::buf;
    f32x16 acc[CHB];
#pragma unroll
    for (int cb = 0; cb < CHB; ++cb)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc[cb][r] = 0.f;
#pragma unroll
    for (int s = 0; s < KS; ++s)
#pragma unroll
      for (int cb = 0; cb < CHB; ++cb) {
        const bf16x8 a = *(const bf16x8*)(sw + (32 * cb + l32) * RB + (2 * s + g2) * 16);
        acc[cb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, xf[s], acc[cb], 0, 0, 0);
      }
    if (tv) {
#pragma unroll
      for (int cb = 0; cb < CHB; ++cb)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int f = c * 32 * CHB + 32 * cb + 8 * q + 4 * g2;
          const f32x4 bq = *(const f32x4*)&sbias[f];
          f32x4 v;
#pragma unroll
          for (int i = 0; i < 4; ++i) v[i] = GELU ? gelu_f(acc[cb][4 * q + i] + bq[i]) : acc[cb][4 * q + i] + bq[i];
          const bf16x4 h = {(bf16)v[0], (bf16)v[1], (bf16)v[2], (bf16)v[3]};
          *(bf16x4*)(out + tok * N + f) = h;
        }
    }
    __syncthreads();
  }
}

// k_oproj3: R += A W^T + b over K = d, then the next LayerNorm into g.out (the
// output projection after attention, A = O in BF16).  Each wave owns 32
// tokens and accumulates all d outputs (acc2, as in the MLP's down
// projection); the contraction walks K in chunks of KCH = 128:
// W[:, k0:k0+128] is DMA'd into LDS (rows padded by 16 bytes) and the A rows'
// k-fragments of the chunk are read from memory one chunk ahead.
template <int D, int KCH>
struct O3Smem {
  static constexpr int RB = KCH * 2 + 16;
  static constexpr size_t w = (size_t)D * RB;
  static constexpr size_t wa = (w + 1023) / 1024 * 1024;
  static constexpr int NCH = D / KCH;
  static constexpr size_t bytes = (NCH > 1 ? 2 : 1) * wa + 3 * D * 4;
  static_assert(D % KCH == 0 && bytes <= 160 * 1024, "LDS");
};

template <int D, bool GATE>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_oproj3(GemmArgs g, const bf16* __restrict__ W) {
  constexpr int KCH = 128;
  using S = O3Smem<D, KCH>;
  constexpr int NW = 8, RB = S::RB, OBK = D / 32, NCH = S::NCH, KSC = KCH / 16;
  constexpr int NB = (int)(S::wa / 1024), NPW = (NB + NW - 1) / NW;
  constexpr size_t BUF = S::wa;
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  float* sv = (float*)(smem + (NCH > 1 ? 2 : 1) * BUF);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;
  const long tok0 = (long)blockIdx.x * kM3BM + wave * 32 + l32;
  const bool tv = tok0 < g.M;
  const bf16* __restrict__ A = (const bf16*)g.A;

  auto dma = [&](int c, int buf) {
    char* base = smem + buf * BUF;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
      const int u = wave + k * NW;
      if (u >= NB) break;
      const int pos = u * 1024 + lane * 16, j = pos / RB, o = pos - j * RB;
      const bool data = o < RB - 16;
      const bf16* src = W + (long)(data ? j : 0) * D + c * KCH + (data ? o / 2 : 0);
      if (pos < (int)S::w)
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(base + u * 1024), 16, 0, 0);
    }
  };
  auto afrag = [&](int c, bf16x8 (&f)[KSC]) {
#pragma unroll
    for (int s = 0; s < KSC; ++s)
      f[s] = tv ? *(const bf16x8*)(A + tok0 * D + c * KCH + 16 * s + 8 * g2) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  };

  f32x16 acc2[OBK][1];
#pragma unroll
  for (int b = 0; b < OBK; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc2[b][0][r] = 0.f;
  bf16x8 fa[KSC], fn[KSC];
  m3_stage_vectors<D>(sv, g, false, tid, 512);
  afrag(0, fa);
  dma(0, 0);
  __syncthreads();
#pragma unroll 1
  for (int c = 0; c < NCH; ++c) {
    const int buf = c & 1;
    if (c + 1 < NCH) {
      dma(c + 1, buf ^ 1);
      afrag(c + 1, fn);
    }
    const char* sw = smem + buf * BUF;
#pragma unroll
    for (int s = 0; s < KSC; ++s)
#pragma unroll
      for (int b = 0; b < OBK; ++b) {
        const bf16x8 w = *(const bf16x8*)(sw + (32 * b + l32) * RB + (2 * s + g2) * 16);
        acc2[b][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, fa[s], acc2[b][0], 0, 0, 0);
      }
    if (c + 1 < NCH) {
#pragma unroll
      for (int s = 0; s < KSC; ++s) fa[s] = fn[s];
      __syncthreads();
    }
  }
  m3_residual_epilogue<D, 1, false, GATE>(acc2, tok0, g, g2, sv);
}

// ---------------------------------------------------------------------------
// User attention with its QKV projection, for the BF16 path at head width 32
// (d = 256): QKV = XN Wqkv^T + b, then for every head the softmax attention
// of each token over the K tokens of its slot; O is written in BF16 and the
// output projection, residual and LayerNorm follow in k_oproj3.  A wave owns
// one group of floor(32/K) columns x K rows of one bin (slot s of the group
// is row s % K of column s / K), so every key a query needs is among the
// wave's own 32 tokens.  The wave keeps the group's XN rows in registers (B
// operand of v_mfma_f32_32x32x16_bf16) and walks the heads; weight chunk h
// holds the Q, K and V rows of head h (96 rows, DMA'd into LDS, double
// buffered).  Per head, in registers:
//   S^T = K Q^T   two MFMAs: the projection's output registers are the
//                 k fragments of both operands, with the same permutation of
//                 the head dimension on both sides;
//   softmax       exp2, masked to the query's column; a lane holds 16 keys
//                 of its query, lane l ^ 32 the other 16;
//   O^T = V^T P^T two MFMAs; V is projected transposed (the projection MFMA
//                 with its operands swapped), which leaves it as the A
//                 operand with the keys in P's register order.
// Only XN is read and only O is written: 4d bytes per token, against 16d for
// a separate projection and attention kernel.
template <int D>
struct UQSmem {
  static constexpr int RB = D * 2 + 16;             // bytes per stored weight row (16 of them pad)
  static constexpr int CR = 96;                      // Q, K and V rows of one head
  static constexpr size_t w = (size_t)CR * RB;
  static constexpr size_t wa = (w + 15) / 16 * 16;
  static constexpr size_t bias = (size_t)3 * D * 4;
  static constexpr size_t bytes = 2 * wa + bias;
  static_assert(bytes <= 160 * 1024, "LDS");
};

template <int D>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_user_qkv_attn(StepCtx c, const bf16* __restrict__ XN, const bf16* __restrict__ W,
                     const float* __restrict__ bqkv, bf16* __restrict__ O) {
  using S = UQSmem<D>;
  constexpr int RB = S::RB, KS = D / 16, HEADS = D / 32;
  constexpr int NB = (int)((S::w + 1023) / 1024), NPW = (NB + 7) / 8;
  static_assert(HEADS % 4 == 0, "heads in batches of four");
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  float* sbias = (float*)(smem + 2 * S::wa);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;

  // ---- this lane's slot of the wave's group
  const int gi = blockIdx.x * 8 + wave;
  int tok = -1, K = 1;
  if (gi < c.total_ugrp32) {
    const int bi = c.ugrp32[2 * gi], c0 = c.ugrp32[2 * gi + 1];
    const DevBin& b = c.bins[bi];
    K = b.K;
    const int C = 32 / K, cl = l32 / K, k = l32 - cl * K;
    if (l32 < C * K && c0 + cl < b.n) tok = b.tok_off + k * b.n + c0 + cl;
  }
  // keys this lane's query may attend to: register r of S^T holds key slot
  // 8(r/4) + 4 g2 + r%4; valid slot in the query's column
  const unsigned long long vmask = __ballot(tok >= 0);
  unsigned okbits = 0;
  const int col_lo = (l32 / K) * K;                 // key slots of this lane's column: col_lo .. col_lo + K - 1
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int kr = 8 * (r >> 2) + 4 * g2 + (r & 3);
    if (((vmask >> kr) & 1ull) && (unsigned)(kr - col_lo) < (unsigned)K) okbits |= 1u << r;
  }

  auto dma = [&](int h, int buf) {
    char* base = smem + buf * S::wa;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
      const int u = wave + k * 8;                   // uniform over the wave
      if (u >= NB) break;
      const int pos = u * 1024 + lane * 16, j = pos / RB, o = pos - j * RB;
      const bool data = o < RB - 16;                 // else a pad (copy something in bounds)
      const int jj = data ? j : 0;
      const bf16* src = W + (long)((jj >> 5) * D + h * 32 + (jj & 31)) * D + (data ? o / 2 : 0);
      if (pos < (int)S::w)
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(base + u * 1024), 16, 0, 0);
    }
  };
  for (int i = tid; i < 3 * D; i += 512) sbias[i] = bqkv[i];
  bf16x8 xf[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s)
    xf[s] = tok >= 0 ? *(const bf16x8*)(XN + (long)tok * D + 16 * s + 8 * g2) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  dma(0, 0);
  __syncthreads();                                  // bias staged, chunk 0 in LDS

  const float scale = 1.4426950408889634f / sqrtf(32.0f);
  // O of HB heads at a time; each batch is stored right after a closing
  // barrier, so its stores overlap the next head's work and are complete by
  // the barrier after it
  constexpr int HB = 4;
  bf16x4 ob[HB][4];
  bf16* orow = O + (long)(tok >= 0 ? tok : 0) * D;
#pragma unroll
  for (int h = 0; h < HEADS; ++h) {
    // buffer (h + 1) & 1 was last read in iteration h - 1, before its closing barrier
    if (h + 1 < HEADS) dma(h + 1, (h + 1) & 1);
    const char* sw = smem + (h & 1) * S::wa;
    // Q, K: register r holds head feature 8(r/4) + 4 g2 + r%4 of token l%32;
    // V^T (operands swapped): register r holds token 8(r/4) + 4 g2 + r%4,
    // feature l%32 -- the A operand of O^T = V^T P^T as it stands
    f32x16 aq, ak, av;
#pragma unroll
    for (int r = 0; r < 16; ++r) aq[r] = ak[r] = av[r] = 0.f;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const bf16x8 wq = *(const bf16x8*)(sw + l32 * RB + (2 * s + g2) * 16);
      const bf16x8 wk = *(const bf16x8*)(sw + (32 + l32) * RB + (2 * s + g2) * 16);
      const bf16x8 wv = *(const bf16x8*)(sw + (64 + l32) * RB + (2 * s + g2) * 16);
      aq = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wq, xf[s], aq, 0, 0, 0);
      ak = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wk, xf[s], ak, 0, 0, 0);
      av = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xf[s], wv, av, 0, 0, 0);
    }
    // + bias, BF16
    bf16x8 qf[2], kf[2], vf[2];
    const float bv = sbias[2 * D + h * 32 + l32];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = h * 32 + 8 * q + 4 * g2;
      const f32x4 bq = *(const f32x4*)&sbias[f];
      const f32x4 bk = *(const f32x4*)&sbias[D + f];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 4 * q + i;
        qf[r >> 3][r & 7] = (bf16)(aq[r] + bq[i]);
        kf[r >> 3][r & 7] = (bf16)(ak[r] + bk[i]);
        vf[r >> 3][r & 7] = (bf16)(av[r] + bv);
      }
    }
    // S^T = K Q^T: lane l holds query l%32, register r key slot 8(r/4) + 4 g2 + r%4
    f32x16 st;
#pragma unroll
    for (int r = 0; r < 16; ++r) st[r] = 0.f;
    st = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf[0], qf[0], st, 0, 0, 0);
    st = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf[1], qf[1], st, 0, 0, 0);
    float mx = -INFINITY;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      st[r] = ((okbits >> r) & 1u) ? st[r] : -INFINITY;
      mx = fmaxf(mx, st[r]);
    }
    mx = xhalf_max(mx);
    // a padding query has no valid key (mx = -inf): p = 0 for it
    const float mxs = mx == -INFINITY ? 0.f : -mx * scale;
    float ps = 0.f;
    bf16x8 pf[2];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float p = __builtin_amdgcn_exp2f(fmaf(st[r], scale, mxs));
      ps += p;
      pf[r >> 3][r & 7] = (bf16)p;
    }
    ps = xhalf_sum(ps);
    f32x16 o;
#pragma unroll
    for (int r = 0; r < 16; ++r) o[r] = 0.f;
    o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf[0], pf[0], o, 0, 0, 0);
    o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf[1], pf[1], o, 0, 0, 0);
    const float inv = ps > 0.f ? 1.0f / ps : 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      ob[h % HB][q] = bf16x4{(bf16)(o[4 * q] * inv), (bf16)(o[4 * q + 1] * inv), (bf16)(o[4 * q + 2] * inv),
                             (bf16)(o[4 * q + 3] * inv)};
    // chunk h + 1 complete in every wave: this wave's memory operations in
    // flight are its part of that DMA and the O stores of the previous batch
    if (h + 1 < HEADS) m3_wait_barrier(0);
    if (h % HB == HB - 1 && tok >= 0) {
#pragma unroll
      for (int hh = 0; hh < HB; ++hh)
#pragma unroll
        for (int q = 0; q < 4; ++q) *(bf16x4*)(orow + (h - HB + 1 + hh) * 32 + 8 * q + 4 * g2) = ob[hh][q];
    }
  }
}

// ---------------------------------------------------------------------------
// The whole user-attention sublayer for the BF16 path at head width 16
// (d = 128): QKV projection, softmax attention of each token over the K
// tokens of its slot, output projection, bias, residual and the next
// LayerNorm, token-resident.  A wave owns one 32-slot group of whole columns
// as in k_user_qkv_attn; the weights go through LDS one head pair at a time:
// the pair's Q, K and V rows (three 32-row MFMA blocks, rows 16 e + j of a
// block = feature j of head 2p + e) and the pair's 32 columns of W_o.  Per
// head the score MFMA takes the 16 features of that head (registers
// 8e .. 8e + 7 of the Q and K blocks).  V is projected transposed (the same
// MFMA with its operands swapped: lane l then holds feature l%32 for 16
// keys, in exactly the key order of P's registers), so it is the A operand
// of O^T = V^T P^T as it stands; that MFMA takes both heads' V rows and the
// head keeps its half.  The pair's O block feeds the output projection at
// once (acc2 += W_o[:, pair] O_pair), so O never leaves registers.  Four
// waves (128 tokens) per workgroup in 74 KB of LDS: two workgroups per CU.
// HBM traffic per token: XN and R in, R and XN out.
template <int D>
struct UBSmem {
  static constexpr int RB1 = D * 2 + 16;               // bytes per stored Wqkv row
  static constexpr int RB2 = 32 * 2 + 16;              // bytes per stored W_o row (the pair's 32 columns)
  static constexpr size_t w1 = (size_t)96 * RB1;
  static constexpr size_t w2 = (size_t)D * RB2;
  static constexpr size_t w1a = (w1 + 15) / 16 * 16;
  static constexpr size_t w2a = (w2 + 15) / 16 * 16;
  static constexpr size_t buf = w1a + w2a;
  static constexpr size_t vec = (size_t)8 * D * 4;     // bqkv [3D], then the epilogue vectors [5D]
  static constexpr size_t bytes = 2 * buf + vec;
  static_assert(bytes <= 80 * 1024, "two workgroups per CU");
};

template <int D, int NW>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_user_block_tr(StepCtx c, GemmArgs g, const bf16* __restrict__ Wqkv, const float* __restrict__ bqkv,
                     const bf16* __restrict__ Wo) {
  using S = UBSmem<D>;
  constexpr int RB1 = S::RB1, RB2 = S::RB2, KS = D / 16, NP = D / 32, OBK = D / 32, NTHR = NW * 64;
  constexpr int N1 = (int)((S::w1 + 1023) / 1024), N2 = (int)((S::w2 + 1023) / 1024), NPW = (N1 + N2 + NW - 1) / NW;
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  float* sbias = (float*)(smem + 2 * S::buf);
  float* sv = sbias + 3 * D;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;

  // ---- this lane's slot of the wave's group
  const int gi = blockIdx.x * NW + wave;
  int tok = -1, K = 1;
  if (gi < c.total_ugrp32) {
    const int bi = c.ugrp32[2 * gi], c0 = c.ugrp32[2 * gi + 1];
    const DevBin& b = c.bins[bi];
    K = b.K;
    const int C = 32 / K, cl = l32 / K, k = l32 - cl * K;
    if (l32 < C * K && c0 + cl < b.n) tok = b.tok_off + k * b.n + c0 + cl;
  }
  const unsigned long long vmask = __ballot(tok >= 0);
  unsigned okbits = 0;                               // register r of S^T: key slot 8(r/4) + 4 g2 + r%4
  const int col_lo = (l32 / K) * K;                 // key slots of this lane's column: col_lo .. col_lo + K - 1
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int kr = 8 * (r >> 2) + 4 * g2 + (r & 3);
    if (((vmask >> kr) & 1ull) && (unsigned)(kr - col_lo) < (unsigned)K) okbits |= 1u << r;
  }

  // head pair p -> LDS: Wqkv rows (j / 32) D + 32 p + j % 32, W_o columns 32 p .. + 32
  auto dma = [&](int p, int buf) {
    char* base = smem + buf * S::buf;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
      const int u = wave + k * NW;                    // uniform over the wave
      if (u >= N1 + N2) break;
      const bool first = u < N1;
      const int pos = (first ? u : u - N1) * 1024 + lane * 16;
      const int rb = first ? RB1 : RB2;
      const int j = pos / rb, o = pos - j * rb;
      const bool data = o < rb - 16;                   // else a pad (copy something in bounds)
      const int jj = data ? j : 0;
      const bf16* src = first ? Wqkv + (long)((jj >> 5) * D + 32 * p + (jj & 31)) * D + (data ? o / 2 : 0)
                              : Wo + (long)jj * D + 32 * p + (data ? o / 2 : 0);
      char* dst = base + (first ? 0 : (int)S::w1a) + (pos - lane * 16);
      if (pos < (first ? (int)S::w1 : (int)S::w2))
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
    }
  };
  for (int i = tid; i < 3 * D; i += NTHR) sbias[i] = bqkv[i];
  m3_stage_vectors<D>(sv, g, false, tid, NTHR);
  const bf16* __restrict__ A = (const bf16*)g.A;
  bf16x8 xf[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s)
    xf[s] = tok >= 0 ? *(const bf16x8*)(A + (long)tok * D + 16 * s + 8 * g2) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  dma(0, 0);
  __syncthreads();                                    // vectors staged, pair 0 in LDS

  const float scale = 1.4426950408889634f / 4.0f;     // log2(e) / sqrt(16)
  f32x16 acc2[OBK][1];
#pragma unroll
  for (int b = 0; b < OBK; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc2[b][0][r] = 0.f;
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    // buffer (p + 1) & 1 was last read in iteration p - 1, before its closing barrier
    if (p + 1 < NP) dma(p + 1, (p + 1) & 1);
    const char* s1 = smem + (p & 1) * S::buf;
    const char* s2 = s1 + S::w1a;
    // Q, K: register r holds pair feature 8(r/4) + 4 g2 + r%4 of token l%32;
    // V^T: register r holds token 8(r/4) + 4 g2 + r%4, feature l%32
    f32x16 aq, ak, av;
#pragma unroll
    for (int r = 0; r < 16; ++r) aq[r] = ak[r] = av[r] = 0.f;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const bf16x8 wq = *(const bf16x8*)(s1 + l32 * RB1 + (2 * s + g2) * 16);
      const bf16x8 wk = *(const bf16x8*)(s1 + (32 + l32) * RB1 + (2 * s + g2) * 16);
      const bf16x8 wv = *(const bf16x8*)(s1 + (64 + l32) * RB1 + (2 * s + g2) * 16);
      aq = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wq, xf[s], aq, 0, 0, 0);
      ak = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wk, xf[s], ak, 0, 0, 0);
      av = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xf[s], wv, av, 0, 0, 0);
    }
    // + bias, BF16; registers 8e .. 8e + 7 of Q and K are head 2p + e
    bf16x8 qf[2], kf[2], vf[2];
    const float bv = sbias[2 * D + 32 * p + l32];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = 32 * p + 8 * q + 4 * g2;
      const f32x4 bq = *(const f32x4*)&sbias[f];
      const f32x4 bk = *(const f32x4*)&sbias[D + f];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 4 * q + i;
        qf[r >> 3][r & 7] = (bf16)(aq[r] + bq[i]);
        kf[r >> 3][r & 7] = (bf16)(ak[r] + bk[i]);
        vf[r >> 3][r & 7] = (bf16)(av[r] + bv);
      }
    }
    f32x16 ob;                                         // O of the pair, pair features as Q's
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      f32x16 st;
#pragma unroll
      for (int r = 0; r < 16; ++r) st[r] = 0.f;
      st = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf[e], qf[e], st, 0, 0, 0);
      float mx = -INFINITY;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        st[r] = ((okbits >> r) & 1u) ? st[r] : -INFINITY;
        mx = fmaxf(mx, st[r]);
      }
      mx = xhalf_max(mx);
      // a padding query has no valid key (mx = -inf): p = 0 for it
      const float mxs = mx == -INFINITY ? 0.f : -mx * scale;
      float ps = 0.f;
      bf16x8 pf[2];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float pv = __builtin_amdgcn_exp2f(fmaf(st[r], scale, mxs));
        ps += pv;
        pf[r >> 3][r & 7] = (bf16)pv;
      }
      ps = xhalf_sum(ps);
      f32x16 o;
#pragma unroll
      for (int r = 0; r < 16; ++r) o[r] = 0.f;
      o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf[0], pf[0], o, 0, 0, 0);
      o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf[1], pf[1], o, 0, 0, 0);
      const float inv = ps > 0.f ? 1.0f / ps : 0.f;
#pragma unroll
      for (int r = 0; r < 8; ++r) ob[8 * e + r] = o[8 * e + r] * inv;
    }
    // output projection of the pair: acc2[b] += W_o[32 b + row][32 p + k] O[k],
    // the k order of O's registers (16 s + 4 g2 + j, 16 s + 8 + 4 g2 + j - 4)
    // on both operands
    bf16x8 of[2];
#pragma unroll
    for (int r = 0; r < 16; ++r) of[r >> 3][r & 7] = (bf16)ob[r];
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const char* wr = s2 + (32 * b + l32) * RB2;
        const bf16x8 w = *(const bf16x8*)(wr + (16 * s + 8 * g2) * 2);   // k-ordered rows
        acc2[b][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, of[s], acc2[b][0], 0, 0, 0);
      }
    // pair p + 1 complete in every wave (this wave's only memory operations in
    // flight are its part of that DMA)
    if (p + 1 < NP) m3_wait_barrier(0);
  }
  m3_residual_epilogue<D, 1, false>(acc2, tok >= 0 ? (long)tok : g.M, g, g2, sv);
}

// ---------------------------------------------------------------------------
// The row-attention sublayer for the BF16 path at head width 16 (d = 128,
// rows of n <= 128 tokens), token-resident: QKV projection, softmax
// attention of each token over the n tokens of its row, output projection,
// bias, residual and the next LayerNorm.  A workgroup of four waves owns one
// row (wave w: slots 32 w .. 32 w + 31); each wave keeps its XN rows in
// registers and walks the head pairs as k_user_block_tr does.  Per pair the
// waves publish their K block (key-major) and V^T block (projected
// transposed) to LDS, then every wave runs its 32 queries over the row's key
// blocks with an online softmax (S^T = K Q^T from the shared K rows, O^T +=
// V^T P^T from the shared V^T rows, both in P's key order), and feeds the
// pair's O to the output projection.  The weights come from fragment-major
// copies of Wqkv (role 5 of om4_fragment_copy) and W_o (role 6), each MFMA
// operand fragment 1 KB with lane l's 16 bytes at 16 l; the pair's Wqkv
// fragments sit in one buffer, refilled once every wave has published K and
// V^T, and its W_o fragments in two, so that a pair costs two barriers (its
// weights in LDS; K and V^T published).  62 KB of LDS: two workgroups per CU.
template <int D>
struct RBFSmem {
  static constexpr size_t w1a = (size_t)3 * (D / 16) * 1024;   // a head pair's Wqkv fragments
  static constexpr size_t w2 = (size_t)2 * (D / 32) * 1024;    // its W_o fragments
  static constexpr size_t w2a = 2 * w2;                        // double-buffered
  // tile pitches of 18 and 66 dwords: the 8-byte accesses of 32 lanes to 32
  // consecutive rows then cover all 64 banks once (a pitch that is a
  // multiple of 4 dwords puts rows l and l + 16 on the same banks)
  static constexpr int LDK = 32 + 4;                   // K row: the pair's 32 features + pad (bf16)
  static constexpr int LDV = 128 + 4;                  // V^T row: 128 keys + pad (bf16)
  static constexpr size_t k = (size_t)128 * LDK * 2;
  static constexpr size_t vt = (size_t)32 * LDV * 2;
  static constexpr size_t ones = (size_t)128 * 2 + 16;  // a V^T row of ones: P's row sums on the MFMA
  static constexpr size_t vec = (size_t)8 * D * 4;     // bqkv [3D], then the epilogue vectors [5D]
  static constexpr size_t bytes = w1a + w2a + k + vt + ones + vec;
  static_assert(bytes <= 80 * 1024, "two workgroups per CU");
};

template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_row_block_tr(StepCtx c, GemmArgs g, const bf16* __restrict__ Wqf, const float* __restrict__ bqkv,
                    const bf16* __restrict__ Wof) {
  using S = RBFSmem<D>;
  constexpr int LDK = S::LDK, LDV = S::LDV;
  constexpr int KS = D / 16, NP = D / 32, OBK = D / 32;
  constexpr int NQ = 3 * KS, NO = 2 * OBK;           // 1 KB fragments of a pair's Wqkv, W_o
  static_assert(NQ % 4 == 0 && NO % 4 == 0, "DMA blocks split evenly over the waves");
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  char* sw1 = smem;
  char* sw2 = smem + S::w1a;
  bf16* sK = (bf16*)(smem + S::w1a + S::w2a);
  bf16* sVt = (bf16*)(smem + S::w1a + S::w2a + S::k);
  bf16* sOnes = (bf16*)(smem + S::w1a + S::w2a + S::k + S::vt);
  float* sbias = (float*)(smem + S::w1a + S::w2a + S::k + S::vt + S::ones);
  float* sv = sbias + 3 * D;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;

  const int row = c.row_first + (int)blockIdx.x;
  const DevBin& b = c.bins[c.row_bin[row]];
  if (b.st->phase == kDone) return;                 // whole workgroup, before any barrier
  const int n = b.n, slot = 32 * wave + l32;
  const int tok = slot < n ? b.tok_off + (row - b.row_off) * n + slot : -1;
  const int nkb = (n + 31) / 32;                    // key blocks holding a token

  // pair p's Wqkv fragments (3 s + m: k-step s of Q, K, V) and W_o fragments
  // (2 b + s), NQ / 4 and NO / 4 DMA blocks per wave
  auto dma_qkv = [&](int p) {
#pragma unroll
    for (int k = 0; k < NQ / 4; ++k) {
      const int u = wave + 4 * k;
      __builtin_amdgcn_global_load_lds(Wqf + ((long)p * NQ + u) * 512 + lane * 8,
                                       (__attribute__((address_space(3))) void*)(sw1 + u * 1024), 16, 0, 0);
    }
  };
  auto dma_o = [&](int p) {
#pragma unroll
    for (int k = 0; k < NO / 4; ++k) {
      const int u = wave + 4 * k;
      __builtin_amdgcn_global_load_lds(Wof + ((long)p * NO + u) * 512 + lane * 8,
                                       (__attribute__((address_space(3))) void*)(sw2 + (p & 1) * S::w2 + u * 1024), 16, 0,
                                       0);
    }
  };
  for (int i = tid; i < 3 * D; i += 256) sbias[i] = bqkv[i];
  if (tid < 128) sOnes[tid] = (bf16)1.0f;
  m3_stage_vectors<D>(sv, g, false, tid, 256);
  const bf16* __restrict__ A = (const bf16*)g.A;
  bf16x8 xf[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s)
    xf[s] = tok >= 0 ? *(const bf16x8*)(A + (long)tok * D + 16 * s + 8 * g2) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  dma_qkv(0);
  dma_o(0);
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // staged vectors written (visible after the first barrier)
  const float scale = 1.4426950408889634f / 4.0f;   // log2(e) / sqrt(16)
  f32x16 acc2[OBK][1];
#pragma unroll
  for (int ob = 0; ob < OBK; ++ob)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc2[ob][0][r] = 0.f;

#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    // Wqkv of pair p in LDS (issued before W_o of pair p, which may still be
    // in flight); every wave done with the previous pair's K and V^T
    m3_wait_barrier(NO / 4);
    const char* sq = sw1 + lane * 16;
    f32x16 aq, ak, av;
#pragma unroll
    for (int r = 0; r < 16; ++r) aq[r] = ak[r] = av[r] = 0.f;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const bf16x8 wq = *(const bf16x8*)(sq + (3 * s) * 1024);
      const bf16x8 wk = *(const bf16x8*)(sq + (3 * s + 1) * 1024);
      const bf16x8 wv = *(const bf16x8*)(sq + (3 * s + 2) * 1024);
      aq = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wq, xf[s], aq, 0, 0, 0);
      ak = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wk, xf[s], ak, 0, 0, 0);
      av = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xf[s], wv, av, 0, 0, 0);
    }
    // + bias, BF16: Q stays in registers (registers 8e .. 8e + 7 = head 2p + e);
    // K (key-major) and V^T (feature-major) are published for the whole row
    bf16x8 qf[2];
    const float bv = sbias[2 * D + 32 * p + l32];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = 32 * p + 8 * q + 4 * g2;
      const f32x4 bq = *(const f32x4*)&sbias[f];
      const f32x4 bk = *(const f32x4*)&sbias[D + f];
      bf16x4 kq, vq;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        qf[q >> 1][4 * (q & 1) + i] = (bf16)(aq[4 * q + i] + bq[i]);
        kq[i] = (bf16)(ak[4 * q + i] + bk[i]);
        vq[i] = (bf16)(av[4 * q + i] + bv);
      }
      *(bf16x4*)&sK[slot * LDK + 8 * q + 4 * g2] = kq;
      *(bf16x4*)&sVt[l32 * LDV + 32 * wave + 8 * q + 4 * g2] = vq;
    }
    // K, V^T of the row published, W_o of pair p in LDS; the Wqkv buffer
    // and the other W_o buffer (last read in pair p - 1) are free
    m3_wait_barrier(0);
    if (p + 1 < NP) {
      dma_qkv(p + 1);
      dma_o(p + 1);
    }

    f32x16 ob;                                       // O of the pair, pair features as Q's
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      // the PV product spans the pair's 32 features; the 16 rows of the other
      // head take the ones row instead of V^T, so that those output rows hold
      // the softmax denominator (the sum of the BF16 P that the product used)
      const bf16* vrow = (l32 >> 4) == e ? &sVt[l32 * LDV] : sOnes;
      float m = -INFINITY;
      f32x16 o;
#pragma unroll
      for (int r = 0; r < 16; ++r) o[r] = 0.f;
      // K fragment of key block kb (read one block ahead of its MFMA)
      auto kfrag = [&](int kb) {
        const bf16* kr = &sK[(32 * kb + l32) * LDK + 16 * e + 4 * g2];
        const bf16x4 k0 = *(const bf16x4*)kr, k1 = *(const bf16x4*)(kr + 8);
        return bf16x8{k0[0], k0[1], k0[2], k0[3], k1[0], k1[1], k1[2], k1[3]};
      };
      bf16x8 kn = kfrag(0);
#pragma unroll 1
      for (int kb = 0; kb < nkb; ++kb) {
        const bf16x8 kfr = kn;
        f32x16 st;
#pragma unroll
        for (int r = 0; r < 16; ++r) st[r] = 0.f;
        st = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kfr, qf[e], st, 0, 0, 0);
        if (kb + 1 < nkb) kn = kfrag(kb + 1);
        // register r: key 32 kb + 8(r/4) + 4 g2 + r%4; only the last block can
        // hold keys past n (a uniform branch)
        if (32 * kb + 32 > n) {
#pragma unroll
          for (int r = 0; r < 16; ++r)
            if (32 * kb + 8 * (r >> 2) + 4 * g2 + (r & 3) >= n) st[r] = -INFINITY;
        }
        float mb = -INFINITY;
#pragma unroll
        for (int r = 0; r < 16; ++r) mb = fmaxf(mb, st[r]);
        mb = xhalf_max(mb);
        // the running max m moves (and o, ls are rescaled) only when some
        // query's block max exceeds it by more than 8 / scale: until then
        // every p is at most 2^8, which FP32 sums and BF16 P carry exactly
        // as well; the first block always sets m (finite: it holds a token)
        if (__ballot(mb > m + 8.0f / scale) != 0ull) {   // wave-uniform
          const float mn = fmaxf(m, mb);
          const float corr = __builtin_amdgcn_exp2f((m - mn) * scale);
#pragma unroll
          for (int r = 0; r < 16; ++r) o[r] *= corr;
          m = mn;
        }
        const float mns = -m * scale;
        bf16x8 pf[2];
#pragma unroll
        for (int r = 0; r < 16; ++r) pf[r >> 3][r & 7] = (bf16)__builtin_amdgcn_exp2f(fmaf(st[r], scale, mns));
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const bf16* vr = vrow + 32 * kb + 16 * s + 4 * g2;
          const bf16x4 v0 = *(const bf16x4*)vr, v1 = *(const bf16x4*)(vr + 8);
          const bf16x8 vfr = bf16x8{v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
          o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vfr, pf[s], o, 0, 0, 0);
        }
      }
      const float inv = 1.0f / o[8 * (1 - e)];     // a ones row of V^T: the denominator
#pragma unroll
      for (int r = 0; r < 8; ++r) ob[8 * e + r] = o[8 * e + r] * inv;
    }
    bf16x8 of[2];
#pragma unroll
    for (int r = 0; r < 16; ++r) of[r >> 3][r & 7] = (bf16)ob[r];
#pragma unroll
    for (int bo = 0; bo < OBK; ++bo)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16x8 w = *(const bf16x8*)(sw2 + (p & 1) * S::w2 + (2 * bo + s) * 1024 + lane * 16);
        acc2[bo][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, of[s], acc2[bo][0], 0, 0, 0);
      }
  }
  // R and XN through the row-store epilogue: the Wqkv buffer was last read
  // before the last pair's publish barrier and W_o buffer NP & 1 before its
  // start barrier (8 KB slices for waves 0-2 and wave 3); row r of the wave
  // is slot 32 wave + r
  static_assert(S::w1a >= 3 * 8192 && S::w2 >= 8192, "an 8 KB slice per wave");
  char* const slice = wave < 3 ? sw1 + wave * 8192 : sw2 + (NP & 1) * S::w2;
  const long tok0 = b.tok_off + (long)(row - b.row_off) * n + 32 * wave;
  m3_residual_rows<D>(acc2, tok >= 0 ? (long)tok : g.M, g, g2, sv, slice, lane,
                      [&](int r) { return 32 * wave + r < n ? tok0 + r : -1L; });
}

// ---------------------------------------------------------------------------
// QKV projection + row attention for the BF16 path at head width 32
// (d = 256, rows of n <= 256 tokens): a workgroup of eight waves owns one
// row (wave w: slots 32 w .. 32 w + 31) and walks the heads; weight chunk h
// holds head h's Q, K and V rows (96 rows, double-buffered DMA).  Per head
// each wave projects its 32 tokens (V transposed, as in k_user_qkv_attn),
// keeps Q in registers and publishes its K block (key-major) and V^T block to
// LDS; then every wave runs its queries over the row's 32-key blocks with the
// online softmax of k_row_block_tr (lazy rescale).  O is written in BF16,
// four heads at a time right after a barrier; the output projection,
// residual and LayerNorm follow in k_oproj3.  HBM traffic: XN in, O out.
template <int D>
struct RQSmem {
  static constexpr int RB = D * 2 + 16;                // bytes per stored weight row
  static constexpr size_t w = (size_t)96 * RB;
  static constexpr size_t wa = (w + 15) / 16 * 16;
  // tile pitches of 18 and 130 dwords (see RBFSmem)
  static constexpr int LDK = 32 + 4;                   // K row: the head's 32 features + pad (bf16)
  static constexpr int LDV = 256 + 4;                  // V^T row: 256 keys + pad (bf16)
  static constexpr size_t k = (size_t)256 * LDK * 2;
  static constexpr size_t vt = (size_t)32 * LDV * 2;
  static constexpr size_t bias = (size_t)3 * D * 4;
  static constexpr size_t os = (size_t)8 * 2048;       // the waves' 2 KB O row-store slices
  static constexpr size_t bytes = 2 * wa + k + vt + bias + os;
  static_assert(bytes <= 160 * 1024 && (bytes - os) % 16 == 0, "LDS");
};

template <int D>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_row_qkv_attn(StepCtx c, const bf16* __restrict__ XN, const bf16* __restrict__ W,
                    const float* __restrict__ bqkv, bf16* __restrict__ O) {
  using S = RQSmem<D>;
  constexpr int RB = S::RB, LDK = S::LDK, LDV = S::LDV, KS = D / 16, HEADS = D / 32;
  constexpr int NB = (int)((S::w + 1023) / 1024), NPW = (NB + 7) / 8;
  static_assert(HEADS % 4 == 0, "heads in batches of four");
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  bf16* sK = (bf16*)(smem + 2 * S::wa);
  bf16* sVt = (bf16*)(smem + 2 * S::wa + S::k);
  float* sbias = (float*)(smem + 2 * S::wa + S::k + S::vt);
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;

  const int row = c.row_first + (int)blockIdx.x;
  const DevBin& b = c.bins[c.row_bin[row]];
  if (b.st->phase == kDone) return;                 // whole workgroup, before any barrier
  const int n = b.n, slot = 32 * wave + l32;
  const int tok = slot < n ? b.tok_off + (row - b.row_off) * n + slot : -1;
  const int nkb = (n + 31) / 32;                    // key blocks holding a token

  auto dma = [&](int h, int buf) {
    char* base = smem + buf * S::wa;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
      const int u = wave + k * 8;                   // uniform over the wave
      if (u >= NB) break;
      const int pos = u * 1024 + lane * 16, j = pos / RB, o = pos - j * RB;
      const bool data = o < RB - 16;                 // else a pad (copy something in bounds)
      const int jj = data ? j : 0;
      const bf16* src = W + (long)((jj >> 5) * D + h * 32 + (jj & 31)) * D + (data ? o / 2 : 0);
      if (pos < (int)S::w)
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(base + u * 1024), 16, 0, 0);
    }
  };
  for (int i = tid; i < 3 * D; i += 512) sbias[i] = bqkv[i];
  bf16x8 xf[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s)
    xf[s] = tok >= 0 ? *(const bf16x8*)(XN + (long)tok * D + 16 * s + 8 * g2) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  dma(0, 0);
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // staged bias written (visible after the first barrier)

  const float scale = 1.4426950408889634f / sqrtf(32.0f);
  constexpr int HB = 4;
  bf16x4 ob[HB][4];
  // O of a batch of heads leaves as whole 64-byte row segments (one head of
  // one row), through the wave's 2 KB LDS slice: 32 rows of 64 bytes, piece p
  // of row r at index p XOR ((r / 2) mod 4), so that both the writes (8 rows
  // of 2 lanes' pieces) and the row-order reads spread over all banks.  Each
  // pair of steps is first exchanged between the wave's halves, so that
  // every lane writes one whole 16-byte piece.  Row r of the wave is slot
  // 32 wave + r.
  char* const oslice = smem + (S::bytes - S::os) + wave * 2048;
  const long orow0 = b.tok_off + (long)(row - b.row_off) * n + 32 * wave;
  auto store_o = [&](int h0) {
    typedef unsigned u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned))));
    typedef unsigned u32x4 __attribute__((__vector_size__(4 * sizeof(unsigned))));
#pragma unroll
    for (int hh = 0; hh < HB; ++hh) {
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const u32x2 a0 = __builtin_bit_cast(u32x2, ob[hh][2 * k]);
        const u32x2 a1 = __builtin_bit_cast(u32x2, ob[hh][2 * k + 1]);
        const auto s0 = __builtin_amdgcn_permlane32_swap(a0[0], a1[0], false, false);
        const auto s1 = __builtin_amdgcn_permlane32_swap(a0[1], a1[1], false, false);
        *(u32x4*)(oslice + l32 * 64 + 16 * ((2 * k + g2) ^ ((l32 >> 1) & 3))) = u32x4{s0[0], s1[0], s0[1], s1[1]};
      }
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int r = 16 * t + (lane >> 2), pp = lane & 3;
        const u32x4 v = *(const u32x4*)(oslice + r * 64 + 16 * (pp ^ ((r >> 1) & 3)));
        if (32 * wave + r < n) *(u32x4*)(O + (orow0 + r) * D + (h0 + hh) * 32 + 8 * pp) = v;
      }
    }
  };
#pragma unroll
  for (int h = 0; h < HEADS; ++h) {
    // chunk h in LDS; every wave is done with the previous head's K, V^T and
    // with the buffer the next DMA refills; the previous batch's O stores
    // are complete too
    m3_wait_barrier(0);
    if (h % HB == 0 && h > 0) store_o(h - HB);      // every lane joins the exchange
    if (h + 1 < HEADS) dma(h + 1, (h + 1) & 1);
    const char* sw = smem + (h & 1) * S::wa;
    f32x16 aq, ak, av;
#pragma unroll
    for (int r = 0; r < 16; ++r) aq[r] = ak[r] = av[r] = 0.f;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const bf16x8 wq = *(const bf16x8*)(sw + l32 * RB + (2 * s + g2) * 16);
      const bf16x8 wk = *(const bf16x8*)(sw + (32 + l32) * RB + (2 * s + g2) * 16);
      const bf16x8 wv = *(const bf16x8*)(sw + (64 + l32) * RB + (2 * s + g2) * 16);
      aq = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wq, xf[s], aq, 0, 0, 0);
      ak = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wk, xf[s], ak, 0, 0, 0);
      av = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xf[s], wv, av, 0, 0, 0);
    }
    bf16x8 qf[2];
    const float bv = sbias[2 * D + h * 32 + l32];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = h * 32 + 8 * q + 4 * g2;
      const f32x4 bq = *(const f32x4*)&sbias[f];
      const f32x4 bk = *(const f32x4*)&sbias[D + f];
      bf16x4 kq, vq;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        qf[q >> 1][4 * (q & 1) + i] = (bf16)(aq[4 * q + i] + bq[i]);
        kq[i] = (bf16)(ak[4 * q + i] + bk[i]);
        vq[i] = (bf16)(av[4 * q + i] + bv);
      }
      *(bf16x4*)&sK[slot * LDK + 8 * q + 4 * g2] = kq;
      *(bf16x4*)&sVt[l32 * LDV + 32 * wave + 8 * q + 4 * g2] = vq;
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();                   // the row's K and V^T published
    asm volatile("" ::: "memory");

    float m = -INFINITY, ls = 0.f;
    f32x16 o;
#pragma unroll
    for (int r = 0; r < 16; ++r) o[r] = 0.f;
    // K fragments of key block kb (read one block ahead of their MFMAs)
    auto kfrag = [&](int kb, int s) {
      const bf16* kr = &sK[(32 * kb + l32) * LDK + 16 * s + 4 * g2];
      const bf16x4 k0 = *(const bf16x4*)kr, k1 = *(const bf16x4*)(kr + 8);
      return bf16x8{k0[0], k0[1], k0[2], k0[3], k1[0], k1[1], k1[2], k1[3]};
    };
    bf16x8 kn[2] = {kfrag(0, 0), kfrag(0, 1)};
#pragma unroll 1
    for (int kb = 0; kb < nkb; ++kb) {
      f32x16 st;
#pragma unroll
      for (int r = 0; r < 16; ++r) st[r] = 0.f;
      const bf16x8 kc0 = kn[0], kc1 = kn[1];
      st = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kc0, qf[0], st, 0, 0, 0);
      st = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kc1, qf[1], st, 0, 0, 0);
      if (kb + 1 < nkb) {
        kn[0] = kfrag(kb + 1, 0);
        kn[1] = kfrag(kb + 1, 1);
      }
      // register r: key 32 kb + 8(r/4) + 4 g2 + r%4; only the last block can
      // hold keys past n (a uniform branch)
      if (32 * kb + 32 > n) {
#pragma unroll
        for (int r = 0; r < 16; ++r)
          if (32 * kb + 8 * (r >> 2) + 4 * g2 + (r & 3) >= n) st[r] = -INFINITY;
      }
      float mb = -INFINITY;
#pragma unroll
      for (int r = 0; r < 16; ++r) mb = fmaxf(mb, st[r]);
      mb = xhalf_max(mb);
      // lazy rescale (see k_row_block_tr): m moves only when some query's
      // block max exceeds it by more than 8 / scale; the first block sets it
      if (__ballot(mb > m + 8.0f / scale) != 0ull) {   // wave-uniform
        const float mn = fmaxf(m, mb);
        const float corr = __builtin_amdgcn_exp2f((m - mn) * scale);
        ls *= corr;
#pragma unroll
        for (int r = 0; r < 16; ++r) o[r] *= corr;
        m = mn;
      }
      const float mns = -m * scale;
      bf16x8 pf[2];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float pv = __builtin_amdgcn_exp2f(fmaf(st[r], scale, mns));
        ls += pv;
        pf[r >> 3][r & 7] = (bf16)pv;
      }
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16* vr = &sVt[l32 * LDV + 32 * kb + 16 * s + 4 * g2];
        const bf16x4 v0 = *(const bf16x4*)vr, v1 = *(const bf16x4*)(vr + 8);
        const bf16x8 vfr = bf16x8{v0[0], v0[1], v0[2], v0[3], v1[0], v1[1], v1[2], v1[3]};
        o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vfr, pf[s], o, 0, 0, 0);
      }
    }
    ls = xhalf_sum(ls);
    const float inv = 1.0f / ls;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      ob[h % HB][q] = bf16x4{(bf16)(o[4 * q] * inv), (bf16)(o[4 * q + 1] * inv), (bf16)(o[4 * q + 2] * inv),
                             (bf16)(o[4 * q + 3] * inv)};
  }
  store_o(HEADS - HB);
}

// ---------------------------------------------------------------------------
// The user-attention sublayer and the MLP of one layer in one kernel (BF16,
// d = 128, head width 16): a wave owns a 32-slot group of whole columns (as
// in k_user_block_tr) for both sublayers, so the residual stream and the
// LayerNorm output between them never leave registers.
//   user:  R1 = R + W_o Attn(Wqkv XN) + b_o, X1 = LN_3(R1)      (registers)
//   MLP:   R2 = R1 + W2 GELU(W1 X1 + b1) + b2, then the next LayerNorm of R2
//          into XN (or, after the last layer, the final LayerNorm and the
//          symbol projection into lbar)
// X1 stays in the output-accumulator layout: k-step s of the up projection
// takes registers 8(s%2) .. 8(s%2) + 7 of block s/2, which hold features
// 16 s + 4 g2 + j and 16 s + 8 + 4 g2 + j - 4; the W1 fragments are read
// from LDS in that order (two 8-byte reads).  Weights go through one LDS
// region: the user sublayer's pair buffers (Wqkv rows refilled after every
// wave's projection, W_o columns after every wave's output projection),
// then the MLP's chunk ring.  HBM traffic per token: XN and R in, R and XN
// out, for two sublayers.
template <int D, int NBUF, int MAXF>
struct UMSmem {
  using U = UBSmem<D>;
  using M = M3Smem<D, NBUF, MAXF>;
  static constexpr size_t wu = U::w1a + U::w2a;            // user sublayer: Wqkv rows | W_o columns of a pair
  static constexpr size_t wm = NBUF * M::buf;              // MLP chunk ring
  static constexpr size_t w = wu > wm ? wu : wm;
  static constexpr size_t vec = (size_t)(3 * D + 3 * D + MAXF + 5 * D) * 4;   // bqkv, (b_o, LN3), b1, epilogue
  static constexpr size_t bytes = w + vec;
  static_assert(bytes <= 160 * 1024, "LDS");
};

struct UserMlpArgs {
  const bf16* Wqkv;
  const float* bqkv;
  const bf16* Wo;
  const float* bo;
  const float* ln3_g;
  const float* ln3_b;
  const bf16* W1;
  const float* b1;
  const bf16* W2;
  int F;
  GemmArgs g;   // A = out = XN, R, bias = b2, next LayerNorm (or final LayerNorm + proj_w / proj_out)
};

// The residual stream of the wave's tokens is final in acc2 (register layout
// as in m3_residual_epilogue, TB = 1): write it to R, then the next
// LayerNorm into g.out or (PROJ) the final LayerNorm and the 2-way
// projection into g.proj_out.
template <int D, bool PROJ>
__device__ __forceinline__ void m3_epilogue_final(f32x16 (&acc2)[D / 32][1], int tok, const GemmArgs& g, int g2,
                                                  const float* sv) {
  constexpr int OBK = D / 32;
  const float* slg = sv + D;
  const float* slb = sv + 2 * D;
  const bool tv = tok >= 0;
  float* Rrow = g.R + (long)(tv ? tok : 0) * D;
  float sum = 0.f;
#pragma unroll
  for (int b = 0; b < OBK; ++b)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = 32 * b + 8 * q + 4 * g2;
#pragma unroll
      for (int i = 0; i < 4; ++i) sum += acc2[b][0][4 * q + i];
      if (tv)
        *(f32x4*)(Rrow + f) = f32x4{acc2[b][0][4 * q], acc2[b][0][4 * q + 1], acc2[b][0][4 * q + 2],
                                    acc2[b][0][4 * q + 3]};
    }
  sum = xhalf_sum(sum);
  const float mean = sum / (float)D;
  float qv = 0.f;
#pragma unroll
  for (int b = 0; b < OBK; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float dv = acc2[b][0][r] - mean;
      qv = fmaf(dv, dv, qv);
    }
  qv = xhalf_sum(qv);
  const float rstd = 1.0f / sqrtf(qv / (float)D + 1e-5f);
  if (!PROJ) {
    if (tv) {
      bf16* xo = (bf16*)g.out + (long)tok * D;
#pragma unroll
      for (int b = 0; b < OBK; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int f = 32 * b + 8 * q + 4 * g2;
          const f32x4 lg = *(const f32x4*)&slg[f];
          const f32x4 lb = *(const f32x4*)&slb[f];
          bf16x4 h;
#pragma unroll
          for (int i = 0; i < 4; ++i) h[i] = (bf16)((acc2[b][0][4 * q + i] - mean) * rstd * lg[i] + lb[i]);
          *(bf16x4*)(xo + f) = h;
        }
    }
  } else {
    const float* sp0 = sv + 3 * D;
    const float* sp1 = sv + 4 * D;
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int f = 32 * b + 8 * q + 4 * g2;
        const f32x4 lg = *(const f32x4*)&slg[f];
        const f32x4 lb = *(const f32x4*)&slb[f];
        const f32x4 w0 = *(const f32x4*)&sp0[f];
        const f32x4 w1 = *(const f32x4*)&sp1[f];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float hv = (acc2[b][0][4 * q + i] - mean) * rstd * lg[i] + lb[i];
          a0 = fmaf(hv, w0[i], a0);
          a1 = fmaf(hv, w1[i], a1);
        }
      }
    a0 = xhalf_sum(a0);
    a1 = xhalf_sum(a1);
    if (tv && g2 == 0) {
      g.proj_out[2 * (long)tok] = a0;
      g.proj_out[2 * (long)tok + 1] = a1;
    }
  }
}

// The same results as m3_epilogue_final, with the R and XN rows stored
// through the wave's 8 KB LDS slice `lds` (rows_store_f32 / rows_store_bf16).
template <int D, bool PROJ, class RowTok>
__device__ __forceinline__ void m3_epilogue_rows(f32x16 (&acc2)[D / 32][1], int tok, const GemmArgs& g, int g2,
                                                 const float* sv, char* lds, int lane, RowTok rowtok) {
  constexpr int OBK = D / 32;
  const float* slg = sv + D;
  const float* slb = sv + 2 * D;
  float sum = 0.f;
#pragma unroll
  for (int b = 0; b < OBK; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) sum += acc2[b][0][r];
  sum = xhalf_sum(sum);
  const float mean = sum / (float)D;
  float qv = 0.f;
#pragma unroll
  for (int b = 0; b < OBK; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float dv = acc2[b][0][r] - mean;
      qv = fmaf(dv, dv, qv);
    }
  qv = xhalf_sum(qv);
  const float rstd = 1.0f / sqrtf(qv / (float)D + 1e-5f);
  // the same values under new names: the compiler would otherwise keep every
  // (acc2 - mean) of the variance loop alive for the LayerNorm below
  float mean2 = mean, rstd2 = rstd;
  asm volatile("" : "+v"(mean2), "+v"(rstd2));
  if (!PROJ) {
    rows_store_bf16<D>(
        [&](int b, int q) {
          const int f = 32 * b + 8 * q + 4 * g2;
          const f32x4 lg = *(const f32x4*)&slg[f];
          const f32x4 lb = *(const f32x4*)&slb[f];
          bf16x4 h;
#pragma unroll
          for (int i = 0; i < 4; ++i) h[i] = (bf16)((acc2[b][0][4 * q + i] - mean2) * rstd2 * lg[i] + lb[i]);
          return h;
        },
        (bf16*)g.out, lds, lane, rowtok);
  } else {
    const float* sp0 = sv + 3 * D;
    const float* sp1 = sv + 4 * D;
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int f = 32 * b + 8 * q + 4 * g2;
        const f32x4 lg = *(const f32x4*)&slg[f];
        const f32x4 lb = *(const f32x4*)&slb[f];
        const f32x4 w0 = *(const f32x4*)&sp0[f];
        const f32x4 w1 = *(const f32x4*)&sp1[f];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float hv = (acc2[b][0][4 * q + i] - mean2) * rstd2 * lg[i] + lb[i];
          a0 = fmaf(hv, w0[i], a0);
          a1 = fmaf(hv, w1[i], a1);
        }
      }
    a0 = xhalf_sum(a0);
    a1 = xhalf_sum(a1);
    if (tok >= 0 && g2 == 0) {
      g.proj_out[2 * (long)tok] = a0;
      g.proj_out[2 * (long)tok + 1] = a1;
    }
  }
  rows_store_f32<D>(
      [&](int b, int q) {
        return f32x4{acc2[b][0][4 * q], acc2[b][0][4 * q + 1], acc2[b][0][4 * q + 2], acc2[b][0][4 * q + 3]};
      },
      g.R, lds, lane, rowtok);
}

template <int D, int NW, int NBUF, int MAXF, bool PROJ, int PF>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_user_mlp_tr(StepCtx c, UserMlpArgs a) {
  using S = UMSmem<D, NBUF, MAXF>;
  // two waves per SIMD: two 4-wave workgroups per CU, or one 8-wave workgroup
  static_assert(NW == 8 || S::bytes <= 80 * 1024, "two workgroups per CU");
  using U = UBSmem<D>;
  using M = typename S::M;
  constexpr int RB1 = U::RB1, RB2 = U::RB2, KS = D / 16, NP = D / 32, OBK = D / 32, NTHR = NW * 64;
  constexpr int U1 = (int)((U::w1 + 1023) / 1024), U2 = (int)((U::w2 + 1023) / 1024);
  constexpr int MRB1 = M::RB1, MRB2 = M::RB2;
  constexpr int N1 = (int)((M::w1 + 1023) / 1024), N2 = (int)((M::w2 + 1023) / 1024);
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  char* su1 = smem;                                 // user: Wqkv rows of the pair
  char* su2 = smem + U::w1a;                        // user: W_o columns of the pair
  float* sbias = (float*)(smem + S::w);             // bqkv [3D]
  float* svu = sbias + 3 * D;                       // b_o, LN3 gain, LN3 bias
  float* sb1 = svu + 3 * D;                         // b1 [MAXF]
  float* svm = sb1 + MAXF;                          // b2, next LayerNorm, projection rows
  const GemmArgs& g = a.g;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;
  const int F = a.F, nch = F / kM3FCH;

  // ---- this lane's slot of the wave's group
  const int gi = blockIdx.x * NW + wave;
  int tok = -1, K = 1;
  if (gi < c.total_ugrp32) {
    const int bi = c.ugrp32[2 * gi], c0 = c.ugrp32[2 * gi + 1];
    const DevBin& b = c.bins[bi];
    K = b.K;
    const int C = 32 / K, cl = l32 / K, k = l32 - cl * K;
    if (l32 < C * K && c0 + cl < b.n) tok = b.tok_off + k * b.n + c0 + cl;
  }
  const unsigned long long vmask = __ballot(tok >= 0);
  unsigned okbits = 0;                               // register r of S^T: key slot 8(r/4) + 4 g2 + r%4
  const int col_lo = (l32 / K) * K;                 // key slots of this lane's column: col_lo .. col_lo + K - 1
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int kr = 8 * (r >> 2) + 4 * g2 + (r & 3);
    if (((vmask >> kr) & 1ull) && (unsigned)(kr - col_lo) < (unsigned)K) okbits |= 1u << r;
  }

  // ---- user-sublayer weights of head pair p (per-wave DMA counts uniform)
  const int nu1 = U1 / NW + (wave < U1 % NW ? 1 : 0), nu2 = U2 / NW + (wave < U2 % NW ? 1 : 0);
  auto dma_qkv = [&](int p) {
#pragma unroll
    for (int k = 0; k < (U1 + NW - 1) / NW; ++k) {
      const int u = wave + NW * k;
      if (u >= U1) break;
      const int pos = u * 1024 + lane * 16, j = pos / RB1, o = pos - j * RB1;
      const bool data = o < RB1 - 16;
      const int jj = data ? j : 0;
      const bf16* src = a.Wqkv + (long)((jj >> 5) * D + 32 * p + (jj & 31)) * D + (data ? o / 2 : 0);
      if (pos < (int)U::w1)
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(su1 + u * 1024), 16, 0, 0);
    }
  };
  auto dma_o = [&](int p) {
#pragma unroll
    for (int k = 0; k < (U2 + NW - 1) / NW; ++k) {
      const int u = wave + NW * k;
      if (u >= U2) break;
      const int pos = u * 1024 + lane * 16, j = pos / RB2, o = pos - j * RB2;
      const bool data = o < RB2 - 16;
      const bf16* src = a.Wo + (long)(data ? j : 0) * D + 32 * p + (data ? o / 2 : 0);
      if (pos < (int)U::w2)
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(su2 + u * 1024), 16, 0, 0);
    }
  };
  // ---- MLP chunk c -> ring buffer
  const int nwm = (N1 + N2) / NW + (wave < (N1 + N2) % NW ? 1 : 0);
  M3ChunkDma<NW, N1, N2, MRB1, MRB2, (int)M::w1, (int)M::w2, (int)M::w1a> mdma;
  mdma.init(wave, lane, D, F);
  auto dma_m = [&](int ch, int buf) { mdma.issue(a.W1, a.W2, ch * kM3FCH, smem + buf * M::buf); };

  for (int i = tid; i < 3 * D; i += NTHR) sbias[i] = a.bqkv[i];
  for (int i = tid; i < D; i += NTHR) {
    svu[i] = a.bo[i];
    svu[D + i] = a.ln3_g[i];
    svu[2 * D + i] = a.ln3_b[i];
  }
  for (int i = tid; i < F; i += NTHR) sb1[i] = a.b1[i];
  m3_stage_vectors<D>(svm, g, PROJ, tid, NTHR);
  const bf16* __restrict__ XN = (const bf16*)g.A;
  bf16x8 xf[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s)
    xf[s] = tok >= 0 ? *(const bf16x8*)(XN + (long)tok * D + 16 * s + 8 * g2) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  dma_qkv(0);
  dma_o(0);
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // staged vectors written (visible after the first barrier)

  // ================= user sublayer (see k_user_block_tr) =================
  const float scale = 1.4426950408889634f / 4.0f;     // log2(e) / sqrt(16)
  f32x16 acc2[OBK][1];
#pragma unroll
  for (int ob = 0; ob < OBK; ++ob)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc2[ob][0][r] = 0.f;
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    m3_wait_barrier(nu2);                            // Wqkv of pair p in LDS (W_o of p may be in flight)
    f32x16 aq, ak, av;
#pragma unroll
    for (int r = 0; r < 16; ++r) aq[r] = ak[r] = av[r] = 0.f;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const bf16x8 wq = *(const bf16x8*)(su1 + l32 * RB1 + (2 * s + g2) * 16);
      const bf16x8 wk = *(const bf16x8*)(su1 + (32 + l32) * RB1 + (2 * s + g2) * 16);
      const bf16x8 wv = *(const bf16x8*)(su1 + (64 + l32) * RB1 + (2 * s + g2) * 16);
      aq = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wq, xf[s], aq, 0, 0, 0);
      ak = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wk, xf[s], ak, 0, 0, 0);
      av = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xf[s], wv, av, 0, 0, 0);
    }
    bf16x8 qf[2], kf[2], vf[2];
    const float bv = sbias[2 * D + 32 * p + l32];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = 32 * p + 8 * q + 4 * g2;
      const f32x4 bq = *(const f32x4*)&sbias[f];
      const f32x4 bk = *(const f32x4*)&sbias[D + f];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 4 * q + i;
        qf[r >> 3][r & 7] = (bf16)(aq[r] + bq[i]);
        kf[r >> 3][r & 7] = (bf16)(ak[r] + bk[i]);
        vf[r >> 3][r & 7] = (bf16)(av[r] + bv);
      }
    }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();                   // every wave is done with the Wqkv buffer
    asm volatile("" ::: "memory");
    if (p + 1 < NP) dma_qkv(p + 1);
    f32x16 ob;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      f32x16 st;
#pragma unroll
      for (int r = 0; r < 16; ++r) st[r] = 0.f;
      st = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf[e], qf[e], st, 0, 0, 0);
      float mx = -INFINITY;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        st[r] = ((okbits >> r) & 1u) ? st[r] : -INFINITY;
        mx = fmaxf(mx, st[r]);
      }
      mx = xhalf_max(mx);
      const float mxs = mx == -INFINITY ? 0.f : -mx * scale;   // a padding query has no valid key
      float ps = 0.f;
      bf16x8 pf[2];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float pv = __builtin_amdgcn_exp2f(fmaf(st[r], scale, mxs));
        ps += pv;
        pf[r >> 3][r & 7] = (bf16)pv;
      }
      ps = xhalf_sum(ps);
      f32x16 o;
#pragma unroll
      for (int r = 0; r < 16; ++r) o[r] = 0.f;
      o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf[0], pf[0], o, 0, 0, 0);
      o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf[1], pf[1], o, 0, 0, 0);
      const float inv = ps > 0.f ? 1.0f / ps : 0.f;
#pragma unroll
      for (int r = 0; r < 8; ++r) ob[8 * e + r] = o[8 * e + r] * inv;
    }
    // W_o of pair p in LDS (the Wqkv DMA of pair p + 1 may be in flight)
    m3_wait_barrier(p + 1 < NP ? nu1 : 0);
    bf16x8 of[2];
#pragma unroll
    for (int r = 0; r < 16; ++r) of[r >> 3][r & 7] = (bf16)ob[r];
#pragma unroll
    for (int bo = 0; bo < OBK; ++bo)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const char* wr = su2 + (32 * bo + l32) * RB2;
        const bf16x8 w = *(const bf16x8*)(wr + (16 * s + 8 * g2) * 2);   // k-ordered rows
        acc2[bo][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, of[s], acc2[bo][0], 0, 0, 0);
      }
    asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
    __builtin_amdgcn_s_barrier();                   // every wave is done with the W_o buffer
    asm volatile("" ::: "memory");
    if (p + 1 < NP) dma_o(p + 1);
  }
  // the user weights are dead: the MLP ring takes the region
  const int pre = min(NBUF - 1, nch);
  for (int ch = 0; ch < pre; ++ch) dma_m(ch, ch);

  // ---- R1 = R + acc2 + b_o in place, X1 = LN3(R1) as the up projection's B
  // operand; acc2 then starts the MLP at R1 + b2, so the down projection
  // accumulates the final residual directly
  bf16x8 x1[KS];
  {
    const bool tv = tok >= 0;
    const float* Rrow = g.R + (long)(tv ? tok : 0) * D;
    float sum = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b) {
      f32x4 rr[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        rr[q] = tv ? *(const f32x4*)(Rrow + 32 * b + 8 * q + 4 * g2) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 bias = *(const f32x4*)&svu[32 * b + 8 * q + 4 * g2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float res = rr[q][i] + (acc2[b][0][4 * q + i] + bias[i]);
          acc2[b][0][4 * q + i] = res;
          sum += res;
        }
      }
      // finish this block before the next block's loads (bounds the registers in flight)
      asm volatile("" : "+v"(acc2[b][0]), "+v"(sum)::"memory");
    }
    sum = xhalf_sum(sum);
    const float mean = sum / (float)D;
    float qv = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float dv = acc2[b][0][r] - mean;
        qv = fmaf(dv, dv, qv);
      }
    qv = xhalf_sum(qv);
    const float rstd = 1.0f / sqrtf(qv / (float)D + 1e-5f);
    // k-step s of the up projection: registers 8(s%2) .. 8(s%2) + 7 of block s/2
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int f = 32 * b + 8 * q + 4 * g2;
        const f32x4 lg = *(const f32x4*)&svu[D + f];
        const f32x4 lb = *(const f32x4*)&svu[2 * D + f];
        const f32x4 b2 = *(const f32x4*)&svm[f];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          x1[2 * b + (q >> 1)][4 * (q & 1) + i] = (bf16)((acc2[b][0][4 * q + i] - mean) * rstd * lg[i] + lb[i]);
          acc2[b][0][4 * q + i] += b2[i];
        }
        if (q & 1) asm volatile("" : "+v"(x1[2 * b + (q >> 1)]), "+v"(acc2[b][0])::"memory");
      }
  }

  // ================= MLP (one chunk of 32 hidden units at a time) =================
  m3_wait_barrier(nwm * max(0, pre - 1));           // chunk 0 in LDS
#pragma unroll 1
  for (int ch = 0; ch < nch; ++ch) {
    // buffer (ch + NBUF - 1) % NBUF was last read in iteration ch - 1, before its closing barrier
    if (ch + NBUF - 1 < nch) dma_m(ch + NBUF - 1, (ch + NBUF - 1) % NBUF);
    const char* s1 = smem + (ch % NBUF) * M::buf;
    const char* s2 = s1 + M::w1a;
    const float* sb = sb1 + ch * kM3FCH;
    f32x16 acc1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 bq = *(const f32x4*)&sb[16 * (q >> 1) + 8 * g2 + 4 * (q & 1)];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc1[4 * q + i] = bq[i];
    }
    // W1 k-values in X1's order (16 s + 4 g2 + j, then 16 s + 8 + 4 g2 + j):
    // the k-ordered copy holds them contiguously
    const char* wr = s1 + l32 * MRB1;
    mfma_pipe<KS, PF>(
        [&](int s) {
          return *(const bf16x8*)(wr + (16 * s + 8 * g2) * 2);   // k-ordered rows
        },
        [&](int s, const bf16x8& w) { acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, x1[s], acc1, 0, 0, 0); });
    bf16x8 hf[2];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) hf[q >> 1][4 * (q & 1) + i] = (bf16)gelu_f(acc1[4 * q + i]);
    mfma_pipe<2 * OBK, PF>(
        [&](int j) { return *(const bf16x8*)(s2 + (32 * (j >> 1) + l32) * MRB2 + (2 * (j & 1) + g2) * 16); },
        [&](int j, const bf16x8& w) {
          acc2[j >> 1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, hf[j & 1], acc2[j >> 1][0], 0, 0, 0);
        });
    // chunk ch + 1 complete in every wave: later chunks (at most NBUF - 2) may be in flight
    if (ch + 1 < nch) m3_wait_barrier(nwm * (min(ch + NBUF - 1, nch - 1) - (ch + 1)));
  }
  m3_epilogue_final<D, PROJ>(acc2, tok, g, g2, svm);
}

// ---------------------------------------------------------------------------
// k_user_mlp_f: the computation of k_user_mlp_tr (the same MFMA sequence for
// every output, so the same bits) on fragment-major weight copies
// (Mat::b16f; see k_oproj_mlp4), four waves per workgroup, two workgroups
// per CU.  The user sublayer's weights of a head pair (its Wqkv fragments,
// then its W_o fragments, 32 KB at d = 128) are double-buffered, so a pair
// costs one barrier instead of four; the MLP's first two chunks are DMA'd
// into the first pair buffer during the last pair, and the MLP chunks (16 KB)
// then run through a ring of two.
template <int D, int MAXF>
struct UMFSmem {
  static constexpr int KS = D / 16, OBK = D / 32;
  static constexpr size_t ub = (size_t)(3 * KS + 2 * OBK) * 1024;   // a head pair's Wqkv and W_o fragments
  static constexpr size_t mb = (size_t)(KS + 2 * OBK) * 1024;       // an MLP chunk's W1 and W2 fragments
  static constexpr size_t vec = ((size_t)(3 * D + 3 * D + MAXF + 5 * D) * 4 + 1023) / 1024 * 1024;
  static constexpr size_t bytes = vec + 2 * ub;
  static_assert(2 * mb <= ub, "the MLP ring fits in the first pair buffer");
  static_assert(ub >= 4 * 8192, "the second pair buffer holds the four waves' 8 KB epilogue slices");
  static_assert(bytes <= 80 * 1024, "two workgroups per CU");
};

template <int D, int MAXF, bool PROJ, int PF>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_user_mlp_f(StepCtx c, UserMlpArgs a) {
  using S = UMFSmem<D, MAXF>;
  constexpr int NW = 4, KS = D / 16, NP = D / 32, OBK = D / 32, NTHR = NW * 64;
  constexpr int NQ = 3 * KS, NO = 2 * OBK, NUB = NQ + NO, NM = KS + NO;   // 1 KB fragments per pair / MLP chunk
  static_assert(NUB % NW == 0 && NM % NW == 0 && NP % 2 == 0, "DMA blocks split evenly; the last pair in buffer 1");
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  float* sbias = (float*)smem;                      // bqkv [3D]
  float* svu = sbias + 3 * D;                       // b_o, LN3 gain, LN3 bias
  float* sb1 = svu + 3 * D;                         // b1 [MAXF]
  float* svm = sb1 + MAXF;                          // b2, next LayerNorm, projection rows
  char* const wreg = smem + S::vec;
  const GemmArgs& g = a.g;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;
  const int F = a.F, nch = F / kM3FCH;

  // ---- this lane's slot of the wave's group
  const int gi = blockIdx.x * NW + wave;
  int tok = -1, K = 1;
  if (gi < c.total_ugrp32) {
    const int bi = c.ugrp32[2 * gi], c0 = c.ugrp32[2 * gi + 1];
    const DevBin& b = c.bins[bi];
    K = b.K;
    const int C = 32 / K, cl = l32 / K, k = l32 - cl * K;
    if (l32 < C * K && c0 + cl < b.n) tok = b.tok_off + k * b.n + c0 + cl;
  }
  const unsigned long long vmask = __ballot(tok >= 0);
  unsigned okbits = 0;                               // register r of S^T: key slot 8(r/4) + 4 g2 + r%4
  const int col_lo = (l32 / K) * K;                 // key slots of this lane's column: col_lo .. col_lo + K - 1
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int kr = 8 * (r >> 2) + 4 * g2 + (r & 3);
    if (((vmask >> kr) & 1ull) && (unsigned)(kr - col_lo) < (unsigned)K) okbits |= 1u << r;
  }

  // head pair p: its NQ Wqkv fragments (3 s + m: k-step s of Q, K, V), then its NO W_o fragments
  auto dma_u = [&](int p, int buf) {
#pragma unroll
    for (int k = 0; k < NUB / NW; ++k) {
      const int u = wave + NW * k;
      const bf16* src = u < NQ ? a.Wqkv + ((long)p * NQ + u) * 512 : a.Wo + ((long)p * NO + (u - NQ)) * 512;
      __builtin_amdgcn_global_load_lds(src + lane * 8,
                                       (__attribute__((address_space(3))) void*)(wreg + buf * S::ub + u * 1024), 16, 0, 0);
    }
  };
  // MLP chunk ch: its KS W1 fragments, then its NO W2 fragments
  auto dma_m = [&](int ch, int buf) {
#pragma unroll
    for (int k = 0; k < NM / NW; ++k) {
      const int u = wave + NW * k;
      const bf16* src = u < KS ? a.W1 + ((long)ch * KS + u) * 512 : a.W2 + ((long)ch * NO + (u - KS)) * 512;
      __builtin_amdgcn_global_load_lds(src + lane * 8,
                                       (__attribute__((address_space(3))) void*)(wreg + buf * S::mb + u * 1024), 16, 0, 0);
    }
  };

  for (int i = tid; i < 3 * D; i += NTHR) sbias[i] = a.bqkv[i];
  for (int i = tid; i < D; i += NTHR) {
    svu[i] = a.bo[i];
    svu[D + i] = a.ln3_g[i];
    svu[2 * D + i] = a.ln3_b[i];
  }
  for (int i = tid; i < F; i += NTHR) sb1[i] = a.b1[i];
  m3_stage_vectors<D>(svm, g, PROJ, tid, NTHR);
  const bf16* __restrict__ XN = (const bf16*)g.A;
  bf16x8 xf[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s)
    xf[s] = tok >= 0 ? *(const bf16x8*)(XN + (long)tok * D + 16 * s + 8 * g2) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  dma_u(0, 0);
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // staged vectors written (visible after the first barrier)

  // ================= user sublayer (as k_user_mlp_tr) =================
  const float scale = 1.4426950408889634f / 4.0f;     // log2(e) / sqrt(16)
  f32x16 acc2[OBK][1];
#pragma unroll
  for (int ob = 0; ob < OBK; ++ob)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc2[ob][0][r] = 0.f;
#pragma unroll 1
  for (int p = 0; p < NP; ++p) {
    // pair p in LDS in every wave, and every wave done with pair p - 1, whose buffer the next DMA refills
    m3_wait_barrier(0);
    if (p + 1 < NP) {
      dma_u(p + 1, (p + 1) & 1);
    } else {
      // the last pair reads buffer 1: the MLP ring's first two chunks go into buffer 0
      dma_m(0, 0);
      if (nch > 1) dma_m(1, 1);
    }
    const char* su = wreg + (p & 1) * S::ub + lane * 16;
    f32x16 aq, ak, av;
#pragma unroll
    for (int r = 0; r < 16; ++r) aq[r] = ak[r] = av[r] = 0.f;
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const bf16x8 wq = *(const bf16x8*)(su + (3 * s) * 1024);
      const bf16x8 wk = *(const bf16x8*)(su + (3 * s + 1) * 1024);
      const bf16x8 wv = *(const bf16x8*)(su + (3 * s + 2) * 1024);
      aq = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wq, xf[s], aq, 0, 0, 0);
      ak = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wk, xf[s], ak, 0, 0, 0);
      av = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xf[s], wv, av, 0, 0, 0);
    }
    bf16x8 qf[2], kf[2], vf[2];
    const float bv = sbias[2 * D + 32 * p + l32];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = 32 * p + 8 * q + 4 * g2;
      const f32x4 bq = *(const f32x4*)&sbias[f];
      const f32x4 bk = *(const f32x4*)&sbias[D + f];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 4 * q + i;
        qf[r >> 3][r & 7] = (bf16)(aq[r] + bq[i]);
        kf[r >> 3][r & 7] = (bf16)(ak[r] + bk[i]);
        vf[r >> 3][r & 7] = (bf16)(av[r] + bv);
      }
    }
    f32x16 ob;
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      f32x16 st;
#pragma unroll
      for (int r = 0; r < 16; ++r) st[r] = 0.f;
      st = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf[e], qf[e], st, 0, 0, 0);
      float mx = -INFINITY;
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        st[r] = ((okbits >> r) & 1u) ? st[r] : -INFINITY;
        mx = fmaxf(mx, st[r]);
      }
      mx = xhalf_max(mx);
      const float mxs = mx == -INFINITY ? 0.f : -mx * scale;   // a padding query has no valid key
      float ps = 0.f;
      bf16x8 pf[2];
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float pv = __builtin_amdgcn_exp2f(fmaf(st[r], scale, mxs));
        ps += pv;
        pf[r >> 3][r & 7] = (bf16)pv;
      }
      ps = xhalf_sum(ps);
      f32x16 o;
#pragma unroll
      for (int r = 0; r < 16; ++r) o[r] = 0.f;
      o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf[0], pf[0], o, 0, 0, 0);
      o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf[1], pf[1], o, 0, 0, 0);
      const float inv = ps > 0.f ? 1.0f / ps : 0.f;
#pragma unroll
      for (int r = 0; r < 8; ++r) ob[8 * e + r] = o[8 * e + r] * inv;
    }
    bf16x8 of[2];
#pragma unroll
    for (int r = 0; r < 16; ++r) of[r >> 3][r & 7] = (bf16)ob[r];
    // W_o fragment 2 bo + s: output block bo, k-step s of the pair's columns
#pragma unroll
    for (int bo = 0; bo < OBK; ++bo)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16x8 w = *(const bf16x8*)(su + (NQ + 2 * bo + s) * 1024);
        acc2[bo][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, of[s], acc2[bo][0], 0, 0, 0);
      }
  }

  // ---- R1 = R + acc2 + b_o in place, X1 = LN3(R1) as the up projection's B
  // operand; acc2 then starts the MLP at R1 + b2
  bf16x8 x1[KS];
  {
    const bool tv = tok >= 0;
    const float* Rrow = g.R + (long)(tv ? tok : 0) * D;
    float sum = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b) {
      f32x4 rr[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        rr[q] = tv ? *(const f32x4*)(Rrow + 32 * b + 8 * q + 4 * g2) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 bias = *(const f32x4*)&svu[32 * b + 8 * q + 4 * g2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float res = rr[q][i] + (acc2[b][0][4 * q + i] + bias[i]);
          acc2[b][0][4 * q + i] = res;
          sum += res;
        }
      }
      asm volatile("" : "+v"(acc2[b][0]), "+v"(sum)::"memory");   // bounds the loads in flight
    }
    sum = xhalf_sum(sum);
    const float mean = sum / (float)D;
    float qv = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float dv = acc2[b][0][r] - mean;
        qv = fmaf(dv, dv, qv);
      }
    qv = xhalf_sum(qv);
    const float rstd = 1.0f / sqrtf(qv / (float)D + 1e-5f);
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int f = 32 * b + 8 * q + 4 * g2;
        const f32x4 lg = *(const f32x4*)&svu[D + f];
        const f32x4 lb = *(const f32x4*)&svu[2 * D + f];
        const f32x4 b2 = *(const f32x4*)&svm[f];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          x1[2 * b + (q >> 1)][4 * (q & 1) + i] = (bf16)((acc2[b][0][4 * q + i] - mean) * rstd * lg[i] + lb[i]);
          acc2[b][0][4 * q + i] += b2[i];
        }
        if (q & 1) asm volatile("" : "+v"(x1[2 * b + (q >> 1)]), "+v"(acc2[b][0])::"memory");
      }
  }

  // ================= MLP (one chunk of 32 hidden units at a time) =================
  m3_wait_barrier(0);                               // chunks 0 and 1 in LDS, every wave done with the user weights
#pragma unroll 1
  for (int ch = 0; ch < nch; ++ch) {
    // the other buffer was last read in iteration ch - 1, before its closing barrier
    if (ch >= 1 && ch + 1 < nch) dma_m(ch + 1, (ch + 1) & 1);
    const char* s1 = wreg + (ch & 1) * S::mb + lane * 16;
    const float* sb = sb1 + ch * kM3FCH;
    f32x16 acc1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 bq = *(const f32x4*)&sb[16 * (q >> 1) + 8 * g2 + 4 * (q & 1)];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc1[4 * q + i] = bq[i];
    }
    mfma_pipe<KS, PF>([&](int s) { return *(const bf16x8*)(s1 + s * 1024); },
                      [&](int s, const bf16x8& w) { acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, x1[s], acc1, 0, 0, 0); });
    // GELU of the first 8 hidden values (the down projection's k-step 0);
    // the other 8 are computed between the k-step 0 MFMAs, which run first
    // (per output block the k-steps keep their order)
    bf16x8 hf[2];
#pragma unroll
    for (int v = 0; v < 8; ++v) hf[0][v] = (bf16)gelu_f(acc1[v]);
    mfma_pipe<NO, PF>(
        [&](int i) { return *(const bf16x8*)(s1 + (KS + 2 * (i % OBK) + i / OBK) * 1024); },
        [&](int i, const bf16x8& w) {
          acc2[i % OBK][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, hf[i / OBK], acc2[i % OBK][0], 0, 0, 0);
          if (i < OBK) {
#pragma unroll
            for (int v = (i * 8) / OBK; v < ((i + 1) * 8) / OBK; ++v) hf[1][v] = (bf16)gelu_f(acc1[8 + v]);
          }
        });
    // chunk ch + 1 complete in every wave, and every wave done with buffer ch & 1
    if (ch + 1 < nch) m3_wait_barrier(0);
  }
  // the second head-pair buffer was last read in the user sublayer, before
  // the barrier ahead of the MLP loop; row r of the wave is lane r's token
  m3_epilogue_rows<D, PROJ>(acc2, tok, g, g2, svm, wreg + S::ub + wave * 8192, lane,
                            [&](int r) { return (long)__shfl(tok, r); });
}

// ---------------------------------------------------------------------------
// The output projection of an attention sublayer and the MLP that follows,
// in one token-resident kernel (BF16, d = 256): the residual stream and the
// LayerNorm output between them stay in registers.
//   R1 = R + O W_o^T + b_o,  X1 = LN(R1)                    (registers)
//   R2 = R1 + W2 GELU(W1 X1 + b1) + b2, then the next LayerNorm of R2 into XN
//   (or, after the last layer, the final LayerNorm and the projection)
// The output projection is k_oproj3's (W_o columns in 128-wide chunks through
// LDS, O fragments read one chunk ahead); X1 stays in the output
// accumulator's layout and the W1 fragments are read in that order (as in
// k_user_mlp_tr); the MLP accumulator starts at R1 + b2.  The weight buffers
// of the two phases share one LDS region.  HBM traffic per token: O, R in;
// R, XN out (12d bytes against 24d for the two kernels).
template <int D, int NBUF, int MAXF>
struct OMSmem {
  using O = O3Smem<D, 128>;
  using M = M3Smem<D, NBUF, MAXF>;
  static constexpr size_t wo = 2 * O::wa;
  static constexpr size_t wm = NBUF * M::buf;
  static constexpr size_t w = wo > wm ? wo : wm;
  static constexpr size_t vec = (size_t)(3 * D + MAXF + 5 * D) * 4;   // (b_o, LN), b1, epilogue vectors
  static constexpr size_t bytes = w + vec;
  static_assert(bytes <= 160 * 1024, "LDS");
};

// F8: the MLP up projection in e4m3 (v_mfma_scale_f32_32x32x64_f8f6f4, unit
// block scales): X1 is quantised per token (amax / 448) straight from the
// LayerNorm, and W1q is the e4m3 copy of W1 (per-tensor scale w1s) with each
// row's columns reordered so that a lane's 32 bytes of a 64-wide k step are
// contiguous: row position 64 t + 32 h + 8 s + e holds feature
// 16 (4 t + s) + 8 (e / 4) + 4 h + e % 4, the feature a lane of half h
// holds in byte 8 s + e of its X1 fragment t.  The result has the BF16 up
// projection's layout, so the GELU and the down projection are unchanged.
template <int D, int NBUF, int MAXF, bool PROJ, int PF, bool F8 = false>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_oproj_mlp3(GemmArgs g, const bf16* __restrict__ Wo, const float* __restrict__ bo, const float* __restrict__ lnx_g,
                  const float* __restrict__ lnx_b, const bf16* __restrict__ W1, const float* __restrict__ b1,
                  const bf16* __restrict__ W2, int F, const uint8_t* __restrict__ W1q, float w1s) {
  constexpr int KCH = 128;
  using S = OMSmem<D, NBUF, MAXF>;
  using O = typename S::O;
  using M = typename S::M;
  constexpr int NW = 8, RB = O::RB, OBK = D / 32, NCH = O::NCH, KSC = KCH / 16, KS = D / 16;
  constexpr int NB = (int)(O::wa / 1024), NPW = (NB + NW - 1) / NW;
  constexpr int MRB1 = M::RB1, MRB2 = M::RB2;
  constexpr int N1 = (int)((M::w1 + 1023) / 1024), N2 = (int)((M::w2 + 1023) / 1024);
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  // the vectors sit at the start of LDS, where one base register plus an
  // immediate offset reaches each of them; the weight buffers follow
  static_assert(S::vec % 1024 == 0, "weight region 1 KB aligned");
  char* const wreg = smem + S::vec;
  float* svo = (float*)smem;                        // b_o, LN gain, LN bias
  float* sb1 = svo + 3 * D;                         // b1 [MAXF]
  float* svm = sb1 + MAXF;                          // b2, next LayerNorm, projection rows
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;
  const long tok0 = (long)blockIdx.x * kM3BM + wave * 32 + l32;
  const bool tv = tok0 < g.M;
  const int tok = tv ? (int)tok0 : -1;
  const int nch = F / kM3FCH;
  const bf16* __restrict__ A = (const bf16*)g.A;

  auto dma_o = [&](int c, int buf) {
    char* base = wreg + buf * O::wa;
#pragma unroll
    for (int k = 0; k < NPW; ++k) {
      const int u = wave + k * NW;
      if (u >= NB) break;
      const int pos = u * 1024 + lane * 16, j = pos / RB, o = pos - j * RB;
      const bool data = o < RB - 16;
      const bf16* src = Wo + (long)(data ? j : 0) * D + c * KCH + (data ? o / 2 : 0);
      if (pos < (int)O::w)
        __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(base + u * 1024), 16, 0, 0);
    }
  };
  auto afrag = [&](int c, bf16x8 (&f)[KSC]) {
#pragma unroll
    for (int s = 0; s < KSC; ++s)
      f[s] = tv ? *(const bf16x8*)(A + tok0 * D + c * KCH + 16 * s + 8 * g2) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  };
  // offsets formed per chunk here: the kernel has no registers to keep them.
  // With F8 the W1 rows are D e4m3 bytes (pitch RB1Q), the first of the
  // BF16 W1 region's bytes
  constexpr int RB1Q = D + 16, W1Q = 32 * RB1Q, N1Q = (W1Q + 1023) / 1024;
  static_assert(W1Q <= (int)M::w1a, "e4m3 W1 chunk fits the BF16 one's region");
  M3ChunkDma<NW, F8 ? N1Q : N1, N2, F8 ? RB1Q : MRB1, MRB2, F8 ? W1Q : (int)M::w1, (int)M::w2, (int)M::w1a, false,
             F8 ? 1 : 2> mdma;
  mdma.init(wave, lane, D, F);
  auto dma_m = [&](int ch, int buf) {
    mdma.issue(F8 ? (const void*)W1q : (const void*)W1, W2, ch * kM3FCH, wreg + buf * M::buf);
  };
  constexpr int NM = (F8 ? N1Q : N1) + N2;          // DMA blocks of a chunk
  const int nwm = NM / NW + (wave < NM % NW ? 1 : 0);

  for (int i = tid; i < D; i += 512) {
    svo[i] = bo[i];
    svo[D + i] = lnx_g[i];
    svo[2 * D + i] = lnx_b[i];
  }
  for (int i = tid; i < F; i += 512) sb1[i] = b1[i];
  m3_stage_vectors<D>(svm, g, PROJ, tid, 512);

  // ================= output projection (see k_oproj3) =================
  f32x16 acc2[OBK][1];
#pragma unroll
  for (int b = 0; b < OBK; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc2[b][0][r] = 0.f;
  bf16x8 fa[KSC], fn[KSC];
  afrag(0, fa);
  dma_o(0, 0);
  __syncthreads();
#pragma unroll 1
  for (int c = 0; c < NCH; ++c) {
    const int buf = c & 1;
    if (c + 1 < NCH) {
      dma_o(c + 1, buf ^ 1);
      afrag(c + 1, fn);
    }
    const char* sw = wreg + buf * O::wa;
    mfma_pipe<KSC * OBK, PF>(
        [&](int i) { return *(const bf16x8*)(sw + (32 * (i % OBK) + l32) * RB + (2 * (i / OBK) + g2) * 16); },
        [&](int i, const bf16x8& w) {
          acc2[i % OBK][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, fa[i / OBK], acc2[i % OBK][0], 0, 0, 0);
        });
    if (c + 1 < NCH) {
#pragma unroll
      for (int s = 0; s < KSC; ++s) fa[s] = fn[s];
    }
    __syncthreads();                                // every wave is done with this buffer
  }
  // the W_o buffers are dead: the MLP ring takes the region (chunks prefetched
  // DIST ahead)
  constexpr int DIST = NBUF - 1;
  const int pre = min(DIST, nch);
  for (int ch = 0; ch < pre; ++ch) dma_m(ch, ch);

  // ---- R1 = R + acc2 + b_o in place, X1 = LN(R1) in the accumulator layout
  // (BF16, or e4m3 fragments with the token's scale), then acc2 = R1 + b2
  bf16x8 x1[KS];
  i32x8 xq[F8 ? D / 64 : 1];
  float xsc = 1.f;
  {
    const float* Rrow = g.R + (long)(tv ? tok0 : 0) * D;
    float sum = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b) {
      f32x4 rr[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        rr[q] = tv ? *(const f32x4*)(Rrow + 32 * b + 8 * q + 4 * g2) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 bias = *(const f32x4*)&svo[32 * b + 8 * q + 4 * g2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float res = rr[q][i] + (acc2[b][0][4 * q + i] + bias[i]);
          acc2[b][0][4 * q + i] = res;
          sum += res;
        }
      }
      asm volatile("" : "+v"(acc2[b][0]), "+v"(sum)::"memory");   // bounds the loads in flight
    }
    sum = xhalf_sum(sum);
    const float mean = sum / (float)D;
    float qv = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float dv = acc2[b][0][r] - mean;
        qv = fmaf(dv, dv, qv);
      }
    qv = xhalf_sum(qv);
    const float rstd = 1.0f / sqrtf(qv / (float)D + 1e-5f);
#pragma unroll
      for (int b = 0; b < OBK; ++b)
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int f = 32 * b + 8 * q + 4 * g2;
          const f32x4 lg = *(const f32x4*)&svo[D + f];
          const f32x4 lb = *(const f32x4*)&svo[2 * D + f];
          const f32x4 b2 = *(const f32x4*)&svm[f];
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            x1[2 * b + (q >> 1)][4 * (q & 1) + i] = (bf16)((acc2[b][0][4 * q + i] - mean) * rstd * lg[i] + lb[i]);
            acc2[b][0][4 * q + i] += b2[i];
          }
          if (q & 1) asm volatile("" : "+v"(x1[2 * b + (q >> 1)]), "+v"(acc2[b][0])::"memory");
        }
    if constexpr (F8) {
      // e4m3 fragments of X1 with the token's scale amax / 448 (amax over the
      // two lanes of the token); value e of x1[s] is byte 8 (s % 4) + e of
      // fragment s / 4
      float amax = 0.f;
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) amax = fmaxf(amax, fabsf((float)x1[s][e]));
      amax = xhalf_max(amax);
      xsc = amax > 0.f ? amax / 448.0f : 1.0f;
      const float inv = 1.0f / xsc;
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          float hq[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) hq[i] = fminf(fmaxf((float)x1[s][4 * h + i] * inv, -448.f), 448.f);
          int pk = __builtin_amdgcn_cvt_pk_fp8_f32(hq[0], hq[1], 0, false);
          pk = __builtin_amdgcn_cvt_pk_fp8_f32(hq[2], hq[3], pk, true);
          xq[s >> 2][2 * (s & 3) + h] = pk;
        }
    }
  }

  // ================= MLP (one chunk of 32 hidden units at a time) =================
  // up: acc1 = b1 + W1 X1 for the chunk's 32 hidden units
  auto up = [&](int ch, f32x16& acc1) {
    const char* s1 = wreg + (ch % NBUF) * M::buf;
    const float* sb = sb1 + ch * kM3FCH;
    if constexpr (F8) {
      // acc1 = b1 + (scale of X1 x w1s) (W1q X1q) over D / 64 steps of 64
      f32x16 a;
#pragma unroll
      for (int r = 0; r < 16; ++r) a[r] = 0.f;
      const char* wr = s1 + l32 * RB1Q + 32 * g2;
#pragma unroll
      for (int t = 0; t < D / 64; ++t) {
        const i32x8 wa = *(const i32x8*)(wr + 64 * t);
        a = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(wa, xq[t], a, 0, 0, 0, 127, 0, 127);
      }
      const float sc = xsc * w1s;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 bq = *(const f32x4*)&sb[16 * (q >> 1) + 8 * g2 + 4 * (q & 1)];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc1[4 * q + i] = a[4 * q + i] * sc + bq[i];
      }
      return;
    }
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const f32x4 bq = *(const f32x4*)&sb[16 * (q >> 1) + 8 * g2 + 4 * (q & 1)];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc1[4 * q + i] = bq[i];
    }
    // W1 k-values in X1's order (16 s + 4 g2 + j, then 16 s + 8 + 4 g2 + j):
    // the k-ordered copy holds them contiguously
    const char* wr = s1 + l32 * MRB1;
    mfma_pipe<KS, PF>(
        [&](int s) {
          return *(const bf16x8*)(wr + (16 * s + 8 * g2) * 2);   // k-ordered rows
        },
        [&](int s, const bf16x8& w) { acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, x1[s], acc1, 0, 0, 0); });
  };
  auto gelu = [&](const f32x16& acc1, bf16x8 (&hf)[2]) {
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) hf[q >> 1][4 * (q & 1) + i] = (bf16)gelu_f(acc1[4 * q + i]);
  };
  // down: acc2 += W2 GELU(.) over the chunk
  auto down = [&](int ch, const bf16x8 (&hf)[2]) {
    const char* s2 = wreg + (ch % NBUF) * M::buf + M::w1a;
    mfma_pipe<2 * OBK, PF>(
        [&](int j) { return *(const bf16x8*)(s2 + (32 * (j >> 1) + l32) * MRB2 + (2 * (j & 1) + g2) * 16); },
        [&](int j, const bf16x8& w) {
          acc2[j >> 1][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, hf[j & 1], acc2[j >> 1][0], 0, 0, 0);
        });
  };
  m3_wait_barrier(nwm * max(0, pre - 1));           // chunk 0 in LDS
#pragma unroll 1
  for (int ch = 0; ch < nch; ++ch) {
    // buffer (ch + DIST) % NBUF was last read in iteration ch - 1, before its closing barrier
    if (ch + DIST < nch) dma_m(ch + DIST, (ch + DIST) % NBUF);
    f32x16 acc1;
    bf16x8 hf[2];
    up(ch, acc1);
    gelu(acc1, hf);
    down(ch, hf);
    // chunk ch + 1 complete in every wave: later chunks (at most DIST - 1) may be in flight
    if (ch + 1 < nch) m3_wait_barrier(nwm * (min(ch + DIST, nch - 1) - (ch + 1)));
  }
  m3_epilogue_final<D, PROJ>(acc2, tok, g, g2, svm);
}

// ---------------------------------------------------------------------------
// k_oproj_mlp4: the computation of k_oproj_mlp3 (same MFMA sequence for every
// output element, so the same bits) in workgroups of four waves and 128
// tokens whose LDS fits twice in a CU (76 KB at d = 256).  Two workgroups per
// CU let one workgroup's loads of O and R and its stores of R and XN, which
// a CU moves at its own limited rate, run while the other computes.  The
// weights come from fragment-major copies (Mat::b16f): each MFMA A-operand
// fragment is 1 KB, lane l's 16 bytes at 16 l, so a chunk is one contiguous
// run of 1 KB DMA blocks and every LDS read is a conflict-free 1 KB read
// with the fragment index in the instruction's offset; nothing is padded.
// W_o goes through LDS in chunks of 64 k-columns (32 fragments), the MLP in
// chunks of 32 hidden units (16 W1 fragments, then 16 W2 fragments), each
// double-buffered in one 64 KB region.
template <int D, int MAXF>
struct OM4Smem {
  static constexpr int KCH = 64;
  static constexpr size_t wo = (size_t)D * KCH * 2;            // a W_o chunk: D rows x 64 k
  static constexpr size_t wm = (size_t)2 * kM3FCH * D * 2;     // an MLP chunk: W1 (32 x D) and W2 (D x 32)
  static constexpr size_t buf = wo > wm ? wo : wm;
  static constexpr size_t vec = ((size_t)(3 * D + MAXF + 5 * D) * 4 + 1023) / 1024 * 1024;
  static constexpr size_t bytes = vec + 2 * buf;
  static_assert(bytes <= 80 * 1024, "two workgroups per CU");
  static_assert(buf >= 4 * 8192, "one buffer holds the four waves' 8 KB epilogue slices");
};

template <int D, int MAXF, bool PROJ, int PF, bool F8 = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_oproj_mlp4(GemmArgs g, const bf16* __restrict__ Wof, const float* __restrict__ bo,
                  const float* __restrict__ lnx_g, const float* __restrict__ lnx_b, const bf16* __restrict__ W1f,
                  const float* __restrict__ b1, const bf16* __restrict__ W2f, int F,
                  const uint8_t* __restrict__ W1qf, float w1s) {
  using S = OM4Smem<D, MAXF>;
  constexpr int NW = 4, KCH = S::KCH, NCH = D / KCH, KSC = KCH / 16, OBK = D / 32, KS = D / 16;
  // 1 KB fragments per chunk; with F8 a W1 k-step of 64 is 2 KB (lane l's
  // 32 e4m3 bytes as two 16-byte halves, at 16 l and 1024 + 16 l)
  constexpr int NBO = (int)(S::wo / 1024), NB1 = F8 ? 2 * (D / 64) : KS, NB2 = 2 * OBK;
  static_assert(NBO % NW == 0 && (NB1 + NB2) % NW == 0 && NB1 % NW == 0, "DMA blocks split evenly over the waves");
  constexpr int TPW = NW * 32;                      // tokens per workgroup
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  float* svo = (float*)smem;                        // b_o, LN gain, LN bias
  float* sb1 = svo + 3 * D;                         // b1 [MAXF]
  float* svm = sb1 + MAXF;                          // b2, next LayerNorm, projection rows
  char* const wreg = smem + S::vec;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;
  const long tok0 = (long)blockIdx.x * TPW + wave * 32 + l32;
  const bool tv = tok0 < g.M;
  const int tok = tv ? (int)tok0 : -1;
  const int nch = F / kM3FCH;
  const bf16* __restrict__ A = (const bf16*)g.A;

  // chunk c of W_o: fragments c * NBO .. c * NBO + NBO - 1 of the copy
  auto dma_o = [&](int c, int buf) {
#pragma unroll
    for (int k = 0; k < NBO / NW; ++k) {
      const int u = wave + NW * k;
      __builtin_amdgcn_global_load_lds(Wof + ((long)c * NBO + u) * 512 + lane * 8,
                                       (__attribute__((address_space(3))) void*)(wreg + buf * S::buf + u * 1024), 16, 0, 0);
    }
  };
  // MLP chunk ch: its NB1 W1 fragments, then its NB2 W2 fragments
  auto dma_m = [&](int ch, int buf) {
#pragma unroll
    for (int k = 0; k < (NB1 + NB2) / NW; ++k) {
      const int u = wave + NW * k;
      const char* src = u < NB1 ? (F8 ? (const char*)W1qf + ((long)ch * NB1 + u) * 1024
                                      : (const char*)(W1f + ((long)ch * NB1 + u) * 512))
                                : (const char*)(W2f + ((long)ch * NB2 + (u - NB1)) * 512);
      __builtin_amdgcn_global_load_lds(src + lane * 16,
                                       (__attribute__((address_space(3))) void*)(wreg + buf * S::buf + u * 1024), 16, 0, 0);
    }
  };
  auto afrag = [&](int c, bf16x8 (&f)[KSC]) {
#pragma unroll
    for (int s = 0; s < KSC; ++s)
      f[s] = tv ? *(const bf16x8*)(A + tok0 * D + c * KCH + 16 * s + 8 * g2) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  };

  for (int i = tid; i < D; i += NW * 64) {
    svo[i] = bo[i];
    svo[D + i] = lnx_g[i];
    svo[2 * D + i] = lnx_b[i];
  }
  for (int i = tid; i < F; i += NW * 64) sb1[i] = b1[i];
  m3_stage_vectors<D>(svm, g, PROJ, tid, NW * 64);

  // ================= output projection =================
  f32x16 acc2[OBK][1];
#pragma unroll
  for (int b = 0; b < OBK; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc2[b][0][r] = 0.f;
  bf16x8 fa[KSC], fn[KSC];
  afrag(0, fa);
  dma_o(0, 0);
  __syncthreads();
#pragma unroll 1
  for (int c = 0; c < NCH; ++c) {
    const int buf = c & 1;
    if (c + 1 < NCH) {
      dma_o(c + 1, buf ^ 1);
      afrag(c + 1, fn);
    }
    const char* sw = wreg + buf * S::buf + lane * 16;
    // fragment i: output block i % OBK, k-step i / OBK of the chunk
    mfma_pipe<KSC * OBK, PF>(
        [&](int i) { return *(const bf16x8*)(sw + i * 1024); },
        [&](int i, const bf16x8& w) {
          acc2[i % OBK][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, fa[i / OBK], acc2[i % OBK][0], 0, 0, 0);
        });
    if (c + 1 < NCH) {
#pragma unroll
      for (int s = 0; s < KSC; ++s) fa[s] = fn[s];
    }
    __syncthreads();                                // every wave is done with this buffer
  }
  dma_m(0, 0);

  // ---- R1 = R + acc2 + b_o in place, X1 = LN(R1) in the accumulator layout, then acc2 = R1 + b2
  bf16x8 x1[KS];
  i32x8 xq[F8 ? D / 64 : 1];
  float xsc = 1.f;
  {
    const float* Rrow = g.R + (long)(tv ? tok0 : 0) * D;
    float sum = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b) {
      f32x4 rr[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        rr[q] = tv ? *(const f32x4*)(Rrow + 32 * b + 8 * q + 4 * g2) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 bias = *(const f32x4*)&svo[32 * b + 8 * q + 4 * g2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float res = rr[q][i] + (acc2[b][0][4 * q + i] + bias[i]);
          acc2[b][0][4 * q + i] = res;
          sum += res;
        }
      }
      asm volatile("" : "+v"(acc2[b][0]), "+v"(sum)::"memory");   // bounds the loads in flight
    }
    sum = xhalf_sum(sum);
    const float mean = sum / (float)D;
    float qv = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float dv = acc2[b][0][r] - mean;
        qv = fmaf(dv, dv, qv);
      }
    qv = xhalf_sum(qv);
    const float rstd = 1.0f / sqrtf(qv / (float)D + 1e-5f);
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int f = 32 * b + 8 * q + 4 * g2;
        const f32x4 lg = *(const f32x4*)&svo[D + f];
        const f32x4 lb = *(const f32x4*)&svo[2 * D + f];
        const f32x4 b2 = *(const f32x4*)&svm[f];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          x1[2 * b + (q >> 1)][4 * (q & 1) + i] = (bf16)((acc2[b][0][4 * q + i] - mean) * rstd * lg[i] + lb[i]);
          acc2[b][0][4 * q + i] += b2[i];
        }
        if (q & 1) asm volatile("" : "+v"(x1[2 * b + (q >> 1)]), "+v"(acc2[b][0])::"memory");
      }
    if constexpr (F8) {
      // e4m3 fragments of X1 with the token's scale amax / 448, as in k_oproj_mlp3
      float amax = 0.f;
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int e = 0; e < 8; ++e) amax = fmaxf(amax, fabsf((float)x1[s][e]));
      amax = xhalf_max(amax);
      xsc = amax > 0.f ? amax / 448.0f : 1.0f;
      const float inv = 1.0f / xsc;
#pragma unroll
      for (int s = 0; s < KS; ++s)
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          float hq[4];
#pragma unroll
          for (int i = 0; i < 4; ++i) hq[i] = fminf(fmaxf((float)x1[s][4 * h + i] * inv, -448.f), 448.f);
          int pk = __builtin_amdgcn_cvt_pk_fp8_f32(hq[0], hq[1], 0, false);
          pk = __builtin_amdgcn_cvt_pk_fp8_f32(hq[2], hq[3], pk, true);
          xq[s >> 2][2 * (s & 3) + h] = pk;
        }
    }
  }

  // ================= MLP (one chunk of 32 hidden units at a time) =================
  m3_wait_barrier(0);                               // chunk 0 in LDS
#pragma unroll 1
  for (int ch = 0; ch < nch; ++ch) {
    // the other buffer was last read in iteration ch - 1, before its closing barrier
    if (ch + 1 < nch) dma_m(ch + 1, (ch + 1) & 1);
    const char* s1 = wreg + (ch & 1) * S::buf + lane * 16;
    const float* sb = sb1 + ch * kM3FCH;
    // up: acc1 = b1 + W1 X1 for the chunk's 32 hidden units (W1 fragments in X1's k order)
    f32x16 acc1;
    if constexpr (F8) {
      // acc1 = b1 + (scale of X1 x w1s) (W1q X1q) over D / 64 steps of 64
      f32x16 a;
#pragma unroll
      for (int r = 0; r < 16; ++r) a[r] = 0.f;
#pragma unroll
      for (int t = 0; t < D / 64; ++t) {
        const int4 lo = *(const int4*)(s1 + 2 * t * 1024), hi = *(const int4*)(s1 + (2 * t + 1) * 1024);
        const i32x8 wa = i32x8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
        a = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(wa, xq[t], a, 0, 0, 0, 127, 0, 127);
      }
      const float sc = xsc * w1s;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 bq = *(const f32x4*)&sb[16 * (q >> 1) + 8 * g2 + 4 * (q & 1)];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc1[4 * q + i] = a[4 * q + i] * sc + bq[i];
      }
    } else {
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 bq = *(const f32x4*)&sb[16 * (q >> 1) + 8 * g2 + 4 * (q & 1)];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc1[4 * q + i] = bq[i];
      }
      mfma_pipe<KS, PF>([&](int s) { return *(const bf16x8*)(s1 + s * 1024); },
                        [&](int s, const bf16x8& w) { acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, x1[s], acc1, 0, 0, 0); });
    }
    // GELU of the first 8 hidden values (the down projection's k-step 0);
    // the other 8 are computed between the k-step 0 MFMAs, which run first
    // (per output block the k-steps keep their order)
    bf16x8 hf[2];
#pragma unroll
    for (int v = 0; v < 8; ++v) hf[0][v] = (bf16)gelu_f(acc1[v]);
    // down: acc2 += W2 GELU(.) over the chunk; step i: output block i % OBK,
    // k-step i / OBK (fragment 2 (i % OBK) + i / OBK)
    mfma_pipe<NB2, PF>(
        [&](int i) { return *(const bf16x8*)(s1 + (NB1 + 2 * (i % OBK) + i / OBK) * 1024); },
        [&](int i, const bf16x8& w) {
          acc2[i % OBK][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, hf[i / OBK], acc2[i % OBK][0], 0, 0, 0);
          if (i < OBK) {
#pragma unroll
            for (int v = (i * 8) / OBK; v < ((i + 1) * 8) / OBK; ++v) hf[1][v] = (bf16)gelu_f(acc1[8 + v]);
          }
        });
    // chunk ch + 1 complete in every wave, and every wave done with buffer ch & 1
    if (ch + 1 < nch) m3_wait_barrier(0);
  }
  // the MLP ring's buffer (nch & 1) was last read before the closing barrier of chunk nch - 2
  const long row0 = (long)blockIdx.x * TPW + wave * 32;
  m3_epilogue_rows<D, PROJ>(acc2, tok, g, g2, svm, wreg + (nch & 1) * S::buf + wave * 8192, lane,
                            [&](int r) { return row0 + r < g.M ? row0 + r : -1L; });
}

// ---------------------------------------------------------------------------
// The row sublayer's output projection followed by the user sublayer's QKV
// projection and attention (BF16, d = 256, head width 32), in one kernel per
// 32-slot user group (the output projection is per token, so it runs on the
// user grouping): R1 = R + O_row W_o^T + b_o is written, X2 = LN2(R1) stays
// in registers in the accumulator's layout and feeds the QKV projection
// (for the transposed V projection both operands use that layout); the user
// attention then proceeds as in k_user_qkv_attn and writes O_user.  Saves the
// XN round trip between the two sublayers.  A workgroup holds four user
// groups and its LDS fits twice in a CU (78 KB at d = 256), so one
// workgroup's loads and stores run under the other's compute.  The weights
// come from fragment-major copies (Mat::b16f; see k_oproj_mlp4): W_o in
// chunks of 64 k-columns (double-buffered), the user QKV projection in
// chunks of half a head's k range (its Q, K and V fragments of eight
// k-steps, 24 KB) in a ring of three.
template <int D>
struct OU4Smem {
  static constexpr int KCH = 64, NBQ = 3;
  static constexpr size_t wo = (size_t)D * KCH * 2;             // a W_o chunk
  static constexpr size_t wq = (size_t)3 * 32 * (D / 2) * 2;    // Q, K, V rows of a head over half of k
  static constexpr size_t vec = (size_t)6 * D * 4;              // bqkv; b_o, LN2 gain, LN2 bias
  static constexpr size_t region = 2 * wo > NBQ * wq ? 2 * wo : NBQ * wq;
  static constexpr size_t bytes = vec + region;
  static_assert(vec % 1024 == 0 && bytes <= 80 * 1024, "two workgroups per CU");
};

template <int D>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_oproj_user_attn4(StepCtx c, const bf16* __restrict__ Orow, const bf16* __restrict__ Wof,
                        const float* __restrict__ bo, const float* __restrict__ ln_g, const float* __restrict__ ln_b,
                        float* __restrict__ R, const bf16* __restrict__ Wqf, const float* __restrict__ bqkv,
                        bf16* __restrict__ O) {
  using S = OU4Smem<D>;
  constexpr int NW = 4, KCH = S::KCH, NCH = D / KCH, KSC = KCH / 16, OBK = D / 32, KS = D / 16, HEADS = D / 32;
  constexpr int NBO = (int)(S::wo / 1024), KH = KS / 2, NBQ = 3 * KH;   // 1 KB fragments per chunk
  constexpr int NQ = 2 * HEADS, NBUF = S::NBQ, DIST = NBUF - 1;        // QKV chunks; ring
  static_assert(NBO % NW == 0 && NBQ % NW == 0, "DMA blocks split evenly over the waves");
  constexpr int QPW = NBQ / NW;                     // DMA blocks per wave per QKV chunk
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  char* const wreg = smem + S::vec;
  float* sbias = (float*)smem;                      // bqkv [3D]
  float* svo = sbias + 3 * D;                       // b_o, LN2 gain, LN2 bias
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;

  // ---- this lane's slot of the wave's group
  const int gi = blockIdx.x * NW + wave;
  int tok = -1, K = 1;
  if (gi < c.total_ugrp32) {
    const int bi = c.ugrp32[2 * gi], c0 = c.ugrp32[2 * gi + 1];
    const DevBin& b = c.bins[bi];
    K = b.K;
    const int C = 32 / K, cl = l32 / K, k = l32 - cl * K;
    if (l32 < C * K && c0 + cl < b.n) tok = b.tok_off + k * b.n + c0 + cl;
  }
  const unsigned long long vmask = __ballot(tok >= 0);
  unsigned okbits = 0;                               // register r of S^T: key slot 8(r/4) + 4 g2 + r%4
  const int col_lo = (l32 / K) * K;                 // key slots of this lane's column: col_lo .. col_lo + K - 1
#pragma unroll
  for (int r = 0; r < 16; ++r) {
    const int kr = 8 * (r >> 2) + 4 * g2 + (r & 3);
    if (((vmask >> kr) & 1ull) && (unsigned)(kr - col_lo) < (unsigned)K) okbits |= 1u << r;
  }
  const bool tv = tok >= 0;

  auto dma_o = [&](int cc, int buf) {
#pragma unroll
    for (int k = 0; k < NBO / NW; ++k) {
      const int u = wave + NW * k;
      __builtin_amdgcn_global_load_lds(Wof + ((long)cc * NBO + u) * 512 + lane * 8,
                                       (__attribute__((address_space(3))) void*)(wreg + buf * S::wo + u * 1024), 16, 0, 0);
    }
  };
  // QKV chunk t: head t / 2, k-steps KH (t % 2) .. KH (t % 2) + KH - 1
  auto dma_q = [&](int t, int buf) {
#pragma unroll
    for (int k = 0; k < QPW; ++k) {
      const int u = wave + NW * k;
      __builtin_amdgcn_global_load_lds(Wqf + ((long)t * NBQ + u) * 512 + lane * 8,
                                       (__attribute__((address_space(3))) void*)(wreg + buf * S::wq + u * 1024), 16, 0, 0);
    }
  };
  auto afrag = [&](int cc, bf16x8 (&f)[KSC]) {
#pragma unroll
    for (int s = 0; s < KSC; ++s)
      f[s] = tv ? *(const bf16x8*)(Orow + (long)tok * D + cc * KCH + 16 * s + 8 * g2) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  };
  for (int i = tid; i < 3 * D; i += NW * 64) sbias[i] = bqkv[i];
  for (int i = tid; i < D; i += NW * 64) {
    svo[i] = bo[i];
    svo[D + i] = ln_g[i];
    svo[2 * D + i] = ln_b[i];
  }

  // ================= row output projection =================
  f32x16 acc2[OBK];
#pragma unroll
  for (int b = 0; b < OBK; ++b)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc2[b][r] = 0.f;
  {
    bf16x8 fa[KSC], fn[KSC];
    afrag(0, fa);
    dma_o(0, 0);
    __syncthreads();
#pragma unroll 1
    for (int cc = 0; cc < NCH; ++cc) {
      const int buf = cc & 1;
      if (cc + 1 < NCH) {
        dma_o(cc + 1, buf ^ 1);
        afrag(cc + 1, fn);
      }
      const char* sw = wreg + buf * S::wo + lane * 16;
      // fragment i: output block i % OBK, k-step i / OBK of the chunk
      mfma_pipe<KSC * OBK, 3>([&](int i) { return *(const bf16x8*)(sw + i * 1024); },
                              [&](int i, const bf16x8& w) {
                                acc2[i % OBK] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, fa[i / OBK], acc2[i % OBK], 0, 0, 0);
                              });
      if (cc + 1 < NCH) {
#pragma unroll
        for (int s = 0; s < KSC; ++s) fa[s] = fn[s];
      }
      __syncthreads();                              // every wave is done with this buffer
    }
  }
  // the W_o buffers are dead: the QKV ring takes the region (DIST chunks ahead)
#pragma unroll
  for (int t = 0; t < DIST; ++t) dma_q(t, t);

  // ---- R1 = R + acc2 + b_o (written), X2 = LN2(R1) in the accumulator layout
  bf16x8 xf[KS];
  {
    float* Rrow = R + (long)(tv ? tok : 0) * D;
    float sum = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b) {
      f32x4 rr[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        rr[q] = tv ? *(const f32x4*)(Rrow + 32 * b + 8 * q + 4 * g2) : f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const f32x4 bias = *(const f32x4*)&svo[32 * b + 8 * q + 4 * g2];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float res = rr[q][i] + (acc2[b][4 * q + i] + bias[i]);
          acc2[b][4 * q + i] = res;
          sum += res;
        }
      }
      asm volatile("" : "+v"(acc2[b]), "+v"(sum)::"memory");   // bounds the loads in flight
    }
    // R1 leaves as whole 128-byte row segments (rows_store_f32) through ring
    // buffer DIST: the last W_o chunk's barrier freed it, and its first DMA
    // is issued after the QKV loop's first barrier; row r of the wave is lane
    // r's token
    static_assert(NW * 4096 <= S::wq, "a 4 KB slice per wave in one ring buffer");
    rows_store_f32<D, 128>([&](int b, int q) {
                        return f32x4{acc2[b][4 * q], acc2[b][4 * q + 1], acc2[b][4 * q + 2], acc2[b][4 * q + 3]};
                      },
                      R, wreg + DIST * S::wq + wave * 4096, lane, [&](int r) { return (long)__shfl(tok, r); });
    sum = xhalf_sum(sum);
    const float mean = sum / (float)D;
    float qv = 0.f;
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float dv = acc2[b][r] - mean;
        qv = fmaf(dv, dv, qv);
      }
    qv = xhalf_sum(qv);
    const float rstd = 1.0f / sqrtf(qv / (float)D + 1e-5f);
#pragma unroll
    for (int b = 0; b < OBK; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int f = 32 * b + 8 * q + 4 * g2;
        const f32x4 lg = *(const f32x4*)&svo[D + f];
        const f32x4 lb = *(const f32x4*)&svo[2 * D + f];
#pragma unroll
        for (int i = 0; i < 4; ++i)
          xf[2 * b + (q >> 1)][4 * (q & 1) + i] = (bf16)((acc2[b][4 * q + i] - mean) * rstd * lg[i] + lb[i]);
        if (q & 1) asm volatile("" : "+v"(xf[2 * b + (q >> 1)])::"memory");
      }
  }

  // ================= user attention (as k_user_qkv_attn; k order of X2) =================
  const float scale = 1.4426950408889634f / sqrtf(32.0f);
  constexpr int HB = 2;                             // heads per O store batch (registers)
  bf16x4 ob[HB][4];
  // O of a batch of heads leaves as whole 128-byte row segments through four
  // 1 KB blocks of a ring buffer that only this wave's DMA refills (blocks
  // wave + 4 j; block j holds rows 8 j .. 8 j + 7, piece p of row r at index
  // p XOR (r mod 8)), after each pair of steps is exchanged between the
  // wave's halves so that every lane writes one whole 16-byte piece; row r
  // of the wave is lane r's token
  static_assert(NW == 4 && QPW >= 4 && HB == 2, "four own DMA blocks per ring buffer; 8 pieces per row");
  auto store_o = [&](int h0, int buf) {
    typedef unsigned u32x2 __attribute__((__vector_size__(2 * sizeof(unsigned))));
    typedef unsigned u32x4 __attribute__((__vector_size__(4 * sizeof(unsigned))));
    char* const blk = wreg + buf * S::wq + wave * 1024;   // block j at blk + 4096 j
#pragma unroll
    for (int hh = 0; hh < HB; ++hh)
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const u32x2 a0 = __builtin_bit_cast(u32x2, ob[hh][2 * k]);
        const u32x2 a1 = __builtin_bit_cast(u32x2, ob[hh][2 * k + 1]);
        const auto s0 = __builtin_amdgcn_permlane32_swap(a0[0], a1[0], false, false);
        const auto s1 = __builtin_amdgcn_permlane32_swap(a0[1], a1[1], false, false);
        *(u32x4*)(blk + (l32 >> 3) * 4096 + (l32 & 7) * 128 + 16 * ((4 * hh + 2 * k + g2) ^ (l32 & 7))) =
            u32x4{s0[0], s1[0], s0[1], s1[1]};
      }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = 8 * j + (lane >> 3), pp = lane & 7;
      const u32x4 v = *(const u32x4*)(blk + j * 4096 + (r & 7) * 128 + 16 * (pp ^ (r & 7)));
      const int tr = __shfl(tok, r);
      if (tr >= 0) *(u32x4*)(O + (long)tr * D + h0 * 32 + 8 * pp) = v;
    }
  };
#pragma unroll
  for (int h = 0; h < HEADS; ++h) {
    f32x16 aq, ak, av;
#pragma unroll
    for (int r = 0; r < 16; ++r) aq[r] = ak[r] = av[r] = 0.f;
#pragma unroll
    for (int half = 0; half < 2; ++half) {
      const int t = 2 * h + half;
      // chunk t complete in every wave (later chunks may be in flight), and
      // every wave done with chunk t - 1, whose buffer the next DMA refills
      m3_wait_barrier(QPW * (min(t + DIST - 1, NQ - 1) - t));
      // the previous batch of heads' O, stored between the wait and the next
      // DMA so that the next wait does not cover that DMA
      // (through the buffer of chunk t - 1, which that DMA refills; every lane
      // joins the exchange)
      if (half == 0 && h % HB == 0 && h > 0) store_o(h - HB, (t + DIST) % NBUF);
      if (t + DIST < NQ) dma_q(t + DIST, (t + DIST) % NBUF);
      const char* sw = wreg + (t % NBUF) * S::wq + lane * 16;
      // fragment 3 s + m: k-step KH half + s of Q (m = 0), K (1) and V (2)
#pragma unroll
      for (int s = 0; s < KH; ++s) {
        const bf16x8 wq = *(const bf16x8*)(sw + (3 * s) * 1024);
        const bf16x8 wk = *(const bf16x8*)(sw + (3 * s + 1) * 1024);
        const bf16x8 wv = *(const bf16x8*)(sw + (3 * s + 2) * 1024);
        aq = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wq, xf[KH * half + s], aq, 0, 0, 0);
        ak = __builtin_amdgcn_mfma_f32_32x32x16_bf16(wk, xf[KH * half + s], ak, 0, 0, 0);
        av = __builtin_amdgcn_mfma_f32_32x32x16_bf16(xf[KH * half + s], wv, av, 0, 0, 0);
      }
    }
    bf16x8 qf[2], kf[2], vf[2];
    const float bv = sbias[2 * D + h * 32 + l32];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = h * 32 + 8 * q + 4 * g2;
      const f32x4 bq = *(const f32x4*)&sbias[f];
      const f32x4 bk = *(const f32x4*)&sbias[D + f];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = 4 * q + i;
        qf[r >> 3][r & 7] = (bf16)(aq[r] + bq[i]);
        kf[r >> 3][r & 7] = (bf16)(ak[r] + bk[i]);
        vf[r >> 3][r & 7] = (bf16)(av[r] + bv);
      }
    }
    f32x16 st;
#pragma unroll
    for (int r = 0; r < 16; ++r) st[r] = 0.f;
    st = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf[0], qf[0], st, 0, 0, 0);
    st = __builtin_amdgcn_mfma_f32_32x32x16_bf16(kf[1], qf[1], st, 0, 0, 0);
    float mx = -INFINITY;
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      st[r] = ((okbits >> r) & 1u) ? st[r] : -INFINITY;
      mx = fmaxf(mx, st[r]);
    }
    mx = xhalf_max(mx);
    const float mxs = mx == -INFINITY ? 0.f : -mx * scale;   // a padding query has no valid key
    float ps = 0.f;
    bf16x8 pf[2];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float p = __builtin_amdgcn_exp2f(fmaf(st[r], scale, mxs));
      ps += p;
      pf[r >> 3][r & 7] = (bf16)p;
    }
    ps = xhalf_sum(ps);
    f32x16 o;
#pragma unroll
    for (int r = 0; r < 16; ++r) o[r] = 0.f;
    o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf[0], pf[0], o, 0, 0, 0);
    o = __builtin_amdgcn_mfma_f32_32x32x16_bf16(vf[1], pf[1], o, 0, 0, 0);
    const float inv = ps > 0.f ? 1.0f / ps : 0.f;
#pragma unroll
    for (int q = 0; q < 4; ++q)
      ob[h % HB][q] = bf16x4{(bf16)(o[4 * q] * inv), (bf16)(o[4 * q + 1] * inv), (bf16)(o[4 * q + 2] * inv),
                             (bf16)(o[4 * q + 3] * inv)};
  }
  // the last batch through the buffer of chunk NQ - 2: every wave was done
  // with it at the last barrier, and no DMA refills it any more
  store_o(HEADS - HB, (NQ - 2) % NBUF);
}

// ---------------------------------------------------------------------------
// Module A for the BF16 path, from the symbol grid to the first LayerNorm in
// one token-resident kernel (method section, Module A; Appendix, one-step
// algorithm):
//   Z = E[x] + P[l] + gamma u,    r[k, a] = softmax over the slot's rows of
//   <Z[k], w_a> / tau,            e = sum_a r[k, a] p[l, a] v_a,
//   R = g Z + (1 - g) e,  g = sigmoid(Wg2 GELU(Wg1 [Z ; e] + bg1) + bg2),
//   XN = LayerNorm_1(R) of the first layer.
// The rows of one slot differ only in E[x]: P[l] + gamma u is common to them
// and cancels in the softmax over rows, so r[k, a] is the softmax over the
// slot's rows of <E[x_k], w_a> / tau, six table values (three symbols, two
// logits) that each workgroup computes once.  Each lane forms Z of its token
// in registers, straight in the B-operand layout of the up MFMAs, and Z and
// e again in the output layout for the blend: neither reaches HBM.  Since
// e = c0 v_0 + c1 v_1, the up projection's e half is c0 (Wg1_e v_0) +
// c1 (Wg1_e v_1), two vectors formed once per weight set, so only Wg1's Z
// half (d x d) and Wg2 (d x d) are DMA'd into LDS, once per workgroup; a
// workgroup then walks 256-token tiles.
template <int D>
struct EG3Smem {
  static constexpr int DIN = D;                          // the Z half of Wg1's columns
  static constexpr int NCH = D / kM3FCH;                 // the gate's hidden width is d
  static constexpr int RB1 = DIN * 2 + 16;
  static constexpr int RB2 = kM3FCH * 2 + 16;
  static constexpr size_t w1 = (size_t)kM3FCH * RB1;
  static constexpr size_t w2 = (size_t)D * RB2;
  static constexpr size_t w1a = (w1 + 1023) / 1024 * 1024;
  static constexpr size_t w2a = (w2 + 1023) / 1024 * 1024;
  static constexpr size_t buf = w1a + w2a;
  // E[3], u, v[2], Wg1_e v_a [2], bg1, bg2, LN gain / bias, <E[x], w_a>: at
  // the start of LDS, so that every vector address is a register base + an
  // immediate
  static constexpr size_t vec = ((size_t)(13 * D + 12) * 4 + 8 * 4 + 1023) / 1024 * 1024;
  static constexpr size_t epi = (size_t)8 * 8192;       // the waves' 8 KB row-store slices
  static constexpr size_t bytes = vec + NCH * buf + epi;
  static_assert(bytes <= 160 * 1024, "LDS");
};

template <int D>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_embed_gate3(StepCtx c, EmbedW m, EmbedGateArgs a, int ntiles) {
  using S = EG3Smem<D>;
  constexpr int DIN = S::DIN, NCH = S::NCH, RB1 = S::RB1, RB2 = S::RB2;
  constexpr int KS1 = DIN / 16, OBK = D / 32, KZ = D / 16;
  constexpr int N1 = (int)(S::w1a / 1024), N2 = (int)(S::w2a / 1024), NB = NCH * (N1 + N2);
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;
  char* wsm = smem + S::vec;                      // the weight chunks
  char* const epi = smem + S::vec + NCH * S::buf + wave * 8192;   // this wave's row-store slice
  // E's three rows at a pitch of D + 4 floats: lanes of different symbols
  // read their row at the same feature, which a pitch of D (a multiple of
  // the bank count) would put on the same banks
  constexpr int EP = D + 4;
  float* sE = (float*)smem;                       // [3][EP]
  float* su = sE + 3 * EP;
  float* sv = su + D;                             // [2][D]
  float* sug = sv + 2 * D;                        // [2][D]: Wg1_e v_a
  float* sbg1 = sug + 2 * D;
  float* sbg2 = sbg1 + D;
  float* slg = sbg2 + D;
  float* slb = slg + D;
  float* sEW = slb + D;                           // [3][2]: <E[x], w_a>

  // small vectors first: their loads complete before the weight DMA is issued
  for (int i = tid; i < 3 * D; i += 512) sE[(i / D) * EP + i % D] = m.E[i];
  for (int i = tid; i < D; i += 512) {
    su[i] = m.u[i];
    sv[i] = m.v[i];
    sv[D + i] = m.v[D + i];
    sug[i] = a.ug[i];
    sug[D + i] = a.ug[D + i];
    sbg1[i] = a.bg1[i];
    sbg2[i] = a.bg2[i];
    slg[i] = a.ln_g[i];
    slb[i] = a.ln_b[i];
  }
  if (wave < 6) {
    const int x = wave >> 1, al = wave & 1;
    float acc = 0.f;
    for (int i = lane; i < D; i += 64) acc = fmaf(m.E[x * D + i], m.W[al * D + i], acc);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) sEW[wave] = acc;
  }
  __syncthreads();
  // the whole gate MLP -> LDS, 1 KB blocks spread over the waves; chunk ch
  // holds hidden units 32 ch + sigma(j) of Wg1's Z half (rows padded to RB1
  // bytes) and columns 32 ch .. + 32 of Wg2 (rows padded to RB2 bytes)
  for (int u = wave; u < NB; u += 8) {
    const int ch = u / (N1 + N2), v = u - ch * (N1 + N2);
    const bool first = v < N1;
    const int pos = (first ? v : v - N1) * 1024 + lane * 16;
    const int rb = first ? RB1 : RB2;
    const int j = pos / rb, o = pos - j * rb;
    const bool data = o < rb - 16;                 // else a pad (copy something in bounds)
    const bf16* src;
    if (first) src = a.Wg1 + (long)(ch * kM3FCH + m3_sigma(data ? j : 0)) * (2 * D) + (data ? o / 2 : 0);
    else src = a.Wg2 + (long)(data ? j : 0) * D + ch * kM3FCH + (data ? o / 2 : 0);
    char* dst = wsm + ch * S::buf + (first ? 0 : (int)S::w1a) + (pos - lane * 16);
    if (pos < (first ? (int)S::w1 : (int)S::w2))
      __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)dst, 16, 0, 0);
  }
  const float inv_tau = 1.0f / c.tau;
  bool weights_ready = false;

  for (int tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
    // the staged vectors are re-read from LDS in every tile, not held in
    // registers across tiles
    asm volatile("" ::: "memory");
    // ---- this lane's token: its bin, row k, slot l, symbol, mask ratio and
    // the demixing coefficients r[k, a] p[l, a]
    const long tok = (long)tile * kM3BM + wave * 32 + l32;
    const bool tv = tok < c.total_tokens;
    const long tq = tv ? tok : c.total_tokens - 1;
    int b = c.tile_bin[tile];
    while (b + 1 < c.num_bins && tq >= c.bins[b + 1].tok_off) ++b;
    const DevBin* bp = &c.bins[b];
    const int K = bp->K, n = bp->n;
    const int rel = (int)(tq - bp->tok_off), k = rel / n, l = rel - k * n;
    const float gamma = c.gamma_override >= 0.f ? c.gamma_override : (float)bp->st->masked / (float)(K * n);
    const uint8_t* Xc = bp->X + l;
    const int x = min((int)Xc[k * n], kMask);
    float mx0 = -INFINITY, mx1 = -INFINITY;
    for (int kk = 0; kk < K; ++kk) {
      const int xk = min((int)Xc[kk * n], kMask);
      mx0 = fmaxf(mx0, sEW[2 * xk] * inv_tau);
      mx1 = fmaxf(mx1, sEW[2 * xk + 1] * inv_tau);
    }
    float den0 = 0.f, den1 = 0.f;
    for (int kk = 0; kk < K; ++kk) {
      const int xk = min((int)Xc[kk * n], kMask);
      den0 += expf(sEW[2 * xk] * inv_tau - mx0);
      den1 += expf(sEW[2 * xk + 1] * inv_tau - mx1);
    }
    const int slot = bp->slot_off + l;
    const float c0 = expf(sEW[2 * x] * inv_tau - mx0) / den0 * a.p[2 * slot];
    const float c1 = expf(sEW[2 * x + 1] * inv_tau - mx1) / den1 * a.p[2 * slot + 1];
    const float* Pl = m.P + (long)l * D;
    const float* Ex = sE + x * EP;

    // ---- Z in the B-operand layout: k-step s holds features 16 s + 8 g2 + 0..7
    // (e = c0 v_0 + c1 v_1 enters the up projection as c0 Wg1_e v_0 + c1 Wg1_e v_1)
    static_assert(KS1 == KZ, "the up projection reads Z only");
    bf16x8 xf[KZ];
#pragma unroll
    for (int s = 0; s < KZ; ++s) {
      const int f = 16 * s + 8 * g2;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const f32x4 pq = *(const f32x4*)(Pl + f + 4 * h);
        const f32x4 eq = *(const f32x4*)(Ex + f + 4 * h);
        const f32x4 uq = *(const f32x4*)(su + f + 4 * h);
#pragma unroll
        for (int i = 0; i < 4; ++i) xf[s][4 * h + i] = (bf16)((eq[i] + pq[i]) + gamma * uq[i]);
      }
      // finish these fragments before the next loads, so that the loaded
      // vectors die here (bounds the registers in flight)
      asm volatile("" : "+v"(xf[s])::"memory");
    }
    if (!weights_ready) {
      __syncthreads();                            // every wave's weight DMA complete
      weights_ready = true;
    }

    // ---- gate MLP: up (d -> d, + c0 Wg1_e v_0 + c1 Wg1_e v_1, GELU), down
    // (d -> d), all weights in LDS
    f32x16 acc2[OBK];
#pragma unroll
    for (int ob = 0; ob < OBK; ++ob)
#pragma unroll
      for (int r = 0; r < 16; ++r) acc2[ob][r] = 0.f;
#pragma unroll 1
    for (int ch = 0; ch < NCH; ++ch) {
      const char* s1 = wsm + ch * S::buf;
      const char* s2 = s1 + S::w1a;
      f32x16 acc1;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int f = ch * kM3FCH + 16 * (q >> 1) + 8 * g2 + 4 * (q & 1);
        const f32x4 bq = *(const f32x4*)&sbg1[f];
        const f32x4 u0 = *(const f32x4*)&sug[f];
        const f32x4 u1 = *(const f32x4*)&sug[D + f];
#pragma unroll
        for (int i = 0; i < 4; ++i) acc1[4 * q + i] = bq[i] + (c0 * u0[i] + c1 * u1[i]);
      }
#pragma unroll
      for (int s = 0; s < KS1; ++s) {
        const bf16x8 w = *(const bf16x8*)(s1 + l32 * RB1 + (2 * s + g2) * 16);
        acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, xf[s], acc1, 0, 0, 0);
      }
      bf16x8 hf[2];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int i = 0; i < 4; ++i) hf[q >> 1][4 * (q & 1) + i] = (bf16)gelu_f(acc1[4 * q + i]);
#pragma unroll
      for (int ob = 0; ob < OBK; ++ob)
#pragma unroll
        for (int s = 0; s < 2; ++s) {
          const bf16x8 w = *(const bf16x8*)(s2 + (32 * ob + l32) * RB2 + (2 * s + g2) * 16);
          acc2[ob] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, hf[s], acc2[ob], 0, 0, 0);
        }
    }

    // ---- blend R = g Z + (1 - g) e, then the first LayerNorm.  Lane l holds
    // output features 32 ob + 8 q + 4 g2 + i of its token in register 4 q + i.
    float sum = 0.f;
#pragma unroll
    for (int ob = 0; ob < OBK; ++ob)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int f = 32 * ob + 8 * q + 4 * g2;
        const f32x4 pq = *(const f32x4*)(Pl + f);
        const f32x4 eq = *(const f32x4*)(Ex + f);
        const f32x4 uq = *(const f32x4*)(su + f);
        const f32x4 v0 = *(const f32x4*)(sv + f);
        const f32x4 v1 = *(const f32x4*)(sv + D + f);
        const f32x4 bq = *(const f32x4*)(sbg2 + f);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const float z = (eq[i] + pq[i]) + gamma * uq[i];
          const float e = c0 * v0[i] + c1 * v1[i];
          const float gt = sigmoid_f(acc2[ob][4 * q + i] + bq[i]);
          const float res = gt * z + (1.0f - gt) * e;
          acc2[ob][4 * q + i] = res;
          sum += res;
        }
        asm volatile("" ::: "memory");            // bound the loads in flight
      }
    sum = xhalf_sum(sum);
    const float mean = sum / (float)D;
    float qv = 0.f;
#pragma unroll
    for (int ob = 0; ob < OBK; ++ob)
#pragma unroll
      for (int r = 0; r < 16; ++r) {
        const float dv = acc2[ob][r] - mean;
        qv = fmaf(dv, dv, qv);
      }
    qv = xhalf_sum(qv);
    const float rstd = 1.0f / sqrtf(qv / (float)D + 1e-5f);
    // R and XN leave as whole row segments (rows_store_*): row r of the wave
    // is token tile * kM3BM + 32 wave + r
    const long row0 = (long)tile * kM3BM + wave * 32;
    const auto rowtok = [&](int r) { return row0 + r < c.total_tokens ? row0 + r : -1L; };
    float mean2 = mean, rstd2 = rstd;
    asm volatile("" : "+v"(mean2), "+v"(rstd2));   // no (acc2 - mean) kept from the variance loop
    rows_store_bf16<D>(
        [&](int ob, int q) {
          const int f = 32 * ob + 8 * q + 4 * g2;
          const f32x4 lg = *(const f32x4*)(slg + f);
          const f32x4 lb = *(const f32x4*)(slb + f);
          bf16x4 h;
#pragma unroll
          for (int i = 0; i < 4; ++i) h[i] = (bf16)((acc2[ob][4 * q + i] - mean2) * rstd2 * lg[i] + lb[i]);
          return h;
        },
        a.XN, epi, lane, rowtok);
    rows_store_f32<D>(
        [&](int ob, int q) {
          return f32x4{acc2[ob][4 * q], acc2[ob][4 * q + 1], acc2[ob][4 * q + 2], acc2[ob][4 * q + 3]};
        },
        a.R, epi, lane, rowtok);
  }
  if (!weights_ready) __syncthreads();            // no tile: drain the DMA before the workgroup ends
}

// ---------------------------------------------------------------------------
// Embedding, Module A and the first LayerNorm for the BF16 path at d = 256, in
// one token-resident kernel.  The gate's input [Z ; e] has e = c0 v_0 + c1 v_1
// (Q = 2: a per-token combination of two fixed vectors), so its
// up-projection is Wg1_Z Z + c0 (Wg1_e v_0) + c1 (Wg1_e v_1), with the two
// products Wg1_e v_a formed once per weight set (exact in real arithmetic;
// here they enter in FP32 where the two-kernel form rounds e to BF16).  What
// remains is a d -> d -> d MLP on Z, run as the MLP chunk ring (rows of Wg1_Z
// and columns of Wg2, 32 hidden units per chunk, through LDS), with the
// sigmoid gate, the blend R = g Z + (1 - g) e and the first LayerNorm in the
// epilogue.  Reads the symbols, the per-slot beliefs and the tables; writes R
// (FP32) and XN (BF16).
template <int D>
struct EGZSmem {
  static constexpr int NBUF = 3;
  using M = M3Smem<D, NBUF, D>;
  // E[3], u, v[2], Wg1_e v_a [2], bg1, bg2, LN gain / bias, <E[x], w_a>: at
  // the start of LDS (one register base plus immediate offsets)
  static constexpr size_t vec = ((size_t)(12 * D + 12) * 4 + 8 * 4 + 1023) / 1024 * 1024;
  static constexpr size_t bytes = vec + NBUF * M::buf;
  static_assert(bytes <= 160 * 1024, "LDS");
};

template <int D>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_embed_gate_z(StepCtx c, EmbedW m, EmbedGateArgs a) {
  using S = EGZSmem<D>;
  using M = typename S::M;
  constexpr int NW = 8, NBUF = S::NBUF, NCH = D / kM3FCH, OBK = D / 32, KZ = D / 16;
  constexpr int MRB1 = M::RB1, MRB2 = M::RB2;
  constexpr int N1 = (int)((M::w1 + 1023) / 1024), N2 = (int)((M::w2 + 1023) / 1024);
  static_assert(NCH > NBUF - 1, "the prefetch covers chunks 0 .. NBUF - 2");
  static_assert(S::vec % 1024 == 0, "weight region 1 KB aligned");
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  char* const wreg = smem + S::vec;               // the chunk ring
  // E's three rows at a pitch of D + 4 floats: lanes of different symbols
  // read their row at the same feature, which a pitch of D (a multiple of
  // the bank count) would put on the same banks
  constexpr int EP = D + 4;
  float* sE = (float*)smem;                       // [3][EP]
  float* su = sE + 3 * EP;
  float* sv = su + D;                             // [2][D]
  float* sug = sv + 2 * D;                        // [2][D]: Wg1_e v_a
  float* sbg1 = sug + 2 * D;
  float* sbg2 = sbg1 + D;
  float* slg = sbg2 + D;
  float* slb = slg + D;
  float* sEW = slb + D;                           // [3][2]: <E[x], w_a>
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g2 = lane >> 5, l32 = lane & 31;

  for (int i = tid; i < 3 * D; i += 512) sE[(i / D) * EP + i % D] = m.E[i];
  for (int i = tid; i < D; i += 512) {
    su[i] = m.u[i];
    sv[i] = m.v[i];
    sv[D + i] = m.v[D + i];
    sug[i] = a.ug[i];
    sug[D + i] = a.ug[D + i];
    sbg1[i] = a.bg1[i];
    sbg2[i] = a.bg2[i];
    slg[i] = a.ln_g[i];
    slb[i] = a.ln_b[i];
  }
  if (wave < 6) {
    const int x = wave >> 1, al = wave & 1;
    float acc = 0.f;
    for (int i = lane; i < D; i += 64) acc = fmaf(m.E[x * D + i], m.W[al * D + i], acc);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (lane == 0) sEW[wave] = acc;
  }
  __syncthreads();

  // ---- chunk ch of the gate MLP -> ring buffer: rows 32 ch + sigma(j) of
  // Wg1's Z half (row stride 2d) and columns 32 ch .. + 32 of Wg2
  const int nwm = (N1 + N2) / NW + (wave < (N1 + N2) % NW ? 1 : 0);
  M3ChunkDma<NW, N1, N2, MRB1, MRB2, (int)M::w1, (int)M::w2, (int)M::w1a> mdma;
  mdma.init(wave, lane, 2 * D, D);
  auto dma_m = [&](int ch, int buf) { mdma.issue(a.Wg1, a.Wg2, ch * kM3FCH, wreg + buf * M::buf); };
  for (int ch = 0; ch < NBUF - 1; ++ch) dma_m(ch, ch);

  // ---- this lane's token: its bin, row k, slot l, symbol, mask ratio and
  // the demixing coefficients r[k, a] p[l, a]
  const float inv_tau = 1.0f / c.tau;
  const long tok = (long)blockIdx.x * kM3BM + wave * 32 + l32;
  const bool tv = tok < c.total_tokens;
  const long tq = tv ? tok : c.total_tokens - 1;
  int b = c.tile_bin[blockIdx.x];
  while (b + 1 < c.num_bins && tq >= c.bins[b + 1].tok_off) ++b;
  const DevBin* bp = &c.bins[b];
  const int K = bp->K, n = bp->n;
  const int rel = (int)(tq - bp->tok_off), k = rel / n, l = rel - k * n;
  const float gamma = c.gamma_override >= 0.f ? c.gamma_override : (float)bp->st->masked / (float)(K * n);
  const uint8_t* Xc = bp->X + l;
  const int x = min((int)Xc[k * n], kMask);
  float mx0 = -INFINITY, mx1 = -INFINITY;
  for (int kk = 0; kk < K; ++kk) {
    const int xk = min((int)Xc[kk * n], kMask);
    mx0 = fmaxf(mx0, sEW[2 * xk] * inv_tau);
    mx1 = fmaxf(mx1, sEW[2 * xk + 1] * inv_tau);
  }
  float den0 = 0.f, den1 = 0.f;
  for (int kk = 0; kk < K; ++kk) {
    const int xk = min((int)Xc[kk * n], kMask);
    den0 += expf(sEW[2 * xk] * inv_tau - mx0);
    den1 += expf(sEW[2 * xk + 1] * inv_tau - mx1);
  }
  const int slot = bp->slot_off + l;
  const float c0 = expf(sEW[2 * x] * inv_tau - mx0) / den0 * a.p[2 * slot];
  const float c1 = expf(sEW[2 * x + 1] * inv_tau - mx1) / den1 * a.p[2 * slot + 1];
  const float* Pl = m.P + (long)l * D;
  const float* Ex = sE + x * EP;

  // ---- Z in the B-operand layout: k-step s holds features 16 s + 8 g2 + 0..7
  bf16x8 xf[KZ];
#pragma unroll
  for (int s = 0; s < KZ; ++s) {
    const int f = 16 * s + 8 * g2;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const f32x4 pq = *(const f32x4*)(Pl + f + 4 * h);
      const f32x4 eq = *(const f32x4*)(Ex + f + 4 * h);
      const f32x4 uq = *(const f32x4*)(su + f + 4 * h);
#pragma unroll
      for (int i = 0; i < 4; ++i) xf[s][4 * h + i] = (bf16)((eq[i] + pq[i]) + gamma * uq[i]);
    }
    asm volatile("" : "+v"(xf[s])::"memory");      // bounds the loads in flight
  }

  // ---- gate MLP over Z: up (d -> d, + c0 Wg1_e v_0 + c1 Wg1_e v_1, GELU), down (d -> d)
  f32x16 acc2[OBK];
#pragma unroll
  for (int ob = 0; ob < OBK; ++ob)
#pragma unroll
    for (int r = 0; r < 16; ++r) acc2[ob][r] = 0.f;
  m3_wait_barrier(nwm * (NBUF - 2));              // chunk 0 in LDS
#pragma unroll 1
  for (int ch = 0; ch < NCH; ++ch) {
    // buffer (ch + NBUF - 1) % NBUF was last read in iteration ch - 1, before its closing barrier
    if (ch + NBUF - 1 < NCH) dma_m(ch + NBUF - 1, (ch + NBUF - 1) % NBUF);
    const char* s1 = wreg + (ch % NBUF) * M::buf;
    const char* s2 = s1 + M::w1a;
    f32x16 acc1;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = ch * kM3FCH + 16 * (q >> 1) + 8 * g2 + 4 * (q & 1);
      const f32x4 bq = *(const f32x4*)&sbg1[f];
      const f32x4 u0 = *(const f32x4*)&sug[f];
      const f32x4 u1 = *(const f32x4*)&sug[D + f];
#pragma unroll
      for (int i = 0; i < 4; ++i) acc1[4 * q + i] = bq[i] + (c0 * u0[i] + c1 * u1[i]);
    }
#pragma unroll
    for (int s = 0; s < KZ; ++s) {
      const bf16x8 w = *(const bf16x8*)(s1 + l32 * MRB1 + (2 * s + g2) * 16);
      acc1 = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, xf[s], acc1, 0, 0, 0);
    }
    bf16x8 hf[2];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int i = 0; i < 4; ++i) hf[q >> 1][4 * (q & 1) + i] = (bf16)gelu_f(acc1[4 * q + i]);
#pragma unroll
    for (int ob = 0; ob < OBK; ++ob)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const bf16x8 w = *(const bf16x8*)(s2 + (32 * ob + l32) * MRB2 + (2 * s + g2) * 16);
        acc2[ob] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, hf[s], acc2[ob], 0, 0, 0);
      }
    // chunk ch + 1 complete in every wave: later chunks (at most NBUF - 2) may be in flight
    if (ch + 1 < NCH) m3_wait_barrier(nwm * (min(ch + NBUF - 1, NCH - 1) - (ch + 1)));
  }

  // ---- blend R = g Z + (1 - g) e, then the first LayerNorm.  Lane l holds
  // output features 32 ob + 8 q + 4 g2 + i of its token in register 4 q + i.
  float sum = 0.f;
#pragma unroll
  for (int ob = 0; ob < OBK; ++ob)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int f = 32 * ob + 8 * q + 4 * g2;
      const f32x4 pq = *(const f32x4*)(Pl + f);
      const f32x4 eq = *(const f32x4*)(Ex + f);
      const f32x4 uq = *(const f32x4*)(su + f);
      const f32x4 v0 = *(const f32x4*)(sv + f);
      const f32x4 v1 = *(const f32x4*)(sv + D + f);
      const f32x4 bq = *(const f32x4*)(sbg2 + f);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const float z = (eq[i] + pq[i]) + gamma * uq[i];
        const float e = c0 * v0[i] + c1 * v1[i];
        const float gt = sigmoid_f(acc2[ob][4 * q + i] + bq[i]);
        const float res = gt * z + (1.0f - gt) * e;
        acc2[ob][4 * q + i] = res;
        sum += res;
      }
      asm volatile("" ::: "memory");              // bounds the loads in flight
    }
  sum = xhalf_sum(sum);
  const float mean = sum / (float)D;
  float qv = 0.f;
#pragma unroll
  for (int ob = 0; ob < OBK; ++ob)
#pragma unroll
    for (int r = 0; r < 16; ++r) {
      const float dv = acc2[ob][r] - mean;
      qv = fmaf(dv, dv, qv);
    }
  qv = xhalf_sum(qv);
  const float rstd = 1.0f / sqrtf(qv / (float)D + 1e-5f);
  // R and XN leave as whole row segments (rows_store_*), through the two ring
  // buffers that do not hold the last chunk: both were last read before the
  // barrier that closed chunk NCH - 2, and no DMA targets them any more.
  // Waves 0-3 use one, waves 4-7 the other; row r of the wave is token
  // 256 blockIdx.x + 32 wave + r.
  static_assert(NW == 8 && 4 * 8192 <= M::buf && NCH >= NBUF - 1, "four 8 KB slices per free ring buffer");
  char* const slice = wreg + ((NCH + (wave >> 2)) % NBUF) * M::buf + (wave & 3) * 8192;
  const long row0 = (long)blockIdx.x * kM3BM + wave * 32;
  const auto rowtok = [&](int r) { return row0 + r < c.total_tokens ? row0 + r : -1L; };
  float mean2 = mean, rstd2 = rstd;
  asm volatile("" : "+v"(mean2), "+v"(rstd2));   // no (acc2 - mean) kept from the variance loop
  rows_store_bf16<D>(
      [&](int ob, int q) {
        const int f = 32 * ob + 8 * q + 4 * g2;
        const f32x4 lg = *(const f32x4*)(slg + f);
        const f32x4 lb = *(const f32x4*)(slb + f);
        bf16x4 h;
#pragma unroll
        for (int i = 0; i < 4; ++i) h[i] = (bf16)((acc2[ob][4 * q + i] - mean2) * rstd2 * lg[i] + lb[i]);
        return h;
      },
      a.XN, slice, lane, rowtok);
  rows_store_f32<D>(
      [&](int ob, int q) {
        return f32x4{acc2[ob][4 * q], acc2[ob][4 * q + 1], acc2[ob][4 * q + 2], acc2[ob][4 * q + 3]};
      },
      a.R, slice, lane, rowtok);
}

}  // namespace

// out = XN W^T + b (BF16), N a multiple of 32.
hipError_t launch_proj3_bf16(const GemmArgs& g, const Mat& W, hipStream_t s, bool gelu) {
  if (g.M == 0) return hipSuccess;
  if (!(g.Kd == 128 || g.Kd == 256 || g.Kd == 384 || g.Kd == 512) || g.N % 32 != 0 || g.N <= 0 || g.N > 1536)
    return hipErrorInvalidValue;
  dim3 grid((unsigned)((g.M + kM3BM - 1) / kM3BM)), block(512);
#define CIDER_P3(KD, CHB, WPE)                                                                     \
  if (g.Kd == KD && g.N % (32 * CHB) == 0) {                                                       \
    if (gelu) hipLaunchKernelGGL((k_proj3<KD, CHB, WPE, true>), grid, block, 0, s, g, W.b16);      \
    else hipLaunchKernelGGL((k_proj3<KD, CHB, WPE, false>), grid, block, 0, s, g, W.b16);          \
    return hipGetLastError();                                                                      \
  }
  CIDER_P3(128, 4, 2) CIDER_P3(128, 1, 4) CIDER_P3(256, 2, 4) CIDER_P3(256, 1, 4) CIDER_P3(384, 2, 2)
  CIDER_P3(384, 1, 2) CIDER_P3(512, 2, 2) CIDER_P3(512, 1, 2)
#undef CIDER_P3
  return hipErrorInvalidValue;
}

// R += A W^T + b (A in BF16, K = N = d), then the next LayerNorm into g.out.
hipError_t launch_oproj3_bf16(const GemmArgs& g, const Mat& W, hipStream_t s, bool gate) {
  if (g.M == 0) return hipSuccess;
  if (!(g.N == 128 || g.N == 256) || g.Kd != g.N || !g.ln_g || g.out_scale || g.proj_out) return hipErrorInvalidValue;
  if (gate && !g.E) return hipErrorInvalidValue;
  dim3 grid((unsigned)((g.M + kM3BM - 1) / kM3BM)), block(512);
  if (g.N == 128) {
    if (gate) hipLaunchKernelGGL((k_oproj3<128, true>), grid, block, 0, s, g, W.b16);
    else hipLaunchKernelGGL((k_oproj3<128, false>), grid, block, 0, s, g, W.b16);
  } else {
    if (gate) hipLaunchKernelGGL((k_oproj3<256, true>), grid, block, 0, s, g, W.b16);
    else hipLaunchKernelGGL((k_oproj3<256, false>), grid, block, 0, s, g, W.b16);
  }
  return hipGetLastError();
}

bool proj3_ok(int d) { return d == 128 || d == 256; }

// The token-resident QKV projection (input width d, 3d outputs).
bool qkv3_ok(int d) { return d == 128 || d == 256 || d == 384 || d == 512; }

bool mlp3_ok(int d, int F) { return (d == 128 || d == 256) && F % kM3FCH == 0 && F >= kM3FCH && F <= kM3MaxF; }

// R += W2 GELU(W1 XN + b1) + b2 with the next LayerNorm into g.out (g.ln_g set)
// or the final LayerNorm and projection into g.proj_out (g.proj_w set).
hipError_t launch_mlp3_bf16(const GemmArgs& g, const Mat& W1, const float* b1, const Mat& W2, int F, hipStream_t s) {
  if (g.M == 0) return hipSuccess;
  if (!mlp3_ok(g.N, F) || !g.ln_g || g.out_scale) return hipErrorInvalidValue;
  if (g.N == 128) {
    // 128 tokens per workgroup, two workgroups per CU when the hidden width allows
    if (F <= 512) return mlp3_t<128, 1, 4, 2, 4, true, 1, 512>(g, W1.b16, b1, W2.b16, F, s);
    return mlp3_t<128, 1, 8, 2, 4, true, 1>(g, W1.b16, b1, W2.b16, F, s);
  }
  return mlp3_t<256, 1, 8, 2, 3, false>(g, W1.b16, b1, W2.b16, F, s);
}

// ---------------------------------------------------------------------------
// Token-resident MLP for wide models (BF16, d = 384): 16 tokens per wave on
// MFMA 16 x 16 x 32, so that the d outputs of a wave's tokens (d / 4
// accumulators per lane) and its XN fragments (d / 8 registers) fit two waves
// per SIMD.  R += W2 GELU(W1 XN + b1) + b2, then the next LayerNorm into
// g.out (or, PROJ, the final LayerNorm and the 2-way projection).
//   up    acc1[u] (hidden 16 u + 4 (l/16) + r of token l % 16) starts at b1;
//         A = W1 rows of the chunk (natural order), B = XN[token][32 s + 8 (l/16) ..]
//   down  B = GELU of the lane's 8 hidden units: k-slot 8 (l/16) + e holds
//         hidden 4 (l/16) + e (e < 4) or 16 + 4 (l/16) + e - 4, and the A
//         operand reads W2's chunk columns in that order (two 8-byte halves)
// Weights go through LDS one chunk of 32 hidden units at a time, two
// buffers, the next chunk's DMA issued before the current one's MFMAs.
namespace {

template <int D, int MAXF>
struct M16Smem {
  static constexpr int RB1 = D * 2 + 16;          // W1 row pitch (bytes)
  static constexpr int RB2 = 32 * 2 + 16;         // W2 chunk row pitch
  static constexpr size_t w1 = (size_t)32 * RB1;
  static constexpr size_t w2 = (size_t)D * RB2;
  static constexpr size_t w1a = (w1 + 15) / 16 * 16;
  static constexpr size_t buf = (w1a + w2 + 1023) / 1024 * 1024;
  // b1, then b2, LN gain and bias, projection rows; the weights from a 1 KB boundary
  static constexpr size_t vec = ((size_t)(MAXF + 5 * D) * 4 + 1023) / 1024 * 1024;
  static constexpr size_t bytes = vec + 2 * buf;
  static_assert(bytes <= 160 * 1024, "LDS");
};

template <int D, int MAXF, bool PROJ>
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2, 2)))
void k_mlp16(GemmArgs g, const bf16* __restrict__ W1, const float* __restrict__ b1, const bf16* __restrict__ W2,
             int F) {
  using S = M16Smem<D, MAXF>;
  constexpr int NW = 8, KS = D / 32, OT = D / 16, RB1 = S::RB1, RB2 = S::RB2;
  constexpr int N1 = (int)((S::w1 + 1023) / 1024), N2 = (int)((S::w2 + 1023) / 1024), NM = N1 + N2;
  __shared__ __attribute__((aligned(1024))) char smem[S::bytes];
  float* sb1 = (float*)smem;
  float* sv = sb1 + MAXF;                           // b2, LN gain, LN bias, projection rows
  char* const wreg = smem + S::vec;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63, g4 = lane >> 4, l16 = lane & 15;
  const long tok0 = (long)blockIdx.x * (NW * 16) + wave * 16 + l16;
  const bool tv = tok0 < g.M;
  const long tok = tv ? tok0 : 0;
  const int nch = F / 32;
  const bf16* __restrict__ A = (const bf16*)g.A;

  auto dma = [&](int ch, int buf) {
    const int c0 = ch * 32;
    char* base = wreg + buf * S::buf;
#pragma unroll
    for (int k = 0; k < (NM + NW - 1) / NW; ++k) {
      const int u = wave + NW * k;
      if (u >= NM) break;
      if (u < N1) {
        const int pos = u * 1024 + lane * 16, j = pos / RB1, o = pos - j * RB1;
        const bool data = o < RB1 - 16;
        const bf16* src = W1 + (long)(c0 + (data ? j : 0)) * D + (data ? o / 2 : 0);
        if (pos < (int)S::w1)
          __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(base + u * 1024), 16, 0, 0);
      } else {
        const int pos = (u - N1) * 1024 + lane * 16, j = pos / RB2, o = pos - j * RB2;
        const bool data = o < RB2 - 16;
        const bf16* src = W2 + (long)(data ? j : 0) * F + c0 + (data ? o / 2 : 0);
        if (pos < (int)S::w2)
          __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void*)(base + S::w1a + (u - N1) * 1024),
                                           16, 0, 0);
      }
    }
  };
  for (int i = tid; i < F; i += NW * 64) sb1[i] = b1[i];
  m3_stage_vectors<D>(sv, g, PROJ, tid, NW * 64);
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");   // staged vectors written (visible after the first barrier)
  dma(0, 0);
  bf16x8 xf[KS];
#pragma unroll
  for (int s = 0; s < KS; ++s)
    xf[s] = tv ? *(const bf16x8*)(A + tok * D + 32 * s + 8 * g4) : bf16x8{0, 0, 0, 0, 0, 0, 0, 0};
  f32x4 acc2[OT];
#pragma unroll
  for (int t = 0; t < OT; ++t) acc2[t] = f32x4{0.f, 0.f, 0.f, 0.f};
  m3_wait_barrier(0);                               // chunk 0 and the vectors in LDS

#pragma unroll 1
  for (int ch = 0; ch < nch; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nch) dma(ch + 1, buf ^ 1);         // its last readers passed the previous barrier
    const char* s1 = wreg + buf * S::buf;
    const char* s2 = s1 + S::w1a;
    f32x4 acc1[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) acc1[u] = *(const f32x4*)&sb1[ch * 32 + 16 * u + 4 * g4];
    mfma_pipe<2 * KS, 3>(
        [&](int i) { return *(const bf16x8*)(s1 + (16 * (i & 1) + l16) * RB1 + (32 * (i >> 1) + 8 * g4) * 2); },
        [&](int i, const bf16x8& w) {
          acc1[i & 1] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, xf[i >> 1], acc1[i & 1], 0, 0, 0);
        });
    bf16x8 hf;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      hf[r] = (bf16)gelu_f(acc1[0][r]);
      hf[4 + r] = (bf16)gelu_f(acc1[1][r]);
    }
    mfma_pipe<OT, 3>(
        [&](int t) {
          const char* wr = s2 + (16 * t + l16) * RB2;
          const bf16x4 a0 = *(const bf16x4*)(wr + 8 * g4);
          const bf16x4 a1 = *(const bf16x4*)(wr + 32 + 8 * g4);
          return bf16x8{a0[0], a0[1], a0[2], a0[3], a1[0], a1[1], a1[2], a1[3]};
        },
        [&](int t, const bf16x8& w) { acc2[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(w, hf, acc2[t], 0, 0, 0); });
    // chunk ch + 1 complete in every wave, and every wave done with buffer buf
    if (ch + 1 < nch) m3_wait_barrier(0);
  }

  // ---- R += acc2 + b2, then the next LayerNorm (or the final one and the projection).
  // Lane l holds features 16 t + 4 (l/16) + r of token l % 16; four lanes per token.
  const float* slg = sv + D;
  const float* slb = sv + 2 * D;
  float* Rrow = g.R + tok * D;
  float sum = 0.f;
#pragma unroll
  for (int t = 0; t < OT; ++t) {
    const int f = 16 * t + 4 * g4;
    const f32x4 rr = tv ? *(const f32x4*)(Rrow + f) : f32x4{0.f, 0.f, 0.f, 0.f};
    const f32x4 bb = *(const f32x4*)&sv[f];
    const f32x4 res = rr + (acc2[t] + bb);
    acc2[t] = res;
    sum += (res[0] + res[1]) + (res[2] + res[3]);
    if (tv) *(f32x4*)(Rrow + f) = res;
    if ((t & 3) == 3) asm volatile("" ::: "memory");   // bounds the loads in flight
  }
  sum += __shfl_xor(sum, 16, 64);
  sum += __shfl_xor(sum, 32, 64);
  const float mean = sum / (float)D;
  float qv = 0.f;
#pragma unroll
  for (int t = 0; t < OT; ++t)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const float dv = acc2[t][r] - mean;
      qv = fmaf(dv, dv, qv);
    }
  qv += __shfl_xor(qv, 16, 64);
  qv += __shfl_xor(qv, 32, 64);
  const float rstd = 1.0f / sqrtf(qv / (float)D + 1e-5f);
  if (!PROJ) {
    bf16* xo = (bf16*)g.out + tok * D;
#pragma unroll
    for (int t = 0; t < OT; ++t) {
      const int f = 16 * t + 4 * g4;
      const f32x4 lg = *(const f32x4*)&slg[f];
      const f32x4 lb = *(const f32x4*)&slb[f];
      bf16x4 h;
#pragma unroll
      for (int r = 0; r < 4; ++r) h[r] = (bf16)((acc2[t][r] - mean) * rstd * lg[r] + lb[r]);
      if (tv) *(bf16x4*)(xo + f) = h;
    }
  } else {
    const float* sp0 = sv + 3 * D;
    const float* sp1 = sv + 4 * D;
    float a0 = 0.f, a1 = 0.f;
#pragma unroll
    for (int t = 0; t < OT; ++t) {
      const int f = 16 * t + 4 * g4;
      const f32x4 lg = *(const f32x4*)&slg[f];
      const f32x4 lb = *(const f32x4*)&slb[f];
      const f32x4 w0 = *(const f32x4*)&sp0[f];
      const f32x4 w1 = *(const f32x4*)&sp1[f];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float hv = (acc2[t][r] - mean) * rstd * lg[r] + lb[r];
        a0 = fmaf(hv, w0[r], a0);
        a1 = fmaf(hv, w1[r], a1);
      }
    }
    a0 += __shfl_xor(a0, 16, 64);
    a0 += __shfl_xor(a0, 32, 64);
    a1 += __shfl_xor(a1, 16, 64);
    a1 += __shfl_xor(a1, 32, 64);
    if (tv && g4 == 0) {
      g.proj_out[2 * tok] = a0;
      g.proj_out[2 * tok + 1] = a1;
    }
  }
}

}  // namespace

bool oproj_user_attn_ok(int d, int heads) { return d == 256 && heads * 32 == d; }

// R += O_row W_o^T + b_o (the row sublayer's output projection), then the
// user sublayer's QKV projection of LN(R) and its attention into O_user
// (BF16, d = 256, head width 32).  Groups from c.ugrp32.
hipError_t launch_oproj_user_attn(const StepCtx& c, const void* Orow, const Mat& Wo, const float* bo,
                                  const float* ln_g, const float* ln_b, float* R, const Mat& Wqkv, const float* bqkv,
                                  void* O, int d, int heads, hipStream_t s) {
  if (c.total_ugrp32 == 0) return hipSuccess;
  if (!oproj_user_attn_ok(d, heads) || !c.ugrp32 || !Wo.b16f || !Wqkv.b16f) return hipErrorInvalidValue;
  // four groups per workgroup, two workgroups per CU, fragment-major weights
  hipLaunchKernelGGL((k_oproj_user_attn4<256>), dim3((c.total_ugrp32 + 3) / 4), dim3(256), 0, s, c,
                     (const bf16*)Orow, Wo.b16f, bo, ln_g, ln_b, R, Wqkv.b16f, bqkv, (bf16*)O);
  return hipGetLastError();
}

bool oproj_mlp3_ok(int d, int F) { return d == 256 && F % kM3FCH == 0 && F >= 64 && F <= 1024; }

// R += O W_o^T + b_o, X = LN(R) with (lnx_g, lnx_b), then the MLP on X into R
// with the next LayerNorm (g.ln_g / g.ln_b into g.out) or the final
// projection (g.proj_w / g.proj_out).  BF16, d = 256.  g.A = O, g.bias = b2.
hipError_t launch_oproj_mlp3_bf16(const GemmArgs& g, const Mat& Wo, const float* bo, const float* lnx_g,
                                  const float* lnx_b, const Mat& W1, const float* b1, const Mat& W2, int F,
                                  hipStream_t s, int variant, bool f8_up) {
  if (g.M == 0) return hipSuccess;
  if (!oproj_mlp3_ok(g.N, F) || !g.ln_g || !Wo.b16 || !W1.b16k || !W2.b16) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((g.M + kM3BM - 1) / kM3BM)), block(512);
#define CIDER_OM(NB, PF)                                                                                          \
  if (g.proj_out)                                                                                                 \
    hipLaunchKernelGGL((k_oproj_mlp3<256, NB, 1024, true, PF>), grid, block, 0, s, g, Wo.b16, bo, lnx_g, lnx_b,    \
                       W1.b16k, b1, W2.b16, F, nullptr, 1.f);                                                      \
  else                                                                                                            \
    hipLaunchKernelGGL((k_oproj_mlp3<256, NB, 1024, false, PF>), grid, block, 0, s, g, Wo.b16, bo, lnx_g, lnx_b,   \
                       W1.b16k, b1, W2.b16, F, nullptr, 1.f);
  if (f8_up && W1.f8f && Wo.b16f && W2.b16f) {
    // the up projection in e4m3 on the four-wave kernel (W1.f8f: the reordered
    // e4m3 copy in fragment order)
    const dim3 grid4((unsigned)((g.M + 127) / 128)), block4(256);
    if (g.proj_out)
      hipLaunchKernelGGL((k_oproj_mlp4<256, 1024, true, 2, true>), grid4, block4, 0, s, g, Wo.b16f, bo, lnx_g, lnx_b,
                         W1.b16f, b1, W2.b16f, F, W1.f8f, W1.f8_scale);
    else
      hipLaunchKernelGGL((k_oproj_mlp4<256, 1024, false, 2, true>), grid4, block4, 0, s, g, Wo.b16f, bo, lnx_g, lnx_b,
                         W1.b16f, b1, W2.b16f, F, W1.f8f, W1.f8_scale);
    return hipGetLastError();
  }
  if (f8_up) {
    // the up projection in e4m3 (W1.f8p, the reordered copy)
    if (!W1.f8p) return hipErrorInvalidValue;
    if (g.proj_out)
      hipLaunchKernelGGL((k_oproj_mlp3<256, 2, 1024, true, 3, true>), grid, block, 0, s, g, Wo.b16, bo, lnx_g, lnx_b,
                         W1.b16k, b1, W2.b16, F, W1.f8p, W1.f8_scale);
    else
      hipLaunchKernelGGL((k_oproj_mlp3<256, 2, 1024, false, 3, true>), grid, block, 0, s, g, Wo.b16, bo, lnx_g, lnx_b,
                         W1.b16k, b1, W2.b16, F, W1.f8p, W1.f8_scale);
    return hipGetLastError();
  }
  // Variants 0-2: the four-wave k_oproj_mlp4 (two workgroups per CU, on the
  // fragment-major weight copies) with 3, 2 or 4 weight fragments in flight
  // ahead of its MFMAs; variants 3-7: the eight-wave k_oproj_mlp3 with MLP
  // weight-chunk rings of 2, 3 or 4 buffers and 2-4 fragments in flight.
  // Every element's arithmetic is the same in all of them.
  if (variant >= 0 && variant <= 2) {
    if (!Wo.b16f || !W1.b16f || !W2.b16f || F > 1024) return hipErrorInvalidValue;
    const dim3 grid4((unsigned)((g.M + 127) / 128)), block4(256);
#define CIDER_OM4(PF)                                                                                             \
  if (g.proj_out)                                                                                                 \
    hipLaunchKernelGGL((k_oproj_mlp4<256, 1024, true, PF>), grid4, block4, 0, s, g, Wo.b16f, bo, lnx_g, lnx_b,     \
                       W1.b16f, b1, W2.b16f, F, nullptr, 1.f);                                                     \
  else                                                                                                            \
    hipLaunchKernelGGL((k_oproj_mlp4<256, 1024, false, PF>), grid4, block4, 0, s, g, Wo.b16f, bo, lnx_g, lnx_b,    \
                       W1.b16f, b1, W2.b16f, F, nullptr, 1.f);
    if (variant == 1) { CIDER_OM4(2) }
    else if (variant == 2) { CIDER_OM4(4) }
    else { CIDER_OM4(3) }
#undef CIDER_OM4
    return hipGetLastError();
  }
  if (variant == 4) { CIDER_OM(3, 3) }
  else if (variant == 5) { CIDER_OM(2, 2) }
  else if (variant == 6) { CIDER_OM(2, 4) }
  else if (variant == 7) { CIDER_OM(4, 3) }
  else { CIDER_OM(2, 3) }
#undef CIDER_OM
  return hipGetLastError();
}

int oproj_mlp3_variants() { return 8; }

// The fragment-major copies k_oproj_mlp4 reads (see there): fragment f is
// elements 512 f .. 512 f + 511, lane l's eight at 8 l, lane l = 32 g2 + l32.
//   role 0, W_o [d][d]: f = (d / 32) (4 c + s) + b -> row 32 b + l32, columns
//     64 c + 16 s + 8 g2 + e (chunk c of 64 columns, k-step s, block b)
//   role 1, W1 [F][d]: f = (d / 16) ch + s -> row 32 ch + sigma(l32), the
//     k-ordered columns 16 s + 8 g2 + e (the order of X1's accumulator layout)
//   role 2, W2 [d][F]: f = (d / 16) ch + 2 b + ks -> row 32 b + l32, columns
//     32 ch + 16 ks + 8 g2 + e
//   role 3, Wqkv [3d][d] (k_oproj_user_attn4): f = (3 d / 32) t + 3 s + m ->
//     row m d + 32 (t / 2) + l32, the k-ordered columns 16 (d / 32 (t % 2) + s)
//     + 8 g2 + e (chunk t: head t / 2, half t % 2 of the k range; m = Q, K, V)
//   role 5, Wqkv [3d][d] (k_user_mlp_f): f = (3 d / 16) p + 3 s + m -> row
//     m d + 32 p + l32, columns 16 s + 8 g2 + e (head pair p, k-step s)
//   role 6, W_o [d][d] (k_user_mlp_f): f = (d / 16) p + 2 b + s -> row
//     32 b + l32, the k-ordered columns 32 p + 16 s + 8 g2 + e
// The e4m3 W1 of k_oproj_mlp4<..., F8>: from the reordered e4m3 rows w1p
// (Mat::f8p's layout, rows of d bytes), fragment (ch, t) of 2 KB holds, for
// lane l = 32 h + l32, bytes 64 t + 32 h .. + 31 of row 32 ch + sigma(l32) as
// two 16-byte halves at 16 l and 1024 + 16 l.
void om4_fragment_copy_f8(int d, int F, const uint8_t* w1p, uint8_t* dst) {
  const int nt = d / 64;
  for (int ch = 0; ch < F / 32; ++ch)
    for (int t = 0; t < nt; ++t)
      for (int l = 0; l < 64; ++l) {
        const int h = l >> 5, l32 = l & 31;
        const int q = l32 >> 3, g = (l32 >> 2) & 1, i = l32 & 3;
        const int row = 32 * ch + 16 * (q >> 1) + 8 * g + 4 * (q & 1) + i;   // sigma(l32)
        for (int half = 0; half < 2; ++half)
          for (int e = 0; e < 16; ++e)
            dst[((size_t)ch * nt + t) * 2048 + half * 1024 + (size_t)l * 16 + e] =
                w1p[(size_t)row * d + 64 * t + 32 * h + 16 * half + e];
      }
}

void om4_fragment_copy(int role, int d, int F, const float* src, uint16_t* dst, uint16_t (*to_bf16)(float)) {
  static const int kperm[16] = {0, 1, 2, 3, 8, 9, 10, 11, 4, 5, 6, 7, 12, 13, 14, 15};
  const int rows = role == 1 ? F : (role == 3 || role == 5) ? 3 * d : d, cols = role == 2 ? F : d;
  const size_t nfrag = (size_t)rows * cols / 512;
  const int obk = d / 32, ks = d / 16;
  for (size_t f = 0; f < nfrag; ++f)
    for (int l = 0; l < 64; ++l)
      for (int e = 0; e < 8; ++e) {
        const int g2 = l >> 5, l32 = l & 31;
        int r, c;
        if (role == 0) {
          const int cs = (int)(f / obk), b = (int)(f % obk);
          r = 32 * b + l32;
          c = 16 * cs + 8 * g2 + e;                 // 16 (4 c + s) = 64 c + 16 s
        } else if (role == 1) {
          const int ch = (int)(f / ks), s = (int)(f % ks);
          const int q = l32 >> 3, g = (l32 >> 2) & 1, i = l32 & 3;
          r = 32 * ch + 16 * (q >> 1) + 8 * g + 4 * (q & 1) + i;   // sigma(l32)
          const int kc = 16 * s + 8 * g2 + e;
          c = (kc & ~15) + kperm[kc & 15];
        } else if (role == 5) {
          const int p = (int)(f / (3 * ks)), i3 = (int)(f % (3 * ks)), s = i3 / 3, m = i3 % 3;
          r = m * d + 32 * p + l32;
          c = 16 * s + 8 * g2 + e;
        } else if (role == 6) {
          const int p = (int)(f / (2 * obk)), j = (int)(f % (2 * obk));
          r = 32 * (j >> 1) + l32;
          const int kc = 32 * p + 16 * (j & 1) + 8 * g2 + e;
          c = (kc & ~15) + kperm[kc & 15];
        } else if (role == 3) {
          const int kh = ks / 2, t = (int)(f / (3 * kh)), i3 = (int)(f % (3 * kh)), s = i3 / 3, m = i3 % 3;
          r = m * d + 32 * (t / 2) + l32;
          const int kc = 16 * (kh * (t % 2) + s) + 8 * g2 + e;
          c = (kc & ~15) + kperm[kc & 15];
        } else {
          const int ch = (int)(f / (2 * obk)), j = (int)(f % (2 * obk));
          r = 32 * (j >> 1) + l32;
          c = 32 * ch + 16 * (j & 1) + 8 * g2 + e;
        }
        dst[f * 512 + (size_t)l * 8 + e] = to_bf16(src[(size_t)r * cols + c]);
      }
}

bool mlp16_ok(int d, int F) { return d == 384 && F % 32 == 0 && F >= 64 && F <= 1536; }

// R += W2 GELU(W1 XN + b1) + b2 for the d = 384 model, 16 tokens per wave,
// with the next LayerNorm (g.ln_g / g.out) or the final LayerNorm and the
// projection (g.proj_out).
hipError_t launch_mlp16_bf16(const GemmArgs& g, const Mat& W1, const float* b1, const Mat& W2, int F, hipStream_t s) {
  if (g.M == 0) return hipSuccess;
  if (!mlp16_ok(g.N, F) || g.Kd != g.N || !g.ln_g || !g.R || !W1.b16 || !W2.b16 || (!g.proj_out && !g.out))
    return hipErrorInvalidValue;
  const dim3 grid((unsigned)((g.M + 127) / 128)), block(512);
  if (g.proj_out) hipLaunchKernelGGL((k_mlp16<384, 1536, true>), grid, block, 0, s, g, W1.b16, b1, W2.b16, F);
  else hipLaunchKernelGGL((k_mlp16<384, 1536, false>), grid, block, 0, s, g, W1.b16, b1, W2.b16, F);
  return hipGetLastError();
}

bool user_mlp_tr_ok(int d, int heads, int F) { return d == 128 && heads * 16 == d && F % kM3FCH == 0 && F >= 64 && F <= 512; }

// The user-attention sublayer and the MLP of one layer (BF16, d = 128, head
// width 16, hidden width <= 512): R and XN in, R and XN (or, with
// g.proj_out set, lbar) out.  Groups from c.ugrp32.
hipError_t launch_user_mlp_tr(const StepCtx& c, void* XN, const DevLayer& L, const GemmArgs& g2, int d, int heads,
                              int F, hipStream_t s, int variant) {
  if (c.total_ugrp32 == 0) return hipSuccess;
  if (!user_mlp_tr_ok(d, heads, F) || !c.ugrp32 || !L.Wqkv_u.b16 || !L.Wo_u.b16k || !L.W1.b16k || !L.W2.b16)
    return hipErrorInvalidValue;
  UserMlpArgs a{};
  // W_o and W1 multiply operands held in the accumulator layout: their k-ordered copies
  a.Wqkv = L.Wqkv_u.b16; a.bqkv = L.bqkv_u; a.Wo = L.Wo_u.b16k; a.bo = L.bo_u;
  a.ln3_g = L.ln3_g; a.ln3_b = L.ln3_b;
  a.W1 = L.W1.b16k; a.b1 = L.b1; a.W2 = L.W2.b16; a.F = F;
  a.g = g2;
  a.g.A = XN;
  a.g.M = c.total_tokens;
#define CIDER_UM(NW, NB, PF)                                                                                   \
  {                                                                                                            \
    const dim3 grid((c.total_ugrp32 + NW - 1) / NW), block(NW * 64);                                          \
    if (g2.proj_out) hipLaunchKernelGGL((k_user_mlp_tr<128, NW, NB, 512, true, PF>), grid, block, 0, s, c, a); \
    else hipLaunchKernelGGL((k_user_mlp_tr<128, NW, NB, 512, false, PF>), grid, block, 0, s, c, a);            \
  }
  // Variants 0-1: k_user_mlp_f (fragment-major weights, double-buffered
  // head-pair weights) with 3 or 2 weight fragments in flight; 2-6:
  // k_user_mlp_tr with 4 waves per workgroup (two workgroups per CU) or 8
  // (one, which halves the weight traffic per token), MLP chunk rings of 2 or
  // 3 and 2-4 fragments in flight.  Each wave's arithmetic on its own 32
  // tokens is the same in all of them.
  if (variant == 0 || variant == 1) {
    if (!L.Wqkv_u.b16f || !L.Wo_u.b16f || !L.W1.b16f || !L.W2.b16f) return hipErrorInvalidValue;
    UserMlpArgs af = a;
    af.Wqkv = L.Wqkv_u.b16f; af.Wo = L.Wo_u.b16f; af.W1 = L.W1.b16f; af.W2 = L.W2.b16f;
    const dim3 grid((c.total_ugrp32 + 3) / 4), block(256);
#define CIDER_UMF(PF)                                                                             \
  if (g2.proj_out) hipLaunchKernelGGL((k_user_mlp_f<128, 512, true, PF>), grid, block, 0, s, c, af); \
  else hipLaunchKernelGGL((k_user_mlp_f<128, 512, false, PF>), grid, block, 0, s, c, af);
    if (variant == 1) { CIDER_UMF(2) }
    else { CIDER_UMF(3) }
#undef CIDER_UMF
    return hipGetLastError();
  }
  if (variant == 3) CIDER_UM(4, 3, 3)
  else if (variant == 4) CIDER_UM(4, 2, 2)
  else if (variant == 5) CIDER_UM(4, 2, 4)
  else if (variant == 6) CIDER_UM(8, 3, 3)
  else CIDER_UM(4, 2, 3)
#undef CIDER_UM
  return hipGetLastError();
}

int user_mlp_tr_variants() { return 7; }

bool row_qkv_attn_ok(int d, int heads, int max_n) { return d == 256 && heads * 32 == d && max_n <= 256; }

// QKV projection + row attention for BF16 at d = 256, head width 32, rows of
// at most 256 tokens: O (BF16 [T][d]) from XN.  One workgroup per row.
hipError_t launch_row_qkv_attn(const StepCtx& c, const void* XN, const Mat& Wqkv, const float* bqkv, void* O, int d,
                               int heads, hipStream_t s) {
  if (c.total_rows == 0) return hipSuccess;
  if (!row_qkv_attn_ok(d, heads, c.max_n) || !Wqkv.b16) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_row_qkv_attn<256>), dim3(c.total_rows), dim3(512), 0, s, c, (const bf16*)XN, Wqkv.b16, bqkv,
                     (bf16*)O);
  return hipGetLastError();
}

bool row_block_tr_ok(int d, int heads, int max_n) { return d == 128 && heads * 16 == d && max_n <= 128; }

// The row-attention sublayer for BF16 at d = 128, head width 16, rows of at
// most 128 tokens: R += O W_o^T + b_o with O the row attention of the QKV
// projection of XN, then the next LayerNorm of R into XN (in place).  One
// workgroup per row.
hipError_t launch_row_block_tr(const StepCtx& c, void* XN, const DevLayer& L, const float* ln_g, const float* ln_b,
                               float* R, int d, int heads, hipStream_t s) {
  if (c.total_rows == 0) return hipSuccess;
  if (!row_block_tr_ok(d, heads, c.max_n) || !L.Wqkv_r.b16f || !L.Wo_r.b16f) return hipErrorInvalidValue;
  GemmArgs g{};
  g.M = c.total_tokens;
  g.N = d;
  g.Kd = d;
  g.A = XN;
  g.out = XN;
  g.bias = L.bo_r;
  g.R = R;
  g.ln_g = ln_g;
  g.ln_b = ln_b;
  // fragment-major weights, W_o double-buffered
  hipLaunchKernelGGL((k_row_block_tr<128>), dim3(c.total_rows), dim3(256), 0, s, c, g, L.Wqkv_r.b16f, L.bqkv_r,
                     L.Wo_r.b16f);
  return hipGetLastError();
}

bool user_block_tr_ok(int d, int heads) { return d == 128 && heads * 16 == d; }

// The user-attention sublayer for BF16 at d = 128, head width 16: R += O W_o^T
// + b_o with O the user attention of the QKV projection of XN, then the next
// LayerNorm of R into XN (in place).  Groups from c.ugrp32.
hipError_t launch_user_block_tr(const StepCtx& c, void* XN, const DevLayer& L, const float* ln_g, const float* ln_b,
                                float* R, int d, int heads, hipStream_t s) {
  if (c.total_ugrp32 == 0) return hipSuccess;
  if (!user_block_tr_ok(d, heads) || !c.ugrp32 || !L.Wqkv_u.b16 || !L.Wo_u.b16k) return hipErrorInvalidValue;
  GemmArgs g{};
  g.M = c.total_tokens;
  g.N = d;
  g.Kd = d;
  g.A = XN;
  g.out = XN;
  g.bias = L.bo_u;
  g.R = R;
  g.ln_g = ln_g;
  g.ln_b = ln_b;
  hipLaunchKernelGGL((k_user_block_tr<128, 4>), dim3((c.total_ugrp32 + 3) / 4), dim3(256), 0, s, c, g,
                     L.Wqkv_u.b16, L.bqkv_u, L.Wo_u.b16k);   // W_o k-ordered
  return hipGetLastError();
}

bool user_qkv_attn_ok(int d, int heads) { return d == 256 && heads * 32 == d; }

// QKV projection + user attention for BF16 at d = 256, head width 32: O (BF16
// [T][d]) from XN; groups from c.ugrp32.
hipError_t launch_user_qkv_attn(const StepCtx& c, const void* XN, const Mat& Wqkv, const float* bqkv, void* O,
                                int d, int heads, hipStream_t s) {
  if (c.total_ugrp32 == 0) return hipSuccess;
  if (!user_qkv_attn_ok(d, heads) || !c.ugrp32 || !Wqkv.b16) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_user_qkv_attn<256>), dim3((c.total_ugrp32 + 7) / 8), dim3(512), 0, s, c, (const bf16*)XN,
                     Wqkv.b16, bqkv, (bf16*)O);
  return hipGetLastError();
}

bool embed_gate3_ok(int d) { return d == 128; }

// Embedding, Module A and the first LayerNorm for the BF16 path (d = 128):
// writes R (FP32) and XN (BF16) of every token of the batch.
hipError_t launch_embed_gate3(const StepCtx& c, const EmbedW& m, const EmbedGateArgs& a, hipStream_t s) {
  if (c.total_tokens == 0) return hipSuccess;
  if (!embed_gate3_ok(m.d) || !c.tile_bin || !a.Wg1 || !a.Wg2 || !a.ug) return hipErrorInvalidValue;
  const int ntiles = (int)((c.total_tokens + kM3BM - 1) / kM3BM);
  int dev = 0, ncu = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
    return hipErrorInvalidValue;
  const int grid = std::min(ntiles, std::max(ncu, 1));
  hipLaunchKernelGGL((k_embed_gate3<128>), dim3(grid), dim3(512), 0, s, c, m, a, ntiles);
  return hipGetLastError();
}

bool embed_gate_z_ok(int d) { return d == 256; }

// Embedding, Module A and the first LayerNorm for the BF16 path (d = 256):
// writes R (FP32) and XN (BF16) of every token of the batch.
hipError_t launch_embed_gate_z(const StepCtx& c, const EmbedW& m, const EmbedGateArgs& a, hipStream_t s) {
  if (c.total_tokens == 0) return hipSuccess;
  if (!embed_gate_z_ok(m.d) || !c.tile_bin || !a.Wg1 || !a.Wg2 || !a.ug) return hipErrorInvalidValue;
  const int ntiles = (int)((c.total_tokens + kM3BM - 1) / kM3BM);
  hipLaunchKernelGGL((k_embed_gate_z<256>), dim3(ntiles), dim3(512), 0, s, c, m, a);
  return hipGetLastError();
}

}  // namespace cider
