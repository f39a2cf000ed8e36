// Re-ranked distances: dense ||x_q - x_g||^2 between query and gallery rows
// of the propagated features (the ranking is read off the updated features).
//
// Split-bfloat16 GEMM over 128 x 128 tiles.  Every float32 feature x is held
// as hi + lo, hi = bf16(x), lo = bf16(x - hi) (x - hi is exact in float32),
// so |x - hi - lo| <= 2^-16 |x|.  The inner product of a pair is the sum of
// the four bfloat16 MFMA products hi.hi + hi.lo + lo.hi + lo.lo, each exact in
// the float32 accumulator; the only departure from the float32 inputs is the
// 2^-16 representation error, whose worst case (2^-15 sum |q_k g_k|) is below
// the float32 accumulation's own (d 2^-24 sum |q_k g_k|) from d = 512 on.
// Four bfloat16 MFMAs take a quarter of the cycles of the sixteen float32
// ones they replace, on the same operand bytes.  The epilogue forms
// n2_q + n2_g - 2 s (n2 from the float32 rows), clamps at 0 and stores.
#include "kernels.h"

namespace gcr {

namespace {
constexpr int BM = 128, NT = 256, LSTR = 144, OPB = BM * LSTR, SMEM = 4 * OPB;
}

// In-place rewrite of the float32 operand into the split form: each
// 32-float group (128 bytes) becomes its 32 hi parts followed by its 32 lo
// parts.  Eight lanes of one wave own a group; each lane reads 4 floats and
// writes their 4 hi and 4 lo parts, which the loads of the same wave
// instruction have already consumed.
__global__ __launch_bounds__(256) void split_bf16_kernel(uint8_t* __restrict__ Xs, int64_t groups) {
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t g = t >> 3;
  const int p = (int)(t & 7);
  if (g >= groups) return;
  uint8_t* base = Xs + g * 128;
  const f32x4 v = *(const f32x4*)(base + p * 16);
  const uint16_t h0 = f32_to_bf16_rne(v.x), h1 = f32_to_bf16_rne(v.y);
  const uint16_t h2 = f32_to_bf16_rne(v.z), h3 = f32_to_bf16_rne(v.w);
  const uint16_t l0 = f32_to_bf16_rne(v.x - bf16_to_f32(h0)), l1 = f32_to_bf16_rne(v.y - bf16_to_f32(h1));
  const uint16_t l2 = f32_to_bf16_rne(v.z - bf16_to_f32(h2)), l3 = f32_to_bf16_rne(v.w - bf16_to_f32(h3));
  uint2 hi, lo;
  hi.x = (uint32_t)h0 | ((uint32_t)h1 << 16);
  hi.y = (uint32_t)h2 | ((uint32_t)h3 << 16);
  lo.x = (uint32_t)l0 | ((uint32_t)l1 << 16);
  lo.y = (uint32_t)l2 | ((uint32_t)l3 << 16);
  *(uint2*)(base + p * 8) = hi;
  *(uint2*)(base + 64 + p * 8) = lo;
}

__global__ __launch_bounds__(NT, 2) void dense_dist_kernel(const uint8_t* __restrict__ Xs, int64_t ld,
                                                           int kch, const float* __restrict__ n2,
                                                           int64_t q0, int64_t nq, int64_t g0,
                                                           int64_t ng, float* __restrict__ out) {
  extern __shared__ __align__(16) uint8_t smem[];
  const int TR = (int)((nq + BM - 1) / BM), TC = (int)((ng + BM - 1) / BM);
  const int id = blockIdx.x, xcd = id & 7, j = id >> 3;
  const int blk = (j >> 6) * 8 + xcd, w = j & 63;
  const int TCg = (TC + 7) / 8;
  const int tr = (blk / TCg) * 8 + (w >> 3), tc = (blk % TCg) * 8 + (w & 7);
  if (tr >= TR || tc >= TC) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t rbase = q0 + (int64_t)tr * BM, cbase = g0 + (int64_t)tc * BM;
  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  const int l32 = lane & 31, half = lane >> 5;
  u32x4 r0, r1, r2, r3, c0, c1, c2, c3;
#define GCR_GL(Q, RV, CV)                                                        \
  {                                                                              \
    const int seg = tid + NT * (Q), lr = seg >> 3, part = seg & 7;               \
    RV = *(const u32x4*)(Xs + (rbase + lr) * ld + ch_ * 128 + part * 16);        \
    CV = *(const u32x4*)(Xs + (cbase + lr) * ld + ch_ * 128 + part * 16);        \
  }
#define GCR_LS(Q, RV, CV)                                                        \
  {                                                                              \
    const int seg = tid + NT * (Q), lr = seg >> 3, part = seg & 7;               \
    *(u32x4*)(Rw + lr * LSTR + part * 16) = RV;                                  \
    *(u32x4*)(Cw + lr * LSTR + part * 16) = CV;                                  \
  }
#define GCR_GLOAD(CH)                                                            \
  {                                                                              \
    const int ch_ = (CH);                                                        \
    GCR_GL(0, r0, c0) GCR_GL(1, r1, c1) GCR_GL(2, r2, c2) GCR_GL(3, r3, c3)      \
  }
#define GCR_LSTORE(ST)                                                           \
  {                                                                              \
    uint8_t* Rw = smem + (ST) * 2 * OPB;                                         \
    uint8_t* Cw = Rw + OPB;                                                      \
    GCR_LS(0, r0, c0) GCR_LS(1, r1, c1) GCR_LS(2, r2, c2) GCR_LS(3, r3, c3)      \
  }
  f32x16 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[a][b][i] = 0.f;
  GCR_GLOAD(0)
  GCR_LSTORE(0)
  __syncthreads();
  for (int ch = 0; ch < kch; ++ch) {
    if (ch + 1 < kch) GCR_GLOAD(ch + 1)
    const uint8_t* R = smem + (ch & 1) * 2 * OPB;
    const uint8_t* Cc = R + OPB;
    // a chunk holds 32 hi then 32 lo parts per row: two k-steps of 16, lane
    // half h taking elements 16 q + 8 h .. + 7 of both operands
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      bf16x8 rh[2], rl[2], chi[2], clo[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const uint8_t* pr = R + (wr + 32 * b + l32) * LSTR + q * 32 + half * 16;
        const uint8_t* pc = Cc + (wc + 32 * b + l32) * LSTR + q * 32 + half * 16;
        rh[b] = *(const bf16x8*)pr;
        rl[b] = *(const bf16x8*)(pr + 64);
        chi[b] = *(const bf16x8*)pc;
        clo[b] = *(const bf16x8*)(pc + 64);
      }
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) {
          acc[cb][rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(clo[cb], rl[rb], acc[cb][rb], 0, 0, 0);
          acc[cb][rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(clo[cb], rh[rb], acc[cb][rb], 0, 0, 0);
          acc[cb][rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(chi[cb], rl[rb], acc[cb][rb], 0, 0, 0);
          acc[cb][rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(chi[cb], rh[rb], acc[cb][rb], 0, 0, 0);
        }
    }
    if (ch + 1 < kch) GCR_LSTORE((ch + 1) & 1)
    __syncthreads();
  }
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
    const int64_t qr = (int64_t)tr * BM + wr + 32 * rb + l32;  // query index
    if (qr >= nq) continue;
    const float nqv = n2[q0 + qr];
    float* orow = out + qr * ng;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int64_t gc = (int64_t)tc * BM + wc + 32 * cb + 8 * (i >> 2) + 4 * half + (i & 3);
        if (gc < ng) orow[gc] = fmaxf(nqv + n2[g0 + gc] - 2.0f * acc[cb][rb][i], 0.f);
      }
  }
}

#undef GCR_GL
#undef GCR_LS
#undef GCR_GLOAD
#undef GCR_LSTORE

void launch_split_bf16(uint8_t* Xs, int64_t rows, int64_t ld_bytes, hipStream_t st) {
  const int64_t groups = rows * (ld_bytes / 128);
  if (groups <= 0) return;
  hipLaunchKernelGGL(split_bf16_kernel, dim3((unsigned)((groups * 8 + 255) / 256)), dim3(256), 0, st, Xs, groups);
}

void launch_dense_dist(const uint8_t* Xs, int64_t ld_bytes, int kchunks, const float* n2, int64_t q0,
                       int64_t nq, int64_t g0, int64_t ng, float* out, hipStream_t st) {
  if (nq <= 0 || ng <= 0) return;
  const int TR = (int)((nq + BM - 1) / BM), TC = (int)((ng + BM - 1) / BM);
  const int blocks = ((TR + 7) / 8) * ((TC + 7) / 8);
  const int grid = (blocks + 7) / 8 * 8 * 64;
  hipFuncSetAttribute((const void*)dense_dist_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, SMEM);
  hipLaunchKernelGGL(dense_dist_kernel, dim3(grid), dim3(NT), SMEM, st, Xs, ld_bytes, kchunks, n2, q0,
                     nq, g0, ng, out);
}

}  // namespace gcr
