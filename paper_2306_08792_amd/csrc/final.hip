// Re-ranked distances: dense ||x_q - x_g||^2 between query and gallery rows
// of the propagated features (the ranking is read off the updated features).
// A float32 MFMA GEMM over 128 x 128 tiles; the epilogue forms
// n2_q + n2_g - 2 s, clamps at 0 and stores.
#include "kernels.h"

namespace gcr {

namespace {
constexpr int BM = 128, NT = 256, LSTR = 144, OPB = BM * LSTR, SMEM = 4 * OPB;
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
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      f32x4 vr[2], vc[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        vr[b] = *(const f32x4*)(R + (wr + 32 * b + l32) * LSTR + half * 64 + q * 16);
        vc[b] = *(const f32x4*)(Cc + (wc + 32 * b + l32) * LSTR + half * 64 + q * 16);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
            acc[cb][rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(vc[cb][s], vr[rb][s], acc[cb][rb], 0, 0, 0);
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
