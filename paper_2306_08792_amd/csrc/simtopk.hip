// Fused all-pairs similarity (MFMA) + streaming per-row top-k screening.
//
// The k-nearest-neighbour sets of Eq. (4) (and the cross-camera sets of
// Eq. (8)) need, for every row i, the k smallest ||x_i - x_j||^2.  For a
// fixed row this ranks columns by the key n2_j - 2 <x_i, x_j>.  Each work-
// group owns 128 rows and sweeps one column split in 128-column tiles; a tile
// of similarities is an MFMA GEMM over the feature dimension (float32,
// bfloat16 or FP8-E4M3 operands, float32 accumulation) and never leaves the
// registers.  Its epilogue screens every score against the row's running
// admission threshold and appends survivors to the row's candidate buffer
// (global memory, one region per row/list/split).
//
// Admission rule.  Let E_i bound |screened key - exact key| (screen_margin)
// and tau_i be the k-th smallest screened key the buffer has seen.  A column
// is admitted while its screened key <= tau_i + 2 E_i.  Because tau_i only
// decreases during the sweep and the true k-th key is <= tau_final + E_i,
// every true neighbour has a screened key <= tau_final + 2 E_i, so the
// buffer always keeps the exact top-k (ties included).  A full buffer is
// compacted by one wave: bitonic sort, new tau_i, drop keys above the
// threshold.  If the margin band alone fills the buffer (a split's local
// k-th neighbour can sit in a dense region of unrelated items), the buffer
// keeps its smallest keys and the admission threshold drops below the first
// key it gave up; the split's final threshold is written out, and the
// refine step falls back to an exhaustive row only if the global cut
// reaches beyond it.
#include "kernels.h"

namespace gcr {

namespace {
constexpr int BM = 128, BN = 128, NT = 256;
constexpr int LSTR = 144;                  // LDS row stride (128 B + 16 B pad)
constexpr int OPB = BM * LSTR;             // one operand tile in LDS
constexpr int SMEM = 4 * OPB;              // 2 stages x (rows, cols)
}  // namespace

int sim_topk_grid(int RB, int S) {
  const int RBg = (RB + 7) / 8;
  const int blocks = RBg * (S / 8);
  const int blocks8 = (blocks + 7) / 8 * 8;
  return blocks8 * 64;
}

template <int PREC>
__device__ __forceinline__ void mma_chunk(const uint8_t* __restrict__ Rt, const uint8_t* __restrict__ Ct,
                                          int wr, int wc, int lane, f32x16 (&acc)[2][2]) {
  const int l32 = lane & 31, half = lane >> 5;
  if constexpr (PREC == GCR_PREC_FP32) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      f32x4 vr[2], vc[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        vr[b] = *(const f32x4*)(Rt + (wr + 32 * b + l32) * LSTR + half * 64 + q * 16);
        vc[b] = *(const f32x4*)(Ct + (wc + 32 * b + l32) * LSTR + half * 64 + q * 16);
      }
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int rb = 0; rb < 2; ++rb)
            acc[cb][rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(vc[cb][s], vr[rb][s], acc[cb][rb], 0, 0, 0);
    }
  } else if constexpr (PREC == GCR_PREC_BF16) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      bf16x8 fr[2], fc[2];
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        fr[b] = *(const bf16x8*)(Rt + (wr + 32 * b + l32) * LSTR + half * 64 + q * 16);
        fc[b] = *(const bf16x8*)(Ct + (wc + 32 * b + l32) * LSTR + half * 64 + q * 16);
      }
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
          acc[cb][rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(fc[cb], fr[rb], acc[cb][rb], 0, 0, 0);
    }
  } else {
    i32x8 fr[2][2], fc[2][2];
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      const uint8_t* pr = Rt + (wr + 32 * b + l32) * LSTR + half * 64;
      const uint8_t* pc = Ct + (wc + 32 * b + l32) * LSTR + half * 64;
#pragma unroll
      for (int q = 0; q < 2; ++q) {
        fr[b][q] = *(const i32x8*)(pr + q * 32);
        fc[b][q] = *(const i32x8*)(pc + q * 32);
      }
    }
#pragma unroll
    for (int s = 0; s < 2; ++s)
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb = 0; rb < 2; ++rb)
          acc[cb][rb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(fc[cb][s], fr[rb][s], acc[cb][rb],
                                                                         0, 0, 0, 127, 0, 127);
  }
}

// Prefetch registers of one K chunk: 4 x 16 B of the row tile and of the
// column tile per thread (named members keep them in VGPRs).
struct Pref {
  u32x4 r0, r1, r2, r3, c0, c1, c2, c3;
};
#define GCR_GL(Q, RV, CV)                                                                   \
  {                                                                                         \
    const int seg = tid + NT * (Q), lr = seg >> 3, part = seg & 7;                          \
    RV = *(const u32x4*)(Xs + (row0 + lr) * ld + ch * 128 + part * 16);                     \
    CV = *(const u32x4*)(Xs + (ct0 + lr) * ld + ch * 128 + part * 16);                      \
  }
__device__ __forceinline__ void tile_gload(const uint8_t* __restrict__ Xs, int64_t ld, int64_t row0, int64_t ct0,
                                           int ch, int tid, Pref& p) {
  GCR_GL(0, p.r0, p.c0) GCR_GL(1, p.r1, p.c1) GCR_GL(2, p.r2, p.c2) GCR_GL(3, p.r3, p.c3)
}
#undef GCR_GL
#define GCR_LS(Q, RV, CV)                                                                   \
  {                                                                                         \
    const int seg = tid + NT * (Q), lr = seg >> 3, part = seg & 7;                          \
    *(u32x4*)(R + lr * LSTR + part * 16) = RV;                                              \
    *(u32x4*)(Cc + lr * LSTR + part * 16) = CV;                                             \
  }
__device__ __forceinline__ void tile_lstore(uint8_t* smem, int stage, int tid, const Pref& p) {
  uint8_t* R = smem + stage * 2 * OPB;
  uint8_t* Cc = R + OPB;
  GCR_LS(0, p.r0, p.c0) GCR_LS(1, p.r1, p.c1) GCR_LS(2, p.r2, p.c2) GCR_LS(3, p.r3, p.c3)
}
#undef GCR_LS

// One wave compacts the candidate buffer of (list L, local row lr): sort,
// tau = k-th smallest key, keep the keys <= tau + 2E.  When that band does
// not fit, keep only the m = max(C/2, k) smallest keys and lower the
// admission threshold below the first dropped key, so the buffer still
// holds every item of the split whose key is <= the threshold.
template <int E>
__device__ void compact_row(uint64_t* base, int* cnt, float* thr, int C, int kk, float twoE) {
  const int lane = threadIdx.x & 63;
  const int n = min(*cnt, C);
  uint64_t v[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = j * 64 + lane;
    v[j] = e < n ? base[e] : GCR_EMPTY;
  }
  wave_bitonic_sort<E>(v);
  auto elem = [&](int e) {
    uint64_t sel = 0;
#pragma unroll
    for (int j = 0; j < E; ++j) {
      const uint64_t t = shfl_u64(v[j], e & 63);
      if (j == (e >> 6)) sel = t;
    }
    return sel;
  };
  float th = *thr;
  if (n >= kk) th = fminf(th, cand_key(elem(kk - 1)) + twoE);
  int newn = 0;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const bool ok = v[j] != GCR_EMPTY && cand_key(v[j]) <= th;
    newn += __popcll(__ballot(ok));
  }
  if (newn > C - 16) {
    const int m = max(C / 2, kk);
    if (m < newn) {
      // admit only keys strictly below the first dropped one
      const float cut = cand_key(elem(m));
      th = fminf(th, nextafterf(cut, -INFINITY));
      newn = 0;
#pragma unroll
      for (int j = 0; j < E; ++j) {
        const bool ok = v[j] != GCR_EMPTY && cand_key(v[j]) <= th;
        newn += __popcll(__ballot(ok));
      }
    }
  }
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = j * 64 + lane;
    if (e < newn) base[e] = v[j];
  }
  if (lane == 0) { *cnt = newn; *thr = th; }
}

template <int PREC, int NL, int E>
__global__ __launch_bounds__(NT, 1) void sim_topk_kernel(SimArgs a) {
  extern __shared__ __align__(16) uint8_t smem[];
  __shared__ float col_n2[BN], col_sc[BN];
  __shared__ int col_cam[BN];
  __shared__ float row_thr[NL][BM];
  __shared__ int row_cnt[NL][BM];
  __shared__ float row_twoE[BM], row_sc[BM];
  __shared__ int row_cam[BM];
  __shared__ int any_flag[2];

  // XCD-aware placement: consecutive ids go round-robin over the 8 XCDs;
  // the 64 workgroups an XCD holds at a time form an 8 row-block x 8 split
  // block, so they share 8 row tiles and 8 column streams in its L2.
  const int id = blockIdx.x;
  const int xcd = id & 7, j = id >> 3;
  const int blk = (j >> 6) * 8 + xcd, w = j & 63;
  const int SG = a.S >> 3;
  const int rb = (blk / SG) * 8 + (w >> 3);
  const int cs = (blk % SG) * 8 + (w & 7);
  if (rb >= a.RB) return;

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t row0 = a.r0 + (int64_t)rb * BM;
  const int64_t sc0 = a.c0 + (int64_t)cs * a.W;
  const int64_t sc1 = min(a.c1, sc0 + a.W);
  const int ntiles = sc1 > sc0 ? (int)((sc1 - sc0 + BN - 1) / BN) : 0;
  const float maxn2 = *a.maxn2;

  if (tid < 2) any_flag[tid] = 0;
  for (int t = tid; t < BM; t += NT) {
    const int64_t r = row0 + t;
    const bool rv = r < a.r1;
    const float n2r = rv ? a.n2[r] : 0.f;
    row_twoE[t] = 2.0f * screen_margin(n2r, maxn2, a.eps_s, a.eps_n);
    row_cam[t] = (a.cam && rv) ? a.cam[r] : 0;
    row_sc[t] = (PREC == GCR_PREC_FP8 && rv) ? a.scale[r] : 1.0f;
#pragma unroll
    for (int L = 0; L < NL; ++L) {
      row_thr[L][t] = (rv && (L == 0 ? a.k0 : a.k1) > 0) ? INFINITY : -INFINITY;
      row_cnt[L][t] = 0;
    }
  }

  const int wr = (wave >> 1) * 64, wc = (wave & 1) * 64;
  const int kch = a.kchunks;
  const int total = ntiles * kch;
  const int64_t ld = a.ld_bytes;
  const uint8_t* __restrict__ Xs = a.Xs;
  Pref pf;

  const int l32 = lane & 31, half = lane >> 5;
  const int64_t rrel0 = row0 - a.r0;
  f32x16 acc[2][2];
#pragma unroll
  for (int cb = 0; cb < 2; ++cb)
#pragma unroll
    for (int rb2 = 0; rb2 < 2; ++rb2)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[cb][rb2][i] = 0.f;

  if (total > 0) {
    tile_gload(Xs, ld, row0, sc0, 0, tid, pf);
    tile_lstore(smem, 0, tid, pf);
  }
  __syncthreads();

  for (int g = 0; g < total; ++g) {
    const int tile = g / kch, ch = g - tile * kch;
    if (g + 1 < total) {
      const int tn = (g + 1) / kch;
      tile_gload(Xs, ld, row0, sc0 + (int64_t)tn * BN, (g + 1) - tn * kch, tid, pf);
    }
    {
      const uint8_t* R = smem + (g & 1) * 2 * OPB;
      mma_chunk<PREC>(R, R + OPB, wr, wc, lane, acc);
    }
    if (g + 1 < total) tile_lstore(smem, (g + 1) & 1, tid, pf);
    __syncthreads();
    if (ch != kch - 1) continue;

    // ---------------- epilogue of one 128 x 128 tile ----------------
    const int64_t ct0 = sc0 + (int64_t)tile * BN;
    if (tid < BN) {
      const int64_t c = ct0 + tid;
      const bool cv = c < sc1;
      col_n2[tid] = cv ? a.n2[c] : INFINITY;
      col_cam[tid] = (a.cam && cv) ? a.cam[c] : 0;
      col_sc[tid] = (PREC == GCR_PREC_FP8 && cv) ? a.scale[c] : 1.0f;
    }
    __syncthreads();

    uint64_t pend0 = 0, pend1 = 0;
    int it = 0;
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int rb2 = 0; rb2 < 2; ++rb2) {
        const int lr = wr + 32 * rb2 + l32;
        const int64_t row = row0 + lr;
        const float t0 = row_thr[0][lr];
        const float t1 = NL > 1 ? row_thr[NL - 1][lr] : -INFINITY;
        const float rs = row_sc[lr];
        const int rc = row_cam[lr];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
          const int lc = wc + 32 * cb + 8 * (i >> 2) + 4 * half + (i & 3);
          const int64_t col = ct0 + lc;
          float s = acc[cb][rb2][i];
          if (PREC == GCR_PREC_FP8) s = s * (rs * col_sc[lc]);
          const float key = col_n2[lc] - 2.0f * s;
          acc[cb][rb2][i] = key;
          const bool valid = col < sc1 && row < a.r1 && !(a.exclude_self && col == row);
          const int bit = cb * 32 + rb2 * 16 + i;
          if (valid && key <= t0) pend0 |= 1ull << bit;
          if (NL > 1 && valid && col_cam[lc] != rc && key <= t1) pend1 |= 1ull << bit;
        }
      }

    while (true) {
#pragma unroll
      for (int cb = 0; cb < 2; ++cb)
#pragma unroll
        for (int rb2 = 0; rb2 < 2; ++rb2)
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int bit = cb * 32 + rb2 * 16 + i;
            const int lr = wr + 32 * rb2 + l32;
            const int lc = wc + 32 * cb + 8 * (i >> 2) + 4 * half + (i & 3);
            const uint32_t colrel = (uint32_t)(ct0 + lc - a.c0);
#pragma unroll
            for (int L = 0; L < NL; ++L) {
              uint64_t& pend = L == 0 ? pend0 : pend1;
              if ((pend >> bit) & 1ull) {
                const int slot = atomicAdd(&row_cnt[L][lr], 1);
                if (slot < a.C) {
                  a.cand[(((rrel0 + lr) * NL + L) * (int64_t)a.S + cs) * a.C + slot] =
                      pack_cand(acc[cb][rb2][i], colrel);
                  pend &= ~(1ull << bit);
                }
              }
            }
          }
      const bool mine = (pend0 | pend1) != 0ull;
      if (__any(mine) && lane == 0) any_flag[it & 1] = 1;
      __syncthreads();
      const int any = any_flag[it & 1];
      if (tid == 0) any_flag[(it + 1) & 1] = 0;
      ++it;
      if (!any) break;
      for (int q = wave; q < NL * BM; q += NT / 64) {
        const int L = q / BM, lr = q - L * BM;
        if (row_cnt[L][lr] >= a.C) {
          uint64_t* base = a.cand + (((rrel0 + lr) * NL + L) * (int64_t)a.S + cs) * a.C;
          compact_row<E>(base, &row_cnt[L][lr], &row_thr[L][lr], a.C,
                         L == 0 ? a.k0 : a.k1, row_twoE[lr]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int rb2 = 0; rb2 < 2; ++rb2) {
        const int lr = wr + 32 * rb2 + l32;
        const float t0 = row_thr[0][lr];
        const float t1 = NL > 1 ? row_thr[NL - 1][lr] : -INFINITY;
#pragma unroll
        for (int cb = 0; cb < 2; ++cb)
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            const int bit = cb * 32 + rb2 * 16 + i;
            if (!(acc[cb][rb2][i] <= t0)) pend0 &= ~(1ull << bit);
            if (NL > 1 && !(acc[cb][rb2][i] <= t1)) pend1 &= ~(1ull << bit);
          }
      }
    }
#pragma unroll
    for (int cb = 0; cb < 2; ++cb)
#pragma unroll
      for (int rb2 = 0; rb2 < 2; ++rb2)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[cb][rb2][i] = 0.f;
  }

  __syncthreads();
  for (int t = tid; t < BM * NL; t += NT) {
    const int L = t / BM, lr = t - L * BM;
    if (row0 + lr < a.r1)
    {
      const int64_t o = ((rrel0 + lr) * NL + L) * (int64_t)a.S + cs;
      a.cnt[o] = min(row_cnt[L][lr], a.C);
      a.thr[o] = row_thr[L][lr];
    }
  }
}

template <int PREC, int NL>
static void launch_prec_nl(const SimArgs& a, hipStream_t st) {
  const dim3 grid(sim_topk_grid(a.RB, a.S)), block(NT);
  if (a.C <= 64) {
    auto k = sim_topk_kernel<PREC, NL, 1>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, SMEM);
    hipLaunchKernelGGL(k, grid, block, SMEM, st, a);
  } else if (a.C <= 128) {
    auto k = sim_topk_kernel<PREC, NL, 2>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, SMEM);
    hipLaunchKernelGGL(k, grid, block, SMEM, st, a);
  } else {
    auto k = sim_topk_kernel<PREC, NL, 4>;
    hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, SMEM);
    hipLaunchKernelGGL(k, grid, block, SMEM, st, a);
  }
}

void launch_sim_topk(int prec, int nl, const SimArgs& a, hipStream_t st) {
  if (prec == GCR_PREC_FP32) {
    if (nl == 1) launch_prec_nl<GCR_PREC_FP32, 1>(a, st); else launch_prec_nl<GCR_PREC_FP32, 2>(a, st);
  } else if (prec == GCR_PREC_BF16) {
    if (nl == 1) launch_prec_nl<GCR_PREC_BF16, 1>(a, st); else launch_prec_nl<GCR_PREC_BF16, 2>(a, st);
  } else {
    if (nl == 1) launch_prec_nl<GCR_PREC_FP8, 1>(a, st); else launch_prec_nl<GCR_PREC_FP8, 2>(a, st);
  }
}

}  // namespace gcr
