// Exact selection of the k nearest neighbours from the screened candidates.
//
// For one (row, list) the candidate buffers of all column splits are
// gathered, sorted by screened key, and cut at tau + 2 E (tau = k-th smallest
// screened key over all splits, E = screening margin): this superset holds
// the exact top-k as long as every split kept all of its items up to that
// cut (each split reports the threshold up to which its buffer is whole).  Its members are re-scored with the squared distance
// ||x_i - x_j||^2 evaluated in float-float arithmetic (error-free
// differences and products, compensated sums), then ordered by
// (distance, index), the order of Eq. (4)'s neighbour sets, and the first k
// are written.  Rows whose buffer overflowed are queued for the exhaustive
// path, which scores every column exactly and extracts the k smallest.
#include "kernels.h"

namespace gcr {

namespace {
constexpr int RT = 256;       // threads per refine block
constexpr int UMAX = 2048;    // max union size (S * C)
}  // namespace

// float-float squared distance of two float32 rows by one wave; the result
// is a packed key (ord(hi) << 32 | ord(lo)) whose unsigned order is the
// order of the exact values.
__device__ __forceinline__ uint64_t wave_exact_sqdist(const float* __restrict__ xa,
                                                      const float* __restrict__ xb, int d) {
  const int lane = threadIdx.x & 63;
  float hi = 0.f, lo = 0.f;
  if ((d & 3) == 0 && ((((uintptr_t)xa) | ((uintptr_t)xb)) & 15) == 0) {
    const int d4 = d >> 2;
    for (int e = lane; e < d4; e += 64) {
      const f32x4 a = ((const f32x4*)xa)[e], b = ((const f32x4*)xb)[e];
      ff_acc_sqdiff(hi, lo, a.x, b.x);
      ff_acc_sqdiff(hi, lo, a.y, b.y);
      ff_acc_sqdiff(hi, lo, a.z, b.z);
      ff_acc_sqdiff(hi, lo, a.w, b.w);
    }
  } else {
    for (int e = lane; e < d; e += 64) ff_acc_sqdiff(hi, lo, xa[e], xb[e]);
  }
  float h, l;
  fast_two_sum(hi, lo, h, l);
  wave_ff_sum(h, l);
  fast_two_sum(h, l, hi, lo);
  return ((uint64_t)ord_f32(hi) << 32) | (uint64_t)ord_f32(lo);
}

__device__ __forceinline__ float exact_hi(uint64_t k) { return unord_f32((uint32_t)(k >> 32)); }

// LDS bitonic sort of n (power of two) entries ordered by (key, aux).
__device__ void block_sort_pairs(uint64_t* key, uint32_t* aux, int n) {
  for (int size = 2; size <= n; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < (n >> 1); t += blockDim.x) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const uint64_t ka = key[lo], kb = key[hi];
        const uint32_t aa = aux[lo], ab = aux[hi];
        const bool gt = (ka > kb) || (ka == kb && aa > ab);
        if (gt == asc) {
          key[lo] = kb; key[hi] = ka;
          aux[lo] = ab; aux[hi] = aa;
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(RT) void refine_kernel(RefineArgs a) {
  __shared__ uint64_t U[UMAX];
  __shared__ uint64_t ek[UMAX];
  __shared__ uint32_t ec[UMAX];
  __shared__ int offs[65];
  __shared__ int s_M;
  __shared__ float s_tmin;

  const int NL = a.NL;
  const int64_t rrel = blockIdx.x / NL;
  const int L = blockIdx.x - (int)rrel * NL;
  const int64_t row = a.r0 + rrel;
  if (row >= a.r1) return;
  const int kk = L == 0 ? a.k0 : a.k1;
  int32_t* oidx = (L == 0 ? a.idx0 : a.idx1) + rrel * kk;
  float* odist = (L == 0 ? a.dist0 : a.dist1) + rrel * kk;
  const int tid = threadIdx.x;

  if (tid == 0) {
    int acc = 0;
    float tmin = INFINITY;
    const int64_t o = (rrel * NL + L) * (int64_t)a.S;
    for (int s = 0; s < a.S; ++s) {
      offs[s] = acc;
      acc += a.cnt[o + s];
      tmin = fminf(tmin, a.thr[o + s]);
    }
    offs[a.S] = acc;
    s_tmin = tmin;
  }
  __syncthreads();
  const int T = offs[a.S];
  int P = 64;
  while (P < T) P <<= 1;
  const uint64_t* cbase = a.cand + (rrel * NL + L) * (int64_t)a.S * a.C;
  for (int s = 0; s < a.S; ++s) {
    const int o = offs[s], c = offs[s + 1] - o;
    for (int t = tid; t < c; t += RT) U[o + t] = cbase[(int64_t)s * a.C + t];
  }
  for (int t = T + tid; t < P; t += RT) U[t] = GCR_EMPTY;
  for (int t = tid; t < P; t += RT) ec[t] = 0u;
  __syncthreads();
  block_sort_pairs(U, ec, P);

  // cut at tau + 2E
  const float twoE = 2.0f * screen_margin(a.n2[row], *a.maxn2, a.eps_s, a.eps_n);
  const float tau = (T >= kk && kk > 0) ? cand_key(U[kk - 1]) : INFINITY;
  const float th = tau + twoE;
  // every split holds all of its items with key <= its threshold; if the
  // cut reaches past one of them, this row needs the exhaustive path
  if (kk > 0 && th > s_tmin) {
    if (tid == 0) {
      const int slot = atomicAdd(a.fb_count, 1);
      a.fb_list[slot] = (int)(rrel * 2 + L);
    }
    return;
  }
  if (tid == 0) s_M = 0;
  __syncthreads();
  int mine = 0;
  for (int t = tid; t < T; t += RT) mine += cand_key(U[t]) <= th ? 1 : 0;
  if (mine) atomicAdd(&s_M, mine);
  __syncthreads();
  const int M = s_M;  // a prefix of the sorted union

  // exact re-score, one wave per candidate
  const int lane = tid & 63, wave = tid >> 6;
  const float* xr = a.X + row * (int64_t)a.d;
  for (int m = wave; m < M; m += RT / 64) {
    const uint32_t col = cand_col(U[m]);
    const uint64_t ex = wave_exact_sqdist(xr, a.X + (a.c0 + (int64_t)col) * a.d, a.d);
    if (lane == 0) { ek[m] = ex; ec[m] = col; }
  }
  int P2 = 64;
  while (P2 < M) P2 <<= 1;
  for (int t = M + tid; t < P2; t += RT) { ek[t] = GCR_EMPTY; ec[t] = 0xffffffffu; }
  __syncthreads();
  block_sort_pairs(ek, ec, P2);
  for (int t = tid; t < kk; t += RT) {
    if (t < M) {
      oidx[t] = (int32_t)ec[t];
      odist[t] = exact_hi(ek[t]);
    } else {
      oidx[t] = -1;
      odist[t] = INFINITY;
    }
  }
  if (tid == 0 && a.stat_cands) atomicAdd(a.stat_cands, (unsigned long long)M);
}

// Exhaustive exact path for (row, list) pairs whose cut reached past a
// split's threshold.  One block per pair (grid-stride); the row's slice of
// the feature vector stays in registers (d <= 2048), each wave scores one
// column at a time in float-float arithmetic, then k rounds of "smallest
// (distance, column) above the previous one" extract the list in order.
__device__ __forceinline__ uint64_t wave_exact_sqdist_reg(const float (&xr)[32], const float* __restrict__ xb,
                                                          int d) {
  const int lane = threadIdx.x & 63;
  float hi = 0.f, lo = 0.f;
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    const int e = lane + 64 * t;
    if (e < d) ff_acc_sqdiff(hi, lo, xr[t], xb[e]);
  }
  float h, l;
  fast_two_sum(hi, lo, h, l);
  wave_ff_sum(h, l);
  fast_two_sum(h, l, hi, lo);
  return ((uint64_t)ord_f32(hi) << 32) | (uint64_t)ord_f32(lo);
}

constexpr int FBT = 512;
__global__ __launch_bounds__(FBT) void fallback_kernel(RefineArgs a) {
  constexpr int NW = FBT / 64;
  __shared__ uint64_t rk[NW];
  __shared__ uint32_t rc[NW];
  __shared__ uint64_t bk;
  __shared__ uint32_t bc;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ncols = a.c1 - a.c0;
  uint64_t* scr = a.fb_scratch + (int64_t)blockIdx.x * ncols;
  const int nfb = *a.fb_count;
  for (int f = blockIdx.x; f < nfb; f += gridDim.x) {
    const int code = a.fb_list[f];
    const int64_t rrel = code >> 1;
    const int L = code & 1;
    const int64_t row = a.r0 + rrel;
    const int kk = L == 0 ? a.k0 : a.k1;
    int32_t* oidx = (L == 0 ? a.idx0 : a.idx1) + rrel * kk;
    float* odist = (L == 0 ? a.dist0 : a.dist1) + rrel * kk;
    const float* xrow = a.X + row * (int64_t)a.d;
    float xr[32];
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const int e = lane + 64 * t;
      xr[t] = e < a.d ? xrow[e] : 0.f;
    }
    const int rcam = a.cam ? a.cam[row] : 0;
    for (int64_t j = wave; j < ncols; j += NW) {
      const int64_t col = a.c0 + j;
      bool ok = !(a.exclude_self && col == row);
      if (L == 1) ok = ok && a.cam[col] != rcam;
      uint64_t v = GCR_EMPTY;
      if (ok) v = wave_exact_sqdist_reg(xr, a.X + col * (int64_t)a.d, a.d);
      if (lane == 0) scr[j] = v;
    }
    __syncthreads();
    uint64_t pk = 0;
    uint32_t pc = 0;
    bool have_prev = false;
    for (int t = 0; t < kk; ++t) {
      uint64_t best = GCR_EMPTY;
      uint32_t bcol = 0xffffffffu;
      for (int64_t j = tid; j < ncols; j += FBT) {
        const uint64_t v = scr[j];
        if (v == GCR_EMPTY) continue;
        const bool after = !have_prev || v > pk || (v == pk && (uint32_t)j > pc);
        const bool better = v < best || (v == best && (uint32_t)j < bcol);
        if (after && better) { best = v; bcol = (uint32_t)j; }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const uint64_t ov = shfl_xor_u64(best, o);
        const uint32_t oc = __shfl_xor(bcol, o, 64);
        if (ov < best || (ov == best && oc < bcol)) { best = ov; bcol = oc; }
      }
      if (lane == 0) { rk[wave] = best; rc[wave] = bcol; }
      __syncthreads();
      if (tid == 0) {
        uint64_t b = rk[0];
        uint32_t c = rc[0];
        for (int q = 1; q < NW; ++q)
          if (rk[q] < b || (rk[q] == b && rc[q] < c)) { b = rk[q]; c = rc[q]; }
        bk = b; bc = c;
        if (b == GCR_EMPTY) { oidx[t] = -1; odist[t] = INFINITY; }
        else { oidx[t] = (int32_t)c; odist[t] = exact_hi(b); }
      }
      __syncthreads();
      pk = bk; pc = bc; have_prev = true;
      if (pk == GCR_EMPTY) {
        for (int u = t + 1 + tid; u < kk; u += FBT) { oidx[u] = -1; odist[u] = INFINITY; }
        break;
      }
    }
    __syncthreads();
  }
}

void launch_refine(const RefineArgs& a, hipStream_t st) {
  const int64_t rows = a.r1 - a.r0;
  if (rows <= 0) return;
  hipLaunchKernelGGL(refine_kernel, dim3((unsigned)(rows * a.NL)), dim3(RT), 0, st, a);
  hipLaunchKernelGGL(fallback_kernel, dim3(a.fb_grid), dim3(FBT), 0, st, a);
}

}  // namespace gcr
