// Exact selection of the k nearest neighbours from the screened candidates.
//
// For one (row, list) the candidate buffers of all column splits are
// gathered, sorted by screened key, and cut at tau + 2 E (tau = k-th smallest
// screened key over all splits, E = screening margin): this superset holds
// the exact top-k as long as every split kept all of its items up to that
// cut (each split reports the threshold up to which its buffer is whole).  Its members are re-scored with the squared distance
// ||x_i - x_j||^2 accumulated in float64 from exactly squared float64
// differences (relative error about 2^-42 at d = 2048), then ordered by
// (distance, index), the order of Eq. (4)'s neighbour sets, and the first k
// are written.  Rows whose buffer overflowed are queued for the exhaustive
// path, which scores every column exactly and extracts the k smallest.
#include "kernels.h"

namespace gcr {

namespace {
constexpr int RT = 256;       // threads per refine block
constexpr int UMAX = 2048;    // max union size (S * C)
constexpr int FB_CW = 2048;   // columns per exhaustive work item
}  // namespace

// Exact squared distance of two float32 rows by one wave (float64
// accumulation of exact squared differences, sqdiff_acc); the result is the
// sum's order-preserving 64-bit key.
__device__ __forceinline__ uint64_t wave_exact_sqdist(const float* __restrict__ xa,
                                                      const float* __restrict__ xb, int d) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  if ((d & 3) == 0 && ((((uintptr_t)xa) | ((uintptr_t)xb)) & 15) == 0) {
    const int d4 = d >> 2;
    for (int e = lane; e < d4; e += 64) {
      const f32x4 a = ((const f32x4*)xa)[e], b = ((const f32x4*)xb)[e];
      s = sqdiff_acc(s, a.x, b.x);
      s = sqdiff_acc(s, a.y, b.y);
      s = sqdiff_acc(s, a.z, b.z);
      s = sqdiff_acc(s, a.w, b.w);
    }
  } else {
    for (int e = lane; e < d; e += 64) s = sqdiff_acc(s, xa[e], xb[e]);
  }
  return ord_f64(wave_sum_f64(s));
}

// The exact squared distance of a key, rounded to float32.
__device__ __forceinline__ float exact_dist(uint64_t k) { return (float)unord_f64(k); }

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

// Block version for the (row, list) pairs the wave kernel passes on (more
// than 128 candidates inside the cut): the union is sorted in LDS.
__global__ __launch_bounds__(RT) void refine_kernel(RefineArgs a) {
  __shared__ uint64_t U[UMAX];
  __shared__ uint64_t ek[UMAX];
  __shared__ uint32_t ec[UMAX];
  __shared__ int offs[65];
  __shared__ int s_M;
  __shared__ float s_tmin;

  const int NL = a.NL;
  const int nheavy = *a.heavy_count;
  for (int f = blockIdx.x; f < nheavy; f += gridDim.x) {
  __syncthreads();
  const int code = a.heavy_list[f];
  const int64_t rrel = code >> 1;
  const int L = code & 1;
  const int64_t row = a.r0 + rrel;
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
  const float twoE = 2.0f * screen_margin(a.n2[row], a.rn[row], a.maxn2[0], a.maxn2[1], a.eps_s, a.eps_n);
  const float tau = (T >= kk && kk > 0) ? cand_key(U[kk - 1]) : INFINITY;
  const float th = tau + twoE;
  // every split holds all of its items with key <= its threshold; if the
  // cut reaches past one of them, this row needs the exhaustive path
  if (kk > 0 && th > s_tmin) {
    if (tid == 0) {
      const int slot = atomicAdd(a.fb_count, 1);
      a.fb_list[slot] = (int)(rrel * 2 + L);
      // the k items with screened key <= tau have exact keys <= tau + E,
      // hence so does the exact k-th smallest key of the row
      a.fb_cut[slot] = tau + 0.5f * twoE;
    }
    continue;
  }
  if (tid == 0) s_M = 0;
  __syncthreads();
  int mine = 0;
  for (int t = tid; t < T; t += RT) mine += (cand_key(U[t]) <= th && cand_key(U[t]) < INFINITY) ? 1 : 0;
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
      odist[t] = exact_dist(ek[t]);
    } else {
      oidx[t] = -1;
      odist[t] = INFINITY;
    }
  }
  if (tid == 0 && a.stat_cands) atomicAdd(a.stat_cands, (unsigned long long)M);
  }  // heavy pairs
}

// ---------------------------------------------------------------------------
// One wave per (row, list): the union of the split buffers goes to the
// wave's LDS region, a radix select over the ordered keys gives tau (the
// k-th smallest screened key), the candidates with key <= tau + 2E (at most
// 128, else the pair goes to the block kernel) are re-scored exactly two at
// a time with the row held in registers, and a wave bitonic sort by
// (distance, index) orders them.
constexpr int WR_MAX = 256;  // re-scored candidates handled by one wave
constexpr int WR_EX = WR_MAX / 64;

__device__ __forceinline__ void wave_lds_sync() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int wave_sum_i(int v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Exact squared distances of the register-held row to two rows
__device__ __forceinline__ void wave_exact_sqdist2_reg(const float (&xr)[32], const float* __restrict__ xa,
                                                       const float* __restrict__ xb, int d, uint64_t& ka,
                                                       uint64_t& kb) {
  const int lane = threadIdx.x & 63;
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    const int e = lane + 64 * t;
    if (e < d) {
      sa = sqdiff_acc(sa, xr[t], xa[e]);
      sb = sqdiff_acc(sb, xr[t], xb[e]);
    }
  }
  ka = ord_f64(wave_sum_f64(sa));
  kb = ord_f64(wave_sum_f64(sb));
}

// The same with 16-byte loads when d is a multiple of 256 (lane l holds
// elements 4 l + 256 t .. + 3 of the row in xr4[t]).
template <int V>
__device__ __forceinline__ void wave_exact_sqdist2_vec(const f32x4 (&xr4)[V], const float* __restrict__ xa,
                                                       const float* __restrict__ xb, uint64_t& ka, uint64_t& kb) {
  const int lane = threadIdx.x & 63;
  f32x4 va[V], vb[V];
#pragma unroll
  for (int t = 0; t < V; ++t) {
    va[t] = ((const f32x4*)xa)[t * 64 + lane];
    vb[t] = ((const f32x4*)xb)[t * 64 + lane];
  }
  double sa = 0.0, sb = 0.0;
#pragma unroll
  for (int t = 0; t < V; ++t) {
    // The empty asm makes the row slice look fresh on every call, so the
    // compiler keeps it in float32 registers instead of hoisting its float64
    // conversion out of the caller's loop (twice the registers, one wave per
    // SIMD fewer).
    f32x4 r = xr4[t];
    asm volatile("" : "+v"(r));
    sa = sqdiff_acc(sa, r.x, va[t].x);
    sa = sqdiff_acc(sa, r.y, va[t].y);
    sa = sqdiff_acc(sa, r.z, va[t].z);
    sa = sqdiff_acc(sa, r.w, va[t].w);
    sb = sqdiff_acc(sb, r.x, vb[t].x);
    sb = sqdiff_acc(sb, r.y, vb[t].y);
    sb = sqdiff_acc(sb, r.z, vb[t].z);
    sb = sqdiff_acc(sb, r.w, vb[t].w);
  }
  ka = ord_f64(wave_sum_f64(sa));
  kb = ord_f64(wave_sum_f64(sb));
}

// ascending bitonic sort of 64 EX (key, index) pairs, EX per lane
// (element j * 64 + lane in k[j], c[j]), by key then index
template <int EX>
__device__ __forceinline__ void wave_sort_pairs(uint64_t (&k)[EX], uint32_t (&c)[EX]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int size = 2; size <= 64 * EX; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= 64) {
        const int rs = stride >> 6;
#pragma unroll
        for (int j = 0; j < EX; ++j) {
          if ((j & rs) == 0) {
            const int e = j * 64 + lane;
            const bool asc = (e & size) == 0;
            const bool gt = k[j] > k[j | rs] || (k[j] == k[j | rs] && c[j] > c[j | rs]);
            if (gt == asc) {
              const uint64_t tk = k[j]; k[j] = k[j | rs]; k[j | rs] = tk;
              const uint32_t tc = c[j]; c[j] = c[j | rs]; c[j | rs] = tc;
            }
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < EX; ++j) {
          const int e = j * 64 + lane;
          const bool asc = (e & size) == 0;
          const bool lower = (lane & stride) == 0;
          const uint64_t ok = shfl_xor_u64(k[j], stride);
          const uint32_t oc = __shfl_xor(c[j], stride, 64);
          const bool mine_le = k[j] < ok || (k[j] == ok && c[j] <= oc);
          const bool keep_mine = (lower == asc) ? mine_le : !mine_le;
          if (!keep_mine) { k[j] = ok; c[j] = oc; }
        }
      }
    }
  }
}

// V > 0: d == 256 V with 16-byte aligned rows; V == 0: any d <= 2048.
// At most 168 VGPRs (three waves per SIMD): the re-score loop is bound by
// the latency of its row gathers, and the third wave hides 15 % of it.
template <int V>
__global__ __launch_bounds__(256, 3) void refine_wave_kernel(RefineArgs a) {
  extern __shared__ uint64_t wsm[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int UW = a.S * a.C;
  uint64_t* U = wsm + (size_t)wave * UW;
  uint32_t* Mc = (uint32_t*)(wsm + (size_t)4 * UW) + wave * WR_MAX;
  const int NL = a.NL;
  const int64_t items = (a.r1 - a.r0) * NL;
  const int64_t p = xcd_position(blockIdx.x, gridDim.x) * 4 + wave;
  if (p >= items) return;
  const int64_t prel = p / NL;
  const int L = (int)(p - prel * NL);
  const int64_t rrel = a.order ? (int64_t)a.order[prel] : prel;
  const int64_t row = a.r0 + rrel;
  const int kk = L == 0 ? a.k0 : a.k1;
  int32_t* oidx = (L == 0 ? a.idx0 : a.idx1) + rrel * kk;
  float* odist = (L == 0 ? a.dist0 : a.dist1) + rrel * kk;

  // split counts (prefix over lanes) and the smallest split threshold
  const int64_t o = (rrel * NL + L) * (int64_t)a.S;
  int c = 0;
  float ts = INFINITY;
  if (lane < a.S) {
    c = min(a.cnt[o + lane], a.C);
    ts = a.thr[o + lane];
  }
  int incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  const int T = __shfl(incl, 63, 64);
  const int excl = incl - c;
  float tmin = ts;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) tmin = fminf(tmin, __shfl_xor(tmin, off, 64));
  const uint64_t* cbase = a.cand + o * a.C;
  for (int s = 0; s < a.S; ++s) {
    const int cs = __shfl(c, s, 64), os = __shfl(excl, s, 64);
    for (int t = lane; t < cs; t += 64) U[os + t] = cbase[(int64_t)s * a.C + t];
  }
  wave_lds_sync();

  // tau: smallest ordered key u with at least kk keys <= u
  float tau = INFINITY;
  if (T >= kk && kk > 0) {
    uint32_t lo = 0u, hi = 0xfffffffeu;
    while (lo < hi) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      int n = 0;
      for (int e = lane; e < T; e += 64) n += (uint32_t)(U[e] >> 32) <= mid ? 1 : 0;
      if (wave_sum_i(n) >= kk) hi = mid;
      else lo = mid + 1u;
    }
    tau = unord_f32(lo);
  }
  const float twoE = 2.0f * screen_margin(a.n2[row], a.rn[row], a.maxn2[0], a.maxn2[1], a.eps_s, a.eps_n);
  const float th = tau + twoE;
  if (kk > 0 && th > tmin) {
    if (lane == 0) {
      const int slot = atomicAdd(a.fb_count, 1);
      a.fb_list[slot] = (int)(rrel * 2 + L);
      a.fb_cut[slot] = tau + 0.5f * twoE;
    }
    return;
  }
  // the candidates inside the cut, compacted (order irrelevant)
  const uint32_t tho = ord_f32(th);
  int M = 0;
  for (int e0 = 0; e0 < T; e0 += 64) {
    const int e = e0 + lane;
    const uint64_t v = e < T ? U[e] : GCR_EMPTY;
    const bool keep = e < T && (uint32_t)(v >> 32) <= tho && cand_key(v) < INFINITY;
    const uint64_t bal = __ballot(keep);
    const int pos = M + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    if (keep && pos < WR_MAX) Mc[pos] = cand_col(v);
    M += __popcll(bal);
  }
  if (M > WR_MAX) {
    if (lane == 0) a.heavy_list[atomicAdd(a.heavy_count, 1)] = (int)(rrel * 2 + L);
    return;
  }
  wave_lds_sync();
  // exact re-score, two candidates per step, the row in registers
  const float* xrow = a.X + row * (int64_t)a.d;
  constexpr int NR = V > 0 ? V : 1;
  constexpr int NS = V > 0 ? 1 : 32;
  f32x4 xr4[NR];
  float xr[NS];
  if constexpr (V > 0) {
#pragma unroll
    for (int t = 0; t < V; ++t) xr4[t] = ((const f32x4*)xrow)[t * 64 + lane];
  } else {
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const int e = lane + 64 * t;
      xr[t] = e < a.d ? xrow[e] : 0.f;
    }
  }
  uint64_t ek[WR_EX];
  uint32_t ec[WR_EX];
#pragma unroll
  for (int j = 0; j < WR_EX; ++j) { ek[j] = GCR_EMPTY; ec[j] = 0xffffffffu; }
  for (int m = 0; m < M; m += 2) {
    const uint32_t ca = Mc[m];
    const uint32_t cb = m + 1 < M ? Mc[m + 1] : ca;
    uint64_t ka, kb;
    const float* pa = a.X + (a.c0 + (int64_t)ca) * a.d;
    const float* pb = a.X + (a.c0 + (int64_t)cb) * a.d;
    if constexpr (V > 0) wave_exact_sqdist2_vec<V>(xr4, pa, pb, ka, kb);
    else wave_exact_sqdist2_reg(xr, pa, pb, a.d, ka, kb);
#pragma unroll
    for (int j = 0; j < WR_EX; ++j) {
      if ((m >> 6) == j && (m & 63) == lane) { ek[j] = ka; ec[j] = ca; }
      if (m + 1 < M && ((m + 1) >> 6) == j && ((m + 1) & 63) == lane) { ek[j] = kb; ec[j] = cb; }
    }
  }
  // sort only as many slots as there are candidates
  if (M <= 64) {
    uint64_t k1[1] = {ek[0]};
    uint32_t c1[1] = {ec[0]};
    wave_sort_pairs<1>(k1, c1);
    ek[0] = k1[0]; ec[0] = c1[0];
  } else if (M <= 128) {
    uint64_t k2[2] = {ek[0], ek[1]};
    uint32_t c2[2] = {ec[0], ec[1]};
    wave_sort_pairs<2>(k2, c2);
    ek[0] = k2[0]; ek[1] = k2[1]; ec[0] = c2[0]; ec[1] = c2[1];
  } else {
    wave_sort_pairs<WR_EX>(ek, ec);
  }
#pragma unroll
  for (int j = 0; j < WR_EX; ++j) {
    const int t = j * 64 + lane;
    if (t < kk) {
      if (t < M) {
        oidx[t] = (int32_t)ec[j];
        odist[t] = exact_dist(ek[j]);
      } else {
        oidx[t] = -1;
        odist[t] = INFINITY;
      }
    }
  }
  if (lane == 0 && a.stat_cands) atomicAdd(a.stat_cands, (unsigned long long)M);
}

// Exhaustive exact path for (row, list) pairs whose cut reached past a
// split's threshold.  One block per pair (grid-stride); the row's slice of
// the feature vector stays in registers (d <= 2048), each wave scores one
// column at a time in float64 arithmetic, then k rounds of "smallest
// (distance, column) above the previous one" extract the list in order.
__device__ __forceinline__ uint64_t wave_exact_sqdist_reg(const float (&xr)[32], const float* __restrict__ xb,
                                                          int d) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    const int e = lane + 64 * t;
    if (e < d) s = sqdiff_acc(s, xr[t], xb[e]);
  }
  return ord_f64(wave_sum_f64(s));
}

// Column-parallel exhaustive path for the first fb_max queued pairs: each
// work item scores one 2,048-column chunk of one pair exactly and keeps the
// chunk's k smallest (distance, column); a merge then takes the k smallest
// over the chunks.  Pairs past fb_max use the one-block-per-pair kernel.
__device__ __forceinline__ bool lex_less(uint64_t ka, uint32_t ca, uint64_t kb, uint32_t cb) {
  return ka < kb || (ka == kb && ca < cb);
}
// block-wide minimum of (key, col) pairs over 256 threads
__device__ __forceinline__ void block_min_pair(uint64_t& k, uint32_t& c, uint64_t* rk, uint32_t* rc) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const uint64_t ok = shfl_xor_u64(k, o);
    const uint32_t oc = __shfl_xor(c, o, 64);
    if (lex_less(ok, oc, k, c)) { k = ok; c = oc; }
  }
  if (lane == 0) { rk[wave] = k; rc[wave] = c; }
  __syncthreads();
  k = rk[0]; c = rc[0];
  for (int q = 1; q < (int)(blockDim.x >> 6); ++q)
    if (lex_less(rk[q], rc[q], k, c)) { k = rk[q]; c = rc[q]; }
  __syncthreads();
}

__global__ __launch_bounds__(256) void fallback_scan_kernel(RefineArgs a) {
  __shared__ uint64_t sk[FB_CW];
  __shared__ uint64_t rk[4];
  __shared__ uint32_t rc[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int64_t ncols = a.c1 - a.c0;
  const int nch = (int)((ncols + FB_CW - 1) / FB_CW);
  const int nfb = min(*a.ovf_count, a.fb_max);
  for (int64_t wi = blockIdx.x; wi < (int64_t)nfb * nch; wi += gridDim.x) {
    const int f = (int)(wi / nch), ch = (int)(wi - (int64_t)f * nch);
    const int code = a.ovf_list[f];
    const int64_t rrel = code >> 1;
    const int L = code & 1;
    const int64_t row = a.r0 + rrel;
    const int kk = L == 0 ? a.k0 : a.k1;
    const float* xrow = a.X + row * (int64_t)a.d;
    float xr[32];
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const int e = lane + 64 * t;
      xr[t] = e < a.d ? xrow[e] : 0.f;
    }
    const int rcam = a.cam ? a.cam[row] : 0;
    const int64_t j0 = (int64_t)ch * FB_CW;
    const int nj = (int)min<int64_t>(FB_CW, ncols - j0);
    for (int j = wave; j < nj; j += 4) {
      const int64_t col = a.c0 + j0 + j;
      bool ok = !(a.exclude_self && col == row) && !column_out(a.filt, col, a.c0, row - a.r0);
      if (L == 1) ok = ok && a.cam[col] != rcam;
      uint64_t v = GCR_EMPTY;
      if (ok) v = wave_exact_sqdist_reg(xr, a.X + col * (int64_t)a.d, a.d);
      if (lane == 0) sk[j] = v;
    }
    __syncthreads();
    // every pair owns nch * kmax slots, whichever list it belongs to
    const int kmax = max(a.k0, a.k1);
    uint64_t* pk = a.fb_part_key + ((int64_t)f * nch + ch) * kmax;
    uint32_t* pc = a.fb_part_col + ((int64_t)f * nch + ch) * kmax;
    uint64_t prevk = 0;
    uint32_t prevc = 0;
    bool have = false;
    for (int t = 0; t < kk; ++t) {
      uint64_t bkey = GCR_EMPTY;
      uint32_t bcol = 0xffffffffu;
      for (int j = tid; j < nj; j += 256) {
        const uint64_t v = sk[j];
        if (v == GCR_EMPTY) continue;
        const uint32_t cj = (uint32_t)(j0 + j);
        if (have && !lex_less(prevk, prevc, v, cj)) continue;
        if (lex_less(v, cj, bkey, bcol)) { bkey = v; bcol = cj; }
      }
      block_min_pair(bkey, bcol, rk, rc);
      if (tid == 0) { pk[t] = bkey; pc[t] = bcol; }
      prevk = bkey; prevc = bcol; have = true;
      if (bkey == GCR_EMPTY) {
        for (int u = t + 1 + tid; u < kk; u += 256) { pk[u] = GCR_EMPTY; pc[u] = 0xffffffffu; }
        break;
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void fallback_merge_kernel(RefineArgs a) {
  __shared__ uint64_t rk[4];
  __shared__ uint32_t rc[4];
  const int tid = threadIdx.x;
  const int64_t ncols = a.c1 - a.c0;
  const int nch = (int)((ncols + FB_CW - 1) / FB_CW);
  const int nfb = min(*a.ovf_count, a.fb_max);
  for (int f = blockIdx.x; f < nfb; f += gridDim.x) {
    const int code = a.ovf_list[f];
    const int64_t rrel = code >> 1;
    const int L = code & 1;
    const int kk = L == 0 ? a.k0 : a.k1;
    int32_t* oidx = (L == 0 ? a.idx0 : a.idx1) + rrel * kk;
    float* odist = (L == 0 ? a.dist0 : a.dist1) + rrel * kk;
    const int kmax = max(a.k0, a.k1);
    const uint64_t* pk = a.fb_part_key + (int64_t)f * nch * kmax;
    const uint32_t* pc = a.fb_part_col + (int64_t)f * nch * kmax;
    uint64_t prevk = 0;
    uint32_t prevc = 0;
    bool have = false;
    for (int t = 0; t < kk; ++t) {
      uint64_t bkey = GCR_EMPTY;
      uint32_t bcol = 0xffffffffu;
      for (int j = tid; j < nch * kk; j += 256) {
        const int64_t o = (int64_t)(j / kk) * kmax + (j % kk);  // chunk j / kk, rank j % kk
        const uint64_t v = pk[o];
        if (v == GCR_EMPTY) continue;
        const uint32_t cj = pc[o];
        if (have && !lex_less(prevk, prevc, v, cj)) continue;
        if (lex_less(v, cj, bkey, bcol)) { bkey = v; bcol = cj; }
      }
      block_min_pair(bkey, bcol, rk, rc);
      if (tid == 0) {
        if (bkey == GCR_EMPTY) { oidx[t] = -1; odist[t] = INFINITY; }
        else { oidx[t] = (int32_t)bcol; odist[t] = exact_dist(bkey); }
      }
      prevk = bkey; prevc = bcol; have = true;
    }
  }
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
  const int nfb = *a.ovf_count;
  for (int f = a.fb_max + blockIdx.x; f < nfb; f += gridDim.x) {
    const int code = a.ovf_list[f];
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
      bool ok = !(a.exclude_self && col == row) && !column_out(a.filt, col, a.c0, row - a.r0);
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
        else { oidx[t] = (int32_t)c; odist[t] = exact_dist(b); }
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


// ---------------------------------------------------------------------------
// Band re-sweep for queued (row, list) pairs.  Pair f carries an upper bound
// ub_f on its exact k-th smallest key.  The sweep scores the pair's row
// against every column in float32 (sequential fused multiply-adds; error at
// most E32 = screen_margin at the float32 coefficient) and keeps each
// eligible column with key32 <= ub_f + E32, which holds every exact top-k
// member; the kept set is the prefix of the key32 order, so its k-th element
// is the global k-th smallest key32, tau32.  The selection then re-scores
// only the items with key32 <= tau32 + 2 E32 exactly.  Pairs whose kept set
// exceeds the band capacity go to the exhaustive path.
namespace {
constexpr int BT_R = 32;   // pairs per sweep tile
constexpr int BT_C = 128;  // columns per sweep tile
constexpr int BT_K = 32;   // feature chunk
}  // namespace

__global__ __launch_bounds__(256) void band_sweep_kernel(RefineArgs a) {
  __shared__ float As[BT_K][BT_R];
  __shared__ float Bs[BT_K][BT_C + 4];
  __shared__ int64_t s_row[BT_R];
  __shared__ int s_list[BT_R];
  __shared__ int s_cam[BT_R];
  __shared__ float s_cut[BT_R];
  const int tid = threadIdx.x;
  const int64_t ncols = a.c1 - a.c0;
  const int nf = min(*a.fb_count, a.band_max);
  const int nrt = (nf + BT_R - 1) / BT_R;
  const int nct = (int)((ncols + BT_C - 1) / BT_C);
  const int d = a.d;
  const bool vec = (d & 3) == 0 && (((uintptr_t)a.X) & 15) == 0;
  const float mx = *a.maxn2;
  const int eg = tid >> 5, cg = tid & 31;   // 4 pairs x 4 columns per thread
  for (int64_t wi = blockIdx.x; wi < (int64_t)nrt * nct; wi += gridDim.x) {
    const int rt = (int)(wi % nrt);
    const int ct = (int)(wi / nrt);
    const int f0 = rt * BT_R;
    const int64_t j0 = (int64_t)ct * BT_C;
    __syncthreads();
    if (tid < BT_R) {
      const int f = f0 + tid;
      if (f < nf) {
        const int code = a.fb_list[f];
        const int64_t row = a.r0 + (code >> 1);
        s_row[tid] = row;
        s_list[tid] = code & 1;
        s_cam[tid] = a.cam ? a.cam[row] : 0;
        const float n2r = a.n2[row];
        s_cut[tid] = a.fb_cut[f] + screen_margin(n2r, 0.f, mx, 0.f, a.eps32, a.eps_n);
      } else {
        s_row[tid] = -1;
        s_list[tid] = 0;
        s_cam[tid] = 0;
        s_cut[tid] = -INFINITY;
      }
    }
    __syncthreads();
    float acc[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = 0.f;
    // staging: pair tid / 8 takes floats 4 (tid % 8) .. +3 of the chunk;
    // column tid / 2 takes floats 16 (tid % 2) .. +15
    const int ar = tid >> 3, ak = (tid & 7) * 4;
    const int bc = tid >> 1, bk = (tid & 1) * 16;
    const int64_t arow = s_row[ar];
    const int64_t bcol = j0 + bc < ncols ? a.c0 + j0 + bc : -1;
    const float* ap = arow >= 0 ? a.X + arow * (int64_t)d : nullptr;
    const float* bp = bcol >= 0 ? a.X + bcol * (int64_t)d : nullptr;
    for (int k0 = 0; k0 < d; k0 += BT_K) {
      float av[4], bv[16];
      if (vec && k0 + BT_K <= d) {
        const f32x4 t = ap ? *(const f32x4*)(ap + k0 + ak) : f32x4{0.f, 0.f, 0.f, 0.f};
        av[0] = t.x; av[1] = t.y; av[2] = t.z; av[3] = t.w;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const f32x4 u = bp ? *(const f32x4*)(bp + k0 + bk + 4 * q) : f32x4{0.f, 0.f, 0.f, 0.f};
          bv[4 * q] = u.x; bv[4 * q + 1] = u.y; bv[4 * q + 2] = u.z; bv[4 * q + 3] = u.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < 4; ++q) av[q] = (ap && k0 + ak + q < d) ? ap[k0 + ak + q] : 0.f;
#pragma unroll
        for (int q = 0; q < 16; ++q) bv[q] = (bp && k0 + bk + q < d) ? bp[k0 + bk + q] : 0.f;
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < 4; ++q) As[ak + q][ar] = av[q];
#pragma unroll
      for (int q = 0; q < 16; ++q) Bs[bk + q][bc] = bv[q];
      __syncthreads();
#pragma unroll 8
      for (int k = 0; k < BT_K; ++k) {
        const f32x4 x = *(const f32x4*)&As[k][eg * 4];
        const f32x4 y = *(const f32x4*)&Bs[k][cg * 4];
        const float xa[4] = {x.x, x.y, x.z, x.w}, ya[4] = {y.x, y.y, y.z, y.w};
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int j = 0; j < 4; ++j) acc[i][j] = fmaf(xa[i], ya[j], acc[i][j]);
      }
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int pr = eg * 4 + i;
      const int64_t row = s_row[pr];
      if (row < 0) continue;
      const int L = s_list[pr];
      const float cut = s_cut[pr];
      const int f = f0 + pr;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int64_t jr = j0 + cg * 4 + j;
        if (jr >= ncols) continue;
        const int64_t col = a.c0 + jr;
        if (a.exclude_self && col == row) continue;
        if (column_out(a.filt, col, a.c0, row - a.r0)) continue;
        if (L == 1 && a.cam[col] == s_cam[pr]) continue;
        const float key = a.n2[col] - 2.0f * acc[i][j];
        if (key <= cut) {
          const int slot = atomicAdd(&a.band_cnt[f], 1);
          if (slot < a.band_cap)
            a.band[(int64_t)f * a.band_cap + slot] = ((uint64_t)ord_f32(key) << 32) | (uint64_t)(uint32_t)jr;
        }
      }
    }
  }
}

__global__ __launch_bounds__(RT) void band_select_kernel(RefineArgs a) {
  __shared__ uint64_t U[UMAX];
  __shared__ uint32_t ux[UMAX];
  __shared__ uint64_t ek[UMAX];
  __shared__ uint32_t ec[UMAX];
  __shared__ int s_M;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int nfb = *a.fb_count;
  const int nf = min(nfb, a.band_max);
  // pairs past the band capacity go straight to the exhaustive path
  for (int f = a.band_max + blockIdx.x * RT + tid; f < nfb; f += gridDim.x * RT) {
    const int slot = atomicAdd(a.ovf_count, 1);
    a.ovf_list[slot] = a.fb_list[f];
  }
  for (int f = blockIdx.x; f < nf; f += gridDim.x) {
    const int code = a.fb_list[f];
    const int64_t rrel = code >> 1;
    const int L = code & 1;
    const int64_t row = a.r0 + rrel;
    const int kk = L == 0 ? a.k0 : a.k1;
    const int T = a.band_cnt[f];
    if (T > a.band_cap) {
      if (tid == 0) {
        const int slot = atomicAdd(a.ovf_count, 1);
        a.ovf_list[slot] = code;
      }
      continue;
    }
    int32_t* oidx = (L == 0 ? a.idx0 : a.idx1) + rrel * kk;
    float* odist = (L == 0 ? a.dist0 : a.dist1) + rrel * kk;
    int P = 64;
    while (P < T) P <<= 1;
    const uint64_t* src = a.band + (int64_t)f * a.band_cap;
    __syncthreads();
    for (int t = tid; t < P; t += RT) {
      U[t] = t < T ? src[t] : GCR_EMPTY;
      ux[t] = 0u;
    }
    if (tid == 0) s_M = 0;
    __syncthreads();
    block_sort_pairs(U, ux, P);
    const float e32 = screen_margin(a.n2[row], 0.f, a.maxn2[0], 0.f, a.eps32, a.eps_n);
    const float th = (T >= kk && kk > 0) ? cand_key(U[kk - 1]) + 2.0f * e32 : INFINITY;
    int mine = 0;
    for (int t = tid; t < T; t += RT) mine += (cand_key(U[t]) <= th && cand_key(U[t]) < INFINITY) ? 1 : 0;
    if (mine) atomicAdd(&s_M, mine);
    __syncthreads();
    const int M = s_M;
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
        odist[t] = exact_dist(ek[t]);
      } else {
        oidx[t] = -1;
        odist[t] = INFINITY;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Split merge: one wave per (row, list, group of GS consecutive splits).
// Every split buffer holds all of its items with key <= its threshold, so the
// group's union holds all of the group's items with key <= tmin (the group's
// smallest threshold).  Items above the group's own k-th key + 2E cannot be
// within 2E of the global k-th key (which is no larger), so the merged buffer
// keeps the union up to cut = min(tmin, tau_g + 2E), and if that is more than
// C items, only the keys below the (C+1)-th smallest, lowering the cut; the
// merged threshold is the cut.  The exactness argument of the refine is
// unchanged: a merged buffer is a split buffer with a recorded threshold.
template <int NK>  // keys per lane: GS * C / 64
__global__ __launch_bounds__(256) void merge_splits_kernel(MergeArgs m) {
  extern __shared__ uint64_t msm[];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int GS = m.GS, C = m.C, S2 = m.S / GS;
  uint64_t* U = msm + (size_t)wave * GS * C;
  const int64_t items = m.rows * m.NL * S2;
  const int64_t it = (int64_t)blockIdx.x * 4 + wave;
  if (it >= items) return;
  const int64_t rl = it / S2;            // (row, list)
  const int g = (int)(it - rl * S2);
  const int64_t rrel = rl / m.NL;
  const int L = (int)(rl - rrel * m.NL);
  const int kk = L == 0 ? m.k0 : m.k1;
  const int64_t o = rl * m.S + (int64_t)g * GS;  // first split of the group
  int c = 0;
  float ts = INFINITY;
  if (lane < GS) {
    c = min(m.cnt[o + lane], C);
    ts = m.thr[o + lane];
  }
  int incl = c;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const int y = __shfl_up(incl, off, 64);
    if (lane >= off) incl += y;
  }
  const int T = __shfl(incl, 63, 64);
  const int excl = incl - c;
  float tmin = ts;
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) tmin = fminf(tmin, __shfl_xor(tmin, off, 64));
  const uint64_t* src = m.cand + o * C;
  for (int s = 0; s < GS; ++s) {
    const int cs = __shfl(c, s, 64), os = __shfl(excl, s, 64);
    for (int t = lane; t < cs; t += 64) U[os + t] = src[(int64_t)s * C + t];
  }
  wave_lds_sync();
  uint32_t key[NK];
#pragma unroll
  for (int j = 0; j < NK; ++j) {
    const int e = j * 64 + lane;
    key[j] = e < T ? (uint32_t)(U[e] >> 32) : 0xffffffffu;
  }
  auto count_le = [&](uint32_t u) {
    int n = 0;
#pragma unroll
    for (int j = 0; j < NK; ++j) n += __popcll(__ballot(key[j] <= u));
    return n;
  };
  auto select = [&](int r) {  // smallest ordered key with at least r keys <= it
    uint32_t lo = 0u, hi = 0xfffffffeu;
    while (lo < hi) {
      const uint32_t mid = lo + ((hi - lo) >> 1);
      if (count_le(mid) >= r) hi = mid;
      else lo = mid + 1u;
    }
    return lo;
  };
  float cut = tmin;
  if (kk > 0 && T >= kk) {
    const int64_t row = m.r0 + rrel;
    const float twoE = 2.0f * screen_margin(m.n2[row], m.rn[row], m.maxn2[0], m.maxn2[1], m.eps_s, m.eps_n);
    cut = fminf(cut, unord_f32(select(kk)) + twoE);
  }
  if (kk == 0) cut = -INFINITY;
  if (count_le(ord_f32(cut)) > C) cut = fminf(cut, nextafterf(unord_f32(select(C + 1)), -INFINITY));
  const uint32_t co = ord_f32(cut);
  uint64_t* dst = m.out_cand + (rl * S2 + g) * C;
  int n = 0;
  for (int e0 = 0; e0 < T; e0 += 64) {
    const int e = e0 + lane;
    const uint64_t v = e < T ? U[e] : GCR_EMPTY;
    const bool keep = e < T && (uint32_t)(v >> 32) <= co;
    const uint64_t bal = __ballot(keep);
    const int pos = n + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(bal >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)bal, 0u));
    if (keep) dst[pos] = v;
    n += __popcll(bal);
  }
  if (lane == 0) {
    m.out_cnt[rl * S2 + g] = n;
    m.out_thr[rl * S2 + g] = cut;
  }
}

void launch_merge_splits(const MergeArgs& m, hipStream_t st) {
  const int64_t items = m.rows * m.NL * (m.S / m.GS);
  if (items <= 0) return;
  const size_t lds = (size_t)4 * m.GS * m.C * sizeof(uint64_t);
  const dim3 grid((unsigned)((items + 3) / 4)), block(256);
  auto go = [&](auto k) {
    (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    hipLaunchKernelGGL(k, grid, block, lds, st, m);
  };
  const int nk = (m.GS * m.C + 63) / 64;
  if (nk <= 2) go(merge_splits_kernel<2>);
  else if (nk <= 4) go(merge_splits_kernel<4>);
  else if (nk <= 8) go(merge_splits_kernel<8>);
  else if (nk <= 16) go(merge_splits_kernel<16>);
  else go(merge_splits_kernel<32>);
}

// One wave per (row, list).  If the previous list of the row has k valid
// members j, the k-th smallest exact key of the row is at most
// U = max_j ||x_i - x_j||^2 - n2_i (up to the float32 error of n2_i), so the
// final screened k-th key tau is <= U + E and the refine's cut tau + 2E is
// <= U + 3E, E being the row's screening margin: the screening never needs
// to keep keys above U + 3E.
template <int V>
__global__ __launch_bounds__(256) void seed_thresholds_kernel(const float* __restrict__ X, int d, int64_t n,
                                                              const int32_t* __restrict__ idx0, int k0,
                                                              const int32_t* __restrict__ idx1, int k1,
                                                              const float* __restrict__ n2,
                                                              const float* __restrict__ rn,
                                                              const float* __restrict__ maxn2, float eps_s,
                                                              float eps_n, float* __restrict__ out,
                                                              const int32_t* __restrict__ order) {
  const int nl = idx1 ? 2 : 1;
  const int lane = threadIdx.x & 63;
  const int64_t p = xcd_position(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (p >= n * nl) return;
  const int64_t prow = p / nl;
  const int L = (int)(p - prow * nl);
  const int64_t row = order ? (int64_t)order[prow] : prow;
  const int64_t w = row * nl + L;
  const int kk = L == 0 ? k0 : k1;
  const int32_t* lst = (L == 0 ? idx0 : idx1) + row * kk;
  const float* xrow = X + row * (int64_t)d;
  constexpr int NR = V > 0 ? V : 1;
  constexpr int NS = V > 0 ? 1 : 32;
  f32x4 xr4[NR];
  float xr[NS];
  if constexpr (V > 0) {
#pragma unroll
    for (int t = 0; t < V; ++t) xr4[t] = ((const f32x4*)xrow)[t * 64 + lane];
  } else {
#pragma unroll
    for (int t = 0; t < 32; ++t) {
      const int e = lane + 64 * t;
      xr[t] = e < d ? xrow[e] : 0.f;
    }
  }
  // the list's valid members come first; two exact distances per step
  float umax = -INFINITY;
  int valid = 0;
  for (int t = 0; t < kk; t += 2) {
    const int32_t ja = lst[t];
    if (ja < 0) break;
    const int32_t jb0 = t + 1 < kk ? lst[t + 1] : -1;
    const int32_t jb = jb0 >= 0 ? jb0 : ja;
    uint64_t ka, kb;
    const float* pa = X + (int64_t)ja * d;
    const float* pb = X + (int64_t)jb * d;
    if constexpr (V > 0) wave_exact_sqdist2_vec<V>(xr4, pa, pb, ka, kb);
    else wave_exact_sqdist2_reg(xr, pa, pb, d, ka, kb);
    umax = fmaxf(umax, exact_dist(ka));
    ++valid;
    if (jb0 < 0) break;
    umax = fmaxf(umax, exact_dist(kb));
    ++valid;
  }
  if (lane != 0) return;
  float res = INFINITY;
  if (kk > 0 && valid == kk) {
    const float mx = *maxn2, n2r = n2[row];
    const float E = screen_margin(n2r, rn[row], mx, maxn2[1], eps_s, eps_n);
    const float u = umax - n2r + eps_n * mx;
    res = u + 3.0f * E + 4e-7f * (fabsf(umax) + n2r + 1.0f);
  }
  out[w] = res;
}

// The same bound from the BF16 screening operand (half the bytes of the
// float32 rows): every member's screened key n2_j - 2 x~_i.x~_j lies within
// E of its exact key (screen_margin holds for any float32 summation order),
// so the k-th exact key is at most the largest screened member key kmax + E,
// the sweep's final k-th screened key tau at most kmax + 2E, and the refine's
// cut tau + 2E at most kmax + 4E: seeding there keeps every split's recorded
// threshold at or above the cut, so a seeded row never needs the re-sweep.
// NV: 16-byte operand parts per lane (ld = 1024 NV bytes).
template <int NV>
__global__ __launch_bounds__(256) void seed_thresholds_bf16_kernel(const uint8_t* __restrict__ Xs, int64_t ld,
                                                                   int64_t n, const int32_t* __restrict__ idx0,
                                                                   int k0, const int32_t* __restrict__ idx1, int k1,
                                                                   const float* __restrict__ n2,
                                                                   const float* __restrict__ rn,
                                                                   const float* __restrict__ maxn2, float eps_s,
                                                                   float eps_n, float* __restrict__ out,
                                                                   const int32_t* __restrict__ order) {
  const int nl = idx1 ? 2 : 1;
  const int lane = threadIdx.x & 63;
  const int64_t p = xcd_position(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (p >= n * nl) return;
  const int64_t prow = p / nl;
  const int L = (int)(p - prow * nl);
  const int64_t row = order ? (int64_t)order[prow] : prow;
  const int kk = L == 0 ? k0 : k1;
  const int32_t* lst = (L == 0 ? idx0 : idx1) + row * kk;
  typedef uint32_t __attribute__((ext_vector_type(4))) u32x4;
  u32x4 xr[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) xr[q] = *(const u32x4*)(Xs + row * ld + (q * 64 + lane) * 16);
  auto dot = [&](const u32x4 (&y)[NV]) {
    float s = 0.f;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const uint32_t a = xr[q][c], b = y[q][c];
        s = fmaf(__uint_as_float(a << 16), __uint_as_float(b << 16), s);
        s = fmaf(__uint_as_float(a & 0xffff0000u), __uint_as_float(b & 0xffff0000u), s);
      }
    }
    return wave_sum(s);
  };
  // the list's members up to the first padding entry, 64 at a time in the
  // lanes, four rows gathered per step
  float kmax = -INFINITY;
  int valid = 0;
  for (int base = 0; base < kk; base += 64) {
    const int m = min(64, kk - base);
    const int32_t jl = lane < m ? lst[base + lane] : -1;
    const uint64_t okb = __ballot(jl >= 0);
    // members before the first -1 of this chunk (all m if there is none)
    const int run = ~okb ? min(m, (int)__builtin_ctzll(~okb)) : m;
    for (int t = 0; t < run; t += 4) {
      int32_t j[4];
      u32x4 y[4][NV];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        j[u] = __shfl(jl, min(t + u, run - 1), 64);
#pragma unroll
        for (int q = 0; q < NV; ++q) y[u][q] = *(const u32x4*)(Xs + (int64_t)j[u] * ld + (q * 64 + lane) * 16);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (t + u < run) kmax = fmaxf(kmax, n2[j[u]] - 2.0f * dot(y[u]));
    }
    valid += run;
    if (run < m) break;
  }
  if (lane != 0) return;
  float res = INFINITY;
  if (kk > 0 && valid == kk) {
    const float mx = *maxn2, n2r = n2[row];
    const float E = screen_margin(n2r, rn[row], mx, maxn2[1], eps_s, eps_n);
    res = kmax + 4.0f * E + 4e-7f * (fabsf(kmax) + n2r + 1.0f);
  }
  out[row * nl + L] = res;
}

void launch_seed_thresholds_bf16(const uint8_t* Xs, int64_t ld, int64_t n, const int32_t* idx0, int k0,
                                 const int32_t* idx1, int k1, const float* n2, const float* rn, const float* maxn2,
                                 float eps_s, float eps_n, float* out, const int32_t* order, hipStream_t st) {
  const int nl = idx1 ? 2 : 1;
  const int64_t waves = n * nl;
  const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
#define GCR_SEED16(V) hipLaunchKernelGGL(seed_thresholds_bf16_kernel<V>, grid, block, 0, st, Xs, ld, n, idx0, k0, \
                                         idx1, k1, n2, rn, maxn2, eps_s, eps_n, out, order)
  if (ld == 4096) GCR_SEED16(4);
  else if (ld == 2048) GCR_SEED16(2);
  else GCR_SEED16(1);
#undef GCR_SEED16
}

void launch_seed_thresholds(const float* X, int d, int64_t n, const int32_t* idx0, int k0, const int32_t* idx1,
                            int k1, const float* n2, const float* rn, const float* maxn2, float eps_s,
                            float eps_n, float* out, const int32_t* order, hipStream_t st) {
  const int nl = idx1 ? 2 : 1;
  const int64_t waves = n * nl;
  const dim3 grid((unsigned)((waves + 3) / 4)), block(256);
  const bool vec = d % 256 == 0 && (((uintptr_t)X) & 15) == 0;
#define GCR_SEED(V) hipLaunchKernelGGL(seed_thresholds_kernel<V>, grid, block, 0, st, X, d, n, idx0, k0, idx1, k1, \
                                       n2, rn, maxn2, eps_s, eps_n, out, order)
  if (vec && d == 2048) GCR_SEED(8);
  else if (vec && d == 1024) GCR_SEED(4);
  else if (vec && d == 512) GCR_SEED(2);
  else if (vec && d == 256) GCR_SEED(1);
  else GCR_SEED(0);
#undef GCR_SEED
}

// ---------------------------------------------------------------------------
// Screening-only selection (the raw precision modes): per (row, list) the k
// smallest screened keys of the union of the split buffers, ties by column,
// with no exact re-score.  The reported distance is n2_i + key (squared norms
// exact in float32, the inner product screened), clamped at zero.  Every
// split buffer holds all of its items up to its threshold, which is at least
// the split's own k-th key, so the union holds the row's k smallest screened
// keys.  One wave per pair: k rounds of "smallest entry above the last one".
__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = ((uint64_t)(uint32_t)__shfl_xor((int)(v >> 32), off, 64) << 32) |
                       (uint64_t)(uint32_t)__shfl_xor((int)(uint32_t)v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}

__global__ __launch_bounds__(256) void raw_select_kernel(RefineArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t items = (a.r1 - a.r0) * a.NL;
  const int64_t p = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (p >= items) return;
  const int64_t rrel = p / a.NL;
  const int L = (int)(p - rrel * a.NL);
  const int64_t row = a.r0 + rrel;
  const int kk = L == 0 ? a.k0 : a.k1;
  int32_t* oidx = (L == 0 ? a.idx0 : a.idx1) + rrel * kk;
  float* odist = (L == 0 ? a.dist0 : a.dist1) + rrel * kk;
  const int64_t o = (rrel * a.NL + L) * (int64_t)a.S;
  const float n2r = a.n2[row];
  uint64_t prev = 0;
  for (int t = 0; t < kk; ++t) {
    uint64_t best = GCR_EMPTY;
    for (int s = 0; s < a.S; ++s) {
      const int cs = min(a.cnt[o + s], a.C);
      const uint64_t* b = a.cand + (o + s) * (int64_t)a.C;
      for (int e = lane; e < cs; e += 64) {
        const uint64_t v = b[e];
        if ((t == 0 || v > prev) && v < best) best = v;
      }
    }
    best = wave_min_u64(best);
    if (lane == 0) {
      if (best == GCR_EMPTY) {
        oidx[t] = -1;
        odist[t] = INFINITY;
      } else {
        oidx[t] = (int32_t)cand_col(best);
        odist[t] = fmaxf(0.0f, n2r + cand_key(best));
      }
    }
    prev = best;
  }
}

void launch_raw_select(const RefineArgs& a, hipStream_t st) {
  const int64_t items = (a.r1 - a.r0) * a.NL;
  if (items <= 0) return;
  hipLaunchKernelGGL(raw_select_kernel, dim3((unsigned)((items + 3) / 4)), dim3(256), 0, st, a);
}

void launch_refine(const RefineArgs& a, hipStream_t st) {
  const int64_t rows = a.r1 - a.r0;
  if (rows <= 0) return;
  {
    const int64_t items = rows * a.NL;
    const size_t lds = (size_t)4 * a.S * a.C * sizeof(uint64_t) + (size_t)4 * WR_MAX * sizeof(uint32_t);
    const dim3 grid((unsigned)((items + 3) / 4)), block(256);
    const bool vec = a.d % 256 == 0 && (((uintptr_t)a.X) & 15) == 0;
    auto go = [&](auto kern) {
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
      hipLaunchKernelGGL(kern, grid, block, lds, st, a);
    };
    if (vec && a.d == 2048) go(refine_wave_kernel<8>);
    else if (vec && a.d == 1024) go(refine_wave_kernel<4>);
    else if (vec && a.d == 512) go(refine_wave_kernel<2>);
    else if (vec && a.d == 256) go(refine_wave_kernel<1>);
    else go(refine_wave_kernel<0>);
  }
  // the follow-up kernels find their work counts on the device and are
  // usually empty: grids of about one workgroup per compute unit keep the
  // empty launches cheap and still fill the GPU when there is work
  hipLaunchKernelGGL(refine_kernel, dim3(256), dim3(RT), 0, st, a);
  hipLaunchKernelGGL(band_sweep_kernel, dim3(512), dim3(256), 0, st, a);
  hipLaunchKernelGGL(band_select_kernel, dim3(256), dim3(RT), 0, st, a);
  hipLaunchKernelGGL(fallback_scan_kernel, dim3(512), dim3(256), 0, st, a);
  hipLaunchKernelGGL(fallback_merge_kernel, dim3(256), dim3(256), 0, st, a);
  hipLaunchKernelGGL(fallback_kernel, dim3(a.fb_grid), dim3(FBT), 0, st, a);
}

}  // namespace gcr
