// Kernels of the serving path: one request's queries against a resident
// gallery whose kNN lists were built on the gallery alone and are frozen
// (precomputed gallery graphs, Sec. IV-F).  The node set of a request is the
// gallery plus its queries; a query row takes its k nearest gallery items
// (Eq. (4)); A = (A~ + A~^T)/2 and P = D^-1/2 A D^-1/2 over that node set
// (Eq. (5)-(7)); L rounds of x <- P x with row renormalisation (Eq. (2),
// (3)) on the fixed graph; then each query's top-K gallery items by squared
// distance over the propagated features.
//
// Gallery node v's row of P changes only when v or one of its neighbours is
// touched by a query (its degree grows by half the query edge weights), so
// after round t only the nodes within t - 1 hops of the touched-or-adjacent
// set R = T u N(T) differ from the gallery-only propagation, which is kept
// resident per round.  These kernels build R's hop sets and recompute
// exactly those rows; every other row reads the resident values.
#include "kernels.h"

namespace gcr {

namespace {
constexpr uint64_t NO_PAIR = ~0ull;
}

// One thread per pair slot i in [0, P): i < b k is query i / k's edge to
// gallery item q_idx[i] with weight exp(-d / gamma) (Eq. (4)); its sort key
// is (gallery item, i).  Threads i < b also write the query degree
// D_q = 1 + (1/2) sum_t w_qt (self weight 1, no gallery row points back).
__global__ void serve_query_edges_kernel(int b, int k, const int32_t* __restrict__ q_idx,
                                         const float* __restrict__ q_dist, float gamma, float* __restrict__ q_w,
                                         float* __restrict__ Dq, uint64_t* __restrict__ keys, int P) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < P) {
    uint64_t key = NO_PAIR;
    if (i < b * k) {
      const int32_t g = q_idx[i];
      const float w = g >= 0 ? expf(-q_dist[i] / gamma) : 0.f;
      q_w[i] = w;
      if (g >= 0) key = ((uint64_t)(uint32_t)g << 32) | (uint32_t)i;
    }
    keys[i] = key;
  }
  if (i < b) {
    float s = 0.f;
    for (int t = 0; t < k; ++t) {
      const int e = i * k + t;
      if (q_idx[e] >= 0) s += expf(-q_dist[e] / gamma);
    }
    Dq[i] = 1.0f + 0.5f * s;
  }
}

// One workgroup sorts the P (a power of two, <= 16,384) pair keys in LDS.
__global__ __launch_bounds__(1024) void serve_sort_pairs_kernel(uint64_t* __restrict__ keys, int P) {
  extern __shared__ uint64_t sk[];
  for (int t = threadIdx.x; t < P; t += blockDim.x) sk[t] = keys[t];
  __syncthreads();
  for (int size = 2; size <= P; size <<= 1) {
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      for (int t = threadIdx.x; t < (P >> 1); t += blockDim.x) {
        const int lo = 2 * t - (t & (stride - 1));
        const int hi = lo + stride;
        const bool asc = (lo & size) == 0;
        const uint64_t a = sk[lo], c = sk[hi];
        if ((a > c) == asc) { sk[lo] = c; sk[hi] = a; }
      }
      __syncthreads();
    }
  }
  for (int t = threadIdx.x; t < P; t += blockDim.x) keys[t] = sk[t];
}

// One thread per sorted pair: the first pair of each gallery item g records
// g as touched, its segment of query edges and its degree increase
// (1/2) sum of the edge weights, summed in segment order.
__global__ void serve_touched_kernel(const uint64_t* __restrict__ keys, int npairs, const float* __restrict__ q_w,
                                     uint32_t stamp, uint32_t* __restrict__ touched, float* __restrict__ dD,
                                     int32_t* __restrict__ seg_start, int32_t* __restrict__ seg_len,
                                     int32_t* __restrict__ T_list, int* __restrict__ T_count) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= npairs) return;
  const uint64_t key = keys[i];
  if (key == NO_PAIR) return;
  const uint32_t g = (uint32_t)(key >> 32);
  if (i > 0 && (uint32_t)(keys[i - 1] >> 32) == g) return;
  int j = i;
  float s = 0.f;
  while (j < npairs && keys[j] != NO_PAIR && (uint32_t)(keys[j] >> 32) == g) {
    s += q_w[(uint32_t)keys[j]];
    ++j;
  }
  touched[g] = stamp;
  dD[g] = 0.5f * s;
  seg_start[g] = i;
  seg_len[g] = j - i;
  T_list[atomicAdd(T_count, 1)] = (int32_t)g;
}

__device__ __forceinline__ void set_insert(int32_t h, uint32_t stamp, uint32_t* mark, int32_t* pos, int32_t* list,
                                           int* count, int cap) {
  if (atomicExch(&mark[h], stamp) != stamp) {
    const int p = atomicAdd(count, 1);
    if (p < cap) {
      list[p] = h;
      pos[h] = p;
    }
  }
}

// One wave per source node v: inserts v and its gallery neighbours (forward
// list and reverse list) into the set (mark == stamp, dense list + position).
__global__ __launch_bounds__(256) void serve_expand_kernel(const int32_t* __restrict__ src, const int* src_count,
                                                           int src_cap, const int32_t* __restrict__ gidx, int k,
                                                           const int32_t* __restrict__ rev_ptr,
                                                           const int32_t* __restrict__ rev_src, uint32_t stamp,
                                                           uint32_t* mark, int32_t* pos, int32_t* list, int* count,
                                                           int cap) {
  const int lane = threadIdx.x & 63;
  const int n = min(*src_count, src_cap);
  for (int w = blockIdx.x * 4 + (threadIdx.x >> 6); w < n; w += gridDim.x * 4) {
    const int32_t v = src[w];
    if (lane == 0) set_insert(v, stamp, mark, pos, list, count, cap);
    for (int t = lane; t < k; t += 64) {
      const int32_t h = gidx[(int64_t)v * k + t];
      if (h >= 0) set_insert(h, stamp, mark, pos, list, count, cap);
    }
    const int b = rev_ptr[v], e = rev_ptr[v + 1];
    for (int p = b + lane; p < e; p += 64) set_insert(rev_src[p], stamp, mark, pos, list, count, cap);
  }
}

namespace {

struct RowSrc {
  const float* X;          // level t - 1 features (gallery rows, then the slot's rows)
  int64_t qbase, pbase;    // slot rows: queries, then recomputed gallery rows
  const uint32_t* mark;    // recomputed at t - 1 (nullptr: none)
  const int32_t* pos;
  uint32_t stamp;
  int d;
  __device__ const float* gallery(int32_t h) const {
    if (mark && mark[h] == stamp) return X + (pbase + pos[h]) * (int64_t)d;
    return X + (int64_t)h * d;
  }
  __device__ const float* query(int q) const { return X + (qbase + q) * (int64_t)d; }
};

template <int NV>
__device__ __forceinline__ void axpy_lane(float (&acc)[NV], float c, const float* __restrict__ x, int d, int lane) {
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const int e = lane + 64 * j;
    if (e < d) acc[j] = fmaf(c, x[e], acc[j]);
  }
}

}  // namespace

// One wave per row of round t: the request's queries, then the gallery
// nodes of the round's set.  Degrees: D'_g = D0_g + dD_g for touched g.
template <int NV>
__global__ __launch_bounds__(256) void serve_propagate_kernel(ServePropArgs a) {
  const int lane = threadIdx.x & 63;
  RowSrc rs{a.Xprev, a.qbase, a.pbase, a.prev_mark, a.prev_pos, a.stamp, a.d};
  const int ncur = min(*a.cur_count, a.cap);
  const int items = a.b + ncur;
  const int d = a.d;
  for (int w = blockIdx.x * 4 + (threadIdx.x >> 6); w < items; w += gridDim.x * 4) {
    float acc[NV];
#pragma unroll
    for (int j = 0; j < NV; ++j) acc[j] = 0.f;
    float* out;
    if (w < a.b) {
      const int q = w;
      const float Dq = a.Dq[q];
      axpy_lane<NV>(acc, 1.0f / Dq, rs.query(q), d, lane);
      for (int t = 0; t < a.k; ++t) {
        const int e = q * a.k + t;
        const int32_t g = a.q_idx[e];
        if (g < 0) continue;
        const float Dg = a.D0[g] + (a.touched[g] == a.stamp ? a.dD[g] : 0.f);
        axpy_lane<NV>(acc, 0.5f * a.q_w[e] / sqrtf(Dq * Dg), rs.gallery(g), d, lane);
      }
      out = a.Xcur + (a.qbase + q) * (int64_t)d;
    } else {
      const int32_t v = a.cur_list[w - a.b];
      const bool tv = a.touched[v] == a.stamp;
      const float Dv = a.D0[v] + (tv ? a.dD[v] : 0.f);
      axpy_lane<NV>(acc, 1.0f / Dv, rs.gallery(v), d, lane);
      for (int t = 0; t < a.k; ++t) {
        const int64_t e = (int64_t)v * a.k + t;
        const int32_t h = a.gidx[e];
        if (h < 0) continue;
        const float Dh = a.D0[h] + (a.touched[h] == a.stamp ? a.dD[h] : 0.f);
        axpy_lane<NV>(acc, 0.5f * a.gw[e] / sqrtf(Dv * Dh), rs.gallery(h), d, lane);
      }
      for (int p = a.rev_ptr[v]; p < a.rev_ptr[v + 1]; ++p) {
        const int32_t h = a.rev_src[p];
        const float Dh = a.D0[h] + (a.touched[h] == a.stamp ? a.dD[h] : 0.f);
        axpy_lane<NV>(acc, 0.5f * a.rev_w[p] / sqrtf(Dv * Dh), rs.gallery(h), d, lane);
      }
      if (tv) {
        const int s0 = a.seg_start[v], s1 = s0 + a.seg_len[v];
        for (int p = s0; p < s1; ++p) {
          const uint32_t e = (uint32_t)a.pair_keys[p];
          const int q = (int)(e / (uint32_t)a.k);
          axpy_lane<NV>(acc, 0.5f * a.q_w[e] / sqrtf(Dv * a.Dq[q]), rs.query(q), d, lane);
        }
      }
      out = a.Xcur + (a.pbase + a.cur_pos[v]) * (int64_t)d;
    }
    float ss = 0.f;
#pragma unroll
    for (int j = 0; j < NV; ++j) ss = fmaf(acc[j], acc[j], ss);
    ss = wave_sum(ss);
    const float inv = 1.0f / fmaxf(sqrtf(ss), 1e-12f);
#pragma unroll
    for (int j = 0; j < NV; ++j) {
      const int e = lane + 64 * j;
      if (e < d) out[e] = acc[j] * inv;
    }
  }
}

// One thread per query: merge the top-K of the unchanged gallery columns
// (A, gallery indices) with the top-K of the recomputed rows (B, positions in
// list) by (distance, gallery index).
__global__ void serve_merge_kernel(int b, int K, const int32_t* __restrict__ ia, const float* __restrict__ da,
                                   const int32_t* __restrict__ ib, const float* __restrict__ db,
                                   const int32_t* __restrict__ list, int32_t* __restrict__ oi,
                                   float* __restrict__ od) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= b) return;
  int x = 0, y = 0;
  for (int t = 0; t < K; ++t) {
    const bool va = x < K && ia[q * K + x] >= 0;
    const bool vb = ib && y < K && ib[q * K + y] >= 0;
    int32_t g = -1;
    float dv = INFINITY;
    if (va && vb) {
      const int32_t ga = ia[q * K + x], gb = list[ib[q * K + y]];
      const float fa = da[q * K + x], fb = db[q * K + y];
      if (fa < fb || (fa == fb && ga < gb)) { g = ga; dv = fa; ++x; }
      else { g = gb; dv = fb; ++y; }
    } else if (va) {
      g = ia[q * K + x]; dv = da[q * K + x]; ++x;
    } else if (vb) {
      g = list[ib[q * K + y]]; dv = db[q * K + y]; ++y;
    }
    oi[q * K + t] = g;
    od[q * K + t] = dv;
  }
}

// Gallery rows stored as BF16 bit patterns -> their exact float32 values.
__global__ void bf16_to_f32_kernel(const uint16_t* __restrict__ in, float* __restrict__ out, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = __uint_as_float((uint32_t)in[i] << 16);
}

__global__ void copy_u32_kernel(const unsigned* __restrict__ src, unsigned* __restrict__ dst, int n) {
  const int i = threadIdx.x;
  if (i < n) dst[i] = src[i];
}

static inline unsigned nblocks(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_serve_query_edges(int b, int k, const int32_t* q_idx, const float* q_dist, float gamma, float* q_w,
                              float* Dq, uint64_t* keys, int P, hipStream_t st) {
  hipLaunchKernelGGL(serve_query_edges_kernel, dim3(nblocks(P, 256)), dim3(256), 0, st, b, k, q_idx, q_dist, gamma,
                     q_w, Dq, keys, P);
}

void launch_serve_sort_pairs(uint64_t* keys, int P, hipStream_t st) {
  const size_t lds = (size_t)P * sizeof(uint64_t);
  (void)hipFuncSetAttribute((const void*)serve_sort_pairs_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)lds);
  hipLaunchKernelGGL(serve_sort_pairs_kernel, dim3(1), dim3(1024), lds, st, keys, P);
}

void launch_serve_touched(const uint64_t* keys, int npairs, const float* q_w, uint32_t stamp, uint32_t* touched,
                          float* dD, int32_t* seg_start, int32_t* seg_len, int32_t* T_list, int* T_count,
                          hipStream_t st) {
  if (npairs <= 0) return;
  hipLaunchKernelGGL(serve_touched_kernel, dim3(nblocks(npairs, 256)), dim3(256), 0, st, keys, npairs, q_w, stamp,
                     touched, dD, seg_start, seg_len, T_list, T_count);
}

void launch_serve_expand(const int32_t* src, const int* src_count, int src_cap, const int32_t* gidx, int k,
                         const int32_t* rev_ptr, const int32_t* rev_src, uint32_t stamp, uint32_t* mark,
                         int32_t* pos, int32_t* list, int* count, int cap, hipStream_t st) {
  const unsigned grid = std::max(1u, std::min(nblocks(src_cap, 4), 2048u));
  hipLaunchKernelGGL(serve_expand_kernel, dim3(grid), dim3(256), 0, st, src, src_count, src_cap, gidx, k, rev_ptr,
                     rev_src, stamp, mark, pos, list, count, cap);
}

void launch_serve_propagate(const ServePropArgs& a, hipStream_t st) {
  const unsigned grid = std::max(1u, std::min(nblocks((int64_t)a.b + a.cap, 4), 2048u));
  const int nv = (a.d + 63) / 64;
  if (nv <= 2) hipLaunchKernelGGL(serve_propagate_kernel<2>, dim3(grid), dim3(256), 0, st, a);
  else if (nv <= 4) hipLaunchKernelGGL(serve_propagate_kernel<4>, dim3(grid), dim3(256), 0, st, a);
  else if (nv <= 8) hipLaunchKernelGGL(serve_propagate_kernel<8>, dim3(grid), dim3(256), 0, st, a);
  else if (nv <= 16) hipLaunchKernelGGL(serve_propagate_kernel<16>, dim3(grid), dim3(256), 0, st, a);
  else hipLaunchKernelGGL(serve_propagate_kernel<32>, dim3(grid), dim3(256), 0, st, a);
}

void launch_serve_merge(int b, int K, const int32_t* ia, const float* da, const int32_t* ib, const float* db,
                        const int32_t* list, int32_t* oi, float* od, hipStream_t st) {
  hipLaunchKernelGGL(serve_merge_kernel, dim3(nblocks(b, 64)), dim3(64), 0, st, b, K, ia, da, ib, db, list, oi, od);
}

void launch_bf16_to_f32(const uint16_t* in, float* out, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(bf16_to_f32_kernel, dim3(nblocks(n, 256)), dim3(256), 0, st, in, out, n);
}

void launch_copy_u32(const unsigned* src, unsigned* dst, int n, hipStream_t st) {
  hipLaunchKernelGGL(copy_u32_kernel, dim3(1), dim3(64), 0, st, src, dst, n);
}

}  // namespace gcr
