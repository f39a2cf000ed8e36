// Sparse symmetric affinity graph from the kNN lists (Eq. (4)-(9)).
//
//   w_ij = beta(cam_i, cam_j) exp(-d_ij / gamma)   for j in N_i     (Eq. (4))
//   A = (A~ + A~^T) / 2 is never formed: row i keeps its forward list
//   (weight w_ij / 2) and a reverse list of the edges j -> i (weight
//   w_ji / 2); a mutual pair simply appears in both, which sums to A_ij.
//   D_i = 1 + sum_fwd w/2 + sum_rev w/2                              (Eq. (5), (7))
//   P_ij = A_ij / sqrt(D_i D_j), P_ii = 1 / D_i                       (Eq. (2))
// Asymmetric variant (Eq. (5), (6)): D_r(i) = 1 + sum_fwd w, D_c(j) = 1 +
// sum_rev w, P = D_r^-1/2 A~ D_c^-1/2 with the forward lists only.
// The reverse lists are a CSR built by a count / exclusive scan / scatter,
// then each row is sorted by source so that sums run in a fixed order.
#include "kernels.h"

namespace gcr {

__global__ void zero_i32_kernel(int32_t* p, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// One thread per forward edge: its weight, and one more entry in the
// reverse row of its target.
__global__ void edge_weight_kernel(GraphBuildArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n * a.k) return;
  const int j = a.idx[e];
  float wv = 0.f;
  if (j >= 0) {
    wv = expf(-a.dist[e] / a.gamma);
    if (a.use_beta && a.cam) wv *= (a.cam[j] == a.cam[e / a.k]) ? a.beta_same : a.beta_cross;
    atomicAdd(&a.tmp_cnt[j], 1);
  }
  a.w[e] = wv;
}

// exclusive scan of tmp_cnt into rev_ptr (n+1 entries): block-local scans of
// 1024-entry tiles, a scan of the tile totals, then the add-back.
__global__ __launch_bounds__(1024) void scan_tiles_kernel(const int32_t* in, int32_t* out,
                                                          int64_t n, int32_t* tile_sum) {
  __shared__ int32_t s[1024];
  const int64_t i = (int64_t)blockIdx.x * 1024 + threadIdx.x;
  const int32_t v = i < n ? in[i] : 0;
  s[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const int32_t t = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
    __syncthreads();
    s[threadIdx.x] += t;
    __syncthreads();
  }
  if (i < n) out[i] = s[threadIdx.x] - v;
  if (threadIdx.x == 1023) tile_sum[blockIdx.x] = s[1023];
}
__global__ __launch_bounds__(1024) void scan_sums_kernel(int32_t* tile_sum, int ntiles, int32_t* total) {
  __shared__ int32_t carry;
  __shared__ int32_t s[1024];
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int base = 0; base < ntiles; base += 1024) {
    const int i = base + threadIdx.x;
    const int32_t v = i < ntiles ? tile_sum[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
      const int32_t t = threadIdx.x >= o ? s[threadIdx.x - o] : 0;
      __syncthreads();
      s[threadIdx.x] += t;
      __syncthreads();
    }
    if (i < ntiles) tile_sum[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) *total = carry;
}
__global__ void scan_add_kernel(int32_t* out, int64_t n, const int32_t* tile_sum) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] += tile_sum[i >> 10];
}

__global__ void rev_scatter_kernel(GraphBuildArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.n * a.k) return;
  const int j = a.idx[e];
  if (j < 0) return;
  const int pos = a.rev_ptr[j] + atomicAdd(&a.tmp_cnt[j], 1);
  a.rev_src[pos] = (int32_t)(e / a.k);
  a.rev_w[pos] = a.w[e];
}

// Sort each reverse row by source and compute the degree: one wave per row.
// The sources of a row are distinct (each forward list names an item once),
// so an entry's slot is the number of entries with a smaller source (ties,
// which well-formed lists never have, go by position); rows
// of up to RS_MAX entries are staged in LDS, ranked, written to their
// sorted slots and summed in sorted order (lane-strided partial sums, then a
// fixed butterfly), so the degree does not depend on the order in which the
// scatter's atomics filled the row.  Longer rows (rare hubs) are sorted by
// one lane.
namespace {
constexpr int RS_MAX = 512;
__device__ __forceinline__ void wave_lds_sync_g() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
  __builtin_amdgcn_wave_barrier();
}
}  // namespace

__global__ __launch_bounds__(256) void rev_sort_degree_kernel(GraphBuildArgs a) {
  __shared__ int32_t ssrc[4][RS_MAX];
  __shared__ float sw[4][RS_MAX], sorted_w[4][RS_MAX];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int64_t i = (int64_t)blockIdx.x * 4 + wave;
  if (i >= a.n) return;
  const int b = a.rev_ptr[i], e = a.rev_ptr[i + 1], m = e - b;
  float rs = 0.f;
  if (m <= RS_MAX) {
    for (int p = lane; p < m; p += 64) {
      ssrc[wave][p] = a.rev_src[b + p];
      sw[wave][p] = a.rev_w[b + p];
    }
    wave_lds_sync_g();
    for (int p = lane; p < m; p += 64) {
      const int32_t s = ssrc[wave][p];
      int r = 0;
      for (int q = 0; q < m; ++q) r += ssrc[wave][q] < s || (ssrc[wave][q] == s && q < p);
      a.rev_src[b + r] = s;
      a.rev_w[b + r] = sw[wave][p];
      sorted_w[wave][r] = sw[wave][p];
    }
    wave_lds_sync_g();
    for (int p = lane; p < m; p += 64) rs += sorted_w[wave][p];
  } else {
    if (lane == 0) {
      for (int p = b + 1; p < e; ++p) {
        const int32_t s = a.rev_src[p];
        const float wv = a.rev_w[p];
        int q = p - 1;
        while (q >= b && a.rev_src[q] > s) {
          a.rev_src[q + 1] = a.rev_src[q];
          a.rev_w[q + 1] = a.rev_w[q];
          --q;
        }
        a.rev_src[q + 1] = s;
        a.rev_w[q + 1] = wv;
      }
      for (int p = b; p < e; ++p) rs += a.rev_w[p];  // lane 0 alone; the others add zeros
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) rs += __shfl_xor(rs, o, 64);
  if (lane == 0) {
    float fs = 0.f;  // forward weights of the row, in list order
    for (int s = 0; s < a.k; ++s) fs += a.w[i * a.k + s];
    if (a.asym) {
      a.deg[i] = 1.0f + fs;  // row degree D_r
      a.deg_c[i] = 1.0f + rs;  // column degree D_c
    } else {
      a.deg[i] = 1.0f + 0.5f * fs + 0.5f * rs;
    }
  }
}

// Normalised values of one row per wave: forward entries, then (symmetric
// graphs) reverse entries.
__global__ __launch_bounds__(256) void values_kernel(GraphBuildArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= a.n) return;
  const float di = a.deg[i];
  if (a.asym) {
    for (int s = lane; s < a.k; s += 64) {
      const int64_t e = i * a.k + s;
      const int j = a.idx[e];
      a.pf[e] = j >= 0 ? a.coef * a.w[e] / sqrtf(di * a.deg_c[j]) : 0.f;
    }
    return;  // no reverse terms
  }
  for (int s = lane; s < a.k; s += 64) {
    const int64_t e = i * a.k + s;
    const int j = a.idx[e];
    a.pf[e] = j >= 0 ? a.coef * 0.5f * a.w[e] / sqrtf(di * a.deg[j]) : 0.f;
  }
  const int b = a.rev_ptr[i], en = a.rev_ptr[i + 1];
  for (int p = b + lane; p < en; p += 64) a.pr[p] = a.coef * 0.5f * a.rev_w[p] / sqrtf(di * a.deg[a.rev_src[p]]);
}

// deg_c / cr_deg_c: column degrees of asymmetric graphs (nullptr: symmetric)
__global__ void self_kernel(int64_t n, const float* deg, const float* deg_c, const float* cr_deg,
                            const float* cr_deg_c, float alpha, float* self) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  float s = deg_c ? alpha / sqrtf(deg[i] * deg_c[i]) : alpha / deg[i];
  if (cr_deg) s += cr_deg_c ? (1.0f - alpha) / sqrtf(cr_deg[i] * cr_deg_c[i]) : (1.0f - alpha) / cr_deg[i];
  self[i] = s;
}

static inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_graph_build(const GraphBuildArgs& a, hipStream_t st) {
  const int64_t n = a.n;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, a.tmp_cnt, n);
  if (n * a.k > 0) hipLaunchKernelGGL(edge_weight_kernel, dim3(nblk(n * a.k, 256)), dim3(256), 0, st, a);
  const int ntiles = (int)((n + 1023) / 1024);
  hipLaunchKernelGGL(scan_tiles_kernel, dim3(ntiles), dim3(1024), 0, st, a.tmp_cnt, a.rev_ptr, n, a.tmp_blk);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, st, a.tmp_blk, ntiles, a.rev_ptr + n);
  hipLaunchKernelGGL(scan_add_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, a.rev_ptr, n, a.tmp_blk);
  hipLaunchKernelGGL(zero_i32_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, a.tmp_cnt, n);
  if (n * a.k > 0)
    hipLaunchKernelGGL(rev_scatter_kernel, dim3(nblk(n * a.k, 256)), dim3(256), 0, st, a);
  hipLaunchKernelGGL(rev_sort_degree_kernel, dim3(nblk(n, 4)), dim3(256), 0, st, a);
}

void launch_finish_values(const GraphBuildArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(values_kernel, dim3(nblk(a.n, 4)), dim3(256), 0, st, a);
}

void launch_self_coef(int64_t n, const float* deg, const float* deg_c, const float* cr_deg, const float* cr_deg_c,
                      float alpha, float* self, hipStream_t st) {
  hipLaunchKernelGGL(self_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, n, deg, deg_c, cr_deg, cr_deg_c, alpha,
                     self);
}

__global__ void label_count_kernel(int64_t n, const int32_t* __restrict__ idx, int k, int32_t* __restrict__ label,
                                   int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  int32_t m = (int32_t)i;
  for (int t = 0; t < k; ++t) {
    const int32_t j = idx[i * k + t];
    if (j >= 0 && j < m) m = j;
  }
  label[i] = m;
  atomicAdd(&cnt[m], 1);
}

__global__ void order_scatter_kernel(int64_t n, const int32_t* __restrict__ label, int32_t* __restrict__ off,
                                     int32_t* __restrict__ order) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  order[atomicAdd(&off[label[i]], 1)] = (int32_t)i;
}

// Label of a row from its screening candidates (list 0, every split).
__global__ void cand_label_count_kernel(int64_t n, const uint64_t* __restrict__ cand, const int32_t* __restrict__ ccnt,
                                        int S, int C, int NL, int32_t* __restrict__ label,
                                        int32_t* __restrict__ cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint32_t m = (uint32_t)i;
  for (int s = 0; s < S; ++s) {
    const int64_t o = (i * NL) * (int64_t)S + s;
    const uint64_t* b = cand + o * C;
    const int c = ccnt[o];
    for (int t = 0; t < c; ++t) {
      const uint32_t j = cand_col(b[t]);
      m = j < m ? j : m;
    }
  }
  label[i] = (int32_t)m;
  atomicAdd(&cnt[m], 1);
}

static void order_from_labels(int64_t n, const int32_t* label, int32_t* cnt, int32_t* blk, int32_t* order,
                              hipStream_t st);

void launch_cand_order(int64_t n, const uint64_t* cand, const int32_t* ccnt, int S, int C, int NL, int32_t* label,
                       int32_t* cnt, int32_t* blk, int32_t* order, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, cnt, n);
  hipLaunchKernelGGL(cand_label_count_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, n, cand, ccnt, S, C, NL, label,
                     cnt);
  order_from_labels(n, label, cnt, blk, order, st);
}

void launch_locality_order(int64_t n, const int32_t* idx, int k, int32_t* label, int32_t* cnt, int32_t* blk,
                           int32_t* order, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(zero_i32_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, cnt, n);
  hipLaunchKernelGGL(label_count_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, n, idx, k, label, cnt);
  order_from_labels(n, label, cnt, blk, order, st);
}

// counts in cnt[label] -> exclusive offsets (in place) -> scatter
static void order_from_labels(int64_t n, const int32_t* label, int32_t* cnt, int32_t* blk, int32_t* order,
                              hipStream_t st) {
  const int ntiles = (int)((n + 1023) / 1024);
  // exclusive offsets, scanned in place
  hipLaunchKernelGGL(scan_tiles_kernel, dim3(ntiles), dim3(1024), 0, st, cnt, cnt, n, blk);
  hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, st, blk, ntiles, cnt + n);
  hipLaunchKernelGGL(scan_add_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, cnt, n, blk);
  hipLaunchKernelGGL(order_scatter_kernel, dim3(nblk(n, 256)), dim3(256), 0, st, n, label, cnt, order);
}

}  // namespace gcr
