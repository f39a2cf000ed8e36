// One synchronous propagation round (Eq. (2), blended as in Eq. (9)):
//   y_i = self_i x_i + sum_{j in fwd(i)} pf_ij x_j + sum_{j in rev(i)} pr_ij x_j
//         (+ the same two sums over the cross-camera graph)
//   x'_i = y_i / max(||y_i||, 1e-12)
// One wave per row.  The row's edge list is loaded lane-parallel (one edge
// per lane) and broadcast with lane shuffles; each lane owns a fixed slice
// of the feature vector, so every neighbour row is read as whole 1 KB
// (f32x4 x 64 lanes) segments.  Edges are summed in a fixed order (self,
// forward list order, reverse rows sorted by source), so results are
// bitwise reproducible.
#include "kernels.h"

namespace gcr {

template <int V>
struct Acc {
  f32x4 v[V];
};

template <int V>
__device__ __forceinline__ void axpy_row(Acc<V>& acc, float p, const float* __restrict__ xj, int lane) {
  const f32x4* x4 = (const f32x4*)xj;
#pragma unroll
  for (int q = 0; q < V; ++q) {
    const f32x4 t = x4[q * 64 + lane];
    acc.v[q].x = fmaf(p, t.x, acc.v[q].x);
    acc.v[q].y = fmaf(p, t.y, acc.v[q].y);
    acc.v[q].z = fmaf(p, t.z, acc.v[q].z);
    acc.v[q].w = fmaf(p, t.w, acc.v[q].w);
  }
}

// Sum over an edge segment: indices/values loaded 64 at a time, then the
// neighbour rows in groups of G whose loads are all issued before the first
// of their multiply-adds, so that G rows (G * V 16-byte loads per lane) are
// in flight per wave: the gather is bound by latency, not bandwidth.  The
// multiply-adds still run in list order (bitwise reproducible).  `safe` is
// a valid row index that stands in for padding entries (-1) in the loads;
// their multiply-adds are skipped.
template <int V, int G>
__device__ __forceinline__ void gather_list(Acc<V>& acc, const float* __restrict__ X, int d,
                                            const int32_t* __restrict__ ids,
                                            const float* __restrict__ vals, int cnt, int lane, int64_t safe) {
  for (int base = 0; base < cnt; base += 64) {
    const int m = min(64, cnt - base);
    int jl = -1;
    float pl = 0.f;
    if (lane < m) { jl = ids[base + lane]; pl = vals[base + lane]; }
    int t = 0;
    for (; t + G <= m; t += G) {
      int jj[G];
      float pp[G];
      f32x4 buf[G][V];
#pragma unroll
      for (int g = 0; g < G; ++g) {
        jj[g] = __shfl(jl, t + g, 64);
        pp[g] = __shfl(pl, t + g, 64);
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const f32x4* x4 = (const f32x4*)(X + (jj[g] >= 0 ? (int64_t)jj[g] : safe) * d);
#pragma unroll
        for (int q = 0; q < V; ++q) buf[g][q] = x4[q * 64 + lane];
      }
#pragma unroll
      for (int g = 0; g < G; ++g) {
        if (jj[g] < 0) continue;
#pragma unroll
        for (int q = 0; q < V; ++q) {
          acc.v[q].x = fmaf(pp[g], buf[g][q].x, acc.v[q].x);
          acc.v[q].y = fmaf(pp[g], buf[g][q].y, acc.v[q].y);
          acc.v[q].z = fmaf(pp[g], buf[g][q].z, acc.v[q].z);
          acc.v[q].w = fmaf(pp[g], buf[g][q].w, acc.v[q].w);
        }
      }
    }
    for (; t < m; ++t) {
      const int j0 = __shfl(jl, t, 64);
      const float p0 = __shfl(pl, t, 64);
      if (j0 >= 0) axpy_row<V>(acc, p0, X + (int64_t)j0 * d, lane);
    }
  }
}

template <int V>
__global__ __launch_bounds__(256) void propagate_vec_kernel(PropArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t pos = xcd_position(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (pos >= a.n) return;
  const int64_t i = a.order ? (int64_t)a.order[pos] : pos;
  const int d = a.d;
  Acc<V> acc;
  {
    const float s = a.self[i];
    const f32x4* x4 = (const f32x4*)(a.X + i * d);
#pragma unroll
    for (int q = 0; q < V; ++q) {
      const f32x4 t = x4[q * 64 + lane];
      acc.v[q] = t * s;
    }
  }
  constexpr int G = V >= 8 ? 2 : 16 / V;  // rows in flight: G * V <= 16 loads per lane
  gather_list<V, G>(acc, a.X, d, a.idx + i * a.k, a.pf + i * a.k, a.k, lane, i);
  if (a.rev_ptr) {
    const int b = a.rev_ptr[i], e = a.rev_ptr[i + 1];
    gather_list<V, G>(acc, a.X, d, a.rev_src + b, a.pr + b, e - b, lane, i);
  }
  if (a.cr_idx) {
    gather_list<V, G>(acc, a.X, d, a.cr_idx + i * a.ck, a.cr_pf + i * a.ck, a.ck, lane, i);
    if (a.cr_rev_ptr) {
      const int b = a.cr_rev_ptr[i], e = a.cr_rev_ptr[i + 1];
      gather_list<V, G>(acc, a.X, d, a.cr_rev_src + b, a.cr_pr + b, e - b, lane, i);
    }
  }
  float ss = 0.f;
#pragma unroll
  for (int q = 0; q < V; ++q)
    ss += acc.v[q].x * acc.v[q].x + acc.v[q].y * acc.v[q].y + acc.v[q].z * acc.v[q].z + acc.v[q].w * acc.v[q].w;
  ss = wave_sum(ss);
  const float inv = 1.0f / fmaxf(sqrtf(ss), 1e-12f);
  f32x4* y4 = (f32x4*)(a.Y + i * d);
#pragma unroll
  for (int q = 0; q < V; ++q)
    y4[q * 64 + lane] = acc.v[q] * inv;
}

// Generic width: lane owns elements lane + 64 t, t < 32 (d <= 2048).
__device__ __forceinline__ void axpy_scalar(float (&acc)[32], float p, const float* __restrict__ xj,
                                            int d, int lane) {
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    const int e = lane + 64 * t;
    if (e < d) acc[t] = fmaf(p, xj[e], acc[t]);
  }
}
__device__ void gather_scalar(float (&acc)[32], const float* __restrict__ X, int d,
                              const int32_t* ids, const float* vals, int cnt, int lane) {
  for (int base = 0; base < cnt; base += 64) {
    const int m = min(64, cnt - base);
    int jl = -1;
    float pl = 0.f;
    if (lane < m) { jl = ids[base + lane]; pl = vals[base + lane]; }
    for (int t = 0; t < m; ++t) {
      const int j = __shfl(jl, t, 64);
      const float p = __shfl(pl, t, 64);
      if (j >= 0) axpy_scalar(acc, p, X + (int64_t)j * d, d, lane);
    }
  }
}
__global__ __launch_bounds__(256) void propagate_scalar_kernel(PropArgs a) {
  const int lane = threadIdx.x & 63;
  const int64_t pos = xcd_position(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (pos >= a.n) return;
  const int64_t i = a.order ? (int64_t)a.order[pos] : pos;
  const int d = a.d;
  float acc[32];
  const float s = a.self[i];
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    const int e = lane + 64 * t;
    acc[t] = e < d ? s * a.X[i * d + e] : 0.f;
  }
  gather_scalar(acc, a.X, d, a.idx + i * a.k, a.pf + i * a.k, a.k, lane);
  if (a.rev_ptr) {
    const int b = a.rev_ptr[i], e = a.rev_ptr[i + 1];
    gather_scalar(acc, a.X, d, a.rev_src + b, a.pr + b, e - b, lane);
  }
  if (a.cr_idx) {
    gather_scalar(acc, a.X, d, a.cr_idx + i * a.ck, a.cr_pf + i * a.ck, a.ck, lane);
    if (a.cr_rev_ptr) {
      const int b = a.cr_rev_ptr[i], e = a.cr_rev_ptr[i + 1];
      gather_scalar(acc, a.X, d, a.cr_rev_src + b, a.cr_pr + b, e - b, lane);
    }
  }
  float ss = 0.f;
#pragma unroll
  for (int t = 0; t < 32; ++t) ss += acc[t] * acc[t];
  ss = wave_sum(ss);
  const float inv = 1.0f / fmaxf(sqrtf(ss), 1e-12f);
#pragma unroll
  for (int t = 0; t < 32; ++t) {
    const int e = lane + 64 * t;
    if (e < d) a.Y[i * d + e] = acc[t] * inv;
  }
}

void launch_propagate(const PropArgs& a, hipStream_t st) {
  if (a.n <= 0) return;
  const dim3 g((unsigned)((a.n + 3) / 4)), b(256);
  const bool aligned = ((((uintptr_t)a.X) | ((uintptr_t)a.Y)) & 15) == 0;
  if (aligned && a.d % 256 == 0 && a.d <= 2048) {
    switch (a.d / 256) {
      case 1: hipLaunchKernelGGL(propagate_vec_kernel<1>, g, b, 0, st, a); return;
      case 2: hipLaunchKernelGGL(propagate_vec_kernel<2>, g, b, 0, st, a); return;
      case 3: hipLaunchKernelGGL(propagate_vec_kernel<3>, g, b, 0, st, a); return;
      case 4: hipLaunchKernelGGL(propagate_vec_kernel<4>, g, b, 0, st, a); return;
      case 5: hipLaunchKernelGGL(propagate_vec_kernel<5>, g, b, 0, st, a); return;
      case 6: hipLaunchKernelGGL(propagate_vec_kernel<6>, g, b, 0, st, a); return;
      case 7: hipLaunchKernelGGL(propagate_vec_kernel<7>, g, b, 0, st, a); return;
      case 8: hipLaunchKernelGGL(propagate_vec_kernel<8>, g, b, 0, st, a); return;
    }
  }
  hipLaunchKernelGGL(propagate_scalar_kernel, g, b, 0, st, a);
}

}  // namespace gcr
