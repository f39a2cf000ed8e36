// Maintenance of a resident gallery's kNN lists under inserts and removals.
//
// The lists stay the lists a fresh build on the current gallery would
// produce: k nearest other items by exact squared distance, ordered by
// (distance, index).
//   Insert (rows appended at the end): an old row's new list is the merge of
//     its list with its nearest items among the appended rows.  Entries carry
//     float32 distances; where an old and an appended entry round to the same
//     float32 value their float64 distances decide, recomputed from the
//     features, and only exactly equal float64 values fall back to the index
//     (every appended index is larger than every old one).  A fresh build
//     orders by float64 distances summed in another order, so the two can
//     differ only for items whose distances agree to the rounding of that
//     sum (about 2^-42 relative at d = 2048).
//   Removal (gallery compacted in place, surviving items keep their relative
//     order): relabelling is monotone, so every list keeps its order; a list
//     that contained a removed item is searched again.
#include "kernels.h"

namespace gcr {

namespace {

// Exact squared distance between gallery rows r and j (float64 sum).
__device__ double exact_d2(const float* __restrict__ X, int d, int64_t r, int64_t j) {
  double s = 0.0;
  for (int e = 0; e < d; ++e) s = sqdiff_acc(s, X[r * d + e], X[j * d + e]);
  return s;
}

// Row r's (distance, index) order between an old entry a and an appended
// entry b, with float32 ties decided in float64.
__device__ __forceinline__ bool before(const float* __restrict__ X, int d, int64_t r, float da, int32_t ia,
                                       float db, int32_t ib) {
  if (da != db) return da < db;
  const double ea = exact_d2(X, d, r, ia), eb = exact_d2(X, d, r, ib);
  if (ea != eb) return ea < eb;
  return ia < ib;
}

// Row r's list (k entries) merged with its m nearest appended items (column
// indices relative to the first appended row, col_offset added), the k
// smallest kept, in place.  A forward pass counts how many entries each side
// contributes; the merge then runs backwards, so a write at position p never
// overwrites an old entry that is still to be read (p >= the old read index).
__global__ void merge_appended_kernel(int64_t rows, int k, int32_t* __restrict__ idx, float* __restrict__ dist, int m,
                                      const int32_t* __restrict__ nidx, const float* __restrict__ ndist,
                                      int32_t col_offset, const float* __restrict__ X, int d) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  int32_t* li = idx + r * k;
  float* ld = dist + r * k;
  const int32_t* ni = nidx + r * m;
  const float* nd = ndist + r * m;
  int x = 0, y = 0;
  for (int t = 0; t < k; ++t) {
    const bool va = x < k && li[x] >= 0;
    const bool vb = y < m && ni[y] >= 0;
    if (va && vb) {
      if (before(X, d, r, ld[x], li[x], nd[y], ni[y] + col_offset)) ++x;
      else ++y;
    } else if (va) {
      ++x;
    } else if (vb) {
      ++y;
    } else {
      break;
    }
  }
  const int nv = x + y;
  int xi = x - 1, yi = y - 1;
  for (int p = nv - 1; p >= 0; --p) {
    bool take_old;
    if (xi >= 0 && yi >= 0) take_old = !before(X, d, r, ld[xi], li[xi], nd[yi], ni[yi] + col_offset);
    else take_old = xi >= 0;
    if (take_old) {
      li[p] = li[xi];
      ld[p] = ld[xi];
      --xi;
    } else {
      li[p] = ni[yi] + col_offset;
      ld[p] = nd[yi];
      --yi;
    }
  }
  for (int t = nv; t < k; ++t) {
    li[t] = -1;
    ld[t] = INFINITY;
  }
}

__global__ void relabel_lists_kernel(int64_t rows_old, int k, const int32_t* __restrict__ new_of_old,
                                     const int32_t* __restrict__ idx_old, const float* __restrict__ dist_old,
                                     int32_t* __restrict__ idx_new, float* __restrict__ dist_new,
                                     int32_t* __restrict__ repair, int* __restrict__ repair_count) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows_old) return;
  const int32_t nr = new_of_old[r];
  if (nr < 0) return;
  int kept = 0;
  bool lost = false;
  for (int t = 0; t < k; ++t) {
    const int32_t j = idx_old[r * k + t];
    if (j < 0) continue;
    const int32_t nj = new_of_old[j];
    if (nj < 0) {
      lost = true;
      continue;
    }
    idx_new[(int64_t)nr * k + kept] = nj;
    dist_new[(int64_t)nr * k + kept] = dist_old[r * k + t];
    ++kept;
  }
  for (int t = kept; t < k; ++t) {
    idx_new[(int64_t)nr * k + t] = -1;
    dist_new[(int64_t)nr * k + t] = INFINITY;
  }
  if (lost) repair[atomicAdd(repair_count, 1)] = nr;
}

__global__ void gather_rows_kernel(const float* __restrict__ src, float* __restrict__ dst,
                                   const int32_t* __restrict__ src_row, int64_t rows, int d) {
  const int64_t r = blockIdx.x;
  if (r >= rows) return;
  const float* s = src + (int64_t)src_row[r] * d;
  float* o = dst + r * d;
  for (int e = threadIdx.x; e < d; e += blockDim.x) o[e] = s[e];
}

__global__ void drop_self_kernel(int64_t rows, int k, const int32_t* __restrict__ self_row,
                                 const int32_t* __restrict__ idx_in, const float* __restrict__ dist_in,
                                 int32_t* __restrict__ idx_out, float* __restrict__ dist_out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= rows) return;
  const int32_t r = self_row[t];
  const int32_t* ii = idx_in + t * (k + 1);
  const float* di = dist_in + t * (k + 1);
  int skip = k;  // no self entry among the k + 1: the last one goes
  for (int e = 0; e <= k; ++e)
    if (ii[e] == r) {
      skip = e;
      break;
    }
  int o = 0;
  for (int e = 0; e <= k; ++e) {
    if (e == skip) continue;
    idx_out[(int64_t)r * k + o] = ii[e];
    dist_out[(int64_t)r * k + o] = di[e];
    ++o;
  }
}

inline unsigned nblk(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

}  // namespace

void launch_merge_appended(int64_t rows, int k, int32_t* idx, float* dist, int m, const int32_t* nidx,
                           const float* ndist, int32_t col_offset, const float* X, int d, hipStream_t st) {
  if (rows <= 0 || k <= 0) return;
  hipLaunchKernelGGL(merge_appended_kernel, dim3(nblk(rows, 64)), dim3(64), 0, st, rows, k, idx, dist, m, nidx, ndist,
                     col_offset, X, d);
}

void launch_relabel_lists(int64_t rows_old, int k, const int32_t* new_of_old, const int32_t* idx_old,
                          const float* dist_old, int32_t* idx_new, float* dist_new, int32_t* repair,
                          int* repair_count, hipStream_t st) {
  if (rows_old <= 0 || k <= 0) return;
  hipLaunchKernelGGL(relabel_lists_kernel, dim3(nblk(rows_old, 256)), dim3(256), 0, st, rows_old, k, new_of_old,
                     idx_old, dist_old, idx_new, dist_new, repair, repair_count);
}

void launch_gather_rows(const float* src, float* dst, const int32_t* src_row, int64_t rows, int d, hipStream_t st) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(gather_rows_kernel, dim3((unsigned)rows), dim3(256), 0, st, src, dst, src_row, rows, d);
}

void launch_drop_self(int64_t rows, int k, const int32_t* self_row, const int32_t* idx_in, const float* dist_in,
                      int32_t* idx_out, float* dist_out, hipStream_t st) {
  if (rows <= 0) return;
  hipLaunchKernelGGL(drop_self_kernel, dim3(nblk(rows, 64)), dim3(64), 0, st, rows, k, self_row, idx_in, dist_in,
                     idx_out, dist_out);
}

}  // namespace gcr
