// Shared device helpers for the GCR kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GCR_WAVE 64

typedef __attribute__((ext_vector_type(16))) float f32x16;
typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(8))) int i32x8;
typedef __attribute__((ext_vector_type(4))) unsigned u32x4;
typedef __attribute__((ext_vector_type(4))) float f32x4;
typedef __attribute__((ext_vector_type(4))) int i32x4;

// ---------------------------------------------------------------------------
// Order-preserving map float -> uint32 (total order for non-NaN values).
__device__ __forceinline__ uint32_t ord_f32(float f) {
  uint32_t b = __float_as_uint(f);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float unord_f32(uint32_t o) {
  uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  return __uint_as_float(b);
}
// Candidate entry: (screened key, column) packed so that unsigned order is
// (key, column) lexicographic.
__device__ __forceinline__ uint64_t pack_cand(float key, uint32_t col) {
  return ((uint64_t)ord_f32(key) << 32) | (uint64_t)col;
}
__device__ __forceinline__ float cand_key(uint64_t e) { return unord_f32((uint32_t)(e >> 32)); }
__device__ __forceinline__ uint32_t cand_col(uint64_t e) { return (uint32_t)e; }
#define GCR_EMPTY (~0ull)

// bfloat16 with round-to-nearest-even (finite inputs) and back.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// ---------------------------------------------------------------------------
// Exact re-scoring arithmetic.  The difference of two float32 values is
// formed in float64 (exact unless their exponents differ by more than 29,
// else rounded once with relative error <= 2^-53), its square is taken
// exactly inside the float64 FMA, and the sum of d non-negative terms then
// carries a relative error below (d + 8) 2^-53 (about 2^-42 at d = 2048),
// far below the float32 rounding of the reported distance.
__device__ __forceinline__ double sqdiff_acc(double acc, float a, float b) {
  const double t = (double)a - (double)b;
  return fma(t, t, acc);
}
// Order-preserving map double -> uint64 (total order for non-NaN values).
__device__ __forceinline__ uint64_t ord_f64(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b & 0x8000000000000000ull) ? ~b : (b | 0x8000000000000000ull);
}
__device__ __forceinline__ double unord_f64(uint64_t o) {
  const uint64_t b = (o & 0x8000000000000000ull) ? (o & 0x7fffffffffffffffull) : ~o;
  return __longlong_as_double((long long)b);
}

// ---------------------------------------------------------------------------
// wave reductions
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ double wave_sum_f64(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = __shfl_xor(lo, m, 64);
  hi = __shfl_xor(hi, m, 64);
  return ((uint64_t)hi << 32) | lo;
}
__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src) {
  uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
  lo = __shfl(lo, src, 64);
  hi = __shfl(hi, src, 64);
  return ((uint64_t)hi << 32) | lo;
}

// Bitonic sort (ascending) of E*64 uint64 values held by one wave; element
// e = j * 64 + lane lives in v[j].
template <int E>
__device__ __forceinline__ void wave_bitonic_sort(uint64_t (&v)[E]) {
  const int lane = threadIdx.x & 63;
  constexpr int N = E * 64;
#pragma unroll
  for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
    for (int stride = size >> 1; stride > 0; stride >>= 1) {
      if (stride >= 64) {
        const int rs = stride >> 6;
#pragma unroll
        for (int j = 0; j < E; ++j) {
          if ((j & rs) == 0) {
            const int e = j * 64 + lane;
            const bool asc = (e & size) == 0;
            uint64_t a = v[j], b = v[j | rs];
            bool sw = asc ? (a > b) : (a < b);
            v[j] = sw ? b : a;
            v[j | rs] = sw ? a : b;
          }
        }
      } else {
#pragma unroll
        for (int j = 0; j < E; ++j) {
          const int e = j * 64 + lane;
          const bool asc = (e & size) == 0;
          const bool lower = (lane & stride) == 0;
          uint64_t o = shfl_xor_u64(v[j], stride);
          uint64_t mn = v[j] < o ? v[j] : o;
          uint64_t mx = v[j] < o ? o : v[j];
          v[j] = (lower == asc) ? mn : mx;
        }
      }
    }
  }
}

// Position of workgroup b among nb workgroups such that each XCD (the
// dispatcher deals workgroups to the 8 XCDs in turn) walks one contiguous
// segment of positions: neighbouring positions then share an L2.
__device__ __forceinline__ int64_t xcd_position(int64_t b, int64_t nb) {
  const int64_t q = nb >> 3, r = nb & 7, x = b & 7, i = b >> 3;
  return x * q + (x < r ? x : r) + i;
}

// Bound on |screened key - exact key| for a row, where key_c = ||x_c||^2 -
// 2 x_r.x_c.  The screening multiplies x~ = x - res (res: the quantisation
// residual, known per row): x~_r.x~_c - x_r.x_c = -res_r.x~_c - x_r.res_c,
// bounded by Cauchy-Schwarz with the row's residual norm rn_r, the largest
// residual norm maxrn and the largest norm; the float32 accumulation adds at
// most eps_acc ||x~_r|| ||x~_c||, the float32 squared norm n2_c at most
// eps_n maxn2, and the key's own rounding a few units of 2^-24.  With
// rn_r = maxrn = 0 this is the bound of a plain float32 product.
__device__ __forceinline__ float screen_margin(float n2r, float rnr, float maxn2, float maxrn, float eps_acc,
                                               float eps_n) {
  const float nr = sqrtf(n2r * (1.0f + eps_n)), nm = sqrtf(maxn2 * (1.0f + eps_n));
  const float tr = nr + rnr, tm = nm + maxrn;  // bounds on ||x~_r||, ||x~_c||
  const float es = rnr * tm + nr * maxrn + eps_acc * tr * tm;
  const float er = 6.0e-8f * (maxn2 + 2.0f * tr * tm);
  return (2.0f * es + eps_n * maxn2 + er) * 1.00001f;
}
