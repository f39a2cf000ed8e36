// Input preparation: row normalisation, squared norms and the padded
// low-precision copies that the similarity screening reads.
#include <algorithm>

#include "kernels.h"

namespace gcr {

// One wave per row: Y[i] = X[i] / max(||X[i]||, 1e-12).
__global__ __launch_bounds__(256) void normalize_rows_kernel(const float* __restrict__ X,
                                                             float* Y, int64_t n, int d) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const float* x = X + row * d;
  float s = 0.f;
  for (int e = lane; e < d; e += 64) s = fmaf(x[e], x[e], s);
  s = wave_sum(s);
  const float inv = 1.0f / fmaxf(sqrtf(s), 1e-12f);
  float* y = Y + row * d;
  for (int e = lane; e < d; e += 64) y[e] = x[e] * inv;
}

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// value of an E4M3 code written by f32_to_e4m3_rne
__device__ __forceinline__ float e4m3_to_f32(uint8_t c) {
  const int E = (c >> 3) & 15, m = c & 7;
  const float a = E == 0 ? (float)m * (1.0f / 512.0f) : ldexpf((float)(8 + m), E - 10);
  return (c & 0x80) ? -a : a;
}

// OCP E4M3 (bias 7, max 448, no infinities), round to nearest even,
// saturating at +-448.
__device__ __forceinline__ uint8_t f32_to_e4m3_rne(float x) {
  uint32_t sign = (__float_as_uint(x) >> 31) << 7;
  float a = fminf(fabsf(x), 448.0f);
  if (a < 0.015625f) {  // below 2^-6: subnormal grid 2^-9
    return (uint8_t)(sign | (uint32_t)rintf(a * 512.0f));
  }
  int e;
  frexpf(a, &e);  // a = f 2^e, f in [0.5, 1)
  int E = e - 1;
  float q = rintf(ldexpf(a, 3 - E));  // in [8, 16]
  if (q >= 16.0f) { E += 1; q = 8.0f; }
  return (uint8_t)(sign | ((uint32_t)(E + 7) << 3) | ((uint32_t)q - 8u));
}

// One wave per row: the screening operand row (ld_bytes, zero past d),
// n2 = ||x||^2 (float32), the FP8 scale, an upper bound rn on the norm of
// the quantisation residual x - x~, and the maxima of n2 and rn into
// maxbits[0] and [1] (atomic max on the bit patterns, valid for
// non-negative floats).
template <int PREC>
__device__ void prep_row(const float* __restrict__ x, int d, uint8_t* out, int64_t ld_bytes, float* n2o,
                         float* scaleo, float* rno, unsigned* maxbits, int lane) {
  float s = 0.f, amax = 0.f;
  for (int e = lane; e < d; e += 64) {
    float v = x[e];
    s = fmaf(v, v, s);
    amax = fmaxf(amax, fabsf(v));
  }
  s = wave_sum(s);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
  if (lane == 0) {
    *n2o = s;
    atomicMax(maxbits, __float_as_uint(s));
  }
  float r2 = 0.f;  // squared residual norm
  if (PREC == GCR_PREC_FP32) {
    float* o = (float*)out;
    const int64_t cnt = ld_bytes / 4;
    for (int64_t e = lane; e < cnt; e += 64) o[e] = e < d ? x[e] : 0.f;
  } else if (PREC == GCR_PREC_BF16) {
    uint16_t* o = (uint16_t*)out;
    const int64_t cnt = ld_bytes / 2;
    for (int64_t e = lane; e < cnt; e += 64) {
      uint16_t h = 0;
      if (e < d) {
        h = f32_to_bf16_rne(x[e]);
        const float r = x[e] - bf16_to_f32(h);  // exact
        r2 = fmaf(r, r, r2);
      }
      o[e] = h;
    }
  } else {
    const float sc = amax > 0.f ? amax / 448.0f : 1.0f;
    if (lane == 0) *scaleo = sc;
    for (int64_t e = lane; e < ld_bytes; e += 64) {
      uint8_t c = 0;
      if (e < d) {
        c = f32_to_e4m3_rne(x[e] / sc);
        const float r = x[e] - e4m3_to_f32(c) * sc;
        r2 = fmaf(r, r, r2);
      }
      out[e] = c;
    }
  }
  if (PREC != GCR_PREC_FP32) {
    r2 = wave_sum(r2);
    // float32 sum of d squares: relative error below (d + 2) 2^-23; each
    // residual itself is off by at most 2^-24 |x_e| (FP8 dequantisation)
    const float rb = sqrtf(r2 * (1.0f + (float)(d + 2) * 1.2e-7f)) * 1.000001f + 1.0e-7f * sqrtf(s);
    if (lane == 0) {
      *rno = rb;
      atomicMax(maxbits + 1, __float_as_uint(rb));
    }
  } else if (lane == 0) {
    *rno = 0.f;
  }
}

// Rows [0, npad): rows past n are zero (operand, n2, rn, scale).
template <int PREC>
__global__ __launch_bounds__(256) void screen_prep_kernel(const float* __restrict__ X, int64_t n,
                                                          int d, int64_t npad, uint8_t* Xs,
                                                          int64_t ld_bytes, float* n2,
                                                          float* scale, float* rn, unsigned* maxn2_bits) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= npad) return;
  uint8_t* out = Xs + row * ld_bytes;
  if (row >= n) {
    for (int64_t b = lane * 4; b < ld_bytes; b += 256) *(uint32_t*)(out + b) = 0u;
    if (lane == 0) { n2[row] = 0.f; rn[row] = 0.f; if (scale) scale[row] = 0.f; }
    return;
  }
  prep_row<PREC>(X + row * d, d, out, ld_bytes, n2 + row, scale ? scale + row : nullptr, rn + row, maxn2_bits,
                 lane);
}

// Rows [r0, r0 + nmax), or only the first *count of them when count is
// given (a row count known on the device); grid-stride over rows.
template <int PREC>
__global__ __launch_bounds__(256) void screen_prep_rows_kernel(const float* __restrict__ X, int64_t r0, int64_t nmax,
                                                               const int* count, int d, uint8_t* Xs,
                                                               int64_t ld_bytes, float* n2, float* scale, float* rn,
                                                               unsigned* maxn2_bits) {
  const int lane = threadIdx.x & 63;
  const int64_t nr = count ? min<int64_t>(nmax, (int64_t)*count) : nmax;
  for (int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); t < nr; t += (int64_t)gridDim.x * 4) {
    const int64_t row = r0 + t;
    prep_row<PREC>(X + row * d, d, Xs + row * ld_bytes, ld_bytes, n2 + row, scale ? scale + row : nullptr,
                   rn + row, maxn2_bits, lane);
  }
}

void launch_normalize_rows(const float* X, float* Y, int64_t n, int d, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(normalize_rows_kernel, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, X, Y, n, d);
}

void launch_screen_prep_rows(int prec, const float* X, int64_t r0, int64_t nmax, const int* count, int d, void* Xs,
                             int64_t ld_bytes, float* n2, float* scale, float* rn, unsigned* maxn2_bits,
                             hipStream_t st) {
  if (nmax <= 0) return;
  const dim3 g((unsigned)std::min<int64_t>((nmax + 3) / 4, 4096)), b(256);
  uint8_t* xs = (uint8_t*)Xs;
  if (prec == GCR_PREC_FP32)
    hipLaunchKernelGGL(screen_prep_rows_kernel<GCR_PREC_FP32>, g, b, 0, st, X, r0, nmax, count, d, xs, ld_bytes, n2,
                       scale, rn, maxn2_bits);
  else if (prec == GCR_PREC_BF16)
    hipLaunchKernelGGL(screen_prep_rows_kernel<GCR_PREC_BF16>, g, b, 0, st, X, r0, nmax, count, d, xs, ld_bytes, n2,
                       scale, rn, maxn2_bits);
  else
    hipLaunchKernelGGL(screen_prep_rows_kernel<GCR_PREC_FP8>, g, b, 0, st, X, r0, nmax, count, d, xs, ld_bytes, n2,
                       scale, rn, maxn2_bits);
}

void launch_screen_prep(int prec, const float* X, int64_t n, int d, int64_t npad, void* Xs,
                        int64_t ld_bytes, float* n2, float* scale, float* rn, unsigned* maxn2_bits,
                        hipStream_t st) {
  dim3 g((unsigned)((npad + 3) / 4)), b(256);
  uint8_t* xs = (uint8_t*)Xs;
  if (prec == GCR_PREC_FP32)
    hipLaunchKernelGGL(screen_prep_kernel<GCR_PREC_FP32>, g, b, 0, st, X, n, d, npad, xs, ld_bytes, n2, scale, rn, maxn2_bits);
  else if (prec == GCR_PREC_BF16)
    hipLaunchKernelGGL(screen_prep_kernel<GCR_PREC_BF16>, g, b, 0, st, X, n, d, npad, xs, ld_bytes, n2, scale, rn, maxn2_bits);
  else
    hipLaunchKernelGGL(screen_prep_kernel<GCR_PREC_FP8>, g, b, 0, st, X, n, d, npad, xs, ld_bytes, n2, scale, rn, maxn2_bits);
}

}  // namespace gcr
