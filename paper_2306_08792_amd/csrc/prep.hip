// Input preparation: row normalisation, squared norms and the padded
// low-precision copies that the similarity screening reads.
#include <algorithm>

#include "kernels.h"

namespace gcr {

// One wave per row: Y[i] = X[i] / max(||X[i]||, 1e-12); X and Y may be the
// same buffer (each lane writes only elements it has read).  VEC: d % 4 == 0
// and 16-byte aligned rows, read and written 16 bytes per lane.
template <bool VEC>
__global__ __launch_bounds__(256) void normalize_rows_kernel(const float* X,
                                                             float* Y, int64_t n, int d) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= n) return;
  const float* x = X + row * d;
  float* y = Y + row * d;
  float s = 0.f;
  if constexpr (VEC) {
    const f32x4* x4 = (const f32x4*)x;
    const int d4 = d >> 2;
    if (d4 <= 8 * 64) {
      // the row stays in registers between the norm and the scaling
      f32x4 r[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = q * 64 + lane;
        r[q] = e < d4 ? x4[e] : f32x4{0.f, 0.f, 0.f, 0.f};
        s = fmaf(r[q].x, r[q].x, s); s = fmaf(r[q].y, r[q].y, s);
        s = fmaf(r[q].z, r[q].z, s); s = fmaf(r[q].w, r[q].w, s);
      }
      s = wave_sum(s);
      const float inv = 1.0f / fmaxf(sqrtf(s), 1e-12f);
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int e = q * 64 + lane;
        if (e < d4) {
          f32x4 v = r[q];
          v.x *= inv; v.y *= inv; v.z *= inv; v.w *= inv;
          ((f32x4*)y)[e] = v;
        }
      }
      return;
    }
    for (int e = lane; e < d4; e += 64) {
      const f32x4 v = x4[e];
      s = fmaf(v.x, v.x, s); s = fmaf(v.y, v.y, s); s = fmaf(v.z, v.z, s); s = fmaf(v.w, v.w, s);
    }
    s = wave_sum(s);
    const float inv = 1.0f / fmaxf(sqrtf(s), 1e-12f);
    for (int e = lane; e < d4; e += 64) {
      f32x4 v = x4[e];
      v.x *= inv; v.y *= inv; v.z *= inv; v.w *= inv;
      ((f32x4*)y)[e] = v;
    }
  } else {
    for (int e = lane; e < d; e += 64) s = fmaf(x[e], x[e], s);
    s = wave_sum(s);
    const float inv = 1.0f / fmaxf(sqrtf(s), 1e-12f);
    for (int e = lane; e < d; e += 64) y[e] = x[e] * inv;
  }
}

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
// the quantisation residual x - x~; lane 0 folds n2 and rn into the running
// maxima maxbits[0] and [1] (bit patterns: their unsigned order is the
// order of non-negative floats).
template <int PREC>
__device__ __forceinline__ void prep_row(const float* __restrict__ x, int d, uint8_t* out, int64_t ld_bytes,
                                         float* n2o, float* scaleo, float* rno, unsigned (&maxbits)[2], int lane) {
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
    maxbits[0] = max(maxbits[0], __float_as_uint(s));
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
      maxbits[1] = max(maxbits[1], __float_as_uint(rb));
    }
  } else if (lane == 0) {
    *rno = 0.f;
  }
}

// prep_row for d % 4 == 0 and 16-byte aligned rows: 16-byte loads, the
// operand written 4 elements per store, the padding past d zeroed.  Float32
// and bfloat16 copies are written in the same pass that sums the squares;
// FP8 needs the row's amax for its scale first and reads the row twice.
template <int PREC>
__device__ __forceinline__ void prep_row_vec(const float* __restrict__ x, int d, uint8_t* out, int64_t ld_bytes,
                                             float* n2o, float* scaleo, float* rno, unsigned (&maxbits)[2],
                                             int lane) {
  const f32x4* x4 = (const f32x4*)x;
  const int d4 = d >> 2;
  float s = 0.f, amax = 0.f, r2 = 0.f;
  for (int e = lane; e < d4; e += 64) {
    const f32x4 v = x4[e];
    s = fmaf(v.x, v.x, s); s = fmaf(v.y, v.y, s); s = fmaf(v.z, v.z, s); s = fmaf(v.w, v.w, s);
    if constexpr (PREC == GCR_PREC_FP32) {
      ((f32x4*)out)[e] = v;
    } else if constexpr (PREC == GCR_PREC_BF16) {
      const uint16_t h0 = f32_to_bf16_rne(v.x), h1 = f32_to_bf16_rne(v.y);
      const uint16_t h2 = f32_to_bf16_rne(v.z), h3 = f32_to_bf16_rne(v.w);
      const float r0 = v.x - bf16_to_f32(h0), r1 = v.y - bf16_to_f32(h1);
      const float q2 = v.z - bf16_to_f32(h2), q3 = v.w - bf16_to_f32(h3);
      r2 = fmaf(r0, r0, r2); r2 = fmaf(r1, r1, r2); r2 = fmaf(q2, q2, r2); r2 = fmaf(q3, q3, r2);
      uint2 w;
      w.x = (uint32_t)h0 | ((uint32_t)h1 << 16);
      w.y = (uint32_t)h2 | ((uint32_t)h3 << 16);
      ((uint2*)out)[e] = w;
    } else {
      amax = fmaxf(amax, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)), fmaxf(fabsf(v.z), fabsf(v.w))));
    }
  }
  s = wave_sum(s);
  if (lane == 0) {
    *n2o = s;
    maxbits[0] = max(maxbits[0], __float_as_uint(s));
  }
  constexpr int ES = PREC == GCR_PREC_FP32 ? 4 : (PREC == GCR_PREC_BF16 ? 2 : 1);
  if constexpr (PREC == GCR_PREC_FP8) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) amax = fmaxf(amax, __shfl_xor(amax, o, 64));
    const float sc = amax > 0.f ? amax / 448.0f : 1.0f;
    if (lane == 0) *scaleo = sc;
    for (int e = lane; e < d4; e += 64) {
      const f32x4 v = x4[e];
      const uint8_t c0 = f32_to_e4m3_rne(v.x / sc), c1 = f32_to_e4m3_rne(v.y / sc);
      const uint8_t c2 = f32_to_e4m3_rne(v.z / sc), c3 = f32_to_e4m3_rne(v.w / sc);
      const float r0 = v.x - e4m3_to_f32(c0) * sc, r1 = v.y - e4m3_to_f32(c1) * sc;
      const float q2 = v.z - e4m3_to_f32(c2) * sc, q3 = v.w - e4m3_to_f32(c3) * sc;
      r2 = fmaf(r0, r0, r2); r2 = fmaf(r1, r1, r2); r2 = fmaf(q2, q2, r2); r2 = fmaf(q3, q3, r2);
      ((uint32_t*)out)[e] = (uint32_t)c0 | ((uint32_t)c1 << 8) | ((uint32_t)c2 << 16) | ((uint32_t)c3 << 24);
    }
  }
  // zero padding past d (whole 4-byte words: d * ES is a multiple of 4)
  for (int64_t b = (int64_t)d * ES + lane * 4; b < ld_bytes; b += 256) *(uint32_t*)(out + b) = 0u;
  if (PREC != GCR_PREC_FP32) {
    r2 = wave_sum(r2);
    const float rb = sqrtf(r2 * (1.0f + (float)(d + 2) * 1.2e-7f)) * 1.000001f + 1.0e-7f * sqrtf(s);
    if (lane == 0) {
      *rno = rb;
      maxbits[1] = max(maxbits[1], __float_as_uint(rb));
    }
  } else if (lane == 0) {
    *rno = 0.f;
  }
}

template <int PREC>
__device__ __forceinline__ void prep_row_any(const float* __restrict__ x, int d, uint8_t* out, int64_t ld_bytes,
                                             float* n2o, float* scaleo, float* rno, unsigned (&maxbits)[2],
                                             int lane) {
  if ((d & 3) == 0 && (((uintptr_t)x) & 15) == 0)
    prep_row_vec<PREC>(x, d, out, ld_bytes, n2o, scaleo, rno, maxbits, lane);
  else
    prep_row<PREC>(x, d, out, ld_bytes, n2o, scaleo, rno, maxbits, lane);
}

// Per-workgroup maxima of the waves' rows, merged with one atomic each.
__device__ __forceinline__ void block_max_merge(unsigned (&mine)[2], unsigned* maxn2_bits) {
  __shared__ unsigned sm[2][4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) { sm[0][wave] = mine[0]; sm[1][wave] = mine[1]; }
  __syncthreads();
  if (threadIdx.x < 2) {
    const unsigned m = max(max(sm[threadIdx.x][0], sm[threadIdx.x][1]), max(sm[threadIdx.x][2], sm[threadIdx.x][3]));
    if (m) atomicMax(maxn2_bits + threadIdx.x, m);
  }
}

// Rows [0, npad), one wave per row (grid-stride): rows past n are zero
// (operand, n2, rn, scale).
template <int PREC>
__global__ __launch_bounds__(256) void screen_prep_kernel(const float* __restrict__ X, int64_t n,
                                                          int d, int64_t npad, uint8_t* Xs,
                                                          int64_t ld_bytes, float* n2,
                                                          float* scale, float* rn, unsigned* maxn2_bits) {
  const int lane = threadIdx.x & 63;
  unsigned mine[2] = {0u, 0u};
  for (int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); row < npad; row += (int64_t)gridDim.x * 4) {
    uint8_t* out = Xs + row * ld_bytes;
    if (row >= n) {
      for (int64_t b = lane * 4; b < ld_bytes; b += 256) *(uint32_t*)(out + b) = 0u;
      if (lane == 0) { n2[row] = 0.f; rn[row] = 0.f; if (scale) scale[row] = 0.f; }
      continue;
    }
    prep_row_any<PREC>(X + row * d, d, out, ld_bytes, n2 + row, scale ? scale + row : nullptr, rn + row, mine,
                       lane);
  }
  block_max_merge(mine, maxn2_bits);
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
  unsigned mine[2] = {0u, 0u};
  for (int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); t < nr; t += (int64_t)gridDim.x * 4) {
    const int64_t row = r0 + t;
    prep_row_any<PREC>(X + row * d, d, Xs + row * ld_bytes, ld_bytes, n2 + row, scale ? scale + row : nullptr,
                       rn + row, mine, lane);
  }
  block_max_merge(mine, maxn2_bits);
}

void launch_normalize_rows(const float* X, float* Y, int64_t n, int d, hipStream_t st) {
  if (n <= 0) return;
  const bool vec = d % 4 == 0 && ((((uintptr_t)X) | ((uintptr_t)Y)) & 15) == 0;
  if (vec)
    hipLaunchKernelGGL(normalize_rows_kernel<true>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, X, Y, n, d);
  else
    hipLaunchKernelGGL(normalize_rows_kernel<false>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, st, X, Y, n, d);
}

void launch_screen_prep_rows(int prec, const float* X, int64_t r0, int64_t nmax, const int* count, int d, void* Xs,
                             int64_t ld_bytes, float* n2, float* scale, float* rn, unsigned* maxn2_bits,
                             hipStream_t st) {
  if (nmax <= 0) return;
  const dim3 g((unsigned)std::min<int64_t>((nmax + 3) / 4, 2048)), b(256);
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
  dim3 g((unsigned)std::min<int64_t>((npad + 3) / 4, 2048)), b(256);
  uint8_t* xs = (uint8_t*)Xs;
  if (prec == GCR_PREC_FP32)
    hipLaunchKernelGGL(screen_prep_kernel<GCR_PREC_FP32>, g, b, 0, st, X, n, d, npad, xs, ld_bytes, n2, scale, rn, maxn2_bits);
  else if (prec == GCR_PREC_BF16)
    hipLaunchKernelGGL(screen_prep_kernel<GCR_PREC_BF16>, g, b, 0, st, X, n, d, npad, xs, ld_bytes, n2, scale, rn, maxn2_bits);
  else
    hipLaunchKernelGGL(screen_prep_kernel<GCR_PREC_FP8>, g, b, 0, st, X, n, d, npad, xs, ld_bytes, n2, scale, rn, maxn2_bits);
}

}  // namespace gcr
