// Tracklet profile vectors for video re-identification.
//   Eq. (10): mu_c = mean of tracklet c's frames (also the "mean" profile).
//   Eq. (16), per camera group with frames F (n of them) and mean mu:
//       (F^T F + lambda n I) w_c = mu_c - mu
// The d x d Gram F^T F is a float32 MFMA GEMM split over frame chunks; the
// shifted system is solved for all tracklets of the group at once with a
// Chebyshev iteration whose spectrum bounds [lambda n, lambda n + tr(F^T F)]
// are exact (F^T F is positive semi-definite with norm <= its trace), so the
// iteration count is fixed in advance; each iteration is one GEMM.
#include "kernels.h"

namespace gcr {

__global__ void segment_means_kernel(const float* __restrict__ F, const int32_t* __restrict__ offs,
                                     int d, float* __restrict__ mu_c) {
  const int c = blockIdx.x;
  const int a = offs[c], b = offs[c + 1];
  const float inv = 1.0f / (float)(b - a);
  for (int e = threadIdx.x; e < d; e += blockDim.x) {
    float s = 0.f;
    for (int f = a; f < b; ++f) s += F[(int64_t)f * d + e];
    mu_c[(int64_t)c * d + e] = s * inv;
  }
}

// mu = sum_c m_c mu_c / sum_c m_c over the group's members, in two passes:
// chunk j of the members sums into part[j][.] (grid: column blocks x
// chunks), then the chunks are added in order and divided by the group's
// frame count.
constexpr int GM_CHUNKS = 64;
__global__ void group_mean_part_kernel(const float* __restrict__ mu_c, const int32_t* __restrict__ offs,
                                       const int32_t* __restrict__ members, int nm, int d,
                                       float* __restrict__ part) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int j = blockIdx.y;
  if (e >= d) return;
  const int per = (nm + GM_CHUNKS - 1) / GM_CHUNKS;
  const int t0 = j * per, t1 = min(nm, t0 + per);
  float s = 0.f;
  for (int t = t0; t < t1; ++t) {
    const int c = members[t];
    s = fmaf((float)(offs[c + 1] - offs[c]), mu_c[(int64_t)c * d + e], s);
  }
  part[(int64_t)j * d + e] = s;
}
__global__ void group_mean_final_kernel(const float* __restrict__ part, int d, float nframes, float* mu) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d) return;
  float s = 0.f;
  for (int j = 0; j < GM_CHUNKS; ++j) s += part[(int64_t)j * d + e];
  mu[e] = s / nframes;
}

// ---------------------------------------------------------------------------
// Gram partials: part[ks][a][b] = sum_{f in chunk ks} F[rows[f]][a] F[rows[f]][b]
namespace {
constexpr int GT = 128, GK = 32, GNT = 256, GSTR = GT + 4;
}

__global__ __launch_bounds__(GNT) void gram_kernel(const float* __restrict__ F, const int32_t* __restrict__ rows,
                                                   int64_t nrows, int d, int ksplit, float* __restrict__ part) {
  __shared__ float As[GK][GSTR], Bs[GK][GSTR];
  const int ntile = (d + GT - 1) / GT;
  const int ta = blockIdx.x % ntile, tb = (blockIdx.x / ntile) % ntile, ks = blockIdx.x / (ntile * ntile);
  const int64_t per = (nrows + ksplit - 1) / ksplit;
  const int64_t f0 = (int64_t)ks * per, f1 = min(nrows, f0 + per);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wa = (wave >> 1) * 64, wb = (wave & 1) * 64;
  const int l32 = lane & 31, half = lane >> 5;
  const int a0 = ta * GT, b0 = tb * GT;
  f32x16 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[x][y][i] = 0.f;
  for (int64_t fb = f0; fb < f1; fb += GK) {
    // load GK frames x 128 features of both column ranges
    for (int t = tid; t < GK * GT; t += GNT) {
      const int kk = t / GT, m = t % GT;
      const int64_t f = fb + kk;
      float va = 0.f, vb = 0.f;
      if (f < f1) {
        const float* fr = F + (int64_t)rows[f] * d;
        if (a0 + m < d) va = fr[a0 + m];
        if (b0 + m < d) vb = fr[b0 + m];
      }
      As[kk][m] = va;
      Bs[kk][m] = vb;
    }
    __syncthreads();
#pragma unroll 4
    for (int s = 0; s < GK / 2; ++s) {
      const int kk = 2 * s + half;
      float fa[2], fbv[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        fa[x] = As[kk][wa + 32 * x + l32];
        fbv[x] = Bs[kk][wb + 32 * x + l32];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[x], fbv[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
  // C[m = a][n = b]: lane holds n = l32, m = 8(i/4) + 4 half + (i%4)
  float* P = part + (int64_t)ks * d * d;
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int a = a0 + wa + 32 * x + 8 * (i >> 2) + 4 * half + (i & 3);
        const int b = b0 + wb + 32 * y + l32;
        if (a < d && b < d) P[(int64_t)a * d + b] = acc[x][y][i];
      }
}

__global__ void gram_reduce_kernel(const float* __restrict__ part, int ksplit, int d, float shift,
                                   float* __restrict__ G) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t dd = (int64_t)d * d;
  if (t >= dd) return;
  float s = 0.f;
  for (int k = 0; k < ksplit; ++k) s += part[(int64_t)k * dd + t];
  const int64_t a = t / d, b = t % d;
  G[t] = s + (a == b ? shift : 0.f);
}

// ---------------------------------------------------------------------------
// C = alpha A B + beta Cin, float32 MFMA; A [M,K] (lda), B [K,N] (ldb), all
// row-major.  128 x 128 tiles, K in chunks of 32.
namespace {
constexpr int MT = 128, MK = 32, MNT = 256, ASTR = MK + 4, BSTR = MT + 4;
}
__global__ __launch_bounds__(MNT) void gemm_nn_f32_kernel(const float* __restrict__ A, int64_t lda,
                                                          const float* __restrict__ B, int64_t ldb,
                                                          float* Cm, int64_t ldc, int M, int N, int K,
                                                          float alpha, float beta, const float* Cin,
                                                          int64_t ldcin) {
  __shared__ float As[MT][ASTR];
  __shared__ float Bs[MK][BSTR];
  const int tn = (N + MT - 1) / MT;
  const int tm = blockIdx.x / tn, tnn = blockIdx.x % tn;
  const int m0 = tm * MT, n0 = tnn * MT;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int l32 = lane & 31, half = lane >> 5;
  f32x16 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[x][y][i] = 0.f;
  for (int k0 = 0; k0 < K; k0 += MK) {
    for (int t = tid; t < MT * MK; t += MNT) {
      const int m = t / MK, kk = t % MK;
      As[m][kk] = (m0 + m < M && k0 + kk < K) ? A[(int64_t)(m0 + m) * lda + k0 + kk] : 0.f;
    }
    for (int t = tid; t < MK * MT; t += MNT) {
      const int kk = t / MT, n = t % MT;
      Bs[kk][n] = (k0 + kk < K && n0 + n < N) ? B[(int64_t)(k0 + kk) * ldb + n0 + n] : 0.f;
    }
    __syncthreads();
#pragma unroll 4
    for (int s = 0; s < MK / 2; ++s) {
      const int kk = 2 * s + half;
      float fa[2], fb[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        fa[x] = As[wm + 32 * x + l32][kk];
        fb[x] = Bs[kk][wn + 32 * x + l32];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[x], fb[y], acc[x][y], 0, 0, 0);
    }
    __syncthreads();
  }
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int m = m0 + wm + 32 * x + 8 * (i >> 2) + 4 * half + (i & 3);
        const int n = n0 + wn + 32 * y + l32;
        if (m < M && n < N) {
          float v = alpha * acc[x][y][i];
          if (Cin) v += beta * Cin[(int64_t)m * ldcin + n];
          Cm[(int64_t)m * ldc + n] = v;
        }
      }
}

// ---------------------------------------------------------------------------
// Pipelined float32 MFMA tiles for d a multiple of 4 (16-byte loads): one
// kernel serves the Gram (GRAM = true: A(k, m) = F[rows[k]][a0 + m],
// B(k, n) = F[rows[k]][b0 + n], upper-triangle tile pairs only, each
// off-diagonal tile also written transposed) and C = alpha A B + beta Cin
// (GRAM = false: A [M, K] row-major, B [K, N] row-major).  Both operands sit
// in LDS k-major (fragment reads are lane-contiguous), double-buffered: the
// global loads of chunk c + 1 are in flight in registers while chunk c is
// multiplied, then stored to the other buffer; one barrier per chunk.
namespace {
constexpr int PT = 128, PK = 32, PNT = 256, PSTR = PT + 4;
}
template <bool GRAM>
__global__ __launch_bounds__(PNT, 2) void mfma_f32_pipe_kernel(const float* __restrict__ A, int64_t lda,
                                                             const float* __restrict__ Bm, int64_t ldb,
                                                             const int32_t* __restrict__ rows, int64_t nrows,
                                                             int ksplit, float* __restrict__ Cm, int64_t ldc,
                                                             int M, int N, int K, float alpha, float beta,
                                                             const float* __restrict__ Cin, int64_t ldcin) {
  __shared__ __align__(16) float As[2][PK][PSTR];
  __shared__ __align__(16) float Bs[2][PK][PSTR];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 64;
  const int l32 = lane & 31, half = lane >> 5;
  int m0, n0, ta = 0, tb = 0;
  int64_t k0, k1;
  if constexpr (GRAM) {
    // tile pair p of the upper triangle (ta <= tb), then its K split
    const int ntile = (M + PT - 1) / PT;
    const int npairs = ntile * (ntile + 1) / 2;
    int p = blockIdx.x % npairs;
    const int ks = blockIdx.x / npairs;
    while (p >= ntile - ta) {
      p -= ntile - ta;
      ++ta;
    }
    tb = ta + p;
    m0 = ta * PT;
    n0 = tb * PT;
    const int64_t per = (nrows + ksplit - 1) / ksplit;
    k0 = (int64_t)ks * per;
    k1 = min(nrows, k0 + per);
    Cm += (int64_t)ks * M * M;
  } else {
    const int tn = (N + PT - 1) / PT;
    m0 = (blockIdx.x / tn) * PT;
    n0 = (blockIdx.x % tn) * PT;
    k0 = 0;
    k1 = K;
  }
  // per-thread load slots: 4 float4 of A and 4 of B per chunk
  f32x4 ra[4], rb[4];
  auto load = [&](int64_t kb) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      if constexpr (GRAM) {
        const int kk = tid >> 3, c4 = (tid & 7) + 8 * j;
        const int64_t f = kb + kk;
        f32x4 va = {0.f, 0.f, 0.f, 0.f}, vb = va;
        if (f < k1) {
          const float* fr = A + (int64_t)rows[f] * lda;
          if (m0 + 4 * c4 < M) va = *(const f32x4*)(fr + m0 + 4 * c4);
          if (n0 + 4 * c4 < M) vb = *(const f32x4*)(fr + n0 + 4 * c4);
        }
        ra[j] = va;
        rb[j] = vb;
      } else {
        // A: row m = tid / 2, k quad (tid & 1) + 2 j; B: k = tid / 8, n quad (tid & 7) + 8 j
        const int m = tid >> 1, q = (tid & 1) + 2 * j;
        const int64_t kq = kb + 4 * q;
        f32x4 va = {0.f, 0.f, 0.f, 0.f};
        if (m0 + m < M && kq < k1) va = *(const f32x4*)(A + (int64_t)(m0 + m) * lda + kq);
        ra[j] = va;
        const int kk = tid >> 3, c4 = (tid & 7) + 8 * j;
        f32x4 vb = {0.f, 0.f, 0.f, 0.f};
        if (kb + kk < k1 && n0 + 4 * c4 < N) vb = *(const f32x4*)(Bm + (kb + kk) * ldb + n0 + 4 * c4);
        rb[j] = vb;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int kk = tid >> 3, c4 = (tid & 7) + 8 * j;
      *(f32x4*)&Bs[buf][kk][4 * c4] = rb[j];
      if constexpr (GRAM) {
        *(f32x4*)&As[buf][kk][4 * c4] = ra[j];
      } else {
        const int m = tid >> 1, q = (tid & 1) + 2 * j;
        As[buf][4 * q + 0][m] = ra[j].x;
        As[buf][4 * q + 1][m] = ra[j].y;
        As[buf][4 * q + 2][m] = ra[j].z;
        As[buf][4 * q + 3][m] = ra[j].w;
      }
    }
  };
  f32x16 acc[2][2];
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 16; ++i) acc[x][y][i] = 0.f;
  const int64_t nch = (k1 - k0 + PK - 1) / PK;
  if (nch > 0) {
    load(k0);
    store(0);
  }
  __syncthreads();
  for (int64_t c = 0; c < nch; ++c) {
    const int buf = (int)(c & 1);
    if (c + 1 < nch) load(k0 + (c + 1) * PK);
#pragma unroll 4
    for (int s2 = 0; s2 < PK / 2; ++s2) {
      const int kk = 2 * s2 + half;
      float fa[2], fb[2];
#pragma unroll
      for (int x = 0; x < 2; ++x) {
        fa[x] = As[buf][kk][wm + 32 * x + l32];
        fb[x] = Bs[buf][kk][wn + 32 * x + l32];
      }
#pragma unroll
      for (int x = 0; x < 2; ++x)
#pragma unroll
        for (int y = 0; y < 2; ++y)
          acc[x][y] = __builtin_amdgcn_mfma_f32_32x32x2f32(fa[x], fb[y], acc[x][y], 0, 0, 0);
    }
    if (c + 1 < nch) store(buf ^ 1);
    __syncthreads();
  }
  // C[m][n]: lane holds n = l32, m = 8 (i / 4) + 4 half + (i % 4)
#pragma unroll
  for (int x = 0; x < 2; ++x)
#pragma unroll
    for (int y = 0; y < 2; ++y)
#pragma unroll
      for (int i = 0; i < 16; ++i) {
        const int m = m0 + wm + 32 * x + 8 * (i >> 2) + 4 * half + (i & 3);
        const int n = n0 + wn + 32 * y + l32;
        if constexpr (GRAM) {
          if (m < M && n < M) {
            Cm[(int64_t)m * M + n] = acc[x][y][i];
            if (ta != tb) Cm[(int64_t)n * M + m] = acc[x][y][i];
          }
        } else if (m < M && n < N) {
          float v = alpha * acc[x][y][i];
          if (Cin) v += beta * Cin[(int64_t)m * ldcin + n];
          Cm[(int64_t)m * ldc + n] = v;
        }
      }
}

// tr(F^T F) = sum over the diagonal of G minus the shift (one workgroup,
// float64 sum)
__global__ __launch_bounds__(256) void gram_trace_kernel(const float* __restrict__ G, int d, float shift,
                                                         double* __restrict__ out) {
  __shared__ double part[4];
  double s = 0.0;
  for (int e = threadIdx.x; e < d; e += 256) s += (double)G[(int64_t)e * (d + 1)] - (double)shift;
  s = wave_sum_f64(s);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) out[0] = part[0] + part[1] + part[2] + part[3];
}

__global__ void build_rhs_kernel(const float* __restrict__ mu_c, const float* __restrict__ mu,
                                 const int32_t* __restrict__ members, int nm, int d, float* B) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nm * d) return;
  const int r = (int)(t / d), e = (int)(t % d);
  B[t] = mu_c[(int64_t)members[r] * d + e] - mu[e];
}

__global__ void scatter_rows_kernel(const float* __restrict__ Wt, const int32_t* __restrict__ members,
                                    int nm, int d, float* W) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)nm * d) return;
  const int r = (int)(t / d), e = (int)(t % d);
  W[(int64_t)members[r] * d + e] = Wt[t];
}

// y = a y + b x
__global__ void axpby_kernel(float* y, const float* x, float a, float b, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t < n) y[t] = a * y[t] + b * x[t];
}

// Chebyshev step: P = R + rho P; W += cR P   (rho = 0 on the first step)
__global__ void cheb_kernel(float* W, float* P, const float* R, float rho, float cR, int64_t n) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n) return;
  const float p = R[t] + rho * P[t];
  P[t] = p;
  W[t] += cR * p;
}

static inline unsigned nb(int64_t n, int b) { return (unsigned)((n + b - 1) / b); }

void launch_segment_means(const float* frames, const int32_t* offsets, int nt, int d, float* mu_c,
                          hipStream_t st) {
  if (nt <= 0) return;
  hipLaunchKernelGGL(segment_means_kernel, dim3(nt), dim3(256), 0, st, frames, offsets, d, mu_c);
}
void launch_group_mean(const float* mu_c, const int32_t* offsets, const int32_t* members, int nm, int d,
                       int64_t nframes, float* scratch, float* mu, hipStream_t st) {
  hipLaunchKernelGGL(group_mean_part_kernel, dim3(nb(d, 256), GM_CHUNKS), dim3(256), 0, st, mu_c, offsets, members,
                     nm, d, scratch);
  hipLaunchKernelGGL(group_mean_final_kernel, dim3(nb(d, 256)), dim3(256), 0, st, scratch, d, (float)nframes, mu);
}
int group_mean_scratch_floats(int d) { return GM_CHUNKS * d; }
void launch_gram(const float* frames, const int32_t* rows, int64_t nrows, int d, float* partial, int ksplit,
                 float* G, float shift, hipStream_t st) {
  if (d % 4 == 0 && ((uintptr_t)frames & 15) == 0) {
    const int ntile = (d + PT - 1) / PT;
    const int npairs = ntile * (ntile + 1) / 2;
    hipLaunchKernelGGL(mfma_f32_pipe_kernel<true>, dim3(npairs * ksplit), dim3(PNT), 0, st, frames, (int64_t)d,
                       nullptr, (int64_t)0, rows, nrows, ksplit, partial, (int64_t)d, d, d, 0, 1.0f, 0.0f, nullptr,
                       (int64_t)0);
  } else {
    const int ntile = (d + GT - 1) / GT;
    hipLaunchKernelGGL(gram_kernel, dim3(ntile * ntile * ksplit), dim3(GNT), 0, st, frames, rows, nrows, d,
                       ksplit, partial);
  }
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(nb((int64_t)d * d, 256)), dim3(256), 0, st, partial, ksplit, d,
                     shift, G);
}
void launch_gemm_nn_f32(const float* A, int64_t lda, const float* B, int64_t ldb, float* Cm, int64_t ldc,
                        int M, int N, int K, float alpha, float beta, const float* Cin, int64_t ldcin,
                        hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  const int grid = ((M + MT - 1) / MT) * ((N + MT - 1) / MT);
  if (K % 4 == 0 && lda % 4 == 0 && ldb % 4 == 0 && (((uintptr_t)A | (uintptr_t)B) & 15) == 0)
    hipLaunchKernelGGL(mfma_f32_pipe_kernel<false>, dim3(grid), dim3(PNT), 0, st, A, lda, B, ldb, nullptr,
                       (int64_t)0, 1, Cm, ldc, M, N, K, alpha, beta, Cin, ldcin);
  else
    hipLaunchKernelGGL(gemm_nn_f32_kernel, dim3(grid), dim3(MNT), 0, st, A, lda, B, ldb, Cm, ldc, M, N, K,
                       alpha, beta, Cin, ldcin);
}
void launch_gram_trace(const float* G, int d, float shift, double* out, hipStream_t st) {
  hipLaunchKernelGGL(gram_trace_kernel, dim3(1), dim3(256), 0, st, G, d, shift, out);
}
void launch_build_rhs(const float* mu_c, const float* mu, const int32_t* members, int nm, int d, float* B,
                      hipStream_t st) {
  hipLaunchKernelGGL(build_rhs_kernel, dim3(nb((int64_t)nm * d, 256)), dim3(256), 0, st, mu_c, mu, members,
                     nm, d, B);
}
void launch_scatter_profiles(const float* Wt, const int32_t* members, int nm, int d, float* W,
                             hipStream_t st) {
  hipLaunchKernelGGL(scatter_rows_kernel, dim3(nb((int64_t)nm * d, 256)), dim3(256), 0, st, Wt, members, nm,
                     d, W);
}
void launch_axpby(float* y, const float* x, float a, float b, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(axpby_kernel, dim3(nb(n, 256)), dim3(256), 0, st, y, x, a, b, n);
}
void launch_cheb_update(float* Wk, float* Wprev, const float* R, float rho, float cR, int64_t n,
                        hipStream_t st) {
  hipLaunchKernelGGL(cheb_kernel, dim3(nb(n, 256)), dim3(256), 0, st, Wk, Wprev, R, rho, cR, n);
}

}  // namespace gcr
