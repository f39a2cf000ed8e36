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

// mu = sum_c m_c mu_c / sum_c m_c over the group's members.
__global__ void group_mean_kernel(const float* __restrict__ mu_c, const int32_t* __restrict__ offs,
                                  const int32_t* __restrict__ members, int nm, int d, float* mu) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d) return;
  float s = 0.f, n = 0.f;
  for (int t = 0; t < nm; ++t) {
    const int c = members[t];
    const float m = (float)(offs[c + 1] - offs[c]);
    s = fmaf(m, mu_c[(int64_t)c * d + e], s);
    n += m;
  }
  mu[e] = s / n;
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
                       float* mu, hipStream_t st) {
  hipLaunchKernelGGL(group_mean_kernel, dim3(nb(d, 256)), dim3(256), 0, st, mu_c, offsets, members, nm, d, mu);
}
void launch_gram(const float* frames, const int32_t* rows, int64_t nrows, int d, float* partial, int ksplit,
                 float* G, float shift, hipStream_t st) {
  const int ntile = (d + GT - 1) / GT;
  hipLaunchKernelGGL(gram_kernel, dim3(ntile * ntile * ksplit), dim3(GNT), 0, st, frames, rows, nrows, d,
                     ksplit, partial);
  hipLaunchKernelGGL(gram_reduce_kernel, dim3(nb((int64_t)d * d, 256)), dim3(256), 0, st, partial, ksplit, d,
                     shift, G);
}
void launch_gemm_nn_f32(const float* A, int64_t lda, const float* B, int64_t ldb, float* Cm, int64_t ldc,
                        int M, int N, int K, float alpha, float beta, const float* Cin, int64_t ldcin,
                        hipStream_t st) {
  if (M <= 0 || N <= 0) return;
  const int grid = ((M + MT - 1) / MT) * ((N + MT - 1) / MT);
  hipLaunchKernelGGL(gemm_nn_f32_kernel, dim3(grid), dim3(MNT), 0, st, A, lda, B, ldb, Cm, ldc, M, N, K,
                     alpha, beta, Cin, ldcin);
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
