// Decentralised synchronous feature propagation, DSFP (Alg. 1).
//
// Node i's local set L = {i} + its listed neighbours (m <= 64 nodes).  On L:
//   A_uv = exp(-||x_u - x_v||^2 / gamma) (1 on the diagonal), D_u = sum_v A_uv,
//   P = D^-1/2 A D^-1/2, and T rounds X_L <- rownorm(P X_L); node i keeps its
//   own row of X_L after round T.
//
// One workgroup per node.  The rounds never need the local features
// themselves: every local row stays a combination of the input rows,
// X_L(t) = C_t X_L(0), with C_0 = I and
//   C_t = diag(1 / max(||y_u||, 1e-12)) P C_{t-1},
//   ||y_u||^2 = (P C_{t-1} G C_{t-1}^T P^T)_uu,  G = X_L(0) X_L(0)^T,
// so the m x d rows are read twice: once for the local Gram G (which also
// gives every local distance, ||x_u||^2 + ||x_v||^2 - 2 G_uv) and once for
// node i's output row sum_a C_T[0][a] x_a, re-normalised from its own values.
// All rounds run on m x m matrices in LDS.
#include "kernels.h"

namespace gcr {

namespace {

constexpr int DS_NT = 256;  // threads per workgroup
// Feature columns per staged chunk: 128 when the local set has at most 32
// members, 64 up to 64 members (the chunk then always fills 4 float4 slots
// per thread, and the transposed chunk fits the LDS of the Gram partials).
constexpr int ds_dc(int mp) { return mp <= 32 ? 128 : 64; }

struct DsLayout {
  int mp;       // local size rounded up to a multiple of 4
  float* G;     // [mp][mp] Gram
  float* P;     // [mp][mp] normalised local affinity
  float* C;     // [mp][mp] coefficients of the local rows
  float* stage; // [mp][DC + 1] feature chunk (odd row stride: the chunk's
                // stores and the Gram's column reads spread over the LDS
                // banks); later the Gram partials and the unscaled
                // coefficients of a round
};

__host__ __device__ inline int ds_mp(int k) { return ((k + 1 + 3) / 4) * 4; }
// LDS floats: G, P, C and the stage, or G and the Gram partials of all 256
// threads (16 each), whichever is larger.  The partials are placed at the
// end of the region, over P, C and the stage, which are unused while the
// partials are summed into G.
__host__ __device__ inline int ds_lds_floats(int k) {
  const int mp = ds_mp(k);
  const int a = 3 * mp * mp + (ds_dc(mp) + 1) * mp, b = mp * mp + DS_NT * 16;
  return a > b ? a : b;
}

__device__ __forceinline__ float block_sum(float v, float* red4) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) red4[w] = v;
  __syncthreads();
  const float s = red4[0] + red4[1] + red4[2] + red4[3];
  __syncthreads();
  return s;
}

// Chunk [c0, c0 + DC) of the m local rows, one float4 per slot: slot e
// covers local row e / (DC / 4), columns c0 + 4 (e % (DC / 4)) + 0..3.
template <bool VEC, int DC>
__device__ __forceinline__ f32x4 load_slot(const float* __restrict__ X, const int* nodes, int m, int d, int c0,
                                           int e) {
  f32x4 v = {0.f, 0.f, 0.f, 0.f};
  const int u = e / (DC / 4), q = e % (DC / 4);
  const int col = c0 + 4 * q;
  if (u < m && col < d) {
    const float* row = X + (int64_t)nodes[u] * d;
    if (VEC) {
      v = *(const f32x4*)(row + col);
    } else {
      v.x = row[col];
      if (col + 1 < d) v.y = row[col + 1];
      if (col + 2 < d) v.z = row[col + 2];
      if (col + 3 < d) v.w = row[col + 3];
    }
  }
  return v;
}

}  // namespace

struct DsfpArgs {
  const float* X;
  const int32_t* idx;
  const int32_t* order;  // visiting order of the nodes or null
  float* Y;
  int64_t n;
  int d, k, rounds;
  float gamma;
};

template <bool VEC, int DC>
__global__ __launch_bounds__(DS_NT) void dsfp_kernel(DsfpArgs a) {
  extern __shared__ f32x4 ds_smem4[];  // 16-byte aligned for the float4 reads
  float* ds_smem = (float*)ds_smem4;
  __shared__ int s_nodes[64];
  __shared__ int s_m;
  __shared__ float s_r[64];    // D_u^-1/2, then the round's row scales
  __shared__ float s_cf[64];   // node i's final coefficients
  __shared__ float s_red[4];
  const int tid = threadIdx.x;
  const int64_t pos = xcd_position(blockIdx.x, gridDim.x);
  const int64_t i = a.order ? (int64_t)a.order[pos] : pos;
  const int k = a.k, d = a.d;

  // ---- local set: node i first, then the valid distinct list entries
  if (tid < 64) {
    int j = -1;
    if (tid < k) {
      j = a.idx[i * k + tid];
      if (j < 0 || (int64_t)j >= a.n || (int64_t)j == i) j = -1;
    }
    bool dup = false;
    for (int v = 0; v < k; ++v) {
      const int jv = __shfl(j, v, 64);
      dup |= (v < tid) && (jv == j);
    }
    const bool keep = (j >= 0) && !dup;
    const uint64_t mask = __ballot(keep);
    if (keep) s_nodes[1 + __popcll(mask & ((1ull << tid) - 1ull))] = j;
    if (tid == 0) {
      s_nodes[0] = (int)i;
      s_m = 1 + __popcll(mask);
    }
  }
  __syncthreads();
  const int m = s_m;
  DsLayout L;
  L.mp = ds_mp(k);
  const int mp = L.mp;
  L.G = ds_smem;
  L.P = L.G + mp * mp;
  L.C = L.P + mp * mp;
  L.stage = L.C + mp * mp;

  // ---- local Gram, 4 x 4 register blocks over the upper block triangle
  const int nb = (m + 3) / 4;
  const int nblk = nb * (nb + 1) / 2;
  const int groups = DS_NT / nblk;  // >= 1 since nblk <= 136
  const bool active = tid < nblk * groups;
  const int blk = tid % nblk, grp = tid / nblk;
  int bi = 0, bj = 0;
  {
    int r = blk;
    while (r >= nb - bi) {
      r -= nb - bi;
      ++bi;
    }
    bj = bi + r;
  }
  float acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int s = 0; s < 4; ++s) acc[r][s] = 0.f;

  constexpr int SLOTS = (DC == 128 ? 32 : 64) * DC / 4 / DS_NT;  // float4 slots per thread
  const int nslot = ((m + 3) / 4) * 4 * (DC / 4);  // rows padded to nb * 4
  f32x4 pre[SLOTS];
#pragma unroll
  for (int s = 0; s < SLOTS; ++s) {
    const int e = tid + s * DS_NT;
    pre[s] = e < nslot ? load_slot<VEC, DC>(a.X, s_nodes, m, d, 0, e) : f32x4{0.f, 0.f, 0.f, 0.f};
  }
  for (int c0 = 0; c0 < d; c0 += DC) {
#pragma unroll
    for (int s = 0; s < SLOTS; ++s) {
      const int e = tid + s * DS_NT;
      if (e < nslot) {
        const int u = e / (DC / 4), q = e % (DC / 4);
        float* dst = L.stage + u * (DC + 1) + 4 * q;
        dst[0] = pre[s].x;
        dst[1] = pre[s].y;
        dst[2] = pre[s].z;
        dst[3] = pre[s].w;
      }
    }
    __syncthreads();
    if (c0 + DC < d) {
#pragma unroll
      for (int s = 0; s < SLOTS; ++s) {
        const int e = tid + s * DS_NT;
        if (e < nslot) pre[s] = load_slot<VEC, DC>(a.X, s_nodes, m, d, c0 + DC, e);
      }
    }
    if (active) {
      const float* xr = L.stage + 4 * bi * (DC + 1);
      const float* yr = L.stage + 4 * bj * (DC + 1);
      for (int c = grp; c < DC; c += groups) {
        float xs[4], ys[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          xs[r] = xr[r * (DC + 1) + c];
          ys[r] = yr[r * (DC + 1) + c];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
          for (int s = 0; s < 4; ++s) acc[r][s] = fmaf(xs[r], ys[s], acc[r][s]);
      }
    }
    __syncthreads();
  }
  // partials -> G (sum over the column groups in group order)
  float* part = ds_smem + ds_lds_floats(k) - nblk * groups * 16;
  if (active) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int s = 0; s < 4; ++s) part[(grp * nblk + blk) * 16 + r * 4 + s] = acc[r][s];
  }
  __syncthreads();
  for (int e = tid; e < nblk * 16; e += DS_NT) {
    const int b = e >> 4, rs = e & 15;
    float sum = 0.f;
    for (int g = 0; g < groups; ++g) sum += part[(g * nblk + b) * 16 + rs];
    int pi = 0, r = b;
    while (r >= nb - pi) {
      r -= nb - pi;
      ++pi;
    }
    const int u = 4 * pi + (rs >> 2), v = 4 * (pi + r) + (rs & 3);
    if (u < m && v < m) {
      L.G[u * mp + v] = sum;
      L.G[v * mp + u] = sum;
    }
  }
  __syncthreads();

  // ---- local affinity, degrees, P = D^-1/2 A D^-1/2
  const float ninv_gamma = -1.0f / a.gamma;
  for (int e = tid; e < m * m; e += DS_NT) {
    const int u = e / m, v = e % m;
    float dist = 0.f;
    if (u != v) dist = fmaxf(L.G[u * mp + u] + L.G[v * mp + v] - 2.0f * L.G[u * mp + v], 0.f);
    L.P[u * mp + v] = u == v ? 1.0f : expf(dist * ninv_gamma);
  }
  __syncthreads();
  if (tid < m) {
    float s = 0.f;
    for (int v = 0; v < m; ++v) s += L.P[tid * mp + v];
    s_r[tid] = 1.0f / sqrtf(s);
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += DS_NT) {
    const int u = e / m, v = e % m;
    L.P[u * mp + v] *= s_r[u] * s_r[v];
  }
  __syncthreads();

  // ---- T local rounds on the coefficients (C_0 = I); the last round only
  // needs node i's row
  float* Cn = L.stage;
  for (int t = 1; t < a.rounds; ++t) {
    for (int e = tid; e < m * m; e += DS_NT) {
      const int u = e / m, v = e % m;
      float s;
      if (t == 1) {
        s = L.P[u * mp + v];
      } else {
        s = 0.f;
        for (int w = 0; w < m; ++w) s = fmaf(L.P[u * mp + w], L.C[w * mp + v], s);
      }
      Cn[u * mp + v] = s;
    }
    __syncthreads();
    // H = Cn G into C (the old coefficients are no longer needed)
    for (int e = tid; e < m * m; e += DS_NT) {
      const int u = e / m, v = e % m;
      float s = 0.f;
      for (int w = 0; w < m; ++w) s = fmaf(Cn[u * mp + w], L.G[w * mp + v], s);
      L.C[u * mp + v] = s;
    }
    __syncthreads();
    if (tid < m) {
      float s = 0.f;
      for (int v = 0; v < m; ++v) s = fmaf(L.C[tid * mp + v], Cn[tid * mp + v], s);
      s_r[tid] = 1.0f / fmaxf(sqrtf(fmaxf(s, 0.f)), 1e-12f);
    }
    __syncthreads();
    for (int e = tid; e < m * m; e += DS_NT) {
      const int u = e / m, v = e % m;
      L.C[u * mp + v] = Cn[u * mp + v] * s_r[u];
    }
    __syncthreads();
  }
  if (tid < m) {
    float s;
    if (a.rounds == 1) {
      s = L.P[tid];
    } else {
      s = 0.f;
      for (int w = 0; w < m; ++w) s = fmaf(L.P[w], L.C[w * mp + tid], s);
    }
    s_cf[tid] = s;
  }
  __syncthreads();

  // ---- node i's row: sum_a cf_a x_a, re-normalised from its own values
  float* yrow = a.Y + i * d;
  if (VEC) {
    constexpr int NV = 2048 / 4 / DS_NT;
    f32x4 y[NV];
    float ss = 0.f;
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      y[q] = f32x4{0.f, 0.f, 0.f, 0.f};
      const int col = 4 * (tid + q * DS_NT);
      if (col < d) {
        // rows in batches of 8 (all loads issued before the sums, which
        // stay in row order)
        for (int u0 = 0; u0 < m; u0 += 8) {
          f32x4 xb[8];
#pragma unroll
          for (int t = 0; t < 8; ++t)
            if (u0 + t < m) xb[t] = *(const f32x4*)(a.X + (int64_t)s_nodes[u0 + t] * d + col);
#pragma unroll
          for (int t = 0; t < 8; ++t)
            if (u0 + t < m) {
              const float c = s_cf[u0 + t];
              y[q].x = fmaf(c, xb[t].x, y[q].x);
              y[q].y = fmaf(c, xb[t].y, y[q].y);
              y[q].z = fmaf(c, xb[t].z, y[q].z);
              y[q].w = fmaf(c, xb[t].w, y[q].w);
            }
        }
        ss += y[q].x * y[q].x + y[q].y * y[q].y + y[q].z * y[q].z + y[q].w * y[q].w;
      }
    }
    const float inv = 1.0f / fmaxf(sqrtf(block_sum(ss, s_red)), 1e-12f);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const int col = 4 * (tid + q * DS_NT);
      if (col < d) *(f32x4*)(yrow + col) = y[q] * inv;
    }
  } else {
    constexpr int NS = 2048 / DS_NT;
    float y[NS];
    float ss = 0.f;
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      y[q] = 0.f;
      const int col = tid + q * DS_NT;
      if (col < d) {
        for (int u0 = 0; u0 < m; u0 += 8) {
          float xb[8];
#pragma unroll
          for (int t = 0; t < 8; ++t)
            if (u0 + t < m) xb[t] = a.X[(int64_t)s_nodes[u0 + t] * d + col];
#pragma unroll
          for (int t = 0; t < 8; ++t)
            if (u0 + t < m) y[q] = fmaf(s_cf[u0 + t], xb[t], y[q]);
        }
        ss += y[q] * y[q];
      }
    }
    const float inv = 1.0f / fmaxf(sqrtf(block_sum(ss, s_red)), 1e-12f);
#pragma unroll
    for (int q = 0; q < NS; ++q) {
      const int col = tid + q * DS_NT;
      if (col < d) yrow[col] = y[q] * inv;
    }
  }
}

void launch_dsfp(const float* X, const int32_t* idx, int64_t n, int d, int k, float gamma, int rounds,
                 const int32_t* order, float* Y, hipStream_t st) {
  if (n <= 0) return;
  DsfpArgs a;
  a.X = X;
  a.idx = idx;
  a.order = order;
  a.Y = Y;
  a.n = n;
  a.d = d;
  a.k = k;
  a.rounds = rounds;
  a.gamma = gamma;
  const size_t lds = (size_t)ds_lds_floats(k) * sizeof(float);
  const bool vec = d % 4 == 0 && ((((uintptr_t)X) | ((uintptr_t)Y)) & 15) == 0;
  const dim3 g((unsigned)n), b(DS_NT);
  if (ds_mp(k) <= 32) {
    if (vec) hipLaunchKernelGGL((dsfp_kernel<true, 128>), g, b, lds, st, a);
    else hipLaunchKernelGGL((dsfp_kernel<false, 128>), g, b, lds, st, a);
  } else {
    if (vec) hipLaunchKernelGGL((dsfp_kernel<true, 64>), g, b, lds, st, a);
    else hipLaunchKernelGGL((dsfp_kernel<false, 64>), g, b, lds, st, a);
  }
}

}  // namespace gcr
