// Fused all-pairs similarity (MFMA) + streaming per-row top-k screening.
//
// The k-nearest-neighbour sets of Eq. (4) (and the cross-camera sets of
// Eq. (8)) need, for every row i, the k smallest ||x_i - x_j||^2.  For a
// fixed row this ranks columns by the key n2_j - 2 <x_i, x_j>.  Each work-
// group owns 128 rows (256 for sweeps of one list over many row blocks) and
// sweeps a range of 256-column tiles; a tile of similarities is an MFMA GEMM
// over the feature dimension (float32, bfloat16 or FP8-E4M3 operands,
// float32 accumulation) and never leaves the registers.  Its epilogue
// screens every score against the row's running admission threshold and
// appends survivors to the row's candidate buffer (global memory, one region
// per row/list/split).
//
// Data movement: the feature dimension is consumed in chunks (128 bytes per
// row, in a 3-stage ring, for 128-row tiles; 64 bytes in a 4-stage ring for
// 256-row tiles).  Each chunk of the row tile and of the column tile is
// copied straight from global memory into LDS by buffer loads with an LDS
// destination (16 bytes per lane, no register staging), so NSTAGE - 1
// chunks are in flight while one is multiplied.  Rows are XOR-swizzled in
// 16-byte units inside LDS so that fragment reads are free of bank
// conflicts.  The column data the epilogue needs comes into LDS the same
// way, so no step waits for more than the ring's own next chunk.  Out-of-
// range reads return zero through the buffer descriptor's range.
//
// Admission rule.  Let E_i bound |screened key - exact key| (screen_margin)
// and tau_i be the k-th smallest screened key the buffer has seen.  A column
// is admitted while its screened key <= tau_i + 2 E_i.  Because tau_i only
// decreases during the sweep and the true k-th key is <= tau_final + E_i,
// every true neighbour has a screened key <= tau_final + 2 E_i, so the
// buffer always keeps the exact top-k (ties included).  A full buffer is
// compacted by one wave: a radix select finds the new tau_i and the keys
// above the threshold are dropped.  If the margin band alone fills the buffer (a split's local
// k-th neighbour can sit in a dense region of unrelated items), the buffer
// keeps its smallest keys and the admission threshold drops below the first
// key it gave up; the split's final threshold is written out, and the
// refine step falls back to an exhaustive row only if the global cut
// reaches beyond it.
#include "kernels.h"

namespace gcr {

namespace {
constexpr int BN = 256, NT = 256;
// s_waitcnt immediate (gfx9 layout) that waits for vmcnt <= n only
constexpr int waitcnt_vm(int n) { return 0xF70 | (n & 0xF) | (((n >> 4) & 3) << 14); }
// ... and for lgkmcnt == 0 (this wave's LDS reads have returned)
constexpr int waitcnt_vm_lgkm0(int n) { return 0x070 | (n & 0xF) | (((n >> 4) & 3) << 14); }
// lgkmcnt == 0 only
constexpr int waitcnt_lgkm0 = 0xC07F;

// Workgroup tiles.  BMT = 128: 128 rows x 256 columns (waves of 64 x 128),
// 128-byte chunks of the feature dimension in a 3-stage ring (144 KB).
// BMT = 256: 256 x 256 (waves of 128 x 128), 64-byte chunks in a 4-stage
// ring (128 KB): per multiply-add it moves two thirds of the operand bytes
// and reads two thirds of the LDS fragments of the smaller tile, for sweeps
// with many row blocks.  A row of a chunk is P 16-byte parts, XOR-swizzled
// in LDS so that the 8 rows one 128-byte bank window serves fall on
// distinct parts.
template <int BMT>
struct Tile {
  static constexpr int BM = BMT;
  static constexpr int CHB = BMT == 256 ? 64 : 128;   // chunk bytes per row
  static constexpr int P = CHB / 16;                   // 16-byte parts per chunk row
  static constexpr int NSTAGE = BMT == 256 ? 4 : 3;
  static constexpr int RBYTES = BM * CHB;              // row tile of one chunk
  static constexpr int STAGE = RBYTES + BN * CHB;
  static constexpr int SMEM = NSTAGE * STAGE;
  // 256-row tiles: after the ring, each wave's admission queue (64 blocks of
  // 16 float32 accumulators, then 64 block tags)
  static constexpr int QBYTES = BMT == 256 ? NT * 16 * 4 + NT * 4 : 0;
  // then the tile's column data (norms, FP8 scales, cameras, stamps) and the
  // thresholds other splits published for the rows (up to two lists)
  static constexpr int COLBYTES = 4 * BN * 4 + 2 * BM * 4;
  static constexpr int DSMEM = SMEM + QBYTES + COLBYTES;
  static constexpr int RPL = 1024 / CHB;               // rows per 1 KB wave load
  static constexpr int DMA_PER_WAVE = (BM + BN) / RPL / 4;
  static constexpr int RBW = BM / 64;                  // 32-row blocks per wave
  __device__ static int swz(int r) { return CHB == 128 ? (r & 7) : ((r >> 1) & 3); }
};
}  // namespace

int sim_topk_grid(int RB, int S) { return RB * S; }

// Balanced schedule for rows [r0, r0 + rows) x ncols columns on G
// workgroups: the largest number of pieces (splits) one row block can be
// cut into, or 0 when the rows are too few for it.
int sim_topk_balanced_splits(int64_t rows, int64_t ncols, int G, int bm) {
  const int64_t RB = (rows + bm - 1) / bm, nt = (ncols + BN - 1) / BN;
  if (RB < 64 || nt < 1) return 0;
  const int64_t T = RB * nt;
  if (T < G) return 0;
  const int64_t per = T / G;  // every workgroup gets per or per + 1 tiles
  return (int)((nt + per - 1) / per + 1);
}
int sim_topk_tile_cols() { return BN; }

typedef uint32_t __attribute__((address_space(3)))* lds_u32_ptr;
extern "C" __device__ void gcr_buffer_load_lds(i32x4 rsrc, lds_u32_ptr lds, int size, int voffset, int soffset,
                                               int offset, int aux) __asm("llvm.amdgcn.raw.buffer.load.lds");

struct BufRes {
  const void* p;
  uint32_t range;
  uint32_t cfg;
};
// Buffer descriptor over [p, p + range): reads past range return zero.
__device__ __forceinline__ i32x4 make_res(const void* p, uint64_t range) {
  BufRes r{p, (uint32_t)(range > 0xffffffffull ? 0xffffffffull : range), 0x00020000u};
  i32x4 v = __builtin_bit_cast(i32x4, r);
  v.x = __builtin_amdgcn_readfirstlane(v.x);
  v.y = __builtin_amdgcn_readfirstlane(v.y);
  v.z = __builtin_amdgcn_readfirstlane(v.z);
  v.w = __builtin_amdgcn_readfirstlane(v.w);
  return v;
}

// Issue this wave's share of one chunk: 1 KB blocks of RPL rows, lane l
// bringing logical part (l % P) ^ swz(row) of row blk * RPL + l / P so the
// data lands swizzled.  Block blk = wave + 4 i has the same swizzle for
// every i, so the per-lane offset voff is the same for every block and
// chunk; the byte offsets of the row tile, the column tile, the chunk and
// the block are wave-uniform and go into the scalar offset of one
// descriptor that spans the whole operand.
template <int BMT>
__device__ __forceinline__ void issue_chunk(uint8_t* stage, i32x4 res, int voff, uint32_t roff, uint32_t coff,
                                            uint32_t step, int wave) {
  using T = Tile<BMT>;
#pragma unroll
  for (int i = 0; i < T::BM / (4 * T::RPL); ++i)
    gcr_buffer_load_lds(res, (lds_u32_ptr)(stage + (wave + 4 * i) * 1024), 16, voff,
                        __builtin_amdgcn_readfirstlane(roff + i * step), 0, 0);
#pragma unroll
  for (int i = 0; i < BN / (4 * T::RPL); ++i)
    gcr_buffer_load_lds(res, (lds_u32_ptr)(stage + T::RBYTES + (wave + 4 * i) * 1024), 16, voff,
                        __builtin_amdgcn_readfirstlane(coff + i * step), 0, 0);
}

template <int BMT>
__device__ __forceinline__ const uint8_t* frag(const uint8_t* base, int r, int lp) {
  return base + r * Tile<BMT>::CHB + ((lp ^ Tile<BMT>::swz(r)) << 4);
}

// Fragments of one MFMA step: RBW row blocks and 4 column blocks of 32.
// acc[cb][rb]: 4 column blocks x RBW row blocks of 32 x 32 (transposed
// orientation: lane l holds row l & 31 of its row block and 16 columns).
// A chunk row of P parts is P / 2 steps of 8 BF16 or 4 float32 values per
// lane (float32: 4 MFMAs of 2 per step) or P / 4 steps of 32 FP8 values.
template <int PREC>
using FragT = typename std::conditional<PREC == GCR_PREC_FP32, f32x4,
                                        typename std::conditional<PREC == GCR_PREC_BF16, bf16x8, i32x8>::type>::type;
template <int PREC, int RBW>
struct Frag {
  FragT<PREC> r[RBW], c[4];
};
template <int PREC, int BMT>
constexpr int steps_per_chunk() { return PREC == GCR_PREC_FP8 ? Tile<BMT>::P / 4 : Tile<BMT>::P / 2; }

template <int PREC, int BMT>
__device__ __forceinline__ void frag_load(Frag<PREC, Tile<BMT>::RBW>& f, const uint8_t* __restrict__ S, int q,
                                          int wr, int wc, int lane) {
  using T = Tile<BMT>;
  const uint8_t* Rt = S;
  const uint8_t* Ct = S + T::RBYTES;
  const int l32 = lane & 31, half = lane >> 5;
  if constexpr (PREC == GCR_PREC_FP8) {
    const int p0 = half * (T::P / 2) + 2 * q;
#pragma unroll
    for (int b = 0; b < T::RBW; ++b) {
      const int r = wr + 32 * b + l32;
      const i32x4 lo = *(const i32x4*)frag<BMT>(Rt, r, p0);
      const i32x4 hi = *(const i32x4*)frag<BMT>(Rt, r, p0 + 1);
      f.r[b] = i32x8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const int r = wc + 32 * b + l32;
      const i32x4 lo = *(const i32x4*)frag<BMT>(Ct, r, p0);
      const i32x4 hi = *(const i32x4*)frag<BMT>(Ct, r, p0 + 1);
      f.c[b] = i32x8{lo.x, lo.y, lo.z, lo.w, hi.x, hi.y, hi.z, hi.w};
    }
  } else {
    using V = FragT<PREC>;
    const int p0 = half * (T::P / 2) + q;
#pragma unroll
    for (int b = 0; b < T::RBW; ++b) f.r[b] = *(const V*)frag<BMT>(Rt, wr + 32 * b + l32, p0);
#pragma unroll
    for (int b = 0; b < 4; ++b) f.c[b] = *(const V*)frag<BMT>(Ct, wc + 32 * b + l32, p0);
  }
}

template <int PREC, int RBW>
__device__ __forceinline__ void frag_mma(const Frag<PREC, RBW>& f, f32x16 (&acc)[4][RBW]) {
  if constexpr (PREC == GCR_PREC_FP32) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int cb = 0; cb < 4; ++cb)
#pragma unroll
        for (int rb = 0; rb < RBW; ++rb)
          acc[cb][rb] = __builtin_amdgcn_mfma_f32_32x32x2f32(f.c[cb][s], f.r[rb][s], acc[cb][rb], 0, 0, 0);
  } else if constexpr (PREC == GCR_PREC_BF16) {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int rb = 0; rb < RBW; ++rb)
        acc[cb][rb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(f.c[cb], f.r[rb], acc[cb][rb], 0, 0, 0);
  } else {
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int rb = 0; rb < RBW; ++rb)
        acc[cb][rb] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(f.c[cb], f.r[rb], acc[cb][rb], 0, 0, 0, 127,
                                                                       0, 127);
  }
}

// LDS fetch-and-add with its wait in the same block.  (Written as a C++
// atomic, it makes the compiler wait first for every load in flight, those
// of the operand ring included, because direct-to-LDS loads count there.)
typedef int __attribute__((address_space(3)))* lds_i32_ptr;
__device__ __forceinline__ int lds_fetch_add(int* p, int v) {
  const uint32_t a = (uint32_t)(uintptr_t)(lds_i32_ptr)p;
  int r;
  asm volatile("ds_add_rtn_u32 %0, %1, %2\n\ts_waitcnt lgkmcnt(0)" : "=v"(r) : "v"(a), "v"(v) : "memory");
  return r;
}

// A serving row's own mask: column c is left out when its stamp matches.
__device__ __forceinline__ bool row_out(const uint32_t* mk, uint32_t stamp, int64_t c) {
  return mk && mk[c] == stamp;
}

// Number of buffer entries whose ordered key is <= u (wave-uniform).
template <int E>
__device__ __forceinline__ int wave_count_le(const uint32_t (&key)[E], uint32_t u) {
  int c = 0;
#pragma unroll
  for (int j = 0; j < E; ++j) c += __popcll(__ballot(key[j] <= u));
  return c;
}
// Smallest ordered key value u with at least r entries <= u (r <= count of
// non-empty entries): binary search over the 32-bit ordered key space.
template <int E>
__device__ __forceinline__ uint32_t wave_select(const uint32_t (&key)[E], int r) {
  uint32_t lo = 0u, hi = 0xfffffffeu;
  while (lo < hi) {
    const uint32_t mid = lo + ((hi - lo) >> 1);
    if (wave_count_le<E>(key, mid) >= r) hi = mid;
    else lo = mid + 1u;
  }
  return lo;
}

// One wave compacts the candidate buffer of (list L, local row lr):
// tau = k-th smallest key, keep the keys <= tau + 2E.  When that band leaves
// fewer than `room` free slots, keep only the keys below the (m+1)-th
// smallest, m = max(C/2, k), and lower the admission threshold below that
// key, so the buffer still holds every item of the split whose key is <=
// the threshold.  Order
// statistics come from a radix select on the ordered keys (ballots and
// popcounts), not from sorting; the kept entries are written back densely
// in no particular order.
template <int E>
__device__ void compact_row(uint64_t* base, int* cnt, float* thr, int C, int kk, float twoE, int room) {
  const int lane = threadIdx.x & 63;
  const int n = min(*cnt, C);
  uint64_t v[E];
  uint32_t key[E];
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const int e = j * 64 + lane;
    v[j] = e < n ? base[e] : GCR_EMPTY;
    key[j] = (uint32_t)(v[j] >> 32);  // empty slots: 0xffffffff, above any key
  }
  float th = *thr;
  if (n >= kk && kk > 0) th = fminf(th, unord_f32(wave_select<E>(key, kk)) + twoE);
  int newn = wave_count_le<E>(key, ord_f32(th));
  if (newn > C - room) {
    const int m = max(C / 2, kk);
    if (m < newn) {
      // admit only keys strictly below the (m+1)-th smallest
      const float cut = unord_f32(wave_select<E>(key, m + 1));
      th = fminf(th, nextafterf(cut, -INFINITY));
      newn = wave_count_le<E>(key, ord_f32(th));
    }
  }
  const uint32_t tho = ord_f32(th);
  int off = 0;
#pragma unroll
  for (int j = 0; j < E; ++j) {
    const bool keep = key[j] <= tho && v[j] != GCR_EMPTY;
    const uint64_t b = __ballot(keep);
    const int pos = off + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
    if (keep) base[pos] = v[j];
    off += __popcll(b);
  }
  if (lane == 0) { *cnt = off; *thr = th; }
}

template <int PREC, int NL, int E, int BMT>
__global__ __launch_bounds__(NT, 1) void sim_topk_kernel(SimArgs a) {
  using T = Tile<BMT>;
  constexpr int BM = T::BM, RBW = T::RBW, NSTAGE = T::NSTAGE, STAGE = T::STAGE, DMA = T::DMA_PER_WAVE;
  constexpr int SH = (BM * NL + NT - 1) / NT;  // shared thresholds prefetched per thread
  // Candidate buffers with room for a whole tile before each admission (C
  // >= 2 BN, 256-row tiles) instead of lost entries screened again after a
  // compaction: the accumulators are then read once, in the admission.
  constexpr bool ROOM = BMT == 256;
  extern __shared__ __align__(16) uint8_t smem[];
  // column data of the tile and the row thresholds other splits published,
  // copied straight into LDS (see the chunk loop)
  float* const col_n2 = reinterpret_cast<float*>(smem + T::SMEM + T::QBYTES);
  float* const col_sc = col_n2 + BN;
  int* const col_cam = reinterpret_cast<int*>(col_n2 + 2 * BN);
  uint32_t* const col_stamp = reinterpret_cast<uint32_t*>(col_n2 + 3 * BN);
  uint32_t* const sh_thr = reinterpret_cast<uint32_t*>(col_n2 + 4 * BN);
  static_assert(NL <= 2, "two lists at most");
  __shared__ float row_thr[NL][BM];
  __shared__ int row_cnt[NL][BM];
  __shared__ float row_twoE[BM], row_sc[BM];
  __shared__ int row_cam[BM];
  __shared__ const uint32_t* row_mk[BM];  // per-row column masks (serving batches)
  __shared__ uint32_t row_stp[BM];
  __shared__ int any_flag[2];
  __shared__ int room_flag[2];  // a buffer passed C - BN in the tile of that parity (room scheme)

  // balanced mode: consecutive pieces (mostly the same row block) go to the
  // same XCD, so its L2 serves the row tile to both workgroups sweeping it
  const int id = a.balanced ? (int)xcd_position(blockIdx.x, gridDim.x) : (int)blockIdx.x;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const float maxn2 = a.maxn2[0];
  const int64_t cend = a.filt.count ? min(a.c1, a.c0 + (int64_t)*a.filt.count) : a.c1;

  // Work pieces.  Split mode: workgroup id sweeps column split id mod S of
  // row block id / S (workgroup ids go round-robin over the 8 XCDs, so with
  // S dividing 8 every workgroup an XCD runs sweeps the same split and
  // shares its column tiles in L2).  Balanced mode (many row blocks): the
  // row-block x tile space is cut into gridDim.x equal ranges, one per
  // workgroup; the part of a row block that one workgroup sweeps is that
  // row's split number (workgroup - first workgroup of the row block).
  int64_t g_cur = 0, g_end = 0;
  if (a.balanced) {
    g_cur = (int64_t)id * a.total_tiles / gridDim.x;
    g_end = (int64_t)(id + 1) * a.total_tiles / gridDim.x;
  }
  for (bool first = true;; first = false) {
  int rb, cs, ntiles;
  int64_t sc0, sc1;
  if (a.balanced) {
    if (g_cur >= g_end) break;
    rb = (int)(g_cur / a.ntr);
    const int64_t x = (int64_t)rb * a.ntr;
    const int t0 = (int)(g_cur - x);
    const int t1 = (int)min<int64_t>(a.ntr, t0 + (g_end - g_cur));
    // first workgroup w with (w + 1) T / G > x, i.e. w = ceil((x + 1) G / T) - 1
    const int64_t G = gridDim.x;
    cs = id - (int)(((x + 1) * G + a.total_tiles - 1) / a.total_tiles - 1);
    sc0 = a.c0 + (int64_t)t0 * BN;
    sc1 = min(cend, a.c0 + (int64_t)t1 * BN);
    ntiles = t1 - t0;
    g_cur += t1 - t0;
  } else {
    if (!first) break;
    cs = id % a.S;
    rb = id / a.S;
    if (rb >= a.RB) break;
    sc0 = a.c0 + (int64_t)cs * a.W;
    sc1 = min(cend, sc0 + a.W);
    ntiles = sc1 > sc0 ? (int)((sc1 - sc0 + BN - 1) / BN) : 0;
  }
  __syncthreads();  // the previous piece is done with the shared state
  const int64_t row0 = a.r0 + (int64_t)rb * BM;

  if (tid < 2) {
    any_flag[tid] = 0;
    room_flag[tid] = 0;
  }
  if (NL > 1 && !a.cam) col_cam[tid] = 0;  // (NT == BN; never loaded then)
  for (int t = tid; t < BM; t += NT) {
    const int64_t r = row0 + t;
    const bool rv = r < a.r1;
    const float n2r = rv ? a.n2[r] : 0.f;
    row_twoE[t] = 2.0f * screen_margin(n2r, rv ? a.rn[r] : 0.f, maxn2, a.maxn2[1], a.eps_s, a.eps_n);
    row_cam[t] = (a.cam && rv) ? a.cam[r] : 0;
    row_mk[t] = (a.filt.row_mark && rv) ? a.filt.row_mark[r - a.r0] : nullptr;
    row_stp[t] = (a.filt.row_mark && rv) ? a.filt.row_stamp[r - a.r0] : 0u;
    row_sc[t] = (PREC == GCR_PREC_FP8 && rv) ? a.scale[r] : 1.0f;
#pragma unroll
    for (int L = 0; L < NL; ++L) {
      row_thr[L][t] = (rv && (L == 0 ? a.k0 : a.k1) > 0)
                          ? (a.thr_init ? a.thr_init[(r - a.r0) * NL + L] : INFINITY)
                          : -INFINITY;
      row_cnt[L][t] = 0;
    }
  }

  const int wr = (wave >> 1) * (BM / 2), wc = (wave & 1) * 128;
  const int kch = (int)(a.ld_bytes / T::CHB);
  const int total = ntiles * kch;
  const uint32_t ld = (uint32_t)a.ld_bytes;
  const int l32 = lane & 31, half = lane >> 5;
  const int64_t rrel0 = row0 - a.r0;
  // one descriptor over the whole operand (its size is below 4 GiB)
  const i32x4 res = make_res(a.Xs, (uint64_t)a.npad * ld);
  const int voff = (wave * T::RPL + lane / T::P) * (int)ld + (((lane % T::P) ^ T::swz(lane / T::P)) << 4);
  const uint32_t roff0 = (uint32_t)row0 * ld;
  const uint32_t step = (uint32_t)(4 * T::RPL) * ld;

  f32x16 acc[4][RBW];

  // Ring: chunk g of the piece (tile g / kch, chunk g % kch of the feature
  // dimension) lands in stage g % NSTAGE.  issue() sends the next
  // chunk (tile pt, chunk pc) to stage ps; past the piece's last chunk it
  // sends the last chunk again (into a stage no live chunk uses), so every
  // step has the same number of loads in flight behind it.
  int pt = 0, pc = 0, ps = 0;
  const int last_g = total > 0 ? total - 1 : 0;
  const int last_t = last_g / kch, last_c = last_g - last_t * kch;
  auto issue = [&]() {
    issue_chunk<BMT>(smem + ps * STAGE, res, voff, roff0 + (uint32_t)(pc * T::CHB),
                     (uint32_t)(sc0 + (int64_t)pt * BN) * ld + (uint32_t)(pc * T::CHB), step, wave);
    ps = ps + 1 == NSTAGE ? 0 : ps + 1;
    const bool at_end = pt == last_t && pc == last_c;
    const int npc = pc + 1 == kch ? 0 : pc + 1;
    const int npt = pc + 1 == kch ? pt + 1 : pt;
    pc = at_end ? pc : npc;
    pt = at_end ? pt : npt;
  };

  constexpr int NSTEP = steps_per_chunk<PREC, BMT>();
  Frag<PREC, RBW> f[2];
  // The vector-memory counter also counts the epilogue's candidate stores
  // and the column-data loads.  Loads return in the order they were issued,
  // so once at most the (NSTAGE - 2) * DMA ops issued after chunk g + 1's
  // loads are pending, chunk g + 1 has landed whatever else was issued in
  // between (other ops only make the wait longer).
  if (total > 0) {
#pragma unroll
    for (int i = 0; i < NSTAGE; ++i) issue();
    __builtin_amdgcn_s_waitcnt(waitcnt_vm((NSTAGE - 1) * DMA));
    asm volatile("s_barrier" ::: "memory");
    frag_load<PREC, BMT>(f[0], smem, 0, wr, wc, lane);
  }

  int g = 0, gs = 0;  // chunk being multiplied and its stage
  for (int tile = 0; tile < ntiles; ++tile) {
    const int64_t ct0 = sc0 + (int64_t)tile * BN;
#pragma unroll
    for (int cb = 0; cb < 4; ++cb)
#pragma unroll
      for (int rb2 = 0; rb2 < RBW; ++rb2)
#pragma unroll
        for (int i = 0; i < 16; ++i) acc[cb][rb2][i] = 0.f;
    for (int ch = 0; ch < kch; ++ch, ++g) {
      const uint8_t* S = smem + gs * STAGE;
      const int gn = gs + 1 == NSTAGE ? 0 : gs + 1;
#pragma unroll
      for (int q = 0; q < NSTEP; ++q) {
        if (q + 1 < NSTEP) {
          frag_load<PREC, BMT>(f[(q + 1) & 1], S, q + 1, wr, wc, lane);
        } else {
          // Every fragment of chunk g has reached the registers (lgkmcnt
          // 0), and chunk g + 1 has landed once at most the loads of the
          // NSTAGE - 2 chunks issued after it are pending; the barrier then
          // makes chunk g + 1 visible and frees
          // stage gs, which receives chunk g + NSTAGE while the last step's
          // MFMAs run.
          __builtin_amdgcn_s_waitcnt(waitcnt_vm_lgkm0((NSTAGE - 2) * DMA));
          asm volatile("s_barrier" ::: "memory");
          if (ch == 0) {
            // Column data of this tile for the epilogue (every wave is past
            // the previous epilogue), copied into LDS ahead of chunk
            // g + NSTAGE: the ring wait that guarantees that chunk at step
            // NSTAGE - 1 of the tile guarantees these too, and no register
            // waits for them (a register load would make the epilogue wait
            // for every load in flight).  One 1 KB load per array; the
            // shared thresholds in 256-byte pieces.
            // (reads past an array's end return zero; the byte offsets are
            // in the per-lane offset, which the descriptor's range checks;
            // the norms and scales have npad entries, a multiple of 128)
            const int cv = (int)(ct0 * 4) + lane * 16;
            if (wave == 0) {
              gcr_buffer_load_lds(make_res(a.n2, (uint64_t)a.npad * 4), (lds_u32_ptr)col_n2, 16, cv, 0, 0, 0);
            } else if (wave == 1) {
              // (arrays that may end at column c1: 4-byte loads, so the range
              // check drops exactly the columns past it)
              const int cw = (int)(ct0 * 4) + lane * 4;
              if (a.filt.stamp_of) {
                const i32x4 rs = make_res(a.filt.stamp_of, (uint64_t)a.c1 * 4);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  gcr_buffer_load_lds(rs, (lds_u32_ptr)(col_stamp + 64 * i), 4, cw + 256 * i, 0, 0, 0);
              }
              if (NL > 1 && a.cam) {
                const i32x4 rc = make_res(a.cam, (uint64_t)a.c1 * 4);
#pragma unroll
                for (int i = 0; i < 4; ++i)
                  gcr_buffer_load_lds(rc, (lds_u32_ptr)(col_cam + 64 * i), 4, cw + 256 * i, 0, 0, 0);
              }
            } else if (wave == 2) {
              if (PREC == GCR_PREC_FP8)
                gcr_buffer_load_lds(make_res(a.scale, (uint64_t)a.npad * 4), (lds_u32_ptr)col_sc, 16, cv, 0, 0, 0);
            } else if (a.thr_shared) {
              const i32x4 rt = make_res(a.thr_shared, (uint64_t)(a.r1 - a.r0) * NL * 4);
#pragma unroll
              for (int i = 0; i < BM * NL / 64; ++i)
                gcr_buffer_load_lds(rt, (lds_u32_ptr)(sh_thr + 64 * i), 4, (int)((rrel0 * NL + 64 * i + lane) * 4), 0, 0, 0);
            }
          }
          issue();
          frag_load<PREC, BMT>(f[(q + 1) & 1], smem + gn * STAGE, 0, wr, wc, lane);
        }
        frag_mma<PREC>(f[q & 1], acc);
      }
      gs = gn;
    }

    // ---------------- epilogue of one tile ----------------
    // (with fewer than NSTAGE chunks per tile the column data may still be
    // in flight)
    if (kch < NSTAGE) {
      __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
      __syncthreads();
    }
    // padding columns and left-out columns get an infinite norm
    if (ct0 + tid >= sc1 || (a.filt.stamp_of && col_stamp[tid] == a.filt.stamp)) col_n2[tid] = INFINITY;
    // adopt the row's threshold published by the other splits of the row
    // (every split's k-th key + 2E bounds the row's k-th key + 2E from above;
    // all ones: none yet)
    if (a.thr_shared) {
#pragma unroll
      for (int j = 0; j < SH; ++j) {
        const int e = tid + NT * j;  // (row, list) = (e / NL, e % NL)
        if (e < BM * NL && row0 + e / NL < a.r1 && sh_thr[e] != 0xffffffffu) {
          float& t = row_thr[e % NL][e / NL];
          t = fminf(t, unord_f32(sh_thr[e]));
        }
      }
    }
    // (a plain barrier after this wave's LDS writes: a full __syncthreads
    // would also wait for the next chunks' loads, which write LDS)
    __builtin_amdgcn_s_waitcnt(waitcnt_lgkm0);
    asm volatile("s_barrier" ::: "memory");
    // every wave read the flag of tile - 1 before this barrier; it is the
    // flag the next tile sets
    if (ROOM && tid == 0) room_flag[(tile + 1) & 1] = 0;

    // Admission.  A lane's entries come in blocks of 16 (one row, 16
    // columns); a block whose lower bound n2_min - 2 s_max is above the row's
    // threshold admits nothing and is dismissed with one max per entry.  The
    // other blocks are screened entry by entry (one multiply-add and one
    // compare against the row's threshold and, for the cross list, its
    // camera), and passing entries are appended at once (one LDS atomic per
    // block and list reserves the slots).
    // 128-row tiles screen a passing block in the lane that holds it (the
    // whole wave runs that path when one lane needs it); an entry that finds
    // its buffer full is marked in the lane's lost mask, then the full
    // buffers are compacted (lower thresholds) and only the lost entries are
    // screened again, until none is left.  256-row tiles keep room for a
    // whole tile in every buffer, and the lanes whose block passes push its
    // 16 accumulators to a queue of the wave in LDS; the queue is then
    // screened one block per lane, so a tile in which a few lanes of the
    // wave pass costs one screening pass instead of one per passing block.
    {
      int lc0 = wc + 4 * half;
      asm volatile("" : "+v"(lc0));
      const uint32_t cbase = (uint32_t)(ct0 - a.c0);
      uint64_t lost[RBW][NL];
      bool near_full = false;  // room scheme: an admission of this lane passed C - BN
      // smallest squared norm among the 16 columns of each of the lane's
      // column blocks (padding and left-out columns carry +inf)
      float n2min[4];
#pragma unroll
      for (int cb = 0; cb < 4; ++cb) {
        float m = INFINITY;
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const f32x4 v = *(const f32x4*)&col_n2[lc0 + 32 * cb + 8 * g];
          m = fminf(m, fminf(fminf(v.x, v.y), fminf(v.z, v.w)));
        }
        n2min[cb] = m;
      }
      if constexpr (ROOM) {
        static_assert(NL == 1 && PREC != GCR_PREC_FP8, "the queue scheme screens one list of float32/BF16 keys");
        float* qv = reinterpret_cast<float*>(smem + T::SMEM) + wave * (64 * 16);
        int* qm = reinterpret_cast<int*>(smem + T::SMEM + NT * 16 * 4) + wave * 64;
        float thr[RBW];
#pragma unroll
        for (int rb2 = 0; rb2 < RBW; ++rb2) thr[rb2] = fminf(row_thr[0][wr + 32 * rb2 + l32], 3.40282347e38f);
        // blocks still to be queued (wave-uniform): a block that does not
        // fit in the 64 free slots of this pass waits for the next pass
        uint32_t todo = (1u << (4 * RBW)) - 1u;
        while (todo) {
          int qn = 0;
          uint32_t next = 0u;
#pragma unroll
          for (int rb2 = 0; rb2 < RBW; ++rb2) {
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
              const int blk = 4 * rb2 + cb;
              if (!(todo & (1u << blk))) continue;
              asm volatile("" : "+a"(acc[cb][rb2]));
              float smax = acc[cb][rb2][0];
#pragma unroll
              for (int i = 1; i < 16; ++i) smax = fmaxf(smax, acc[cb][rb2][i]);
              const bool pass = fmaf(-2.0f, smax, n2min[cb]) <= thr[rb2];
              const uint64_t b = __ballot(pass);
              if (b == 0ull) continue;
              const int nb = __popcll(b);
              if (qn + nb > 64) {
                next |= 1u << blk;
                continue;
              }
              if (pass) {
                const int slot =
                    qn + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
                f32x4* d = reinterpret_cast<f32x4*>(qv + slot * 16);
#pragma unroll
                for (int g = 0; g < 4; ++g)
                  d[g] = f32x4{acc[cb][rb2][4 * g], acc[cb][rb2][4 * g + 1], acc[cb][rb2][4 * g + 2],
                               acc[cb][rb2][4 * g + 3]};
                qm[slot] = rb2 | (cb << 2) | (lane << 4);
              }
              // (qn and todo are wave-uniform; readfirstlane keeps them in
              // scalar registers, so the tests above are scalar branches)
              qn = __builtin_amdgcn_readfirstlane(qn + nb);
            }
          }
          todo = __builtin_amdgcn_readfirstlane(next);
          // (LDS operations of one wave complete in order: the reads below
          // see this pass's queue)
          if (lane < qn) {
            const int meta = qm[lane];
            const int rb2 = meta & 3, cb = (meta >> 2) & 3, sl = meta >> 4;
            const int lr = wr + 32 * rb2 + (sl & 31);
            // entry 4 g + j of the block holds column lcb + 8 g + j of the tile
            const int lcb = wc + 4 * (sl >> 5) + 32 * cb;
            const float t = fminf(row_thr[0][lr], 3.40282347e38f);
            const f32x4* src = reinterpret_cast<const f32x4*>(qv + lane * 16);
            float keys[16];
            uint32_t m = 0u;
#pragma unroll
            for (int g = 0; g < 4; ++g) {
              const f32x4 sv = src[g];
              const f32x4 nv = *(const f32x4*)&col_n2[lcb + 8 * g];
#pragma unroll
              for (int j = 0; j < 4; ++j) {
                keys[4 * g + j] = fmaf(-2.0f, sv[j], nv[j]);
                if (keys[4 * g + j] <= t) m |= 1u << (4 * g + j);
              }
            }
            const int64_t ds = row0 + lr - ct0 - lcb;  // the row's own column, relative to the block
            if (a.exclude_self && ds >= 0 && ds < 32 && (ds & 4) == 0)
              m &= ~(1u << (4 * (int)(ds >> 3) + (int)(ds & 3)));
            if (a.filt.row_mark) {
#pragma unroll
              for (int i = 0; i < 16; ++i)
                if (row_out(row_mk[lr], row_stp[lr], ct0 + lcb + 8 * (i >> 2) + (i & 3))) m &= ~(1u << i);
            }
            if (m != 0u) {
              const int nm = __popc(m);
              const int pos = lds_fetch_add(&row_cnt[0][lr], nm);
              near_full |= pos + nm > a.C - BN;
              uint64_t* buf = a.cand + ((rrel0 + lr) * NL * (int64_t)a.S + cs) * a.C;
              const uint32_t cbv = cbase + (uint32_t)lcb;
              // store step j writes each lane's j-th admitted entry (its key
              // recomputed from the queued accumulator), so a pass issues as
              // many store instructions as the most entries one lane admits
              // rather than one per entry index that some lane admits
              uint32_t mm = m;
              for (int q = pos; mm != 0u; ++q) {
                const int i = __builtin_ctz(mm);
                mm &= mm - 1u;
                const int lc = lcb + 8 * (i >> 2) + (i & 3);
                const float key = fmaf(-2.0f, qv[lane * 16 + i], col_n2[lc]);
                if (q < a.C) buf[q] = pack_cand(key, cbase + (uint32_t)lc);
              }
            }
          }
        }
      } else
#pragma unroll
      for (int rb2 = 0; rb2 < RBW; ++rb2) {
        const int lr = wr + 32 * rb2 + l32;
        // thresholds clamped to the largest finite float: ineligible entries
        // (padding columns, the row itself) carry an infinite key and are
        // never admitted, not even under an infinite threshold; rows past
        // the range have -inf thresholds
        const float t0 = fminf(row_thr[0][lr], 3.40282347e38f);
        const float t1 = NL > 1 ? fminf(row_thr[NL - 1][lr], 3.40282347e38f) : -INFINITY;
        const float rs = row_sc[lr];
        const int rc = row_cam[lr];
        // the row's own column in this tile, if it is left out (its key is
        // the smallest of the row, so its block always reaches the
        // per-entry test below)
        const int64_t selfc64 = row0 + lr - ct0;
        const int selfc = (a.exclude_self && selfc64 >= 0 && selfc64 < BN) ? (int)selfc64 : -1;
        uint64_t* buf0 = a.cand + (((rrel0 + lr) * NL) * (int64_t)a.S + cs) * a.C;
        uint64_t* buf1 = a.cand + (((rrel0 + lr) * NL + NL - 1) * (int64_t)a.S + cs) * a.C;
#pragma unroll
        for (int L = 0; L < NL; ++L) lost[rb2][L] = 0ull;
        // either list admits an entry only if its key is <= the larger of
        // the two thresholds: a block of 16 entries whose smallest key is
        // above it (nearly every block once the thresholds are tight) is
        // dismissed with one compare
        const float tmax = NL > 1 ? fmaxf(t0, t1) : t0;
#pragma unroll
        for (int cb = 0; cb < 4; ++cb) {
          // the block's accumulators are read here and not earlier (an
          // early copy of all of them would not fit in the registers)
          asm volatile("" : "+a"(acc[cb][rb2]));
          if constexpr (PREC != GCR_PREC_FP8) {
            // n2_min - 2 s_max bounds every key of the block from below
            // (fma with one rounding is monotone in both operands), so a
            // block whose bound is above the threshold admits nothing: one
            // max per entry instead of a key and a min
            float smax = acc[cb][rb2][0];
#pragma unroll
            for (int i = 1; i < 16; ++i) smax = fmaxf(smax, acc[cb][rb2][i]);
            if (!(fmaf(-2.0f, smax, n2min[cb]) <= tmax)) continue;
          }
          f32x4 n2v[4], scv[4];
#pragma unroll
          for (int g = 0; g < 4; ++g) {
            const int c4 = lc0 + 32 * cb + 8 * g;
            n2v[g] = *(const f32x4*)&col_n2[c4];
            if (PREC == GCR_PREC_FP8) scv[g] = *(const f32x4*)&col_sc[c4];
          }
          float keys[16];
          float kmin = INFINITY;
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            float sv = acc[cb][rb2][i];
            if (PREC == GCR_PREC_FP8) sv = sv * (rs * scv[i >> 2][i & 3]);
            // n2 - 2 s with one rounding (2 s is exact)
            keys[i] = fmaf(-2.0f, sv, n2v[i >> 2][i & 3]);
            kmin = fminf(kmin, keys[i]);
          }
          if (PREC == GCR_PREC_FP8 && !(kmin <= tmax)) continue;
          i32x4 camv[4];
          if (NL > 1) {
#pragma unroll
            for (int g = 0; g < 4; ++g) camv[g] = *(const i32x4*)&col_cam[lc0 + 32 * cb + 8 * g];
          }
          // the block's admissions to each list as a 16-bit mask; one LDS
          // atomic per list reserves their slots, which they take in order
          uint32_t m0 = 0, m1 = 0;
#pragma unroll
          for (int i = 0; i < 16; ++i) {
            if (keys[i] <= t0) m0 |= 1u << i;
            if (NL > 1 && camv[i >> 2][i & 3] != rc && keys[i] <= t1) m1 |= 1u << i;
          }
          // the row's own column (entry 4 g + j holds column lc0 + 32 cb + 8 g + j)
          const int ds = selfc - (lc0 + 32 * cb);
          if (ds >= 0 && ds < 32 && (ds & 4) == 0) {
            const uint32_t keep = ~(1u << (4 * (ds >> 3) + (ds & 3)));
            m0 &= keep;
            m1 &= keep;
          }
          if (a.filt.row_mark) {
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              if (row_out(row_mk[lr], row_stp[lr], ct0 + lc0 + 32 * cb + 8 * (i >> 2) + (i & 3))) {
                m0 &= ~(1u << i);
                m1 &= ~(1u << i);
              }
            }
          }
#pragma unroll
          for (int L = 0; L < NL; ++L) {
            const uint32_t m = L == 0 ? m0 : m1;
            if (m == 0u) continue;
            const int nm = __popc(m);
            const int pos = lds_fetch_add(&row_cnt[L][lr], nm);
            uint64_t* buf = L == 0 ? buf0 : buf1;
            // (the entries are packed after the atomic returns, not before it
            // with sixteen more registers live)
            uint32_t cbv = cbase + (uint32_t)(lc0 + 32 * cb);
            asm volatile("" : "+v"(cbv) : "v"(pos));
#pragma unroll
            for (int i = 0; i < 16; ++i) {
              if (m & (1u << i)) {
                const int q = pos + __popc(m & ((1u << i) - 1u));
                if (q < a.C) buf[q] = pack_cand(keys[i], cbv + (uint32_t)(8 * (i >> 2) + (i & 3)));
                else lost[rb2][L] |= 1ull << (cb * 16 + i);
              }
            }
          }
        }
      }
      if constexpr (ROOM) {
        // Room scheme: every buffer entered this tile with at least BN free
        // slots (a row gets at most BN entries per list per tile), so no
        // entry was lost.  Buffers past C - BN entries are compacted for the
        // next tile, and at the first tile every buffer with k entries, to
        // set its threshold; the next epilogue's barrier orders this before
        // its admissions.
        if (__any(near_full) && lane == 0) room_flag[tile & 1] = 1;
        __syncthreads();
        // (rows are scanned only at the first tile and when an admission of
        // this tile reached past C - BN)
        const bool scan = tile == 0 || room_flag[tile & 1];
        for (int q = wave; scan && q < NL * BM; q += NT / 64) {
          const int L = q / BM, lr = q - L * BM;
          const int kk = L == 0 ? a.k0 : a.k1;
          const int n = row_cnt[L][lr];
          if (kk > 0 && (n > a.C - BN || (tile == 0 && n >= kk))) {
            uint64_t* base = a.cand + (((rrel0 + lr) * NL + L) * (int64_t)a.S + cs) * a.C;
            compact_row<E>(base, &row_cnt[L][lr], &row_thr[L][lr], a.C, kk, row_twoE[lr], BN);
            if (a.thr_shared && lane == 0)
              atomicMin(&a.thr_shared[(rrel0 + lr) * NL + L], ord_f32(row_thr[L][lr]));
          }
        }
      } else
      for (int it = 0;; ++it) {
        bool left = false;
#pragma unroll
        for (int rb2 = 0; rb2 < RBW; ++rb2)
#pragma unroll
          for (int L = 0; L < NL; ++L) left |= lost[rb2][L] != 0ull;
        if (__any(left) && lane == 0) any_flag[it & 1] = 1;
        __syncthreads();
        const int more = any_flag[it & 1];
        if (tid == 0) any_flag[(it + 1) & 1] = 0;
        if (!more) break;
          // compact the full buffers (a count past C counts lost entries too)
        for (int q = wave; q < NL * BM; q += NT / 64) {
          const int L = q / BM, lr = q - L * BM;
          if (row_cnt[L][lr] >= a.C) {
            uint64_t* base = a.cand + (((rrel0 + lr) * NL + L) * (int64_t)a.S + cs) * a.C;
            compact_row<E>(base, &row_cnt[L][lr], &row_thr[L][lr], a.C, L == 0 ? a.k0 : a.k1, row_twoE[lr], 16);
            if (a.thr_shared && lane == 0)
              atomicMin(&a.thr_shared[(rrel0 + lr) * NL + L], ord_f32(row_thr[L][lr]));
          }
        }
        __syncthreads();
        // the lost entries against the lowered thresholds
#pragma unroll
        for (int rb2 = 0; rb2 < RBW; ++rb2) {
          const int lr = wr + 32 * rb2 + l32;
          const float rs = row_sc[lr];
#pragma unroll
          for (int L = 0; L < NL; ++L) {
            uint64_t m = lost[rb2][L];
            if (m == 0ull) continue;
            const float t = row_thr[L][lr];
            uint64_t* buf = a.cand + (((rrel0 + lr) * NL + L) * (int64_t)a.S + cs) * a.C;
#pragma unroll
            for (int cb = 0; cb < 4; ++cb) {
#pragma unroll
              for (int i = 0; i < 16; ++i) {
                const uint64_t bit = 1ull << (cb * 16 + i);
                if (m & bit) {
                  const int lc = lc0 + 32 * cb + 8 * (i >> 2) + (i & 3);
                  float sv = acc[cb][rb2][i];
                  if (PREC == GCR_PREC_FP8) sv = sv * (rs * col_sc[lc]);
                  const float key = fmaf(-2.0f, sv, col_n2[lc]);
                  if (!(key <= t)) {
                    m &= ~bit;
                  } else {
                    const int pos = atomicAdd(&row_cnt[L][lr], 1);
                    if (pos < a.C) {
                      buf[pos] = pack_cand(key, cbase + (uint32_t)lc);
                      m &= ~bit;
                    }
                  }
                }
              }
            }
            lost[rb2][L] = m;
          }
        }
      }
    }
    if (!ROOM && tile == 0) {
      // set every row's threshold from its first tile instead of waiting
      // for its buffer to fill
      for (int q = wave; q < NL * BM; q += NT / 64) {
        const int L = q / BM, lr = q - L * BM;
        const int kk = L == 0 ? a.k0 : a.k1;
        if (kk > 0 && row_cnt[L][lr] >= kk) {
          uint64_t* base = a.cand + (((rrel0 + lr) * NL + L) * (int64_t)a.S + cs) * a.C;
          compact_row<E>(base, &row_cnt[L][lr], &row_thr[L][lr], a.C, kk, row_twoE[lr], 16);
          if (a.thr_shared && lane == 0)
            atomicMin(&a.thr_shared[(rrel0 + lr) * NL + L], ord_f32(row_thr[L][lr]));
        }
      }
      __syncthreads();
    }
  }
  // the loads of the chunks past the end are still landing in the ring
  __builtin_amdgcn_s_waitcnt(waitcnt_vm(0));
  __syncthreads();
  for (int t = tid; t < BM * NL; t += NT) {
    const int L = t / BM, lr = t - L * BM;
    if (row0 + lr < a.r1) {
      const int64_t o = ((rrel0 + lr) * NL + L) * (int64_t)a.S + cs;
      a.cnt[o] = min(row_cnt[L][lr], a.C);
      a.thr[o] = row_thr[L][lr];
    }
  }
  }  // pieces
}

template <int PREC, int NL, int E, int BMT>
static void launch_one(const SimArgs& a, hipStream_t st) {
  const dim3 grid(a.balanced ? a.grid : sim_topk_grid(a.RB, a.S)), block(NT);
  auto k = sim_topk_kernel<PREC, NL, E, BMT>;
  (void)hipFuncSetAttribute((const void*)k, hipFuncAttributeMaxDynamicSharedMemorySize, Tile<BMT>::DSMEM);
  hipLaunchKernelGGL(k, grid, block, Tile<BMT>::DSMEM, st, a);
}

template <int PREC, int NL, int BMT>
static void launch_prec_nl(const SimArgs& a, hipStream_t st) {
  if (a.C <= 64) launch_one<PREC, NL, 1, BMT>(a, st);
  else if (a.C <= 128) launch_one<PREC, NL, 2, BMT>(a, st);
  else if (a.C <= 256) launch_one<PREC, NL, 4, BMT>(a, st);
  else launch_one<PREC, NL, 8, BMT>(a, st);
}

template <int PREC, int BMT>
static void launch_prec(int nl, const SimArgs& a, hipStream_t st) {
  if (nl == 1) launch_prec_nl<PREC, 1, BMT>(a, st);
  else launch_prec_nl<PREC, 2, BMT>(a, st);
}

// 256-row tiles exist for float32 and BF16 screening of one list (the FP8
// fragments and a second list's state do not fit beside the 256
// accumulators of a 128 x 128 wave tile).
int sim_topk_large_tile(int prec, int nl) { return prec != GCR_PREC_FP8 && nl == 1; }

void launch_sim_topk(int prec, int nl, const SimArgs& a, hipStream_t st) {
  const bool big = a.bm == 256 && sim_topk_large_tile(prec, nl);
  if (prec == GCR_PREC_FP32) {
    if (big) launch_prec_nl<GCR_PREC_FP32, 1, 256>(a, st); else launch_prec<GCR_PREC_FP32, 128>(nl, a, st);
  } else if (prec == GCR_PREC_BF16) {
    if (big) launch_prec_nl<GCR_PREC_BF16, 1, 256>(a, st); else launch_prec<GCR_PREC_BF16, 128>(nl, a, st);
  } else {
    launch_prec<GCR_PREC_FP8, 128>(nl, a, st);
  }
}

}  // namespace gcr
