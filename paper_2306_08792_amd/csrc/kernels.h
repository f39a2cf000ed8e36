// Internal launchers shared between the kernel files and the C ABI layer.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "common.h"

#define GCR_PREC_FP32 0
#define GCR_PREC_BF16 1
#define GCR_PREC_FP8 2

namespace gcr {

// ---- prep.hip
void launch_normalize_rows(const float* X, float* Y, int64_t n, int d, hipStream_t st);
// Rows [r0, r0 + nmax) of X (only the first *count when count != nullptr)
// into the operand rows of the same index; maxima into maxn2_bits.
void launch_screen_prep_rows(int prec, const float* X, int64_t r0, int64_t nmax, const int* count, int d, void* Xs,
                             int64_t ld_bytes, float* n2, float* scale, float* rn, unsigned* maxn2_bits,
                             hipStream_t st);
// maxn2_bits[0], [1]: maxima of n2 and rn (zero before the launch)
void launch_screen_prep(int prec, const float* X, int64_t n, int d, int64_t npad, void* Xs,
                        int64_t ld_bytes, float* n2, float* scale, float* rn, unsigned* maxn2_bits,
                        hipStream_t st);

// Columns of [c0, c1) excluded from a search: column c is out when
// stamp_of[c] == stamp (a per-request mark array), or when c - c0 is at or
// past *count (a column count known only on the device).
struct ColumnFilter {
  const uint32_t* stamp_of = nullptr;
  uint32_t stamp = 0;
  const int* count = nullptr;
  // per-row masks: row r of the search (relative to its first row) leaves
  // out column c when row_mark[r] is set and row_mark[r][c] == row_stamp[r]
  // (rows of different serving requests in one batch skip different rows)
  const uint32_t* const* row_mark = nullptr;
  const uint32_t* row_stamp = nullptr;
};
__device__ __forceinline__ bool column_out(const ColumnFilter& f, int64_t c, int64_t c0, int64_t rrel) {
  if ((f.stamp_of && f.stamp_of[c] == f.stamp) || (f.count && c - c0 >= (int64_t)*f.count)) return true;
  if (f.row_mark) {
    const uint32_t* m = f.row_mark[rrel];
    if (m && m[c] == f.row_stamp[rrel]) return true;
  }
  return false;
}

// ---- simtopk.hip : fused MFMA similarity tiles + streaming per-row top-k
struct SimArgs {
  const uint8_t* Xs;  // screening operand, [npad, ld_bytes]
  int64_t npad;       // rows of Xs (reads beyond return zero)
  int64_t ld_bytes;   // multiple of 128
  const float* n2;    // [npad]
  const float* scale; // [npad] FP8 row scales or nullptr
  const int* cam;     // [n] or nullptr
  const float* rn;    // [npad] quantisation residual norms
  const float* maxn2; // device [max n2, max rn]
  int64_t r0, r1;     // rows [r0, r1)
  int64_t c0, c1;     // columns [c0, c1)
  int64_t W;          // split width (multiple of the 256-column tile)
  int S;              // number of column splits (multiple of 8)
  int RB;             // row blocks of bm rows
  int bm = 128;       // rows per workgroup tile: 128, or 256 (see sim_topk_large_tile)
  int exclude_self;   // skip column == row
  int k0, k1;         // list sizes (global, cross)
  int C;              // candidate capacity per (row, list, split)
  float eps_s, eps_n; // accumulation / squared-norm error coefficients
  uint64_t* cand;     // [(r1-r0), NL, S, C]
  const float* thr_init;  // [(r1-r0), NL] initial admission thresholds or nullptr
  int* cnt;           // [(r1-r0), NL, S] entries kept
  float* thr;         // [(r1-r0), NL, S] final admission threshold: the buffer
                      // holds every item of the split with key <= thr
  ColumnFilter filt;  // columns left out of the search
  unsigned* thr_shared = nullptr;  // [(r1-r0), NL] ordered-bits admission thresholds shared by
                                   // the splits of a row (all ones = none yet), or nullptr
  int balanced = 0;   // balanced schedule (S = most pieces of a row block)
  int grid = 0;       // balanced: workgroups
  int ntr = 0;        // balanced: 256-column tiles per row
  int64_t total_tiles = 0;  // balanced: RB * ntr
};
int sim_topk_grid(int RB, int S);
int sim_topk_balanced_splits(int64_t rows, int64_t ncols, int G, int bm);
// Whether the 256-row workgroup tile exists for a screening precision and
// number of lists.
int sim_topk_large_tile(int prec, int nl);
// Initial admission thresholds from earlier neighbour lists (any k items give
// an upper bound on the k-th distance): out[row * nl + L].
void launch_seed_thresholds(const float* X, int d, int64_t n, const int32_t* idx0, int k0, const int32_t* idx1,
                            int k1, const float* n2, const float* rn, const float* maxn2, float eps_s,
                            float eps_n, float* out, const int32_t* order, hipStream_t st);
int sim_topk_tile_cols();
// The same bounds from a BF16 screening operand with ld in {1024, 2048,
// 4096} bytes (its rows zero past d).
void launch_seed_thresholds_bf16(const uint8_t* Xs, int64_t ld, int64_t n, const int32_t* idx0, int k0,
                                 const int32_t* idx1, int k1, const float* n2, const float* rn, const float* maxn2,
                                 float eps_s, float eps_n, float* out, const int32_t* order, hipStream_t st);
void launch_sim_topk(int prec, int nl, const SimArgs& a, hipStream_t st);

// ---- refine.hip : union of split candidates, exact re-score, selection
struct RefineArgs {
  const uint64_t* cand;
  const int* cnt;
  const float* thr;
  int S, C, NL;
  int k0, k1;
  int64_t r0, r1, c0, c1;
  int exclude_self;
  const float* X;     // [n, d] float32 features (exact re-score)
  int d;
  const int* cam;
  const float* n2;
  const float* rn;
  const float* maxn2;
  float eps_s, eps_n;
  int32_t* idx0; float* dist0;   // [(r1-r0), k0]
  int32_t* idx1; float* dist1;   // [(r1-r0), k1] (cross list) or nullptr
  int* fb_list;       // [(r1-r0) * NL] packed (row_rel * 2 + list)
  int* fb_count;      // device counter
  unsigned long long* stat_cands;  // device counter
  uint64_t* fb_scratch;            // [fb_grid, c1 - c0]
  int fb_grid;
  int fb_max;                      // pairs taken by the column-chunked path
  uint64_t* fb_part_key;           // [min(fb_max, pairs), chunks, k] chunk winners
  uint32_t* fb_part_col;
  float* fb_cut;      // [(r1-r0) * NL] upper bound on the exact k-th key of queued pair f
  float eps32;        // screening coefficient of the float32 band sweep
  const int32_t* order;  // processing order of the rows [0, n) (r0 == 0) or nullptr
  uint64_t* band;     // [band_max, band_cap] (key32, column) of the swept band
  int* band_cnt;      // [band_max] zero before the launch
  int band_cap, band_max;
  int* ovf_list;      // [(r1-r0) * NL] pairs for the exhaustive path
  int* ovf_count;     // device counter, zero before the launch
  int* heavy_list;    // [(r1-r0) * NL] pairs for the block refine kernel
  int* heavy_count;   // device counter, zero before the launch
  ColumnFilter filt;  // columns left out of the search
};
// Merge of groups of GS consecutive split buffers into one buffer each
// (S / GS splits out), keeping every item within reach of the exact top-k.
struct MergeArgs {
  const uint64_t* cand; const int* cnt; const float* thr;  // [rows, NL, S, C]
  int64_t rows, r0; int NL, S, GS, C, k0, k1;
  const float* n2; const float* rn; const float* maxn2; float eps_s, eps_n;
  uint64_t* out_cand; int* out_cnt; float* out_thr;        // [rows, NL, S / GS, C]
};
void launch_merge_splits(const MergeArgs& m, hipStream_t st);
// queued pairs handled by the column-parallel exhaustive path (batch calls)
constexpr int FB_MAX = 8192;
void launch_refine(const RefineArgs& a, hipStream_t st);
// k smallest screened keys per (row, list), no exact re-score (raw modes).
void launch_raw_select(const RefineArgs& a, hipStream_t st);

// ---- graph.hip : affinities, reverse CSR, degrees, normalised values
struct GraphBuildArgs {
  int64_t n; int k;
  const int32_t* idx; const float* dist;
  const int* cam; float beta_same, beta_cross; int use_beta;
  float gamma;
  float* w; int32_t* rev_ptr; int32_t* rev_src; float* rev_w; float* deg;
  float* pf; float* pr;
  float coef;          // alpha or 1 - alpha
  int32_t* tmp_cnt;    // [n]
  int32_t* tmp_blk;    // scan block sums
  int asym = 0;        // asymmetric normalisation: deg = row degrees, deg_c = column degrees
  float* deg_c = nullptr;
};
void launch_graph_build(const GraphBuildArgs& a, hipStream_t st);
void launch_self_coef(int64_t n, const float* deg, const float* deg_c, const float* cr_deg, const float* cr_deg_c,
                      float alpha, float* self, hipStream_t st);
void launch_finish_values(const GraphBuildArgs& a, hipStream_t st);
// Row processing order that keeps rows sharing neighbours together: rows
// sorted (counting sort) by the smallest index among themselves and their
// list members.  label: [n], cnt: [n + 1], blk: scan tile sums.
void launch_locality_order(int64_t n, const int32_t* idx, int k, int32_t* label, int32_t* cnt, int32_t* blk,
                           int32_t* order, hipStream_t st);
// The same order with labels taken from the screening candidate buffers of
// rows [0, n) (list 0, all splits): usable before the lists exist.
void launch_cand_order(int64_t n, const uint64_t* cand, const int32_t* ccnt, int S, int C, int NL, int32_t* label,
                       int32_t* cnt, int32_t* blk, int32_t* order, hipStream_t st);

// ---- propagate.hip
// DSFP (Alg. 1): one workgroup per node over its local set (the node and
// its distinct valid list entries).  Requires rounds >= 1, 0 <= k <=
// DSFP_K_MAX (the local matrices then fit 64 KB of LDS), d <= 2048, Y != X.
constexpr int DSFP_K_MAX = 59;
void launch_dsfp(const float* X, const int32_t* idx, int64_t n, int d, int k, float gamma, int rounds,
                 const int32_t* order, float* Y, hipStream_t st);

struct PropArgs {
  const float* X; float* Y; int64_t n; int d;
  const float* self;
  const int32_t* idx; const float* pf; int k;
  const int32_t* rev_ptr; const int32_t* rev_src; const float* pr;
  const int32_t* cr_idx; const float* cr_pf; int ck;
  const int32_t* cr_rev_ptr; const int32_t* cr_rev_src; const float* cr_pr;
  const int32_t* order;  // row processing order or nullptr
};
void launch_propagate(const PropArgs& a, hipStream_t st);

// ---- final.hip : dense squared distances between two row ranges
// Rewrites the float32 screening operand (rows x ld_bytes, ld_bytes a
// multiple of 128) in place into the split-bfloat16 form launch_dense_dist
// reads.
void launch_split_bf16(uint8_t* Xs, int64_t rows, int64_t ld_bytes, hipStream_t st);
void launch_dense_dist(const uint8_t* Xs, int64_t ld_bytes, int kchunks, const float* n2,
                       int64_t q0, int64_t nq, int64_t g0, int64_t ng, float* out,
                       hipStream_t st);

// ---- pvg.hip : tracklet profile vectors
void launch_segment_means(const float* frames, const int32_t* offsets, int nt, int d,
                          float* mu_c, hipStream_t st);
// scratch: group_mean_scratch_floats(d) floats
void launch_group_mean(const float* mu_c, const int32_t* offsets, const int32_t* members,
                       int nm, int d, int64_t nframes, float* scratch, float* mu, hipStream_t st);
int group_mean_scratch_floats(int d);
void launch_gram(const float* frames, const int32_t* rows, int64_t nrows, int d, float* partial,
                 int ksplit, float* G, float shift, hipStream_t st);
void launch_gemm_nn_f32(const float* A, int64_t lda, const float* B, int64_t ldb, float* Cm,
                        int64_t ldc, int M, int N, int K, float alpha, float beta,
                        const float* Cin, int64_t ldcin, hipStream_t st);
// out[0] = trace of the d x d Gram G minus d * shift (float64)
void launch_gram_trace(const float* G, int d, float shift, double* out, hipStream_t st);
void launch_build_rhs(const float* mu_c, const float* mu, const int32_t* members, int nm, int d,
                      float* B, hipStream_t st);
void launch_scatter_profiles(const float* Wt, const int32_t* members, int nm, int d, float* W,
                             hipStream_t st);
void launch_axpby(float* y, const float* x, float a, float b, int64_t n, hipStream_t st);
void launch_cheb_update(float* Wk, float* Wprev, const float* R, float rho, float cR, int64_t n,
                        hipStream_t st);

// ---- serve.hip : one request against a resident gallery
void launch_serve_query_edges(int b, int k, const int32_t* q_idx, const float* q_dist, float gamma, float* q_w,
                              float* Dq, uint64_t* keys, int P, hipStream_t st);
void launch_serve_sort_pairs(uint64_t* keys, int P, hipStream_t st);  // P: power of two <= 16,384
void launch_serve_touched(const uint64_t* keys, int npairs, const float* q_w, uint32_t stamp, uint32_t* touched,
                          float* dD, int32_t* seg_start, int32_t* seg_len, int32_t* T_list, int* T_count,
                          hipStream_t st);
void launch_serve_expand(const int32_t* src, const int* src_count, int src_cap, const int32_t* gidx, int k,
                         const int32_t* rev_ptr, const int32_t* rev_src, uint32_t stamp, uint32_t* mark,
                         int32_t* pos, int32_t* list, int* count, int cap, hipStream_t st);
struct ServePropArgs {
  int d, k, b;
  const float* Xprev; float* Xcur;    // level t - 1 and t feature arrays
  int64_t qbase, pbase;               // slot rows: queries, recomputed gallery rows
  const int32_t* gidx; const float* gw;                    // gallery forward lists [G, k]
  const int32_t* rev_ptr; const int32_t* rev_src; const float* rev_w;
  const float* D0;                    // gallery degrees without queries
  uint32_t stamp;
  const uint32_t* touched; const float* dD; const int32_t* seg_start; const int32_t* seg_len;
  const uint64_t* pair_keys;          // sorted (gallery item, query edge) pairs
  const int32_t* q_idx; const float* q_w; const float* Dq;
  const uint32_t* prev_mark; const int32_t* prev_pos;      // set of round t - 1 (nullptr at t = 1)
  const int32_t* cur_list; const int32_t* cur_pos; const int* cur_count; int cap;
};
void launch_serve_propagate(const ServePropArgs& a, hipStream_t st);
void launch_serve_merge(int b, int K, const int32_t* ia, const float* da, const int32_t* ib, const float* db,
                        const int32_t* list, int32_t* oi, float* od, hipStream_t st);
// Gallery list maintenance (exact under inserts and removals).
// Merge each of `rows` lists [rows, k] with its m nearest appended items
// (indices + col_offset), keeping the k smallest by (distance, index);
// float32 ties between the two sides are decided by float64 distances from
// the gallery features X [*, d].
void launch_merge_appended(int64_t rows, int k, int32_t* idx, float* dist, int m, const int32_t* nidx,
                           const float* ndist, int32_t col_offset, const float* X, int d, hipStream_t st);
// Lists of the surviving rows renumbered by new_of_old (-1: removed) into
// distinct buffers; rows that lost a neighbour are appended to repair.
void launch_relabel_lists(int64_t rows_old, int k, const int32_t* new_of_old, const int32_t* idx_old,
                          const float* dist_old, int32_t* idx_new, float* dist_new, int32_t* repair,
                          int* repair_count, hipStream_t st);
// dst[r] = src[src_row[r]] (float rows of width d; dst distinct from src).
void launch_gather_rows(const float* src, float* dst, const int32_t* src_row, int64_t rows, int d, hipStream_t st);
// k + 1 nearest items of row self_row[t] (itself included) -> its k nearest
// other items, written to row self_row[t] of idx_out / dist_out.
void launch_drop_self(int64_t rows, int k, const int32_t* self_row, const int32_t* idx_in, const float* dist_in,
                      int32_t* idx_out, float* dist_out, hipStream_t st);
void launch_bf16_to_f32(const uint16_t* in, float* out, int64_t n, hipStream_t st);
void launch_copy_u32(const unsigned* src, unsigned* dst, int n, hipStream_t st);

}  // namespace gcr
