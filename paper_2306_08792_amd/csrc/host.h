// Host-side internals shared by the C ABI layer (api.hip) and the serving
// loop (server.hip): the context, the workspace planner, kNN planning and
// launch sequences, graph assembly.  Not part of the public interface.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

#include "gcr.h"
#include "kernels.h"

struct gcr_timer_rec {
  hipEvent_t a, b;
  int cls;
};
struct gcr_ctx {
  int device = 0;
  int timing = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<gcr_timer_rec> recs;
  std::string err;
  void* ws = nullptr;
  size_t ws_bytes = 0;
  unsigned long long* stats = nullptr;  // device: [0] candidates, [1] re-swept pairs, [2] exhaustive pairs
  int64_t knn_rows = 0;
  int64_t splits = 0;
  int64_t tile_rows = 0;
};

namespace gcr {
namespace host {

inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }
inline int64_t roundup(int64_t x, int64_t a) { return (x + a - 1) / a * a; }

// Two-pass bump planner over the context workspace.
struct Arena {
  char* base = nullptr;
  size_t off = 0;
  template <class T>
  T* take(size_t count) {
    off = align_up(off, 256);
    T* p = base ? (T*)(base + off) : nullptr;
    off += count * sizeof(T);
    return p;
  }
};

struct KnnPlan {
  int prec, nl, C, S, RB, kch, fb_grid;
  int balanced = 0, grid = 0, ntr = 0, bm = 128;  // balanced similarity schedule, tile rows
  int64_t total_tiles = 0;
  int64_t n, npad, ld, W, rows, ncols;
  uint8_t* Xs; float* n2; float* scale; float* rn; unsigned* maxn2;
  uint64_t* cand; int* cnt; float* thr; int* fb_list; int* fb_count; uint64_t* fb_scr;
  uint64_t* fb_pk; uint32_t* fb_pc;
  float* seed;
  unsigned* thr_shared;
  float* fb_cut; uint64_t* band; int* band_cnt; int band_cap, band_max; int* ovf_list; int* heavy_list;
  int32_t *ord, *ord_label, *ord_cnt, *ord_blk;  // refine row order (square sweeps)
  int tsweep = 0, trefine = 1;  // timer classes of the screening sweep and its refine
  int raw = 0;                  // 1: screened keys decide the lists (no exact re-score)
};

struct GraphTmp {
  int32_t* cnt; int32_t* blk;
  int32_t* label; int32_t* order;  // locality order of the last graph built
  float* dc; float* dc_cr;         // column degrees of asymmetric graphs
};

gcr_status fail(gcr_ctx* c, gcr_status s, const char* fmt, ...);
gcr_status reserve_ws(gcr_ctx* c, size_t bytes);
gcr_status need_ws(gcr_ctx* c, size_t bytes);
void fill_u32(void* p, unsigned v, int64_t n, hipStream_t st);
int esize_of(int prec);
// Screening operand precision of a gcr_precision value, and whether it is a
// screening-only (raw) mode.
int screen_prec_of(int precision);
int is_raw_precision(int precision);
int final_screen_prec(int precision);
gcr_status check_operand(gcr_ctx* c, int precision, int64_t rows, int d);
int compute_units();
float eps_accumulation(int prec, int d);
float eps_norm(int d);
int capacity_for(int prec, int kmax, int nl);
gcr_status check_params(gcr_ctx* c, const gcr_params* p);
int cross_k_of(const gcr_params* p);
void plan_knn(Arena& ar, KnnPlan& kp, int prec, int64_t n, int d, int64_t r0, int64_t r1, int64_t c0,
              int64_t c1, int k0, int k1);
// Screening + refine for rows [r0, r1) against columns [c0, c1) of X.
void run_knn(gcr_ctx* c, const KnnPlan& kp, const float* X, int d, const int* cam, int64_t r0, int64_t r1,
             int64_t c0, int64_t c1, int exclude_self, int k0, int k1, int32_t* idx0, float* dist0,
             int32_t* idx1, float* dist1, hipStream_t st, const int32_t* prev0 = nullptr,
             const int32_t* prev1 = nullptr, const int32_t* order = nullptr);
size_t layout_graph(Arena& ar, gcr_graph* g, int64_t n, int k, int ck, int has_cross);
void plan_graph_tmp(Arena& ar, GraphTmp& t, int64_t n);
void enqueue_build_graph(gcr_ctx* c, const KnnPlan& kp, const GraphTmp& gt, const float* X, int64_t n, int d,
                         const int* cam, const gcr_params* p, const gcr_graph* g, hipStream_t st,
                         bool seed_from_previous = false);
void enqueue_graph_from_lists(gcr_ctx* c, const GraphTmp& gt, int64_t n, const int* cam, const gcr_params* p,
                              const gcr_graph* g, hipStream_t st);
void enqueue_propagate(gcr_ctx* c, const gcr_graph* g, const float* Xin, float* Xout, int64_t n, int d,
                       hipStream_t st, const int32_t* order);

}  // namespace host
}  // namespace gcr

#define HIP_TRY(c, expr)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return gcr::host::fail(c, GCR_ERR_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)
