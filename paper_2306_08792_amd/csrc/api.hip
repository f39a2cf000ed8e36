// C ABI of the GCR library: argument checks, workspace planning and the
// launch sequence of each entry point.  All device work is enqueued on the
// caller's stream.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <string>
#include <vector>

#include "host.h"

// Scratch of gcr_propagate_noalloc: a file-scope device array (each GPU the
// library runs on holds its own copy until the process ends).  In host code
// its name is only a stand-in; the device address comes from
// hipGetSymbolAddress, taken once per device in gcr_create with that device
// current, and is kept in noalloc_scratch[device].
#define GCR_NOALLOC_SCRATCH_BYTES (32u << 20)
#define GCR_NOALLOC_MAX_DEVICES 64
static __device__ __align__(256) uint8_t scratch[GCR_NOALLOC_SCRATCH_BYTES];
static std::mutex noalloc_mu;
static void* noalloc_scratch[GCR_NOALLOC_MAX_DEVICES] = {};


namespace gcr {
namespace host {

hipEvent_t pool_event(gcr_ctx* c) {
  if (!c->ev_pool.empty()) {
    hipEvent_t e = c->ev_pool.back();
    c->ev_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  (void)hipEventCreate(&e);
  return e;
}

// RAII scope recording a start/stop event pair around launches of one class.
struct TimedScope {
  gcr_ctx* c;
  hipStream_t st;
  gcr_timer_rec r;
  bool on;
  TimedScope(gcr_ctx* c_, int cls, hipStream_t st_) : c(c_), st(st_), on(c_ && c_->timing) {
    if (on) {
      r.a = pool_event(c);
      r.b = pool_event(c);
      r.cls = cls;
      (void)hipEventRecord(r.a, st);
    }
  }
  ~TimedScope() {
    if (on) {
      (void)hipEventRecord(r.b, st);
      c->recs.push_back(r);
    }
  }
};

gcr_status fail(gcr_ctx* c, gcr_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  if (c) c->err = buf;
  return s;
}



// Grow the context workspace (the only allocation a context makes after
// creation): synchronises the device, frees the old block, allocates anew.
gcr_status reserve_ws(gcr_ctx* c, size_t bytes) {
  if (bytes <= c->ws_bytes) return GCR_OK;
  HIP_TRY(c, hipSetDevice(c->device));
  if (c->ws) {
    HIP_TRY(c, hipDeviceSynchronize());
    HIP_TRY(c, hipFree(c->ws));
    c->ws = nullptr;
    c->ws_bytes = 0;
  }
  size_t want = align_up(bytes, 1 << 20);
  if (hipMalloc(&c->ws, want) != hipSuccess) {
    c->ws = nullptr;
    (void)hipGetLastError();
    return fail(c, GCR_ERR_NOMEM, "workspace allocation of %zu bytes failed", want);
  }
  c->ws_bytes = want;
  return GCR_OK;
}

// A batch call never allocates: it runs in the workspace the context holds
// or fails with NOMEM naming the size it needs.
gcr_status need_ws(gcr_ctx* c, size_t bytes) {
  if (bytes <= c->ws_bytes) return GCR_OK;
  return fail(c, GCR_ERR_NOMEM,
              "this call needs a workspace of %zu bytes and the context holds %zu "
              "(size it with gcr_workspace_size at gcr_create, or grow it with gcr_reserve)",
              bytes, c->ws_bytes);
}

__global__ void fill_u32_kernel(unsigned* p, unsigned v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
void fill_u32(void* p, unsigned v, int64_t n, hipStream_t st) {
  if (n <= 0) return;
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, (unsigned*)p, v, n);
}
__global__ void add_count_kernel(unsigned long long* dst, const int* src) { *dst += (unsigned long long)*src; }

int esize_of(int prec) { return prec == GCR_PREC_FP32 ? 4 : (prec == GCR_PREC_BF16 ? 2 : 1); }
int screen_prec_of(int precision) {
  return precision == GCR_BF16_RAW ? GCR_PREC_BF16 : (precision == GCR_FP8_RAW ? GCR_PREC_FP8 : precision);
}
int is_raw_precision(int precision) { return precision == GCR_BF16_RAW || precision == GCR_FP8_RAW; }
// Screening of the final top-K: FP8's margin (about 0.13 in squared distance
// for unit rows) spans thousands of unrelated items at a K beyond the
// natural neighbourhood size, which would send queries to the refine's
// exhaustive path, so the exact FP8 mode screens the final top-K in BF16.
int final_screen_prec(int precision) { return precision == GCR_FP8 ? GCR_BF16 : precision; }

// The similarity kernel reads its screening operand [npad, ld] through one
// buffer descriptor with 32-bit byte offsets, so the operand must stay below
// 4 GiB (e.g. about 1M rows of BF16 or 524k rows of float32 at d = 2048).
gcr_status check_operand(gcr_ctx* c, int precision, int64_t rows, int d) {
  const int64_t npad = roundup(rows, 128) + 128;
  const int64_t ld = roundup((int64_t)d * esize_of(screen_prec_of(precision)), 128);
  // a 256-row tile of the last row block reads up to 128 rows past npad
  if ((npad + 128) * ld >= ((int64_t)1 << 32))
    return fail(c, GCR_ERR_UNSUPPORTED,
                "%lld rows of width %d exceed the 4 GiB screening operand of the similarity kernel",
                (long long)rows, d);
  return GCR_OK;
}

// Compute units of the current device (one similarity workgroup each).
int compute_units() {
  int dev = 0, n = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n <= 0) {
    (void)hipGetLastError();
    return 256;
  }
  return n;
}

// Relative error of the float32 accumulation of the screening products:
// |fl(sum) - sum| <= eps * ||x~_r|| ||x~_c||.  BF16 and FP8 products are
// exact in float32 (m = d rounded additions); float32 products round too
// (m = d + 1); FP8 similarities are multiplied by the two row scales after
// the accumulation (two more roundings).
float eps_accumulation(int prec, int d) {
  const double u23 = ldexp(1.0, -23);
  const double m = prec == GCR_PREC_FP32 ? d + 1.0 : (double)d;
  double e = m * u23 / (1.0 - m * u23);
  if (prec == GCR_PREC_FP8) e += 4.0 * u23;
  return (float)(e * 1.01);
}
float eps_norm(int d) {
  const double u23 = ldexp(1.0, -23), m = d + 8;
  return (float)(m * u23 / (1.0 - m * u23) * 1.01);
}

// Candidate capacity per (row, list, split).  When a row's k-th neighbour
// lies among many unrelated items at nearly the same distance (a cross-camera
// list whose identity has few other-camera samples), the screening band holds
// hundreds of items; a buffer that keeps 256 of them leaves the split's
// threshold far enough above the cut that the exact step rarely needs the
// exhaustive path.  Rows with a tight neighbourhood compact once and stay
// small, so the large buffer costs little for them.
int capacity_for(int prec, int kmax, int nl) {
  (void)prec;
  (void)nl;
  return kmax + 8 <= 512 ? 512 : 1024;
}


void plan_knn(Arena& ar, KnnPlan& kp, int precision, int64_t n, int d, int64_t r0, int64_t r1, int64_t c0,
              int64_t c1, int k0, int k1) {
  const int prec = screen_prec_of(precision);
  kp.prec = prec;
  kp.raw = is_raw_precision(precision);
  kp.nl = k1 > 0 ? 2 : 1;
  kp.n = n;
  kp.npad = roundup(n, 128) + 128;
  kp.ld = roundup((int64_t)d * esize_of(prec), 128);
  kp.kch = (int)(kp.ld / 128);
  kp.rows = r1 - r0;
  kp.ncols = c1 - c0;
  kp.C = capacity_for(prec, std::max(k0, k1), kp.nl);
  kp.RB = (int)((kp.rows + 127) / 128);
  const int TC = sim_topk_tile_cols();
  // Whole-row sweeps keep a row's neighbourhood in one candidate buffer
  // (its running threshold then tightens to the true k-th key); rows are
  // split over columns only while there are too few row blocks to occupy
  // the GPU.
  int S = 1;
  while ((int64_t)kp.RB * S < 128 && (int64_t)S * 2 * TC <= kp.ncols && S * 2 * kp.C <= 2048 && S < 64) S *= 2;
  // With many row blocks the sweep is cut evenly over one workgroup per
  // compute unit instead (a row block split over workgroups becomes extra
  // splits), so that no unit idles behind the last row blocks; it uses
  // 256-row tiles when there are enough of them.
  const int G = compute_units();
  kp.balanced = 0;
  kp.bm = 128;
  for (const int bm : {256, 128}) {
    // (the 256-row kernel keeps room for a whole 256-column tile in every
    // candidate buffer, so it needs C >= 512)
    if (bm == 256 && (!sim_topk_large_tile(prec, kp.nl) || kp.C < 2 * TC)) continue;
    const int Sb = sim_topk_balanced_splits(kp.rows, kp.ncols, G, bm);
    if (Sb > 0 && Sb * kp.C <= 2048) {
      S = Sb;
      kp.balanced = 1;
      kp.bm = bm;
      kp.RB = (int)((kp.rows + bm - 1) / bm);
      kp.grid = G;
      kp.ntr = (int)((kp.ncols + TC - 1) / TC);
      kp.total_tiles = (int64_t)kp.RB * kp.ntr;
      break;
    }
  }
  kp.S = S;
  kp.W = roundup((kp.ncols + S - 1) / S, TC);
  kp.fb_grid = 256;
  kp.Xs = ar.take<uint8_t>((size_t)(kp.npad * kp.ld));
  kp.n2 = ar.take<float>(kp.npad);
  kp.scale = ar.take<float>(kp.npad);
  kp.rn = ar.take<float>(kp.npad);
  kp.maxn2 = ar.take<unsigned>(64);
  kp.cand = ar.take<uint64_t>((size_t)kp.rows * kp.nl * S * kp.C);
  kp.cnt = ar.take<int>((size_t)kp.rows * kp.nl * S);
  kp.seed = ar.take<float>((size_t)kp.rows * kp.nl);
  kp.thr_shared = ar.take<unsigned>((size_t)kp.rows * kp.nl);
  kp.thr = ar.take<float>((size_t)kp.rows * kp.nl * S);
  kp.fb_list = ar.take<int>((size_t)kp.rows * kp.nl + 1);
  kp.fb_cut = ar.take<float>((size_t)kp.rows * kp.nl + 1);
  kp.ovf_list = ar.take<int>((size_t)kp.rows * kp.nl + 1);
  kp.heavy_list = ar.take<int>((size_t)kp.rows * kp.nl + 1);
  kp.band_max = (int)std::min<int64_t>(2048, kp.rows * kp.nl);
  kp.band_cap = 2048;
  kp.band = ar.take<uint64_t>((size_t)kp.band_max * kp.band_cap + 1);
  kp.band_cnt = ar.take<int>((size_t)kp.band_max + 1);
  const bool square = r0 == 0 && c0 == 0 && r1 == c1;
  kp.ord = square ? ar.take<int32_t>((size_t)r1) : nullptr;
  kp.ord_label = square ? ar.take<int32_t>((size_t)r1) : nullptr;
  kp.ord_cnt = square ? ar.take<int32_t>((size_t)r1 + 1) : nullptr;
  kp.ord_blk = square ? ar.take<int32_t>((size_t)(r1 / 1024 + 2)) : nullptr;
  kp.fb_count = ar.take<int>(64);
  kp.fb_scr = ar.take<uint64_t>((size_t)kp.fb_grid * std::max<int64_t>(kp.ncols, 1));
  {
    const int64_t pairs = std::min<int64_t>(FB_MAX, kp.rows * kp.nl);
    const int64_t nch = (kp.ncols + 2047) / 2048;
    const int64_t kmx = std::max(k0, k1);
    kp.fb_pk = ar.take<uint64_t>((size_t)(pairs * nch * kmx + 1));
    kp.fb_pc = ar.take<uint32_t>((size_t)(pairs * nch * kmx + 1));
  }
}

// Screening + refine for rows [r0, r1) against columns [c0, c1) of X.
// prev0 / prev1: earlier neighbour lists of the same rows (graph rebuilt
// from updated features) used to seed the admission thresholds, or nullptr.
// order: processing order of the rows (rows [0, n) only) or nullptr.
void run_knn(gcr_ctx* c, const KnnPlan& kp, const float* X, int d, const int* cam, int64_t r0, int64_t r1,
             int64_t c0, int64_t c1, int exclude_self, int k0, int k1, int32_t* idx0, float* dist0,
             int32_t* idx1, float* dist1, hipStream_t st, const int32_t* prev0, const int32_t* prev1,
             const int32_t* order) {
  if (r0 != 0) order = nullptr;
  fill_u32(kp.maxn2, 0u, 2, st);
  fill_u32(kp.fb_count, 0u, 3, st);
  fill_u32(kp.band_cnt, 0u, kp.band_max, st);
  {
    TimedScope ts(c, 5, st);
    launch_screen_prep(kp.prec, X, kp.n, d, kp.npad, kp.Xs, kp.ld, kp.n2, kp.scale, kp.rn, kp.maxn2, st);
  }
  SimArgs sa;
  sa.Xs = kp.Xs; sa.npad = kp.npad; sa.ld_bytes = kp.ld; sa.n2 = kp.n2;
  sa.scale = kp.prec == GCR_PREC_FP8 ? kp.scale : nullptr;
  sa.cam = cam; sa.maxn2 = (const float*)kp.maxn2; sa.rn = kp.rn;
  sa.r0 = r0; sa.r1 = r1; sa.c0 = c0; sa.c1 = c1; sa.W = kp.W; sa.S = kp.S; sa.RB = kp.RB;
  sa.exclude_self = exclude_self; sa.k0 = k0; sa.k1 = k1; sa.C = kp.C;
  sa.eps_s = eps_accumulation(kp.prec, d); sa.eps_n = eps_norm(d);
  sa.cand = kp.cand; sa.cnt = kp.cnt; sa.thr = kp.thr;
  sa.thr_init = nullptr;
  sa.balanced = kp.balanced; sa.grid = kp.grid; sa.ntr = kp.ntr; sa.total_tiles = kp.total_tiles; sa.bm = kp.bm;
  sa.thr_shared = nullptr;
  if (kp.S > 1) {
    fill_u32(kp.thr_shared, 0xffffffffu, kp.rows * kp.nl, st);
    sa.thr_shared = kp.thr_shared;
  }
  if (kp.balanced) {
    // a row block has up to S pieces; the ones no workgroup sweeps stay
    // empty with an infinite threshold
    fill_u32(kp.cnt, 0u, kp.rows * kp.nl * kp.S, st);
    fill_u32(kp.thr, 0x7f800000u, kp.rows * kp.nl * kp.S, st);
  }
  if (prev0 && r0 == 0 && c0 == 0 && r1 == c1 && (k1 == 0 || prev1)) {
    TimedScope ts(c, kp.trefine, st);
    if (kp.prec == GCR_PREC_BF16 && (kp.ld == 1024 || kp.ld == 2048 || kp.ld == 4096))
      launch_seed_thresholds_bf16(kp.Xs, kp.ld, r1, prev0, k0, k1 ? prev1 : nullptr, k1, kp.n2, kp.rn,
                                  (const float*)kp.maxn2, sa.eps_s, sa.eps_n, kp.seed, order, st);
    else
      launch_seed_thresholds(X, d, r1, prev0, k0, k1 ? prev1 : nullptr, k1, kp.n2, kp.rn, (const float*)kp.maxn2,
                             sa.eps_s, sa.eps_n, kp.seed, order, st);
    sa.thr_init = kp.seed;
  }
  {
    TimedScope ts(c, kp.tsweep, st);
    launch_sim_topk(kp.prec, kp.nl, sa, st);
  }
  RefineArgs ra;
  ra.cand = kp.cand; ra.cnt = kp.cnt; ra.thr = kp.thr; ra.S = kp.S; ra.C = kp.C; ra.NL = kp.nl; ra.k0 = k0; ra.k1 = k1;
  ra.r0 = r0; ra.r1 = r1; ra.c0 = c0; ra.c1 = c1; ra.exclude_self = exclude_self;
  ra.X = X; ra.d = d; ra.cam = cam; ra.n2 = kp.n2; ra.rn = kp.rn; ra.maxn2 = (const float*)kp.maxn2;
  ra.eps_s = sa.eps_s; ra.eps_n = sa.eps_n;
  ra.idx0 = idx0; ra.dist0 = dist0; ra.idx1 = idx1; ra.dist1 = dist1;
  ra.fb_list = kp.fb_list; ra.fb_count = kp.fb_count; ra.stat_cands = c->stats;
  ra.fb_scratch = kp.fb_scr; ra.fb_grid = kp.fb_grid;
  ra.fb_part_key = kp.fb_pk; ra.fb_part_col = kp.fb_pc; ra.fb_max = FB_MAX;
  ra.fb_cut = kp.fb_cut; ra.eps32 = eps_accumulation(GCR_PREC_FP32, d);
  ra.band = kp.band; ra.band_cnt = kp.band_cnt; ra.band_cap = kp.band_cap; ra.band_max = kp.band_max;
  ra.ovf_list = kp.ovf_list; ra.ovf_count = kp.fb_count + 1;
  ra.heavy_list = kp.heavy_list; ra.heavy_count = kp.fb_count + 2;
  ra.order = nullptr;
  if (kp.raw) {
    TimedScope ts(c, kp.trefine, st);
    launch_raw_select(ra, st);
    c->knn_rows += kp.rows;
    c->splits = kp.S;
    c->tile_rows = kp.bm;
    return;
  }
  if (kp.ord && r0 == 0 && c0 == 0 && r1 == c1 && k0 > 0) {
    TimedScope ts(c, kp.trefine, st);
    launch_cand_order(r1, kp.cand, kp.cnt, kp.S, kp.C, kp.nl, kp.ord_label, kp.ord_cnt, kp.ord_blk, kp.ord, st);
    ra.order = kp.ord;
  }
  {
    TimedScope ts(c, kp.trefine, st);
    launch_refine(ra, st);
  }
  hipLaunchKernelGGL(add_count_kernel, dim3(1), dim3(1), 0, st, c->stats + 1, kp.fb_count);
  hipLaunchKernelGGL(add_count_kernel, dim3(1), dim3(1), 0, st, c->stats + 2, kp.fb_count + 1);
  c->knn_rows += kp.rows;
  c->splits = kp.S;
  c->tile_rows = kp.bm;
}

gcr_status check_params(gcr_ctx* c, const gcr_params* p) {
  if (!p) return fail(c, GCR_ERR_INVALID, "params is NULL");
  if (p->k < 0) return fail(c, GCR_ERR_INVALID, "k must be >= 0 (got %d)", p->k);
  if (p->k > 120 || p->cross_k > 120)
    return fail(c, GCR_ERR_UNSUPPORTED, "k and cross_k above 120 are not supported");
  if (!(p->gamma > 0.f)) return fail(c, GCR_ERR_INVALID, "gamma must be > 0");
  if (!(p->alpha >= 0.f && p->alpha <= 1.f)) return fail(c, GCR_ERR_INVALID, "alpha must be in [0, 1]");
  if (!(p->beta_same > 0.f && p->beta_cross > 0.f)) return fail(c, GCR_ERR_INVALID, "beta factors must be > 0");
  if (p->precision < 0 || p->precision > 4) return fail(c, GCR_ERR_INVALID, "unknown precision %d", p->precision);
  if (p->rounds < 0) return fail(c, GCR_ERR_INVALID, "rounds must be >= 0");
  if (p->symmetric != 0 && p->symmetric != 1) return fail(c, GCR_ERR_INVALID, "symmetric must be 0 or 1");
  return GCR_OK;
}

int cross_k_of(const gcr_params* p) { return p->cross_k < 0 ? p->k : p->cross_k; }

// ---- graph layout
struct GraphLayout {
  size_t bytes;
};
size_t graph_part(Arena& ar, gcr_graph* g, int64_t n, int k, bool cross) {
  (void)cross;
  int32_t* idx = ar.take<int32_t>((size_t)n * k);
  float* dist = ar.take<float>((size_t)n * k);
  float* w = ar.take<float>((size_t)n * k);
  int32_t* rp = ar.take<int32_t>((size_t)n + 1);
  int32_t* rs = ar.take<int32_t>((size_t)n * k);
  float* rw = ar.take<float>((size_t)n * k);
  float* deg = ar.take<float>((size_t)n);
  float* pf = ar.take<float>((size_t)n * k);
  float* pr = ar.take<float>((size_t)n * k);
  if (g) {
    if (!cross) {
      g->idx = idx; g->dist = dist; g->w = w; g->rev_ptr = rp; g->rev_src = rs; g->rev_w = rw;
      g->deg = deg; g->pf = pf; g->pr = pr;
    } else {
      g->cr_idx = idx; g->cr_dist = dist; g->cr_w = w; g->cr_rev_ptr = rp; g->cr_rev_src = rs;
      g->cr_rev_w = rw; g->cr_deg = deg; g->cr_pf = pf; g->cr_pr = pr;
    }
  }
  return ar.off;
}
size_t layout_graph(Arena& ar, gcr_graph* g, int64_t n, int k, int ck, int has_cross) {
  if (g) {
    memset(g, 0, sizeof(*g));
    g->n = n; g->k = k; g->cross_k = ck; g->has_cross = has_cross;
  }
  graph_part(ar, g, n, k, false);
  if (has_cross) graph_part(ar, g, n, ck, true);
  float* self = ar.take<float>((size_t)n);
  if (g) g->self = self;
  return ar.off;
}

void plan_graph_tmp(Arena& ar, GraphTmp& t, int64_t n) {
  t.cnt = ar.take<int32_t>((size_t)n + 1);
  t.blk = ar.take<int32_t>((size_t)(n / 1024 + 2));
  t.label = ar.take<int32_t>((size_t)n);
  t.order = ar.take<int32_t>((size_t)n);
  t.dc = ar.take<float>((size_t)n);
  t.dc_cr = ar.take<float>((size_t)n);
}

void build_one(const gcr_graph* g, bool cross, int64_t n, const int* cam, const gcr_params* p, float coef,
               const GraphTmp& t, hipStream_t st, bool finish) {
  GraphBuildArgs a;
  a.n = n;
  a.k = cross ? g->cross_k : g->k;
  a.idx = cross ? g->cr_idx : g->idx;
  a.dist = cross ? g->cr_dist : g->dist;
  a.cam = cam;
  a.use_beta = (!cross && cam && (p->beta_same != 1.f || p->beta_cross != 1.f)) ? 1 : 0;
  a.beta_same = p->beta_same; a.beta_cross = p->beta_cross;
  a.gamma = p->gamma;
  a.w = cross ? g->cr_w : g->w;
  a.rev_ptr = cross ? g->cr_rev_ptr : g->rev_ptr;
  a.rev_src = cross ? g->cr_rev_src : g->rev_src;
  a.rev_w = cross ? g->cr_rev_w : g->rev_w;
  a.deg = cross ? g->cr_deg : g->deg;
  a.pf = cross ? g->cr_pf : g->pf;
  a.pr = cross ? g->cr_pr : g->pr;
  a.coef = coef;
  a.tmp_cnt = t.cnt; a.tmp_blk = t.blk;
  a.asym = p->symmetric ? 0 : 1;
  a.deg_c = cross ? t.dc_cr : t.dc;
  if (!finish) launch_graph_build(a, st);
  else launch_finish_values(a, st);
}

// kNN + affinity + CSR + degrees + normalised values into g.
// seed_from_previous: g already holds the lists of the same rows from the
// previous round; they bound this round's k-th distances from above.
void enqueue_build_graph(gcr_ctx* c, const KnnPlan& kp, const GraphTmp& gt, const float* X, int64_t n, int d,
                         const int* cam, const gcr_params* p, const gcr_graph* g, hipStream_t st,
                         bool seed_from_previous) {
  const bool cross = g->has_cross != 0;
  if (g->k > 0 || (cross && g->cross_k > 0))
    run_knn(c, kp, X, d, cam, 0, n, 0, n, 1, g->k, cross ? g->cross_k : 0, g->idx, g->dist,
            cross ? g->cr_idx : nullptr, cross ? g->cr_dist : nullptr, st,
            seed_from_previous ? g->idx : nullptr, seed_from_previous && cross ? g->cr_idx : nullptr,
            seed_from_previous && g->k > 0 ? gt.order : nullptr);
  enqueue_graph_from_lists(c, gt, n, cam, p, g, st);
}

// Affinities, reverse lists, degrees, normalised values, self coefficients
// and the locality order from the forward lists already in g.
void enqueue_graph_from_lists(gcr_ctx* c, const GraphTmp& gt, int64_t n, const int* cam, const gcr_params* p,
                              const gcr_graph* g, hipStream_t st) {
  const bool cross = g->has_cross != 0;
  const float alpha = cross ? p->alpha : 1.0f;
  TimedScope ts(c, 2, st);
  build_one(g, false, n, cam, p, alpha, gt, st, false);
  if (cross) build_one(g, true, n, cam, p, 1.0f - alpha, gt, st, false);
  build_one(g, false, n, cam, p, alpha, gt, st, true);
  if (cross) build_one(g, true, n, cam, p, 1.0f - alpha, gt, st, true);
  const bool asym = p->symmetric == 0;
  launch_self_coef(n, g->deg, asym ? gt.dc : nullptr, cross ? g->cr_deg : nullptr, asym && cross ? gt.dc_cr : nullptr,
                   alpha, g->self, st);
  const_cast<gcr_graph*>(g)->asymmetric = asym ? 1 : 0;
  if (g->k > 0) launch_locality_order(n, g->idx, g->k, gt.label, gt.cnt, gt.blk, gt.order, st);
}

void enqueue_propagate(gcr_ctx* c, const gcr_graph* g, const float* Xin, float* Xout, int64_t n, int d,
                       hipStream_t st, const int32_t* order) {
  TimedScope ts(c, 3, st);
  PropArgs a;
  a.X = Xin; a.Y = Xout; a.n = n; a.d = d; a.self = g->self;
  a.order = g->k > 0 ? order : nullptr;
  a.idx = g->idx; a.pf = g->pf; a.k = g->k; a.rev_ptr = g->rev_ptr; a.rev_src = g->rev_src; a.pr = g->pr;
  if (g->asymmetric) a.rev_ptr = nullptr;  // Eq. (6): forward lists only
  if (g->has_cross) {
    a.cr_idx = g->cr_idx; a.cr_pf = g->cr_pf; a.ck = g->cross_k; a.cr_rev_ptr = g->cr_rev_ptr;
    a.cr_rev_src = g->cr_rev_src; a.cr_pr = g->cr_pr;
    if (g->asymmetric) a.cr_rev_ptr = nullptr;
  } else {
    a.cr_idx = nullptr; a.cr_pf = nullptr; a.ck = 0; a.cr_rev_ptr = nullptr; a.cr_rev_src = nullptr;
    a.cr_pr = nullptr;
  }
  launch_propagate(a, st);
}

}  // namespace host
}  // namespace gcr

using namespace gcr;
using namespace gcr::host;

extern "C" {

void gcr_params_default(gcr_params* p) {
  if (!p) return;
  p->k = 15;
  p->cross_k = -1;
  p->rounds = 3;
  p->rebuild_each_round = 1;
  p->normalize_input = 1;
  p->precision = GCR_FP32;
  p->topk_out = 100;
  p->symmetric = 1;
  p->gamma = 0.2f;
  p->alpha = 1.0f;
  p->beta_same = 1.0f;
  p->beta_cross = 1.0f;
  p->lambda = 10.0f;
}

gcr_status gcr_create(gcr_ctx** out, int device, size_t workspace_bytes) {
  if (!out) return GCR_ERR_INVALID;
  *out = nullptr;
  int nd = 0;
  if (hipGetDeviceCount(&nd) != hipSuccess || device < 0 || device >= nd) {
    (void)hipGetLastError();
    return GCR_ERR_INVALID;
  }
  if (hipSetDevice(device) != hipSuccess) {
    (void)hipGetLastError();
    return GCR_ERR_HIP;
  }
  if (device < GCR_NOALLOC_MAX_DEVICES) {
    // the no-allocation entry point's scratch on this device (device current)
    std::lock_guard<std::mutex> lk(noalloc_mu);
    if (!noalloc_scratch[device]) {
      void* ptr = nullptr;
      if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
        (void)hipGetLastError();
        return GCR_ERR_HIP;
      }
      noalloc_scratch[device] = ptr;
    }
  }
  gcr_ctx* c = new gcr_ctx();
  c->device = device;
  if (hipMalloc(&c->stats, 4 * sizeof(unsigned long long)) != hipSuccess ||
      hipMemset(c->stats, 0, 4 * sizeof(unsigned long long)) != hipSuccess) {
    (void)hipGetLastError();
    if (c->stats) (void)hipFree(c->stats);
    delete c;
    return GCR_ERR_HIP;
  }
  if (workspace_bytes > 0 && reserve_ws(c, workspace_bytes) != GCR_OK) {
    (void)hipFree(c->stats);
    delete c;
    return GCR_ERR_NOMEM;
  }
  *out = c;
  return GCR_OK;
}

gcr_status gcr_reserve(gcr_ctx* c, size_t workspace_bytes) {
  if (!c) return GCR_ERR_INVALID;
  return reserve_ws(c, workspace_bytes);
}

size_t gcr_workspace_bytes(const gcr_ctx* c) { return c ? c->ws_bytes : 0; }

gcr_status gcr_destroy(gcr_ctx* c) {
  if (!c) return GCR_ERR_INVALID;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  for (const gcr_timer_rec& r : c->recs) {
    (void)hipEventDestroy(r.a);
    (void)hipEventDestroy(r.b);
  }
  for (hipEvent_t e : c->ev_pool) (void)hipEventDestroy(e);
  if (c->ws) (void)hipFree(c->ws);
  if (c->stats) (void)hipFree(c->stats);
  delete c;
  return GCR_OK;
}

const char* gcr_last_error(const gcr_ctx* c) { return c ? c->err.c_str() : "context is NULL"; }

gcr_status gcr_get_stats(gcr_ctx* c, gcr_stats* out) {
  if (!c || !out) return GCR_ERR_INVALID;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipDeviceSynchronize());
  unsigned long long h[4];
  HIP_TRY(c, hipMemcpy(h, c->stats, sizeof h, hipMemcpyDeviceToHost));
  out->knn_rows = c->knn_rows;
  out->knn_candidates = (int64_t)h[0];
  out->knn_fallback_rows = (int64_t)h[1];
  out->knn_exhaustive_rows = (int64_t)h[2];
  out->splits = c->splits;
  out->tile_rows = c->tile_rows;
  return GCR_OK;
}

gcr_status gcr_reset_stats(gcr_ctx* c) {
  if (!c) return GCR_ERR_INVALID;
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipDeviceSynchronize());
  HIP_TRY(c, hipMemset(c->stats, 0, 4 * sizeof(unsigned long long)));
  c->knn_rows = 0;
  return GCR_OK;
}

gcr_status gcr_set_timing(gcr_ctx* c, int32_t on) {
  if (!c) return GCR_ERR_INVALID;
  c->timing = on ? 1 : 0;
  return GCR_OK;
}

gcr_status gcr_get_timing(gcr_ctx* c, gcr_timing* out) {
  if (!c || !out) return GCR_ERR_INVALID;
  memset(out, 0, sizeof(*out));
  HIP_TRY(c, hipSetDevice(c->device));
  HIP_TRY(c, hipDeviceSynchronize());
  for (const gcr_timer_rec& r : c->recs) {
    float ms = 0.f;
    HIP_TRY(c, hipEventElapsedTime(&ms, r.a, r.b));
    out->ms[r.cls] += ms;
    out->launches[r.cls] += 1;
    c->ev_pool.push_back(r.a);
    c->ev_pool.push_back(r.b);
  }
  c->recs.clear();
  return GCR_OK;
}

gcr_status gcr_normalize_rows(gcr_ctx* c, const float* X, float* Y, int64_t n, int32_t d, void* stream) {
  if (!c) return GCR_ERR_INVALID;
  if (n < 0 || d <= 0 || (n > 0 && (!X || !Y))) return fail(c, GCR_ERR_INVALID, "bad normalize arguments");
  HIP_TRY(c, hipSetDevice(c->device));
  launch_normalize_rows(X, Y, n, d, (hipStream_t)stream);
  HIP_TRY(c, hipGetLastError());
  return GCR_OK;
}

gcr_status gcr_knn(gcr_ctx* c, const float* X, int64_t n, int32_t d, const int32_t* cam, const gcr_params* p,
                   int32_t* idx, float* dist, int32_t* cr_idx, float* cr_dist, void* stream) {
  if (!c) return GCR_ERR_INVALID;
  gcr_status s = check_params(c, p);
  if (s != GCR_OK) return s;
  if (n < 1 || d <= 0 || !X) return fail(c, GCR_ERR_INVALID, "bad X / n / d");
  if (d > 2048) return fail(c, GCR_ERR_UNSUPPORTED, "d above 2048 is not supported");
  if (n > (int64_t)INT32_MAX / 2) return fail(c, GCR_ERR_UNSUPPORTED, "n too large");
  if ((s = check_operand(c, p->precision, n, d)) != GCR_OK) return s;
  const bool cross = cr_idx != nullptr;
  if (cross && (!cam || !cr_dist)) return fail(c, GCR_ERR_INVALID, "cross list needs cam and cr_dist");
  if (p->k > 0 && (!idx || !dist)) return fail(c, GCR_ERR_INVALID, "idx / dist are NULL");
  const int ck = cross ? cross_k_of(p) : 0;
  HIP_TRY(c, hipSetDevice(c->device));
  Arena dry;
  KnnPlan kp;
  plan_knn(dry, kp, p->precision, n, d, 0, n, 0, n, p->k, ck);
  if ((s = need_ws(c, dry.off)) != GCR_OK) return s;
  Arena ar{(char*)c->ws, 0};
  plan_knn(ar, kp, p->precision, n, d, 0, n, 0, n, p->k, ck);
  hipStream_t st = (hipStream_t)stream;
  // a zero-size list is allowed: give the kernels harmless pointers
  run_knn(c, kp, X, d, cam, 0, n, 0, n, 1, p->k, ck, idx, dist, cr_idx, cr_dist, st);
  HIP_TRY(c, hipGetLastError());
  return GCR_OK;
}

size_t gcr_graph_bytes(int64_t n, int32_t k, int32_t cross_k, int32_t has_cross) {
  Arena dry;
  return layout_graph(dry, nullptr, n, k, has_cross ? (cross_k < 0 ? k : cross_k) : 0, has_cross) + 256;
}

gcr_status gcr_graph_bind(gcr_graph* g, void* buf, int64_t n, int32_t k, int32_t cross_k, int32_t has_cross) {
  if (!g || !buf || n < 1 || k < 0) return GCR_ERR_INVALID;
  if (((uintptr_t)buf) & 255) return GCR_ERR_INVALID;
  Arena ar{(char*)buf, 0};
  layout_graph(ar, g, n, k, has_cross ? (cross_k < 0 ? k : cross_k) : 0, has_cross);
  return GCR_OK;
}

gcr_status gcr_build_graph(gcr_ctx* c, const float* X, int64_t n, int32_t d, const int32_t* cam,
                           const gcr_params* p, gcr_graph* g, void* stream) {
  if (!c) return GCR_ERR_INVALID;
  gcr_status s = check_params(c, p);
  if (s != GCR_OK) return s;
  if (!g || !X || n < 1 || d <= 0 || g->n != n || g->k != p->k)
    return fail(c, GCR_ERR_INVALID, "graph / X shape mismatch");
  if (d > 2048) return fail(c, GCR_ERR_UNSUPPORTED, "d above 2048 is not supported");
  if (g->has_cross && !cam) return fail(c, GCR_ERR_INVALID, "cross graph needs camera labels");
  if ((s = check_operand(c, p->precision, n, d)) != GCR_OK) return s;
  HIP_TRY(c, hipSetDevice(c->device));
  Arena dry;
  KnnPlan kp;
  GraphTmp gt;
  plan_knn(dry, kp, p->precision, n, d, 0, n, 0, n, g->k, g->has_cross ? g->cross_k : 0);
  plan_graph_tmp(dry, gt, n);
  if ((s = need_ws(c, dry.off)) != GCR_OK) return s;
  Arena ar{(char*)c->ws, 0};
  plan_knn(ar, kp, p->precision, n, d, 0, n, 0, n, g->k, g->has_cross ? g->cross_k : 0);
  plan_graph_tmp(ar, gt, n);
  enqueue_build_graph(c, kp, gt, X, n, d, cam, p, g, (hipStream_t)stream);
  HIP_TRY(c, hipGetLastError());
  return GCR_OK;
}

gcr_status gcr_propagate(gcr_ctx* c, const gcr_graph* g, const float* X_in, float* X_out, int64_t n, int32_t d,
                         void* stream) {
  if (!c) return GCR_ERR_INVALID;
  if (!g || !X_in || !X_out || g->n != n || d <= 0) return fail(c, GCR_ERR_INVALID, "bad propagate arguments");
  if (X_in == X_out) return fail(c, GCR_ERR_INVALID, "in-place propagation is not allowed");
  if (d > 2048) return fail(c, GCR_ERR_UNSUPPORTED, "d above 2048 is not supported by propagation");
  HIP_TRY(c, hipSetDevice(c->device));
  GraphTmp gt;
  Arena dry;
  plan_graph_tmp(dry, gt, n);
  gcr_status s = need_ws(c, dry.off);
  if (s != GCR_OK) return s;
  Arena ar{(char*)c->ws, 0};
  plan_graph_tmp(ar, gt, n);
  if (g->k > 0) {
    TimedScope ts(c, 2, (hipStream_t)stream);
    launch_locality_order(n, g->idx, g->k, gt.label, gt.cnt, gt.blk, gt.order, (hipStream_t)stream);
  }
  enqueue_propagate(c, g, X_in, X_out, n, d, (hipStream_t)stream, gt.order);
  HIP_TRY(c, hipGetLastError());
  return GCR_OK;
}

gcr_status gcr_propagate_noalloc(gcr_ctx* c, const gcr_graph* g, const float* X_in, float* X_out, int64_t n,
                                 int32_t d, void* stream) {
  if (!c) return GCR_ERR_INVALID;
  if (!g || !X_in || !X_out || g->n != n || n < 1 || d <= 0)
    return fail(c, GCR_ERR_INVALID, "bad propagate arguments");
  if (X_in == X_out) return fail(c, GCR_ERR_INVALID, "in-place propagation is not allowed");
  if (d > 2048) return fail(c, GCR_ERR_UNSUPPORTED, "d above 2048 is not supported by propagation");
  GraphTmp gt;
  Arena dry;
  plan_graph_tmp(dry, gt, n);
  if (dry.off > GCR_NOALLOC_SCRATCH_BYTES)
    return fail(c, GCR_ERR_UNSUPPORTED,
                "n = %lld needs %zu bytes of scratch; the no-allocation entry point holds %u (about %u nodes)",
                (long long)n, dry.off, GCR_NOALLOC_SCRATCH_BYTES, GCR_NOALLOC_SCRATCH_BYTES / 24u);
  void* base = c->device < GCR_NOALLOC_MAX_DEVICES ? noalloc_scratch[c->device] : nullptr;
  if (!base) return fail(c, GCR_ERR_UNSUPPORTED, "no scratch for device %d", c->device);
  HIP_TRY(c, hipSetDevice(c->device));
  Arena ar{(char*)base, 0};
  plan_graph_tmp(ar, gt, n);
  // the locality order clears its counters with a fill kernel every call
  if (g->k > 0) {
    TimedScope ts(c, 2, (hipStream_t)stream);
    launch_locality_order(n, g->idx, g->k, gt.label, gt.cnt, gt.blk, gt.order, (hipStream_t)stream);
  }
  enqueue_propagate(c, g, X_in, X_out, n, d, (hipStream_t)stream, gt.order);
  HIP_TRY(c, hipGetLastError());
  return GCR_OK;
}

size_t gcr_propagate_noalloc_max_nodes(void) {
  // largest n whose locality-order arrays fit the scratch
  int64_t lo = 1, hi = (int64_t)GCR_NOALLOC_SCRATCH_BYTES;
  while (lo < hi) {
    const int64_t mid = lo + (hi - lo + 1) / 2;
    GraphTmp gt;
    Arena dry;
    plan_graph_tmp(dry, gt, mid);
    if (dry.off <= GCR_NOALLOC_SCRATCH_BYTES) lo = mid;
    else hi = mid - 1;
  }
  return (size_t)lo;
}

struct FinalPlan {
  KnnPlan kd, kt;
};
static void plan_final(Arena& ar, FinalPlan& fp, const gcr_params* p, int64_t nq, int64_t ng, int d,
                       bool dense, bool topk) {
  const int64_t n = nq + ng;
  if (dense) plan_knn(ar, fp.kd, GCR_PREC_FP32, n, d, 0, nq, nq, n, 1, 0);
  if (topk) {
    plan_knn(ar, fp.kt, final_screen_prec(p->precision), n, d, 0, nq, nq, n, p->topk_out, 0);
    fp.kt.tsweep = 6;
    fp.kt.trefine = 7;
  }
}

// Workspace of a whole re-ranking: the two feature buffers, the graph (unless
// the caller's last_graph is used), the locality-order scratch, then the kNN
// plan of the rounds and the final plan overlaid on the same bytes (the
// final launches follow the last round's on the same stream).
struct RerankLayout {
  float *xa = nullptr, *xb = nullptr;
  gcr_graph g;
  KnnPlan kp;
  GraphTmp gt;
  FinalPlan fp;
};
static void layout_rerank(Arena& ar, RerankLayout& L, const gcr_params* p, int64_t nq, int64_t ng, int d,
                          int has_cross, int ck, bool own_graph, bool dense, bool topk) {
  const int64_t n = nq + ng;
  L.xa = ar.take<float>((size_t)n * d);
  L.xb = ar.take<float>((size_t)n * d);
  memset(&L.g, 0, sizeof(L.g));
  if (own_graph) {
    void* gbuf = ar.take<char>(gcr_graph_bytes(n, p->k, ck, has_cross));
    if (gbuf) gcr_graph_bind(&L.g, gbuf, n, p->k, ck, has_cross);
  }
  plan_graph_tmp(ar, L.gt, n);
  Arena fin = ar;
  plan_knn(ar, L.kp, p->precision, n, d, 0, n, 0, n, p->k, ck);
  plan_final(fin, L.fp, p, nq, ng, d, dense, topk);
  ar.off = std::max(ar.off, fin.off);
}

// GCR_Local: feature buffers, the neighbour lists, the locality-order
// scratch, then the kNN plan and the final plan overlaid.
struct LocalLayout {
  float *xa = nullptr, *xb = nullptr, *dist = nullptr;
  int32_t* idx = nullptr;
  KnnPlan kp;
  GraphTmp gt;
  FinalPlan fp;
};
static void layout_local(Arena& ar, LocalLayout& L, const gcr_params* p, int64_t nq, int64_t ng, int d, bool dense,
                         bool topk) {
  const int64_t n = nq + ng;
  const int k = p->k;
  L.xa = ar.take<float>((size_t)n * d);
  L.xb = ar.take<float>((size_t)n * d);
  L.idx = ar.take<int32_t>((size_t)n * (k > 0 ? k : 1));
  L.dist = ar.take<float>((size_t)n * (k > 0 ? k : 1));
  plan_graph_tmp(ar, L.gt, n);
  Arena fin = ar;
  plan_knn(ar, L.kp, p->precision, n, d, 0, n, 0, n, k, 0);
  plan_final(fin, L.fp, p, nq, ng, d, dense, topk);
  ar.off = std::max(ar.off, fin.off);
}
static void run_final(gcr_ctx* c, const FinalPlan& fp, const float* X, int64_t nq, int64_t ng, int32_t d,
                      const gcr_params* p, float* dist_out, int32_t* topk_idx, float* topk_dist, hipStream_t st) {
  const int64_t n = nq + ng;
  if (dist_out) {
    const KnnPlan& kd = fp.kd;
    fill_u32(kd.maxn2, 0u, 2, st);
    {
      TimedScope ts(c, 5, st);
      launch_screen_prep(GCR_PREC_FP32, X, n, d, kd.npad, kd.Xs, kd.ld, kd.n2, kd.scale, kd.rn, kd.maxn2, st);
      launch_split_bf16(kd.Xs, kd.npad, kd.ld, st);
    }
    TimedScope ts(c, 4, st);
    launch_dense_dist(kd.Xs, kd.ld, kd.kch, kd.n2, 0, nq, nq, ng, dist_out, st);
  }
  if (topk_idx)
    run_knn(c, fp.kt, X, d, nullptr, 0, nq, nq, n, 0, p->topk_out, 0, topk_idx, topk_dist, nullptr, nullptr, st);
}

gcr_status gcr_final_distances(gcr_ctx* c, const float* X, int64_t nq, int64_t ng, int32_t d, const gcr_params* p,
                               float* dist_out, int32_t* topk_idx, float* topk_dist, void* stream) {
  if (!c) return GCR_ERR_INVALID;
  if (!p) return fail(c, GCR_ERR_INVALID, "params is NULL");
  if (!X || nq < 1 || ng < 1 || d <= 0) return fail(c, GCR_ERR_INVALID, "bad X / nq / ng / d");
  if (d > 2048) return fail(c, GCR_ERR_UNSUPPORTED, "d above 2048 is not supported");
  if (topk_idx && (!topk_dist || p->topk_out < 1 || p->topk_out > 120))
    return fail(c, p->topk_out > 120 ? GCR_ERR_UNSUPPORTED : GCR_ERR_INVALID, "bad top-K output (K in 1..120)");
  if (p->precision < 0 || p->precision > 4) return fail(c, GCR_ERR_INVALID, "unknown precision");
  gcr_status s = GCR_OK;
  if (dist_out && (s = check_operand(c, GCR_FP32, nq + ng, d)) != GCR_OK) return s;
  if (topk_idx && (s = check_operand(c, final_screen_prec(p->precision), nq + ng, d)) != GCR_OK) return s;
  HIP_TRY(c, hipSetDevice(c->device));
  FinalPlan fp;
  Arena dry;
  plan_final(dry, fp, p, nq, ng, d, dist_out != nullptr, topk_idx != nullptr);
  if ((s = need_ws(c, dry.off)) != GCR_OK) return s;
  Arena ar{(char*)c->ws, 0};
  plan_final(ar, fp, p, nq, ng, d, dist_out != nullptr, topk_idx != nullptr);
  run_final(c, fp, X, nq, ng, d, p, dist_out, topk_idx, topk_dist, (hipStream_t)stream);
  HIP_TRY(c, hipGetLastError());
  return GCR_OK;
}

gcr_status gcr_rerank(gcr_ctx* c, const float* X, int64_t nq, int64_t ng, int32_t d, const int32_t* cam,
                      const gcr_params* p, float* dist_out, int32_t* topk_idx, float* topk_dist, float* X_final,
                      gcr_graph* last_graph, void* stream) {
  if (!c) return GCR_ERR_INVALID;
  gcr_status s = check_params(c, p);
  if (s != GCR_OK) return s;
  const int64_t n = nq + ng;
  if (!X || nq < 1 || ng < 1 || d <= 0) return fail(c, GCR_ERR_INVALID, "bad X / nq / ng / d");
  if (d > 2048) return fail(c, GCR_ERR_UNSUPPORTED, "d above 2048 is not supported");
  if (topk_idx && (!topk_dist || p->topk_out < 1 || p->topk_out > 120))
    return fail(c, p->topk_out > 120 ? GCR_ERR_UNSUPPORTED : GCR_ERR_INVALID, "bad top-K output (K in 1..120)");
  const int has_cross = (cam && p->alpha < 1.0f) ? 1 : 0;
  const int ck = has_cross ? cross_k_of(p) : 0;
  if ((s = check_operand(c, p->precision, n, d)) != GCR_OK) return s;
  if (dist_out && (s = check_operand(c, GCR_FP32, n, d)) != GCR_OK) return s;
  if (last_graph && (last_graph->n != n || last_graph->k != p->k || last_graph->has_cross != has_cross ||
                     (has_cross && last_graph->cross_k != ck) || !last_graph->idx || !last_graph->self))
    return fail(c, GCR_ERR_INVALID, "last_graph must be bound for n = %lld, k = %d, cross_k = %d, has_cross = %d",
                (long long)n, p->k, ck, has_cross);
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;

  const bool dense = dist_out != nullptr, topk = topk_idx != nullptr;
  RerankLayout L;
  Arena dry;
  layout_rerank(dry, L, p, nq, ng, d, has_cross, ck, last_graph == nullptr, dense, topk);
  if ((s = need_ws(c, dry.off)) != GCR_OK) return s;
  Arena ar{(char*)c->ws, 0};
  layout_rerank(ar, L, p, nq, ng, d, has_cross, ck, last_graph == nullptr, dense, topk);
  const gcr_graph& g = last_graph ? *last_graph : L.g;
  float* xa = L.xa;
  float* xb = L.xb;
  const KnnPlan& kp = L.kp;
  const GraphTmp& gt = L.gt;
  const FinalPlan& fp = L.fp;

  if (p->normalize_input) {
    TimedScope ts(c, 5, st);
    launch_normalize_rows(X, xa, n, d, st);
  }
  else HIP_TRY(c, hipMemcpyAsync(xa, X, (size_t)n * d * sizeof(float), hipMemcpyDeviceToDevice, st));
  for (int t = 0; t < p->rounds; ++t) {
    if (t == 0 || p->rebuild_each_round) enqueue_build_graph(c, kp, gt, xa, n, d, cam, p, &g, st, t > 0);
    enqueue_propagate(c, &g, xa, xb, n, d, st, gt.order);
    std::swap(xa, xb);
  }
  run_final(c, fp, xa, nq, ng, d, p, dist_out, topk_idx, topk_dist, st);
  if (X_final) HIP_TRY(c, hipMemcpyAsync(X_final, xa, (size_t)n * d * sizeof(float), hipMemcpyDeviceToDevice, st));
  HIP_TRY(c, hipGetLastError());
  return GCR_OK;
}

// DSFP (Alg. 1) over given neighbour lists.  The nodes are visited in the
// locality order of their lists so that workgroups running together on one
// XCD share most of the rows they gather.
static hipError_t enqueue_dsfp(gcr_ctx* c, const GraphTmp& gt, const float* X, const int32_t* idx, int64_t n,
                               int d, int k, float gamma, int rounds, float* Y, hipStream_t st) {
  if (rounds == 0) return hipMemcpyAsync(Y, X, (size_t)n * d * sizeof(float), hipMemcpyDeviceToDevice, st);
  const int32_t* order = nullptr;
  if (k > 0) {
    launch_locality_order(n, idx, k, gt.label, gt.cnt, gt.blk, gt.order, st);
    order = gt.order;
  }
  TimedScope ts(c, 3, st);
  launch_dsfp(X, idx, n, d, k, gamma, rounds, order, Y, st);
  return hipSuccess;
}

static gcr_status check_dsfp_args(gcr_ctx* c, int64_t n, int32_t d, int32_t k, float gamma, int32_t rounds) {
  if (n < 1 || d <= 0 || k < 0 || rounds < 0) return fail(c, GCR_ERR_INVALID, "bad n / d / k / rounds");
  if (!(gamma > 0.f) || !std::isfinite(gamma)) return fail(c, GCR_ERR_INVALID, "gamma must be finite and > 0");
  if (k > DSFP_K_MAX) return fail(c, GCR_ERR_UNSUPPORTED, "DSFP supports k <= %d", DSFP_K_MAX);
  if (d > 2048) return fail(c, GCR_ERR_UNSUPPORTED, "d above 2048 is not supported");
  if (n > (int64_t)INT32_MAX / 2) return fail(c, GCR_ERR_UNSUPPORTED, "n too large");
  return GCR_OK;
}

gcr_status gcr_dsfp(gcr_ctx* c, const float* X, const int32_t* idx, int64_t n, int32_t d, int32_t k, float gamma,
                    int32_t rounds, float* Y, void* stream) {
  if (!c) return GCR_ERR_INVALID;
  gcr_status s = check_dsfp_args(c, n, d, k, gamma, rounds);
  if (s != GCR_OK) return s;
  if (!X || !Y || (k > 0 && !idx)) return fail(c, GCR_ERR_INVALID, "X / Y / idx are NULL");
  const size_t bytes = (size_t)n * d * sizeof(float);
  const uintptr_t xb = (uintptr_t)X, yb = (uintptr_t)Y;
  if (xb < yb + bytes && yb < xb + bytes) return fail(c, GCR_ERR_INVALID, "Y overlaps X");
  HIP_TRY(c, hipSetDevice(c->device));
  Arena dry;
  GraphTmp gt;
  plan_graph_tmp(dry, gt, n);
  if ((s = need_ws(c, dry.off)) != GCR_OK) return s;
  Arena ar{(char*)c->ws, 0};
  plan_graph_tmp(ar, gt, n);
  HIP_TRY(c, enqueue_dsfp(c, gt, X, idx, n, d, k, gamma, rounds, Y, (hipStream_t)stream));
  HIP_TRY(c, hipGetLastError());
  return GCR_OK;
}

gcr_status gcr_rerank_local(gcr_ctx* c, const float* X, int64_t nq, int64_t ng, int32_t d, const gcr_params* p,
                            float* dist_out, int32_t* topk_idx, float* topk_dist, float* X_final, void* stream) {
  if (!c) return GCR_ERR_INVALID;
  gcr_status s = check_params(c, p);
  if (s != GCR_OK) return s;
  const int64_t n = nq + ng;
  if (!X || nq < 1 || ng < 1) return fail(c, GCR_ERR_INVALID, "bad X / nq / ng");
  if ((s = check_dsfp_args(c, n, d, p->k, p->gamma, p->rounds)) != GCR_OK) return s;
  if ((s = check_operand(c, p->precision, n, d)) != GCR_OK) return s;
  if (dist_out && (s = check_operand(c, GCR_FP32, n, d)) != GCR_OK) return s;
  if (topk_idx && (!topk_dist || p->topk_out < 1 || p->topk_out > 120))
    return fail(c, p->topk_out > 120 ? GCR_ERR_UNSUPPORTED : GCR_ERR_INVALID, "bad top-K output (K in 1..120)");
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const int k = p->k;
  const bool dense = dist_out != nullptr, topk = topk_idx != nullptr;
  LocalLayout L;
  Arena dry;
  layout_local(dry, L, p, nq, ng, d, dense, topk);
  if ((s = need_ws(c, dry.off)) != GCR_OK) return s;
  Arena ar{(char*)c->ws, 0};
  layout_local(ar, L, p, nq, ng, d, dense, topk);
  float* xa = L.xa;
  float* xb = L.xb;
  float* dist = L.dist;
  int32_t* idx = L.idx;
  const KnnPlan& kp = L.kp;
  const GraphTmp& gt = L.gt;
  const FinalPlan& fp = L.fp;

  if (p->normalize_input) {
    TimedScope ts(c, 5, st);
    launch_normalize_rows(X, xa, n, d, st);
  }
  else HIP_TRY(c, hipMemcpyAsync(xa, X, (size_t)n * d * sizeof(float), hipMemcpyDeviceToDevice, st));
  if (k > 0) run_knn(c, kp, xa, d, nullptr, 0, n, 0, n, 1, k, 0, idx, dist, nullptr, nullptr, st);
  HIP_TRY(c, enqueue_dsfp(c, gt, xa, idx, n, d, k, p->gamma, p->rounds, xb, st));
  run_final(c, fp, xb, nq, ng, d, p, dist_out, topk_idx, topk_dist, st);
  if (X_final) HIP_TRY(c, hipMemcpyAsync(X_final, xb, (size_t)n * d * sizeof(float), hipMemcpyDeviceToDevice, st));
  HIP_TRY(c, hipGetLastError());
  return GCR_OK;
}

static int profile_ksplit(int64_t nf) { return (int)std::min<int64_t>(64, std::max<int64_t>(1, nf / 2048)); }

// Workspace of the profile vectors: per-tracklet means, the group mean, the
// member and frame row lists, split-K Gram partials and the Gram, and the
// Chebyshev iterates of the largest group (maxm members).
struct ProfileLayout {
  float *mu_c, *mu, *part, *G, *B, *Wt, *P, *R, *tr, *gm;
  int32_t *dm, *dr;
};
static void layout_profile(Arena& ar, ProfileLayout& L, int64_t nt, int64_t nf, int64_t maxm, int d, int mode,
                           int ksplit) {
  L.mu_c = ar.take<float>((size_t)nt * d);
  L.mu = ar.take<float>((size_t)d);
  L.dm = ar.take<int32_t>((size_t)nt);
  L.dr = ar.take<int32_t>((size_t)nf);
  L.part = mode == 0 ? ar.take<float>((size_t)ksplit * d * d) : nullptr;
  L.G = mode == 0 ? ar.take<float>((size_t)d * d) : nullptr;
  L.B = ar.take<float>((size_t)maxm * d);
  L.Wt = ar.take<float>((size_t)maxm * d);
  L.P = ar.take<float>((size_t)maxm * d);
  L.R = ar.take<float>((size_t)maxm * d);
  L.tr = ar.take<float>(64);
  L.gm = mode == 0 ? ar.take<float>((size_t)group_mean_scratch_floats(d)) : nullptr;
}

size_t gcr_profile_workspace_size(int32_t nt, int64_t nf, int32_t d, int32_t mode) {
  if (nt < 1 || nf < nt || d < 1 || d > 8192 || (mode != 0 && mode != 1)) return 0;
  ProfileLayout L;
  Arena dry;
  layout_profile(dry, L, nt, nf, nt, d, mode, profile_ksplit(nf));
  return dry.off + 256;
}

// Largest workspace any batch entry point needs at these sizes.
size_t gcr_workspace_size(const gcr_params* p, int64_t nq, int64_t ng, int32_t d, int32_t with_cameras) {
  if (!p || nq < 0 || ng < 0 || nq + ng < 1 || d < 1 || d > 2048) return 0;
  if (check_params(nullptr, p) != GCR_OK) return 0;
  const int64_t n = nq + ng;
  if (n > (int64_t)INT32_MAX / 2) return 0;
  if (check_operand(nullptr, p->precision, n, d) != GCR_OK || check_operand(nullptr, GCR_FP32, n, d) != GCR_OK)
    return 0;
  const int ck = with_cameras ? cross_k_of(p) : 0;
  size_t best = 0;
  {  // gcr_knn, gcr_build_graph, gcr_propagate, gcr_dsfp over n rows
    Arena a;
    KnnPlan kp;
    GraphTmp gt;
    plan_knn(a, kp, p->precision, n, d, 0, n, 0, n, p->k, ck);
    plan_graph_tmp(a, gt, n);
    best = std::max(best, a.off);
  }
  if (nq >= 1 && ng >= 1) {
    const bool topk = p->topk_out >= 1 && p->topk_out <= 120;
    {
      Arena a;
      FinalPlan fp;
      plan_final(a, fp, p, nq, ng, d, true, topk);
      best = std::max(best, a.off);
    }
    {
      Arena a;
      RerankLayout L;
      layout_rerank(a, L, p, nq, ng, d, with_cameras ? 1 : 0, ck, true, true, topk);
      best = std::max(best, a.off);
    }
    if (p->k <= DSFP_K_MAX) {
      Arena a;
      LocalLayout L;
      layout_local(a, L, p, nq, ng, d, true, topk);
      best = std::max(best, a.off);
    }
  }
  return best + 256;
}

gcr_status gcr_profile_vectors(gcr_ctx* c, const float* frames, const int32_t* offsets, const int32_t* group,
                               const int32_t* offsets_host, const int32_t* group_host, int32_t nt, int32_t d,
                               int32_t mode, float lambda, float* W_out, void* stream) {
  if (!c) return GCR_ERR_INVALID;
  if (!frames || !offsets || !offsets_host || !W_out || nt < 1 || d <= 0)
    return fail(c, GCR_ERR_INVALID, "bad profile-vector arguments");
  if (mode != 0 && mode != 1) return fail(c, GCR_ERR_INVALID, "mode must be 0 (PVG) or 1 (mean)");
  if (mode == 0 && !(lambda > 0.f)) return fail(c, GCR_ERR_INVALID, "lambda must be > 0");
  if (group && !group_host) return fail(c, GCR_ERR_INVALID, "group needs group_host");
  if (d > 8192) return fail(c, GCR_ERR_UNSUPPORTED, "d above 8192 is not supported");
  for (int t = 0; t < nt; ++t)
    if (offsets_host[t + 1] <= offsets_host[t]) return fail(c, GCR_ERR_INVALID, "tracklet %d is empty", t);
  if (offsets_host[0] != 0) return fail(c, GCR_ERR_INVALID, "offsets[0] must be 0");
  HIP_TRY(c, hipSetDevice(c->device));
  hipStream_t st = (hipStream_t)stream;
  const int64_t nf = offsets_host[nt];

  // host plan: members and frame rows per group
  std::vector<int> gid(nt, 0);
  if (group_host) for (int t = 0; t < nt; ++t) gid[t] = group_host[t];
  std::vector<int> ug(gid.begin(), gid.end());
  std::sort(ug.begin(), ug.end());
  ug.erase(std::unique(ug.begin(), ug.end()), ug.end());
  std::vector<int32_t> members, rows;
  std::vector<int64_t> mstart, rstart;
  for (int gv : ug) {
    mstart.push_back((int64_t)members.size());
    rstart.push_back((int64_t)rows.size());
    for (int t = 0; t < nt; ++t)
      if (gid[t] == gv) {
        members.push_back(t);
        for (int f = offsets_host[t]; f < offsets_host[t + 1]; ++f) rows.push_back(f);
      }
  }
  mstart.push_back((int64_t)members.size());
  rstart.push_back((int64_t)rows.size());
  int maxm = 0;
  for (size_t q = 0; q + 1 < mstart.size(); ++q) maxm = std::max<int>(maxm, (int)(mstart[q + 1] - mstart[q]));
  const int ksplit = profile_ksplit(nf);

  ProfileLayout L;
  Arena dry;
  layout_profile(dry, L, nt, (int64_t)rows.size(), maxm, d, mode, ksplit);
  gcr_status s = need_ws(c, dry.off);
  if (s != GCR_OK) return s;
  Arena ar{(char*)c->ws, 0};
  layout_profile(ar, L, nt, (int64_t)rows.size(), maxm, d, mode, ksplit);
  float *mu_c = L.mu_c, *mu = L.mu, *part = L.part, *G = L.G, *B = L.B, *Wt = L.Wt, *P = L.P, *R = L.R;
  int32_t *dm = L.dm, *dr = L.dr;
  HIP_TRY(c, hipMemcpyAsync(dm, members.data(), members.size() * 4, hipMemcpyHostToDevice, st));
  HIP_TRY(c, hipMemcpyAsync(dr, rows.data(), rows.size() * 4, hipMemcpyHostToDevice, st));
  launch_segment_means(frames, offsets, nt, d, mu_c, st);
  if (mode == 1) {
    launch_normalize_rows(mu_c, W_out, nt, d, st);
    HIP_TRY(c, hipGetLastError());
    return GCR_OK;
  }
  for (size_t q = 0; q + 1 < mstart.size(); ++q) {
    const int nm = (int)(mstart[q + 1] - mstart[q]);
    const int64_t nr = rstart[q + 1] - rstart[q];
    const int32_t* mem = dm + mstart[q];
    const int32_t* rw = dr + rstart[q];
    launch_group_mean(mu_c, offsets, mem, nm, d, nr, L.gm, mu, st);
    const float shift = lambda * (float)nr;
    const int ks = (int)std::min<int64_t>(ksplit, std::max<int64_t>(1, nr / 32));
    launch_gram(frames, rw, nr, d, part, ks, G, shift, st);
    // spectrum bounds of M = F^T F + lambda n I: [lambda n, lambda n + tr(F^T F)]
    launch_gram_trace(G, d, shift, (double*)L.tr, st);
    double trace = 0.0;
    HIP_TRY(c, hipMemcpyAsync(&trace, L.tr, sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(c, hipStreamSynchronize(st));
    trace = std::max(trace, 0.0) * 1.0001 + 1e-6 * shift;
    const double lmin = shift, lmax = shift + trace;
    const double dd = 0.5 * (lmax + lmin), cc = 0.5 * (lmax - lmin);
    const double kap = lmax / lmin;
    const double rate = (sqrt(kap) + 1.0) / std::max(sqrt(kap) - 1.0, 1e-30);
    int iters = (int)ceil(log(2.0 / 1e-9) / log(std::max(rate, 1.0000001))) + 2;
    iters = std::max(2, std::min(iters, 400));
    launch_build_rhs(mu_c, mu, mem, nm, d, B, st);
    const int64_t tot = (int64_t)nm * d;
    fill_u32(Wt, 0u, tot, st);
    fill_u32(P, 0u, tot, st);
    // Chebyshev iteration on M W^T = B^T (rows of W are profile vectors;
    // M is symmetric so W M is the row form of M w_c).
    double alpha_c = 0.0, beta_c = 0.0;
    for (int it = 0; it < iters; ++it) {
      // R = B - W M
      launch_gemm_nn_f32(Wt, d, G, d, R, d, nm, d, d, -1.0f, 1.0f, B, d, st);
      if (it == 0) {
        alpha_c = 1.0 / dd;
        beta_c = 0.0;
      } else if (it == 1) {
        beta_c = 0.5 * (cc * alpha_c) * (cc * alpha_c);
        alpha_c = 1.0 / (dd - beta_c / alpha_c);
      } else {
        beta_c = (cc * alpha_c * 0.5) * (cc * alpha_c * 0.5);
        alpha_c = 1.0 / (dd - beta_c / alpha_c);
      }
      launch_cheb_update(Wt, P, R, (float)beta_c, (float)alpha_c, tot, st);
    }
    launch_normalize_rows(Wt, Wt, nm, d, st);
    launch_scatter_profiles(Wt, mem, nm, d, W_out, st);
  }
  // no synchronisation at the end: the host arrays were consumed by the
  // copies above (complete at the first group's trace read)
  HIP_TRY(c, hipGetLastError());
  return GCR_OK;
}

}  // extern "C"
