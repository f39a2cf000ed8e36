// Serving loop.  A gallery stays resident in HBM with its frozen kNN graph,
// degrees and the gallery-only propagated features of every round (graphs
// of the database computed in advance, Sec. IV-F).  A worker thread admits
// query batches into slots as slots free up; a slot is a fixed partition of
// device memory with its own HIP stream, so requests that arrive while
// others run overlap on the device.  Each request is computed exactly over
// the node set gallery + its queries (see serve.hip), independently of the
// other requests in flight.
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "host.h"

using namespace gcr;
using namespace gcr::host;

namespace {

struct Operand {
  int prec;
  int64_t npad, ld;
  int kch;
  uint8_t* Xs;
  float* n2;
  float* scale;
  float* rn;
};

// Per-slot scratch of one screened search (rows <= rows_cap, ncols columns).
struct KnnScratch {
  int C = 0, S = 0, GS = 1, fb_grid = 8, fb_max = 32, band_cap = 2048, band_max = 0;
  int64_t rows_cap = 0, ncols = 0;
  uint64_t* cand; int* cnt; float* thr;
  uint64_t* cand2; int* cnt2; float* thr2;  // merged groups of GS splits
  unsigned* thr_shared;                       // per-row thresholds shared by the splits
  int* fb_list; int* fb_count; uint64_t* fb_scr;
  uint64_t* fb_pk; uint32_t* fb_pc; float* fb_cut; uint64_t* band; int* band_cnt; int* ovf_list;
  int* heavy_list;
};

void plan_scratch(Arena& ar, KnnScratch& s, int64_t rows_cap, int64_t ncols, int k) {
  s.rows_cap = rows_cap;
  s.ncols = ncols;
  s.C = k + 16 <= 64 ? 64 : (k + 16 <= 128 ? 128 : 256);
  // few rows per request: split the columns over up to 256 workgroups so
  // that the sweep fills the GPU; groups of GS splits are merged before the
  // refine, whose union holds at most 2,048 entries
  int S = 1;
  while ((int64_t)S * 2 * sim_topk_tile_cols() <= ncols && S < 256) S *= 2;
  int GS = 1;
  while ((int64_t)(S / GS) * s.C > 2048) GS *= 2;
  s.S = S;
  s.GS = GS;
  s.band_max = (int)std::min<int64_t>(64, rows_cap);
  s.cand = ar.take<uint64_t>((size_t)rows_cap * S * s.C);
  s.cnt = ar.take<int>((size_t)rows_cap * S);
  s.thr = ar.take<float>((size_t)rows_cap * S);
  s.thr_shared = ar.take<unsigned>((size_t)rows_cap);
  s.cand2 = ar.take<uint64_t>((size_t)rows_cap * (S / GS) * s.C);
  s.cnt2 = ar.take<int>((size_t)rows_cap * (S / GS));
  s.thr2 = ar.take<float>((size_t)rows_cap * (S / GS));
  s.fb_list = ar.take<int>((size_t)rows_cap + 1);
  s.fb_count = ar.take<int>(64);
  s.fb_scr = ar.take<uint64_t>((size_t)s.fb_grid * std::max<int64_t>(ncols, 1));
  const int64_t nch = (ncols + 2047) / 2048;
  const int64_t pairs = std::min<int64_t>(s.fb_max, rows_cap);
  s.fb_pk = ar.take<uint64_t>((size_t)(pairs * nch * k + 1));
  s.fb_pc = ar.take<uint32_t>((size_t)(pairs * nch * k + 1));
  s.fb_cut = ar.take<float>((size_t)rows_cap + 1);
  s.band = ar.take<uint64_t>((size_t)s.band_max * s.band_cap + 1);
  s.band_cnt = ar.take<int>((size_t)s.band_max + 1);
  s.ovf_list = ar.take<int>((size_t)rows_cap + 1);
  s.heavy_list = ar.take<int>((size_t)rows_cap + 1);
}

// Rows [r0, r0 + b) against columns [c0, c1) of the operand: the k nearest
// (distance, index) per row, exact (screening + exact re-score).
void serve_knn(const Operand& op, const float* maxn2, const float* X, int d, const KnnScratch& s, int64_t r0, int b,
               int64_t c0, int64_t c1, int k, int32_t* idx, float* dist, const ColumnFilter& filt, hipStream_t st) {
  fill_u32(s.fb_count, 0u, 3, st);
  fill_u32(s.band_cnt, 0u, s.band_max, st);
  SimArgs sa;
  sa.Xs = op.Xs; sa.npad = op.npad; sa.ld_bytes = op.ld; sa.kchunks = op.kch; sa.n2 = op.n2;
  sa.scale = op.prec == GCR_PREC_FP8 ? op.scale : nullptr;
  sa.cam = nullptr; sa.maxn2 = maxn2; sa.rn = op.rn;
  sa.r0 = r0; sa.r1 = r0 + b; sa.c0 = c0; sa.c1 = c1;
  sa.S = s.S;
  sa.W = roundup((c1 - c0 + s.S - 1) / s.S, sim_topk_tile_cols());
  sa.RB = (b + 127) / 128;
  sa.exclude_self = 0; sa.k0 = k; sa.k1 = 0; sa.C = s.C;
  sa.eps_s = eps_accumulation(op.prec, d); sa.eps_n = eps_norm(d);
  sa.cand = s.cand; sa.cnt = s.cnt; sa.thr = s.thr; sa.thr_init = nullptr;
  sa.filt = filt;
  fill_u32(s.thr_shared, 0xffffffffu, b, st);
  sa.thr_shared = s.thr_shared;
  launch_sim_topk(op.prec, 1, sa, st);
  const uint64_t* cand = s.cand;
  const int* cnt = s.cnt;
  const float* thr = s.thr;
  if (s.GS > 1) {
    MergeArgs m;
    m.cand = s.cand; m.cnt = s.cnt; m.thr = s.thr;
    m.rows = b; m.r0 = r0; m.NL = 1; m.S = s.S; m.GS = s.GS; m.C = s.C; m.k0 = k; m.k1 = 0;
    m.n2 = op.n2; m.rn = op.rn; m.maxn2 = maxn2; m.eps_s = sa.eps_s; m.eps_n = sa.eps_n;
    m.out_cand = s.cand2; m.out_cnt = s.cnt2; m.out_thr = s.thr2;
    launch_merge_splits(m, st);
    cand = s.cand2; cnt = s.cnt2; thr = s.thr2;
  }
  RefineArgs ra;
  ra.cand = cand; ra.cnt = cnt; ra.thr = thr; ra.S = s.S / s.GS; ra.C = s.C; ra.NL = 1; ra.k0 = k; ra.k1 = 0;
  ra.r0 = r0; ra.r1 = r0 + b; ra.c0 = c0; ra.c1 = c1; ra.exclude_self = 0;
  ra.X = X; ra.d = d; ra.cam = nullptr; ra.n2 = op.n2; ra.rn = op.rn; ra.maxn2 = maxn2;
  ra.eps_s = sa.eps_s; ra.eps_n = sa.eps_n;
  ra.idx0 = idx; ra.dist0 = dist; ra.idx1 = nullptr; ra.dist1 = nullptr;
  ra.fb_list = s.fb_list; ra.fb_count = s.fb_count; ra.stat_cands = nullptr;
  ra.fb_scratch = s.fb_scr; ra.fb_grid = s.fb_grid; ra.fb_max = s.fb_max;
  ra.fb_part_key = s.fb_pk; ra.fb_part_col = s.fb_pc;
  ra.fb_cut = s.fb_cut; ra.eps32 = eps_accumulation(GCR_PREC_FP32, d);
  ra.band = s.band; ra.band_cnt = s.band_cnt; ra.band_cap = s.band_cap; ra.band_max = s.band_max;
  ra.ovf_list = s.ovf_list; ra.ovf_count = s.fb_count + 1;
  ra.heavy_list = s.heavy_list; ra.heavy_count = s.fb_count + 2;
  ra.order = nullptr;
  ra.filt = filt;
  launch_refine(ra, st);
}

struct Request {
  uint64_t ticket = 0;
  int b = 0;
  std::vector<float> q;
  std::vector<int32_t> idx;
  std::vector<float> dist;
  gcr_status status = GCR_OK;
  std::string err;
  bool done = false;
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  Request* req = nullptr;
  uint32_t stamp = 0;
  int64_t qbase = 0, pbase = 0;
  KnnScratch kn0, knA, knB;
  int32_t* q_idx; float* q_dist; float* q_w; float* Dq; uint64_t* keys;
  uint32_t* touched; float* dD; int32_t* seg_start; int32_t* seg_len; int32_t* T_list;
  int* counts;  // [0] touched items, [t] rows recomputed in round t
  std::vector<uint32_t*> mark;
  std::vector<int32_t*> pos, list;
  int32_t* ia; float* da; int32_t* ib; float* db; int32_t* oi; float* od;
  unsigned* maxL; unsigned* scratch_max;
  float* h_q = nullptr; int32_t* h_idx = nullptr; float* h_dist = nullptr; int* h_counts = nullptr;
};

}  // namespace

struct gcr_server {
  int device = 0;
  gcr_params p;
  int64_t G = 0;
  int d = 0, k = 0, L = 0, K = 0, S = 0, Rq = 0, Rc = 0, P = 0, prec = 0;
  int64_t rows_total = 0;
  void* mem = nullptr;
  std::vector<float*> X;
  Operand op0, opL;
  unsigned* max0 = nullptr;
  unsigned* maxLg = nullptr;
  gcr_graph g;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Request*> pending;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  bool stop = false;
  std::thread worker;
  std::string err;
  gcr_server_stats stats;
};

namespace {

gcr_status sfail(gcr_server* s, gcr_status st, const std::string& m) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->err = m;
  return st;
}

#define SRV_HIP(expr)                                                                             \
  do {                                                                                            \
    hipError_t e_ = (expr);                                                                       \
    if (e_ != hipSuccess) return std::string(#expr) + ": " + hipGetErrorString(e_);               \
  } while (0)

int pow2_at_least(int x) {
  int p = 64;
  while (p < x) p <<= 1;
  return p;
}

// Enqueue one request on its slot's stream; returns "" or an error message.
std::string enqueue_request(gcr_server* s, Slot& sl, Request& r) {
  const hipStream_t st = sl.st;
  const int b = r.b, d = s->d, k = s->k, K = s->K, L = s->L;
  if (++sl.stamp == 0) sl.stamp = 1;
  const uint32_t stamp = sl.stamp;
  memcpy(sl.h_q, r.q.data(), (size_t)b * d * sizeof(float));
  float* q0 = s->X[0] + sl.qbase * d;
  SRV_HIP(hipMemcpyAsync(q0, sl.h_q, (size_t)b * d * sizeof(float), hipMemcpyHostToDevice, st));
  if (s->p.normalize_input) launch_normalize_rows(q0, q0, b, d, st);
  launch_screen_prep_rows(s->prec, s->X[0], sl.qbase, b, nullptr, d, s->op0.Xs, s->op0.ld, s->op0.n2, s->op0.scale,
                          s->op0.rn, sl.scratch_max, st);
  if (L == 0) {
    serve_knn(s->op0, (const float*)s->max0, s->X[0], d, sl.knA, sl.qbase, b, 0, s->G, K, sl.oi, sl.od,
              ColumnFilter{}, st);
  } else {
    serve_knn(s->op0, (const float*)s->max0, s->X[0], d, sl.kn0, sl.qbase, b, 0, s->G, k, sl.q_idx, sl.q_dist,
              ColumnFilter{}, st);
    const int P = pow2_at_least(b * k);
    launch_serve_query_edges(b, k, sl.q_idx, sl.q_dist, s->p.gamma, sl.q_w, sl.Dq, sl.keys, P, st);
    launch_serve_sort_pairs(sl.keys, P, st);
    fill_u32(sl.counts, 0u, L + 1, st);
    launch_serve_touched(sl.keys, b * k, sl.q_w, stamp, sl.touched, sl.dD, sl.seg_start, sl.seg_len, sl.T_list,
                         sl.counts, st);
    for (int t = 1; t <= L; ++t) {
      const int32_t* src = t == 1 ? sl.T_list : sl.list[t - 1];
      const int src_cap = t == 1 ? s->Rq * k : s->Rc;
      launch_serve_expand(src, sl.counts + (t - 1), src_cap, s->g.idx, k, s->g.rev_ptr, s->g.rev_src, stamp,
                          sl.mark[t], sl.pos[t], sl.list[t], sl.counts + t, s->Rc, st);
      ServePropArgs a;
      a.d = d; a.k = k; a.b = b;
      a.Xprev = s->X[t - 1]; a.Xcur = s->X[t];
      a.qbase = sl.qbase; a.pbase = sl.pbase;
      a.gidx = s->g.idx; a.gw = s->g.w; a.rev_ptr = s->g.rev_ptr; a.rev_src = s->g.rev_src; a.rev_w = s->g.rev_w;
      a.D0 = s->g.deg;
      a.stamp = stamp;
      a.touched = sl.touched; a.dD = sl.dD; a.seg_start = sl.seg_start; a.seg_len = sl.seg_len;
      a.pair_keys = sl.keys; a.q_idx = sl.q_idx; a.q_w = sl.q_w; a.Dq = sl.Dq;
      a.prev_mark = t > 1 ? sl.mark[t - 1] : nullptr;
      a.prev_pos = t > 1 ? sl.pos[t - 1] : nullptr;
      a.cur_list = sl.list[t]; a.cur_pos = sl.pos[t]; a.cur_count = sl.counts + t; a.cap = s->Rc;
      launch_serve_propagate(a, st);
    }
    // final top-K over the round-L features: unchanged gallery rows from the
    // resident copy (recomputed ones masked out), recomputed rows from the
    // slot, merged
    launch_copy_u32(s->maxLg, sl.maxL, 2, st);
    launch_screen_prep_rows(s->prec, s->X[L], sl.qbase, b, nullptr, d, s->opL.Xs, s->opL.ld, s->opL.n2,
                            s->opL.scale, s->opL.rn, sl.scratch_max, st);
    launch_screen_prep_rows(s->prec, s->X[L], sl.pbase, s->Rc, sl.counts + L, d, s->opL.Xs, s->opL.ld, s->opL.n2,
                            s->opL.scale, s->opL.rn, sl.maxL, st);
    ColumnFilter fa;
    fa.stamp_of = sl.mark[L];
    fa.stamp = stamp;
    serve_knn(s->opL, (const float*)sl.maxL, s->X[L], d, sl.knA, sl.qbase, b, 0, s->G, K, sl.ia, sl.da, fa, st);
    ColumnFilter fb;
    fb.count = sl.counts + L;
    serve_knn(s->opL, (const float*)sl.maxL, s->X[L], d, sl.knB, sl.qbase, b, sl.pbase, sl.pbase + s->Rc, K, sl.ib,
              sl.db, fb, st);
    launch_serve_merge(b, K, sl.ia, sl.da, sl.ib, sl.db, sl.list[L], sl.oi, sl.od, st);
    SRV_HIP(hipMemcpyAsync(sl.h_counts, sl.counts, (size_t)(L + 1) * sizeof(int), hipMemcpyDeviceToHost, st));
  }
  SRV_HIP(hipMemcpyAsync(sl.h_idx, sl.oi, (size_t)b * K * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SRV_HIP(hipMemcpyAsync(sl.h_dist, sl.od, (size_t)b * K * sizeof(float), hipMemcpyDeviceToHost, st));
  SRV_HIP(hipGetLastError());
  SRV_HIP(hipEventRecord(sl.ev, st));
  return "";
}

// Results of a finished slot into its request (worker thread, unlocked).
void collect(gcr_server* s, Slot& sl) {
  Request& r = *sl.req;
  const size_t m = (size_t)r.b * s->K;
  r.idx.assign(sl.h_idx, sl.h_idx + m);
  r.dist.assign(sl.h_dist, sl.h_dist + m);
  int worst = 0;
  for (int t = 1; t <= s->L; ++t) worst = std::max(worst, sl.h_counts[t]);
  if (worst > s->Rc) {
    r.status = GCR_ERR_UNSUPPORTED;
    r.err = "request touches " + std::to_string(worst) + " gallery rows within the propagation depth, more than the "
            "slot capacity of " + std::to_string(s->Rc);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  s->stats.requests_done += 1;
  s->stats.queries_done += r.b;
  s->stats.max_recomputed_rows = std::max<int64_t>(s->stats.max_recomputed_rows, worst);
}

void worker_main(gcr_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool busy = false;
    for (Slot& sl : s->slots) {
      if (!sl.req && !s->pending.empty() && !s->stop) {
        Request* r = s->pending.front();
        s->pending.pop_front();
        sl.req = r;
        lk.unlock();
        const std::string e = enqueue_request(s, sl, *r);
        lk.lock();
        if (!e.empty()) {
          (void)hipStreamSynchronize(sl.st);
          r->status = GCR_ERR_HIP;
          r->err = e;
          r->done = true;
          sl.req = nullptr;
          s->cv_done.notify_all();
        }
      }
      if (sl.req) busy = true;
    }
    if (s->stop) {
      while (!s->pending.empty()) {
        Request* r = s->pending.front();
        s->pending.pop_front();
        r->status = GCR_ERR_INVALID;
        r->err = "server destroyed before the request started";
        r->done = true;
      }
      s->cv_done.notify_all();
      if (!busy) break;
    }
    if (!busy) {
      s->cv_work.wait(lk, [&] { return s->stop || !s->pending.empty(); });
      continue;
    }
    lk.unlock();
    bool progressed = false;
    for (Slot& sl : s->slots) {
      if (!sl.req) continue;
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipErrorNotReady) continue;
      if (q == hipSuccess) {
        collect(s, sl);
      } else {
        sl.req->status = GCR_ERR_HIP;
        sl.req->err = std::string("request failed on the device: ") + hipGetErrorString(q);
      }
      std::lock_guard<std::mutex> g2(s->mu);
      sl.req->done = true;
      sl.req = nullptr;
      s->cv_done.notify_all();
      progressed = true;
    }
    if (!progressed) std::this_thread::sleep_for(std::chrono::microseconds(20));
    lk.lock();
  }
}

// Device memory of the server (two-pass planner: dry run for the size).
void plan_server(Arena& ar, gcr_server* s) {
  const int64_t npad = roundup(s->rows_total, 128) + 128;
  s->X.assign(s->L + 1, nullptr);
  for (int t = 0; t <= s->L; ++t) s->X[t] = ar.take<float>((size_t)s->rows_total * s->d);
  auto plan_op = [&](Operand& o) {
    o.prec = s->prec;
    o.npad = npad;
    o.ld = roundup((int64_t)s->d * esize_of(s->prec), 128);
    o.kch = (int)(o.ld / 128);
    o.Xs = ar.take<uint8_t>((size_t)(npad * o.ld));
    o.n2 = ar.take<float>(npad);
    o.scale = ar.take<float>(npad);
    o.rn = ar.take<float>(npad);
  };
  plan_op(s->op0);
  if (s->L > 0) plan_op(s->opL);
  else s->opL = s->op0;
  s->max0 = ar.take<unsigned>(64);
  s->maxLg = ar.take<unsigned>(64);
  void* gbuf = ar.take<char>(gcr_graph_bytes(s->G, s->k, 0, 0));
  if (gbuf) gcr_graph_bind(&s->g, gbuf, s->G, s->k, 0, 0);
  for (Slot& sl : s->slots) {
    plan_scratch(ar, sl.kn0, s->Rq, s->G, s->k);
    plan_scratch(ar, sl.knA, s->Rq, s->G, s->K);
    plan_scratch(ar, sl.knB, s->Rq, s->Rc, s->K);
    const int64_t qk = (int64_t)s->Rq * s->k;
    sl.q_idx = ar.take<int32_t>((size_t)qk);
    sl.q_dist = ar.take<float>((size_t)qk);
    sl.q_w = ar.take<float>((size_t)s->P);
    sl.Dq = ar.take<float>((size_t)s->Rq);
    sl.keys = ar.take<uint64_t>((size_t)s->P);
    sl.touched = ar.take<uint32_t>((size_t)s->G);
    sl.dD = ar.take<float>((size_t)s->G);
    sl.seg_start = ar.take<int32_t>((size_t)s->G);
    sl.seg_len = ar.take<int32_t>((size_t)s->G);
    sl.T_list = ar.take<int32_t>((size_t)qk);
    sl.counts = ar.take<int>(64);
    sl.mark.assign(s->L + 1, nullptr);
    sl.pos.assign(s->L + 1, nullptr);
    sl.list.assign(s->L + 1, nullptr);
    for (int t = 1; t <= s->L; ++t) {
      sl.mark[t] = ar.take<uint32_t>((size_t)s->G);
      sl.pos[t] = ar.take<int32_t>((size_t)s->G);
      sl.list[t] = ar.take<int32_t>((size_t)s->Rc);
    }
    const int64_t qK = (int64_t)s->Rq * s->K;
    sl.ia = ar.take<int32_t>((size_t)qK); sl.da = ar.take<float>((size_t)qK);
    sl.ib = ar.take<int32_t>((size_t)qK); sl.db = ar.take<float>((size_t)qK);
    sl.oi = ar.take<int32_t>((size_t)qK); sl.od = ar.take<float>((size_t)qK);
    sl.maxL = ar.take<unsigned>(64);
    sl.scratch_max = ar.take<unsigned>(64);
  }
}

void release(gcr_server* s) {
  for (Slot& sl : s->slots) {
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.h_q) (void)hipHostFree(sl.h_q);
    if (sl.h_idx) (void)hipHostFree(sl.h_idx);
    if (sl.h_dist) (void)hipHostFree(sl.h_dist);
    if (sl.h_counts) (void)hipHostFree(sl.h_counts);
  }
  if (s->mem) (void)hipFree(s->mem);
  delete s;
}

}  // namespace

extern "C" {

void gcr_server_config_default(gcr_server_config* c) {
  if (!c) return;
  c->slots = 4;
  c->max_batch = 512;
  c->max_recomputed = 65536;
}

gcr_status gcr_server_create(gcr_ctx* ctx, const void* gallery, int32_t gallery_dtype, int64_t ng, int32_t d,
                             const gcr_params* p, const gcr_server_config* cfg, gcr_server** out) {
  if (!ctx || !out) return GCR_ERR_INVALID;
  *out = nullptr;
  const gcr_status pst = check_params(ctx, p);
  if (pst != GCR_OK) return pst;
  if (!gallery || ng < 2 || d <= 0) return fail(ctx, GCR_ERR_INVALID, "bad gallery / ng / d");
  if (gallery_dtype != 0 && gallery_dtype != 1) return fail(ctx, GCR_ERR_INVALID, "gallery_dtype must be 0 or 1");
  if (d > 2048) return fail(ctx, GCR_ERR_UNSUPPORTED, "d above 2048 is not supported");
  if (ng > (int64_t)1 << 30) return fail(ctx, GCR_ERR_UNSUPPORTED, "galleries above 2^30 items are not supported");
  if (p->k < 1) return fail(ctx, GCR_ERR_INVALID, "serving needs k >= 1");
  if (p->topk_out < 1 || p->topk_out > 120) return fail(ctx, GCR_ERR_UNSUPPORTED, "top-K output must be in 1..120");
  if (p->rebuild_each_round) return fail(ctx, GCR_ERR_INVALID, "serving keeps the gallery graph fixed "
                                                               "(rebuild_each_round must be 0)");
  if (p->symmetric != 1) return fail(ctx, GCR_ERR_UNSUPPORTED, "serving uses the symmetric normalisation");
  gcr_server_config c;
  gcr_server_config_default(&c);
  if (cfg) c = *cfg;
  if (c.slots < 1 || c.slots > 16) return fail(ctx, GCR_ERR_INVALID, "slots must be in 1..16");
  if (c.max_batch < 1 || c.max_recomputed < 1) return fail(ctx, GCR_ERR_INVALID, "bad slot capacities");
  HIP_TRY(ctx, hipSetDevice(ctx->device));

  gcr_server* s = new gcr_server();
  s->device = ctx->device;
  s->p = *p;
  s->G = ng;
  s->d = d;
  s->k = p->k;
  s->L = p->rounds;
  s->K = p->topk_out;
  s->prec = p->precision;
  s->S = c.slots;
  s->Rq = std::min(c.max_batch, 16384 / p->k);
  s->Rc = (int)std::min<int64_t>(c.max_recomputed, ng);
  s->P = pow2_at_least(s->Rq * p->k);
  s->rows_total = ng + (int64_t)s->S * (s->Rq + s->Rc);
  s->slots.resize(s->S);
  for (int i = 0; i < s->S; ++i) {
    s->slots[i].qbase = ng + (int64_t)i * (s->Rq + s->Rc);
    s->slots[i].pbase = s->slots[i].qbase + s->Rq;
  }
  memset(&s->stats, 0, sizeof s->stats);
  s->stats.slots = s->S;
  s->stats.max_batch = s->Rq;
  s->stats.max_recomputed = s->Rc;

  Arena dry;
  plan_server(dry, s);
  s->stats.device_bytes = (int64_t)dry.off;
  if (hipMalloc(&s->mem, dry.off) != hipSuccess) {
    (void)hipGetLastError();
    s->mem = nullptr;
    release(s);
    return fail(ctx, GCR_ERR_NOMEM, "server allocation of %zu bytes failed", dry.off);
  }
  Arena ar{(char*)s->mem, 0};
  plan_server(ar, s);

  hipStream_t st = nullptr;
  auto bail = [&](gcr_status code, const char* what, hipError_t e) {
    if (st) (void)hipStreamDestroy(st);
    release(s);
    return fail(ctx, code, "%s: %s", what, hipGetErrorString(e));
  };
  hipError_t e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
  if (e != hipSuccess) return bail(GCR_ERR_HIP, "stream", e);
  // resident gallery: level-0 features as given (float32, or BF16 widened)
  if (gallery_dtype == 0)
    e = hipMemcpyAsync(s->X[0], gallery, (size_t)ng * d * sizeof(float), hipMemcpyDeviceToDevice, st);
  else
    launch_bf16_to_f32((const uint16_t*)gallery, s->X[0], ng * d, st);
  if (e != hipSuccess) return bail(GCR_ERR_HIP, "gallery copy", e);
  // frozen gallery graph (fixed mode, one list, no camera weighting)
  gcr_params gp = *p;
  gp.alpha = 1.0f;
  gp.beta_same = gp.beta_cross = 1.0f;
  {
    Arena d1;
    KnnPlan kp;
    GraphTmp gt;
    plan_knn(d1, kp, gp.precision, ng, d, 0, ng, 0, ng, gp.k, 0);
    plan_graph_tmp(d1, gt, ng);
    if (ensure_ws(ctx, d1.off) != GCR_OK) {
      (void)hipStreamDestroy(st);
      release(s);
      return GCR_ERR_NOMEM;
    }
    Arena a1{(char*)ctx->ws, 0};
    plan_knn(a1, kp, gp.precision, ng, d, 0, ng, 0, ng, gp.k, 0);
    plan_graph_tmp(a1, gt, ng);
    enqueue_build_graph(ctx, kp, gt, s->X[0], ng, d, nullptr, &gp, &s->g, st, false);
    for (int t = 1; t <= s->L; ++t) enqueue_propagate(ctx, &s->g, s->X[t - 1], s->X[t], ng, d, st, gt.order);
    fill_u32(s->max0, 0u, 2, st);
    launch_screen_prep_rows(s->prec, s->X[0], 0, ng, nullptr, d, s->op0.Xs, s->op0.ld, s->op0.n2, s->op0.scale,
                            s->op0.rn, s->max0, st);
    if (s->L > 0) {
      fill_u32(s->maxLg, 0u, 2, st);
      launch_screen_prep_rows(s->prec, s->X[s->L], 0, ng, nullptr, d, s->opL.Xs, s->opL.ld, s->opL.n2,
                              s->opL.scale, s->opL.rn, s->maxLg, st);
    }
    // marks start clear; positions start in range, so a row marked in a
    // request whose set overflowed still reads inside the slot (that
    // request is reported as failed)
    for (Slot& sl : s->slots) {
      fill_u32(sl.touched, 0u, ng, st);
      for (int t = 1; t <= s->L; ++t) {
        fill_u32(sl.mark[t], 0u, ng, st);
        fill_u32(sl.pos[t], 0u, ng, st);
      }
    }
    e = hipStreamSynchronize(st);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return bail(GCR_ERR_HIP, "gallery preparation", e);
  }
  (void)hipStreamDestroy(st);
  st = nullptr;
  for (Slot& sl : s->slots) {
    e = hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_q, (size_t)s->Rq * d * sizeof(float), hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&sl.h_idx, (size_t)s->Rq * s->K * sizeof(int32_t), hipHostMallocDefault);
    if (e == hipSuccess)
      e = hipHostMalloc((void**)&sl.h_dist, (size_t)s->Rq * s->K * sizeof(float), hipHostMallocDefault);
    if (e == hipSuccess) e = hipHostMalloc((void**)&sl.h_counts, 64 * sizeof(int), hipHostMallocDefault);
    if (e != hipSuccess) return bail(GCR_ERR_HIP, "slot set-up", e);
    memset(sl.h_counts, 0, 64 * sizeof(int));
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return GCR_OK;
}

gcr_status gcr_server_submit(gcr_server* s, const float* q_host, int32_t b, uint64_t* ticket) {
  if (!s || !ticket) return GCR_ERR_INVALID;
  if (!q_host || b < 1) return sfail(s, GCR_ERR_INVALID, "queries must be a host array of b >= 1 rows");
  if (b > s->Rq)
    return sfail(s, GCR_ERR_INVALID, "batch of " + std::to_string(b) + " queries exceeds the slot capacity of " +
                                         std::to_string(s->Rq));
  auto r = std::make_unique<Request>();
  r->b = b;
  r->q.assign(q_host, q_host + (size_t)b * s->d);
  std::lock_guard<std::mutex> lk(s->mu);
  if (s->stop) {
    s->err = "server is shutting down";
    return GCR_ERR_INVALID;
  }
  r->ticket = s->next_ticket++;
  *ticket = r->ticket;
  s->pending.push_back(r.get());
  s->reqs.emplace(r->ticket, std::move(r));
  s->cv_work.notify_one();
  return GCR_OK;
}

gcr_status gcr_server_wait(gcr_server* s, uint64_t ticket, int32_t* idx_host, float* dist_host, int32_t timeout_ms) {
  if (!s) return GCR_ERR_INVALID;
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(ticket);
  if (it == s->reqs.end()) {
    s->err = "unknown ticket";
    return GCR_ERR_INVALID;
  }
  Request* r = it->second.get();
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, [&] { return r->done; });
  } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), [&] { return r->done; })) {
    return GCR_ERR_TIMEOUT;
  }
  const gcr_status st = r->status;
  if (st == GCR_OK) {
    if (idx_host) memcpy(idx_host, r->idx.data(), r->idx.size() * sizeof(int32_t));
    if (dist_host) memcpy(dist_host, r->dist.data(), r->dist.size() * sizeof(float));
  } else {
    s->err = r->err;
  }
  s->reqs.erase(it);
  return st;
}

gcr_status gcr_server_get_stats(gcr_server* s, gcr_server_stats* out) {
  if (!s || !out) return GCR_ERR_INVALID;
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->stats;
  return GCR_OK;
}

const char* gcr_server_last_error(const gcr_server* s) { return s ? s->err.c_str() : "server is NULL"; }

gcr_status gcr_server_destroy(gcr_server* s) {
  if (!s) return GCR_ERR_INVALID;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
  }
  s->cv_work.notify_all();
  if (s->worker.joinable()) s->worker.join();
  (void)hipSetDevice(s->device);
  for (Slot& sl : s->slots)
    if (sl.st) (void)hipStreamSynchronize(sl.st);
  release(s);
  return GCR_OK;
}

}  // extern "C"
