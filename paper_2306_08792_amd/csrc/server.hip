// Serving loop.  A gallery stays resident in HBM with its frozen kNN graph,
// degrees and the gallery-only propagated features of every round (graphs
// of the database computed in advance, Sec. IV-F).  Requests are batched
// continuously: a worker thread hands the queued requests to a scheduler
// (scheduler.h) that forms a batch whenever one of the server's lanes is
// free, taking requests in order while their query rows fit the lane's
// query region and a request scratch slot (the per-request device memory,
// counted from the memory budget) is free.  A batch runs on its lane's HIP
// stream, so batches overlap on the device while new requests queue.
//
// Within a batch the two gallery sweeps are shared by all its queries: one
// screened kNN search of every query row over the gallery, and one final
// top-K search over the gallery's round-L features in which every row
// leaves out the gallery rows its own request recomputed (a per-row mask).
// Between them each request is computed exactly over the node set
// gallery + its own queries (see serve.hip), independently of the other
// requests, in its own scratch slot; its recomputed rows get a small search
// of their own and are merged into its rows' lists.  A query row's result
// therefore does not depend on which requests share its batch.
//
// The gallery is mutable: rows are appended or removed between requests and
// its kNN lists are maintained exactly (gallery.hip), after which the graph,
// degrees, gallery-only rounds and screening operands are recomputed from
// the lists.  Items carry external ids; the device gallery stays dense.
#include <stdio.h>
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
#include "scheduler.h"

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
  sa.Xs = op.Xs; sa.npad = op.npad; sa.ld_bytes = op.ld; sa.n2 = op.n2;
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

// Scratch of one request (a scheduler slot): its query edges, the hop sets
// of every round (stamped marks and positions over the gallery) and the
// rows it recomputes, which live in the slot's region [pbase, pbase + Rc)
// of the feature arrays.
struct ReqSlot {
  int64_t pbase = 0;
  float* q_w; float* Dq; uint64_t* keys; int32_t* T_list;
  int* counts;  // [0] touched items, [t] rows recomputed in round t
  std::vector<uint32_t*> mark;
  std::vector<int32_t*> pos, list;
};

// A lane runs one batch at a time on its own stream: query rows
// [qbase, qbase + max_batch) of the feature arrays, the shared sweeps'
// scratch and outputs, and pinned host buffers for the batch's queries and
// results.
struct Lane {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  int64_t qbase = 0;
  KnnScratch kn0, knA, knB;
  int32_t* q_idx; float* q_dist;               // [max_batch, k] the queries' gallery lists
  int32_t* ia; float* da; int32_t* ib; float* db;
  int32_t* oi; float* od;                      // [max_batch, K]
  uint32_t* touched; float* dD; int32_t* seg_start; int32_t* seg_len;  // [Gcap], stamped
  unsigned* maxL; unsigned* scratch_max;
  const uint32_t** row_mark; uint32_t* row_stamp;  // [max_batch] final sweep masks
  float* h_q = nullptr; int32_t* h_idx = nullptr; float* h_dist = nullptr; int* h_counts = nullptr;
  const uint32_t** h_row_mark = nullptr; uint32_t* h_row_stamp = nullptr;
  bool busy = false;
  SchedBatch batch;
  std::vector<Request*> reqs;
};

}  // namespace

struct gcr_server {
  int device = 0;
  gcr_params p;
  int64_t G = 0;      // live gallery rows (dense, rows [0, G))
  int64_t Gcap = 0;   // gallery capacity (rows reserved)
  gcr_ctx* mctx = nullptr;         // private context for gallery maintenance
  hipStream_t mst = nullptr;       // its stream
  std::vector<int32_t> ext;        // external id of every gallery row, increasing
  int64_t next_id = 0;
  bool paused = false;             // no new request starts while set
  std::mutex mut_mu;               // one gallery mutation at a time
  int32_t* tmp_idx = nullptr;      // [Gcap, k + 1] list scratch
  float* tmp_dist = nullptr;
  int32_t* map_a = nullptr;        // [Gcap] row maps
  int32_t* map_b = nullptr;
  int32_t* repair = nullptr;       // [Gcap] rows whose lists are searched again
  int* mcount = nullptr;           // [64] device counters
  int d = 0, k = 0, L = 0, K = 0, prec = 0;
  int NL = 0;       // lanes (batches in flight)
  int Rq = 0;       // query rows of one batch (= the largest request)
  int MR = 0;       // requests of one batch
  int NS = 0;       // request scratch slots
  int Rc = 0;       // gallery rows recomputed per round and request
  int P = 0;        // sort size of one request's query edges
  int64_t rows_total = 0;
  void* mem = nullptr;
  std::vector<float*> X;
  Operand op0, opL;
  unsigned* max0 = nullptr;
  unsigned* maxLg = nullptr;
  gcr_graph g;
  std::vector<ReqSlot> rslots;
  std::vector<Lane> lanes;
  std::unique_ptr<Scheduler> sched;
  uint32_t next_stamp = 0;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::unordered_map<uint64_t, std::unique_ptr<Request>> reqs;
  uint64_t next_ticket = 1;
  int lanes_signalled = 0;  // completions reported by stream callbacks
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

// Host callback at the end of a batch's stream work: wake the worker.
void batch_done_cb(void* arg) {
  gcr_server* s = (gcr_server*)arg;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->lanes_signalled += 1;
  }
  s->cv_work.notify_all();
}

// Enqueue one batch on its lane's stream; returns "" or an error message.
std::string enqueue_batch(gcr_server* s, Lane& ln) {
  const hipStream_t st = ln.st;
  const SchedBatch& bt = ln.batch;
  const int B = bt.rows, d = s->d, k = s->k, K = s->K, L = s->L;
  for (size_t r = 0; r < bt.items.size(); ++r)
    memcpy(ln.h_q + (size_t)bt.items[r].row0 * d, ln.reqs[r]->q.data(), (size_t)bt.items[r].b * d * sizeof(float));
  float* q0 = s->X[0] + ln.qbase * d;
  SRV_HIP(hipMemcpyAsync(q0, ln.h_q, (size_t)B * d * sizeof(float), hipMemcpyHostToDevice, st));
  if (s->p.normalize_input) launch_normalize_rows(q0, q0, B, d, st);
  launch_screen_prep_rows(s->op0.prec, s->X[0], ln.qbase, B, nullptr, d, s->op0.Xs, s->op0.ld, s->op0.n2,
                          s->op0.scale, s->op0.rn, ln.scratch_max, st);
  if (L == 0) {
    // no rounds: the final top-K of every query over the gallery as given
    serve_knn(s->op0, (const float*)s->max0, s->X[0], d, ln.knA, ln.qbase, B, 0, s->G, K, ln.oi, ln.od,
              ColumnFilter{}, st);
  } else {
    // the shared sweep: every query's k nearest gallery items
    serve_knn(s->op0, (const float*)s->max0, s->X[0], d, ln.kn0, ln.qbase, B, 0, s->G, k, ln.q_idx, ln.q_dist,
              ColumnFilter{}, st);
    launch_copy_u32(s->maxLg, ln.maxL, 2, st);
    // each request over gallery + its own queries, in its own slot
    for (size_t r = 0; r < bt.items.size(); ++r) {
      const SchedItem& it = bt.items[r];
      ReqSlot& rs = s->rslots[it.slot];
      const uint32_t stamp = ln.h_row_stamp[it.row0];
      const int b = it.b;
      const int P = pow2_at_least(b * k);
      launch_serve_query_edges(b, k, ln.q_idx + (int64_t)it.row0 * k, ln.q_dist + (int64_t)it.row0 * k, s->p.gamma,
                               rs.q_w, rs.Dq, rs.keys, P, st);
      launch_serve_sort_pairs(rs.keys, P, st);
      fill_u32(rs.counts, 0u, L + 1, st);
      launch_serve_touched(rs.keys, b * k, rs.q_w, stamp, ln.touched, ln.dD, ln.seg_start, ln.seg_len, rs.T_list,
                           rs.counts, st);
      for (int t = 1; t <= L; ++t) {
        const int32_t* src = t == 1 ? rs.T_list : rs.list[t - 1];
        const int src_cap = t == 1 ? s->Rq * k : s->Rc;
        launch_serve_expand(src, rs.counts + (t - 1), src_cap, s->g.idx, k, s->g.rev_ptr, s->g.rev_src, stamp,
                            rs.mark[t], rs.pos[t], rs.list[t], rs.counts + t, s->Rc, st);
        ServePropArgs a;
        a.d = d; a.k = k; a.b = b;
        a.Xprev = s->X[t - 1]; a.Xcur = s->X[t];
        a.qbase = ln.qbase + it.row0; a.pbase = rs.pbase;
        a.gidx = s->g.idx; a.gw = s->g.w; a.rev_ptr = s->g.rev_ptr; a.rev_src = s->g.rev_src; a.rev_w = s->g.rev_w;
        a.D0 = s->g.deg;
        a.stamp = stamp;
        a.touched = ln.touched; a.dD = ln.dD; a.seg_start = ln.seg_start; a.seg_len = ln.seg_len;
        a.pair_keys = rs.keys; a.q_idx = ln.q_idx + (int64_t)it.row0 * k; a.q_w = rs.q_w; a.Dq = rs.Dq;
        a.prev_mark = t > 1 ? rs.mark[t - 1] : nullptr;
        a.prev_pos = t > 1 ? rs.pos[t - 1] : nullptr;
        a.cur_list = rs.list[t]; a.cur_pos = rs.pos[t]; a.cur_count = rs.counts + t; a.cap = s->Rc;
        launch_serve_propagate(a, st);
      }
      // the request's recomputed rows into the round-L operand (their
      // maxima widen the batch's screening margin)
      launch_screen_prep_rows(s->opL.prec, s->X[L], rs.pbase, s->Rc, rs.counts + L, d, s->opL.Xs, s->opL.ld,
                              s->opL.n2, s->opL.scale, s->opL.rn, ln.maxL, st);
      SRV_HIP(hipMemcpyAsync(ln.h_counts + r * 64, rs.counts, (size_t)(L + 1) * sizeof(int), hipMemcpyDeviceToHost,
                             st));
    }
    // the shared final sweep over the unchanged gallery rows: every row
    // leaves out the rows its own request recomputed
    launch_screen_prep_rows(s->opL.prec, s->X[L], ln.qbase, B, nullptr, d, s->opL.Xs, s->opL.ld, s->opL.n2,
                            s->opL.scale, s->opL.rn, ln.scratch_max, st);
    SRV_HIP(hipMemcpyAsync(ln.row_mark, ln.h_row_mark, (size_t)B * sizeof(uint32_t*), hipMemcpyHostToDevice, st));
    SRV_HIP(hipMemcpyAsync(ln.row_stamp, ln.h_row_stamp, (size_t)B * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    ColumnFilter fa;
    fa.row_mark = ln.row_mark;
    fa.row_stamp = ln.row_stamp;
    serve_knn(s->opL, (const float*)ln.maxL, s->X[L], d, ln.knA, ln.qbase, B, 0, s->G, K, ln.ia, ln.da, fa, st);
    // each request's recomputed rows, merged into its rows' lists
    for (size_t r = 0; r < bt.items.size(); ++r) {
      const SchedItem& it = bt.items[r];
      ReqSlot& rs = s->rslots[it.slot];
      ColumnFilter fb;
      fb.count = rs.counts + L;
      serve_knn(s->opL, (const float*)ln.maxL, s->X[L], d, ln.knB, ln.qbase + it.row0, it.b, rs.pbase,
                rs.pbase + s->Rc, K, ln.ib, ln.db, fb, st);
      launch_serve_merge(it.b, K, ln.ia + (int64_t)it.row0 * K, ln.da + (int64_t)it.row0 * K, ln.ib, ln.db,
                         rs.list[L], ln.oi + (int64_t)it.row0 * K, ln.od + (int64_t)it.row0 * K, st);
    }
  }
  SRV_HIP(hipMemcpyAsync(ln.h_idx, ln.oi, (size_t)B * K * sizeof(int32_t), hipMemcpyDeviceToHost, st));
  SRV_HIP(hipMemcpyAsync(ln.h_dist, ln.od, (size_t)B * K * sizeof(float), hipMemcpyDeviceToHost, st));
  SRV_HIP(hipGetLastError());
  SRV_HIP(hipEventRecord(ln.ev, st));
  SRV_HIP(hipLaunchHostFunc(st, batch_done_cb, s));
  return "";
}

// Results of a finished batch into its requests (worker thread, unlocked).
void collect(gcr_server* s, Lane& ln) {
  const int K = s->K;
  for (size_t r = 0; r < ln.batch.items.size(); ++r) {
    const SchedItem& it = ln.batch.items[r];
    Request& q = *ln.reqs[r];
    const size_t m = (size_t)it.b * K, o = (size_t)it.row0 * K;
    q.idx.assign(ln.h_idx + o, ln.h_idx + o + m);
    for (int32_t& v : q.idx)
      if (v >= 0) v = s->ext[v];
    q.dist.assign(ln.h_dist + o, ln.h_dist + o + m);
    int worst = 0;
    for (int t = 1; t <= s->L; ++t) worst = std::max(worst, ln.h_counts[r * 64 + t]);
    if (worst > s->Rc) {
      q.status = GCR_ERR_UNSUPPORTED;
      q.err = "request touches " + std::to_string(worst) + " gallery rows within the propagation depth, more than "
              "the per-request capacity of " + std::to_string(s->Rc);
    }
    std::lock_guard<std::mutex> lk(s->mu);
    s->stats.requests_done += 1;
    s->stats.queries_done += it.b;
    s->stats.max_recomputed_rows = std::max<int64_t>(s->stats.max_recomputed_rows, worst);
  }
  std::lock_guard<std::mutex> lk(s->mu);
  s->stats.batches_done += 1;
  s->stats.max_batch_requests = std::max<int64_t>(s->stats.max_batch_requests, (int64_t)ln.batch.items.size());
  s->stats.max_batch_rows = std::max<int64_t>(s->stats.max_batch_rows, ln.batch.rows);
}

void worker_main(gcr_server* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    // start batches on the free lanes
    while (!s->stop && !s->paused) {
      SchedBatch bt;
      if (!s->sched->next(&bt)) break;
      Lane& ln = s->lanes[bt.lane];
      ln.batch = bt;
      ln.reqs.clear();
      for (size_t r = 0; r < bt.items.size(); ++r) {
        const SchedItem& it = bt.items[r];
        ln.reqs.push_back(s->reqs.at(it.ticket).get());
        // a stamp per request (never 0): marks of earlier requests in the
        // same slot stay below it and need no clearing
        if (++s->next_stamp == 0) s->next_stamp = 1;
        for (int j = 0; j < it.b; ++j) {
          ln.h_row_mark[it.row0 + j] = s->L > 0 ? s->rslots[it.slot].mark[s->L] : nullptr;
          ln.h_row_stamp[it.row0 + j] = s->next_stamp;
        }
      }
      ln.busy = true;
      lk.unlock();
      const auto te0 = std::chrono::steady_clock::now();
      const std::string e = enqueue_batch(s, ln);
      const auto te1 = std::chrono::steady_clock::now();
      lk.lock();
      s->stats.enqueue_us += std::chrono::duration_cast<std::chrono::microseconds>(te1 - te0).count();
      if (!e.empty()) {
        lk.unlock();
        (void)hipStreamSynchronize(ln.st);
        lk.lock();
        for (Request* r : ln.reqs) {
          r->status = GCR_ERR_HIP;
          r->err = e;
          r->done = true;
        }
        ln.busy = false;
        s->sched->finish(bt.lane);
        s->cv_done.notify_all();
      }
    }
    bool busy = false;
    for (const Lane& ln : s->lanes) busy = busy || ln.busy;
    if (s->stop) {
      for (uint64_t t : s->sched->drain()) {
        Request* r = s->reqs.at(t).get();
        r->status = GCR_ERR_INVALID;
        r->err = "server destroyed before the request started";
        r->done = true;
      }
      s->cv_done.notify_all();
      if (!busy) break;
    }
    if (!busy) {
      s->cv_work.wait(lk, [&] { return s->stop || (s->sched->pending() > 0 && !s->paused); });
      continue;
    }
    // sleep until a stream callback reports a finished batch (or new work
    // can start on a free lane); the timed wait only guards against a lost
    // wake-up
    s->cv_work.wait_for(lk, std::chrono::milliseconds(5), [&] {
      return s->stop || s->lanes_signalled > 0 ||
             (!s->paused && s->sched->pending() > 0 && s->sched->free_lanes() > 0);
    });
    s->lanes_signalled = 0;
    lk.unlock();
    for (size_t l = 0; l < s->lanes.size(); ++l) {
      Lane& ln = s->lanes[l];
      if (!ln.busy) continue;
      const hipError_t q = hipEventQuery(ln.ev);
      if (q == hipErrorNotReady) continue;
      if (q == hipSuccess) {
        collect(s, ln);
      } else {
        for (Request* r : ln.reqs) {
          r->status = GCR_ERR_HIP;
          r->err = std::string("request failed on the device: ") + hipGetErrorString(q);
        }
      }
      std::lock_guard<std::mutex> g2(s->mu);
      for (Request* r : ln.reqs) r->done = true;
      ln.busy = false;
      s->sched->finish((int)l);
      s->cv_done.notify_all();
    }
    lk.lock();
  }
}

// Device memory of one request scratch slot.
void plan_req_slot(Arena& ar, const gcr_server* s, ReqSlot& rs) {
  const int64_t qk = (int64_t)s->Rq * s->k;
  rs.q_w = ar.take<float>((size_t)s->P);
  rs.Dq = ar.take<float>((size_t)s->Rq);
  rs.keys = ar.take<uint64_t>((size_t)s->P);
  rs.T_list = ar.take<int32_t>((size_t)qk);
  rs.counts = ar.take<int>(64);
  rs.mark.assign(s->L + 1, nullptr);
  rs.pos.assign(s->L + 1, nullptr);
  rs.list.assign(s->L + 1, nullptr);
  for (int t = 1; t <= s->L; ++t) {
    rs.mark[t] = ar.take<uint32_t>((size_t)s->Gcap);
    rs.pos[t] = ar.take<int32_t>((size_t)s->Gcap);
    rs.list[t] = ar.take<int32_t>((size_t)s->Rc);
  }
}

// Device memory of the server (two-pass planner: dry run for the size).
void plan_server(Arena& ar, gcr_server* s) {
  const int64_t npad = roundup(s->rows_total, 128) + 128;
  s->X.assign(s->L + 1, nullptr);
  for (int t = 0; t <= s->L; ++t) s->X[t] = ar.take<float>((size_t)s->rows_total * s->d);
  // The final top-K screens in BF16 when the kNN screening is FP8: at
  // K = 100 the K-th neighbour lies among unrelated items, and FP8's margin
  // would admit thousands of them per query (the refine's exhaustive path).
  const int prec_final = final_screen_prec(s->prec);
  auto plan_op = [&](Operand& o, int prec) {
    o.prec = prec;
    o.npad = npad;
    o.ld = roundup((int64_t)s->d * esize_of(prec), 128);
    o.kch = (int)(o.ld / 128);
    o.Xs = ar.take<uint8_t>((size_t)(npad * o.ld));
    o.n2 = ar.take<float>(npad);
    o.scale = ar.take<float>(npad);
    o.rn = ar.take<float>(npad);
  };
  // with no rounds the round-0 operand serves only the final top-K
  plan_op(s->op0, s->L > 0 ? s->prec : prec_final);
  if (s->L > 0) plan_op(s->opL, prec_final);
  else s->opL = s->op0;
  s->max0 = ar.take<unsigned>(64);
  s->maxLg = ar.take<unsigned>(64);
  // graph arrays sized for the capacity; kernels run on the first G rows
  void* gbuf = ar.take<char>(gcr_graph_bytes(s->Gcap, s->k, 0, 0));
  if (gbuf) gcr_graph_bind(&s->g, gbuf, s->Gcap, s->k, 0, 0);
  s->tmp_idx = ar.take<int32_t>((size_t)s->Gcap * (s->k + 1));
  s->tmp_dist = ar.take<float>((size_t)s->Gcap * (s->k + 1));
  s->map_a = ar.take<int32_t>((size_t)s->Gcap);
  s->map_b = ar.take<int32_t>((size_t)s->Gcap);
  s->repair = ar.take<int32_t>((size_t)s->Gcap);
  s->mcount = ar.take<int>(64);
  for (ReqSlot& rs : s->rslots) plan_req_slot(ar, s, rs);
  for (Lane& ln : s->lanes) {
    plan_scratch(ar, ln.kn0, s->Rq, s->Gcap, s->k);
    plan_scratch(ar, ln.knA, s->Rq, s->Gcap, s->K);
    plan_scratch(ar, ln.knB, s->Rq, s->Rc, s->K);
    const int64_t qk = (int64_t)s->Rq * s->k;
    ln.q_idx = ar.take<int32_t>((size_t)qk);
    ln.q_dist = ar.take<float>((size_t)qk);
    ln.touched = ar.take<uint32_t>((size_t)s->Gcap);
    ln.dD = ar.take<float>((size_t)s->Gcap);
    ln.seg_start = ar.take<int32_t>((size_t)s->Gcap);
    ln.seg_len = ar.take<int32_t>((size_t)s->Gcap);
    const int64_t qK = (int64_t)s->Rq * s->K;
    ln.ia = ar.take<int32_t>((size_t)qK); ln.da = ar.take<float>((size_t)qK);
    ln.ib = ar.take<int32_t>((size_t)qK); ln.db = ar.take<float>((size_t)qK);
    ln.oi = ar.take<int32_t>((size_t)qK); ln.od = ar.take<float>((size_t)qK);
    ln.maxL = ar.take<unsigned>(64);
    ln.scratch_max = ar.take<unsigned>(64);
    ln.row_mark = (const uint32_t**)ar.take<uint64_t>((size_t)s->Rq);
    ln.row_stamp = ar.take<uint32_t>((size_t)s->Rq);
  }
}

void release(gcr_server* s) {
  for (Lane& ln : s->lanes) {
    if (ln.ev) (void)hipEventDestroy(ln.ev);
    if (ln.st) (void)hipStreamDestroy(ln.st);
    if (ln.h_q) (void)hipHostFree(ln.h_q);
    if (ln.h_idx) (void)hipHostFree(ln.h_idx);
    if (ln.h_dist) (void)hipHostFree(ln.h_dist);
    if (ln.h_counts) (void)hipHostFree(ln.h_counts);
    if (ln.h_row_mark) (void)hipHostFree(ln.h_row_mark);
    if (ln.h_row_stamp) (void)hipHostFree(ln.h_row_stamp);
  }
  if (s->mst) (void)hipStreamDestroy(s->mst);
  if (s->mem) (void)hipFree(s->mem);
  if (s->mctx) (void)gcr_destroy(s->mctx);
  delete s;
}

}  // namespace

namespace {

// Validation, sizes and the one device allocation of a server over an
// initial gallery of ng rows (nothing computed yet).
gcr_status server_new(gcr_ctx* ctx, const gcr_params* p, const gcr_server_config* cfg, int64_t ng, int32_t d,
                      gcr_server** out) {
  *out = nullptr;
  const gcr_status pst = check_params(ctx, p);
  if (pst != GCR_OK) return pst;
  if (ng < 2 || d <= 0) return fail(ctx, GCR_ERR_INVALID, "bad gallery size / d");
  if (d > 2048) return fail(ctx, GCR_ERR_UNSUPPORTED, "d above 2048 is not supported");
  if (p->k < 1) return fail(ctx, GCR_ERR_INVALID, "serving needs k >= 1");
  if (p->topk_out < 1 || p->topk_out > 120) return fail(ctx, GCR_ERR_UNSUPPORTED, "top-K output must be in 1..120");
  if (p->rebuild_each_round) return fail(ctx, GCR_ERR_INVALID, "serving keeps the gallery graph fixed "
                                                               "(rebuild_each_round must be 0)");
  if (p->symmetric != 1) return fail(ctx, GCR_ERR_UNSUPPORTED, "serving uses the symmetric normalisation");
  if (is_raw_precision(p->precision))
    return fail(ctx, GCR_ERR_UNSUPPORTED, "serving needs an exact mode (raw screening is not served)");
  gcr_server_config c;
  gcr_server_config_default(&c);
  if (cfg) c = *cfg;
  if (c.lanes < 1 || c.lanes > 8) return fail(ctx, GCR_ERR_INVALID, "lanes must be in 1..8");
  if (c.max_batch < 1 || c.max_requests < 1 || c.max_requests > 256 || c.max_recomputed < 1)
    return fail(ctx, GCR_ERR_INVALID, "bad batch capacities (max_batch >= 1, max_requests in 1..256, "
                                      "max_recomputed >= 1)");
  const int64_t cap = c.gallery_capacity > 0 ? c.gallery_capacity : ng;
  if (cap < ng) return fail(ctx, GCR_ERR_INVALID, "gallery_capacity is below the gallery size");
  if (cap > (int64_t)1 << 30) return fail(ctx, GCR_ERR_UNSUPPORTED, "galleries above 2^30 items are not supported");
  HIP_TRY(ctx, hipSetDevice(ctx->device));

  gcr_server* s = new gcr_server();
  s->device = ctx->device;
  s->p = *p;
  s->G = ng;
  s->Gcap = cap;
  s->d = d;
  s->k = p->k;
  s->L = p->rounds;
  s->K = p->topk_out;
  s->prec = p->precision;
  s->NL = c.lanes;
  s->Rq = std::min(c.max_batch, 16384 / p->k);
  s->MR = c.max_requests;
  s->Rc = (int)std::min<int64_t>(c.max_recomputed, cap);
  s->P = pow2_at_least(s->Rq * p->k);
  // request scratch slots: as many as the memory budget holds (at most one
  // per request a full set of lanes can carry), else lanes x max_requests
  Arena one;
  ReqSlot probe;
  plan_req_slot(one, s, probe);
  const int64_t slot_bytes = (int64_t)one.off + (int64_t)s->Rc * d * sizeof(float) * (s->L + 1);
  const int64_t most = (int64_t)s->NL * s->MR;
  int64_t ns = most;
  if (c.mem_budget > 0) {
    ns = std::min<int64_t>(most, (int64_t)(c.mem_budget / (uint64_t)slot_bytes));
    if (ns < 1) {
      delete s;
      return fail(ctx, GCR_ERR_NOMEM, "memory budget of %llu bytes is below one request's scratch (%lld bytes)",
                  (unsigned long long)c.mem_budget, (long long)slot_bytes);
    }
  }
  s->NS = (int)ns;
  s->rows_total = cap + (int64_t)s->NL * s->Rq + (int64_t)s->NS * s->Rc;
  {
    const gcr_status ost = check_operand(ctx, p->precision, s->rows_total, d);
    if (ost != GCR_OK) {
      delete s;
      return ost;
    }
  }
  s->lanes.resize(s->NL);
  for (int i = 0; i < s->NL; ++i) s->lanes[i].qbase = cap + (int64_t)i * s->Rq;
  s->rslots.resize(s->NS);
  for (int i = 0; i < s->NS; ++i) s->rslots[i].pbase = cap + (int64_t)s->NL * s->Rq + (int64_t)i * s->Rc;
  SchedConfig sc;
  sc.lanes = s->NL;
  sc.max_batch = s->Rq;
  sc.max_requests = s->MR;
  sc.slots = s->NS;
  s->sched.reset(new Scheduler(sc));
  s->ext.resize(ng);
  for (int64_t i = 0; i < ng; ++i) s->ext[i] = (int32_t)i;
  s->next_id = ng;
  memset(&s->stats, 0, sizeof s->stats);
  s->stats.lanes = s->NL;
  s->stats.max_batch = s->Rq;
  s->stats.max_requests = s->MR;
  s->stats.request_slots = s->NS;
  s->stats.slot_bytes = slot_bytes;
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
  hipError_t e = hipStreamCreateWithFlags(&s->mst, hipStreamNonBlocking);
  if (e == hipSuccess && gcr_create(&s->mctx, ctx->device, 0) != GCR_OK) e = hipErrorOutOfMemory;
  if (e != hipSuccess) {
    release(s);
    return fail(ctx, GCR_ERR_HIP, "server set-up: %s", hipGetErrorString(e));
  }
  // rows past the live gallery stay zero (they are screened as padding)
  fill_u32((unsigned*)s->X[0] + ng * d, 0u, (cap - ng) * d, s->mst);
  for (const Operand* o : {&s->op0, &s->opL}) fill_u32(o->Xs + ng * o->ld, 0u, (o->npad - ng) * o->ld / 4, s->mst);
  *out = s;
  return GCR_OK;
}

// Workspace of the private context for a plan of `bytes`.
std::string mctx_ws(gcr_server* s, size_t bytes) {
  if (reserve_ws(s->mctx, bytes) != GCR_OK) return std::string("maintenance workspace: ") + gcr_last_error(s->mctx);
  return "";
}

// Exact k nearest other items of gallery rows [r0, r1) among columns
// [c0, c1) (run on the private context; kk <= k + 1 entries per row).
std::string gallery_knn(gcr_server* s, int64_t n_prep, int64_t r0, int64_t r1, int64_t c0, int64_t c1, int excl,
                        int kk, int32_t* idx, float* dist) {
  Arena dry;
  KnnPlan kp;
  plan_knn(dry, kp, s->prec, n_prep, s->d, r0, r1, c0, c1, kk, 0);
  std::string e = mctx_ws(s, dry.off);
  if (!e.empty()) return e;
  Arena a1{(char*)s->mctx->ws, 0};
  plan_knn(a1, kp, s->prec, n_prep, s->d, r0, r1, c0, c1, kk, 0);
  run_knn(s->mctx, kp, s->X[0], s->d, nullptr, r0, r1, c0, c1, excl, kk, 0, idx, dist, nullptr, nullptr, s->mst);
  return "";
}

// Graph, degrees, gallery-only rounds and screening operands of the live
// gallery, from its lists.
std::string refresh_gallery(gcr_server* s) {
  const hipStream_t st = s->mst;
  gcr_params gp = s->p;
  gp.alpha = 1.0f;
  gp.beta_same = gp.beta_cross = 1.0f;
  Arena dry;
  GraphTmp gt;
  plan_graph_tmp(dry, gt, s->G);
  std::string e = mctx_ws(s, dry.off);
  if (!e.empty()) return e;
  Arena a1{(char*)s->mctx->ws, 0};
  plan_graph_tmp(a1, gt, s->G);
  enqueue_graph_from_lists(s->mctx, gt, s->G, nullptr, &gp, &s->g, st);
  for (int t = 1; t <= s->L; ++t) enqueue_propagate(s->mctx, &s->g, s->X[t - 1], s->X[t], s->G, s->d, st, gt.order);
  fill_u32(s->max0, 0u, 2, st);
  launch_screen_prep_rows(s->op0.prec, s->X[0], 0, s->G, nullptr, s->d, s->op0.Xs, s->op0.ld, s->op0.n2, s->op0.scale,
                          s->op0.rn, s->max0, st);
  if (s->L > 0) {
    fill_u32(s->maxLg, 0u, 2, st);
    launch_screen_prep_rows(s->opL.prec, s->X[s->L], 0, s->G, nullptr, s->d, s->opL.Xs, s->opL.ld, s->opL.n2,
                            s->opL.scale, s->opL.rn, s->maxLg, st);
  }
  SRV_HIP(hipStreamSynchronize(st));
  SRV_HIP(hipGetLastError());
  return "";
}

// Slot state, streams and the worker thread (after the gallery is ready).
std::string server_start(gcr_server* s) {
  // marks start clear; positions start in range, so a row marked in a
  // request whose set overflowed still reads inside its slot (that request
  // is reported as failed)
  for (ReqSlot& rs : s->rslots)
    for (int t = 1; t <= s->L; ++t) {
      fill_u32(rs.mark[t], 0u, s->Gcap, s->mst);
      fill_u32(rs.pos[t], 0u, s->Gcap, s->mst);
    }
  for (Lane& ln : s->lanes) fill_u32(ln.touched, 0u, s->Gcap, s->mst);
  std::string e = refresh_gallery(s);
  if (!e.empty()) return e;
  for (Lane& ln : s->lanes) {
    SRV_HIP(hipStreamCreateWithFlags(&ln.st, hipStreamNonBlocking));
    SRV_HIP(hipEventCreateWithFlags(&ln.ev, hipEventDisableTiming));
    SRV_HIP(hipHostMalloc((void**)&ln.h_q, (size_t)s->Rq * s->d * sizeof(float), hipHostMallocDefault));
    SRV_HIP(hipHostMalloc((void**)&ln.h_idx, (size_t)s->Rq * s->K * sizeof(int32_t), hipHostMallocDefault));
    SRV_HIP(hipHostMalloc((void**)&ln.h_dist, (size_t)s->Rq * s->K * sizeof(float), hipHostMallocDefault));
    SRV_HIP(hipHostMalloc((void**)&ln.h_counts, (size_t)s->MR * 64 * sizeof(int), hipHostMallocDefault));
    SRV_HIP(hipHostMalloc((void**)&ln.h_row_mark, (size_t)s->Rq * sizeof(uint32_t*), hipHostMallocDefault));
    SRV_HIP(hipHostMalloc((void**)&ln.h_row_stamp, (size_t)s->Rq * sizeof(uint32_t), hipHostMallocDefault));
    memset(ln.h_counts, 0, (size_t)s->MR * 64 * sizeof(int));
  }
  s->worker = std::thread(worker_main, s);
  return "";
}

// Stop admitting requests and wait for the ones on the device.
void pause_and_drain(gcr_server* s) {
  std::unique_lock<std::mutex> lk(s->mu);
  s->paused = true;
  s->cv_done.wait(lk, [&] {
    for (const Lane& ln : s->lanes)
      if (ln.busy) return false;
    return true;
  });
}

void resume(gcr_server* s) {
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->paused = false;
  }
  s->cv_work.notify_all();
}

std::string insert_rows(gcr_server* s, const float* rows, int32_t m) {
  const hipStream_t st = s->mst;
  const int64_t G0 = s->G, G1 = G0 + m;
  const int k = s->k, d = s->d;
  SRV_HIP(hipMemcpyAsync(s->X[0] + G0 * d, rows, (size_t)m * d * sizeof(float), hipMemcpyHostToDevice, st));
  // the appended rows' lists over the whole gallery
  std::string e = gallery_knn(s, G1, G0, G1, 0, G1, 1, k, s->g.idx + G0 * k, s->g.dist + G0 * k);
  if (!e.empty()) return e;
  // the old rows' nearest appended items, merged into their lists
  const int km = (int)std::min<int64_t>(k, m);
  e = gallery_knn(s, G1, 0, G0, G0, G1, 0, km, s->tmp_idx, s->tmp_dist);
  if (!e.empty()) return e;
  launch_merge_appended(G0, k, s->g.idx, s->g.dist, km, s->tmp_idx, s->tmp_dist, (int32_t)G0, s->X[0], d, st);
  SRV_HIP(hipGetLastError());
  s->G = G1;
  return refresh_gallery(s);
}

std::string remove_rows(gcr_server* s, const std::vector<int32_t>& new_of_old, const std::vector<int32_t>& old_of_new) {
  const hipStream_t st = s->mst;
  const int64_t G0 = s->G, G1 = (int64_t)old_of_new.size();
  const int k = s->k, d = s->d;
  SRV_HIP(hipMemcpyAsync(s->map_a, new_of_old.data(), (size_t)G0 * sizeof(int32_t), hipMemcpyHostToDevice, st));
  SRV_HIP(hipMemcpyAsync(s->map_b, old_of_new.data(), (size_t)G1 * sizeof(int32_t), hipMemcpyHostToDevice, st));
  // lists renumbered (order kept: the renumbering is monotone)
  fill_u32((unsigned*)s->mcount, 0u, 1, st);
  launch_relabel_lists(G0, k, s->map_a, s->g.idx, s->g.dist, s->tmp_idx, s->tmp_dist, s->repair, s->mcount, st);
  SRV_HIP(hipMemcpyAsync(s->g.idx, s->tmp_idx, (size_t)G1 * k * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
  SRV_HIP(hipMemcpyAsync(s->g.dist, s->tmp_dist, (size_t)G1 * k * sizeof(float), hipMemcpyDeviceToDevice, st));
  // features compacted through a staging copy past the gallery capacity
  // (rows [Gcap, rows_total) belong to the idle slots), in pieces
  const int64_t stage_rows = s->rows_total - s->Gcap;
  for (int64_t r = 0; r < G1; r += stage_rows) {
    const int64_t b = std::min<int64_t>(stage_rows, G1 - r);
    launch_gather_rows(s->X[0], s->X[0] + s->Gcap * d, s->map_b + r, b, d, st);
    SRV_HIP(hipMemcpyAsync(s->X[0] + r * d, s->X[0] + s->Gcap * d, (size_t)b * d * sizeof(float),
                           hipMemcpyDeviceToDevice, st));
  }
  fill_u32((unsigned*)s->X[0] + G1 * d, 0u, (G0 - G1) * d, st);
  int nrep = 0;
  SRV_HIP(hipMemcpyAsync(&nrep, s->mcount, sizeof(int), hipMemcpyDeviceToHost, st));
  SRV_HIP(hipStreamSynchronize(st));
  s->G = G1;
  // lists that lost a neighbour: k + 1 nearest of a staged copy of the row
  // (the copy finds the row itself), then the row itself dropped
  for (int64_t r = 0; r < nrep; r += stage_rows) {
    const int64_t b = std::min<int64_t>(stage_rows, nrep - r);
    launch_gather_rows(s->X[0], s->X[0] + s->Gcap * d, s->repair + r, b, d, st);
    std::string e = gallery_knn(s, s->Gcap + b, s->Gcap, s->Gcap + b, 0, G1, 0, k + 1, s->tmp_idx, s->tmp_dist);
    if (!e.empty()) return e;
    launch_drop_self(b, k, s->repair + r, s->tmp_idx, s->tmp_dist, s->g.idx, s->g.dist, st);
    SRV_HIP(hipGetLastError());
  }
  return refresh_gallery(s);
}

const char kMagic[8] = {'G', 'C', 'R', 'S', 'R', 'V', '0', '1'};

}  // namespace

extern "C" {

void gcr_server_config_default(gcr_server_config* c) {
  if (!c) return;
  c->lanes = 2;
  c->max_batch = 512;
  c->max_requests = 16;
  c->max_recomputed = 65536;
  c->gallery_capacity = 0;
  c->reserved = 0;
  c->mem_budget = 0;
}

gcr_status gcr_server_create(gcr_ctx* ctx, const void* gallery, int32_t gallery_dtype, int64_t ng, int32_t d,
                             const gcr_params* p, const gcr_server_config* cfg, gcr_server** out) {
  if (!ctx || !out || !p) return GCR_ERR_INVALID;
  *out = nullptr;
  if (!gallery) return fail(ctx, GCR_ERR_INVALID, "gallery is NULL");
  if (gallery_dtype != 0 && gallery_dtype != 1) return fail(ctx, GCR_ERR_INVALID, "gallery_dtype must be 0 or 1");
  gcr_server* s = nullptr;
  gcr_status st = server_new(ctx, p, cfg, ng, d, &s);
  if (st != GCR_OK) return st;
  // resident gallery: level-0 features as given (float32, or BF16 widened).
  // The copy runs on the server's own stream: finish whatever the caller
  // enqueued on any stream first (it may still be writing the gallery).
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    release(s);
    return fail(ctx, GCR_ERR_HIP, "hipDeviceSynchronize before the gallery copy: %s", hipGetErrorString(e));
  }
  if (gallery_dtype == 0)
    e = hipMemcpyAsync(s->X[0], gallery, (size_t)ng * d * sizeof(float), hipMemcpyDeviceToDevice, s->mst);
  else
    launch_bf16_to_f32((const uint16_t*)gallery, s->X[0], ng * d, s->mst);
  std::string err = e == hipSuccess ? "" : std::string("gallery copy: ") + hipGetErrorString(e);
  // the gallery's kNN lists (fixed mode, one list, no camera weighting)
  if (err.empty()) err = gallery_knn(s, ng, 0, ng, 0, ng, 1, s->k, s->g.idx, s->g.dist);
  if (err.empty()) err = server_start(s);
  if (!err.empty()) {
    if (s->worker.joinable()) gcr_server_destroy(s);
    else release(s);
    return fail(ctx, GCR_ERR_HIP, "%s", err.c_str());
  }
  *out = s;
  return GCR_OK;
}

gcr_status gcr_server_insert(gcr_server* s, const float* rows_host, int32_t m, int32_t* ids_out) {
  if (!s) return GCR_ERR_INVALID;
  if (!rows_host || m < 1) return sfail(s, GCR_ERR_INVALID, "rows must be a host array of m >= 1 rows");
  std::lock_guard<std::mutex> mg(s->mut_mu);
  if (s->G + m > s->Gcap)
    return sfail(s, GCR_ERR_UNSUPPORTED, "inserting " + std::to_string(m) + " rows exceeds the gallery capacity of " +
                                             std::to_string(s->Gcap));
  if (s->next_id + m > (int64_t)INT32_MAX) return sfail(s, GCR_ERR_UNSUPPORTED, "external ids exhausted");
  pause_and_drain(s);
  (void)hipSetDevice(s->device);
  const std::string e = insert_rows(s, rows_host, m);
  if (e.empty()) {
    for (int32_t t = 0; t < m; ++t) {
      s->ext.push_back((int32_t)s->next_id);
      if (ids_out) ids_out[t] = (int32_t)s->next_id;
      ++s->next_id;
    }
  }
  resume(s);
  return e.empty() ? GCR_OK : sfail(s, GCR_ERR_HIP, e);
}

gcr_status gcr_server_remove(gcr_server* s, const int32_t* ids_host, int32_t m) {
  if (!s) return GCR_ERR_INVALID;
  if (!ids_host || m < 1) return sfail(s, GCR_ERR_INVALID, "ids must be a host array of m >= 1 ids");
  std::lock_guard<std::mutex> mg(s->mut_mu);
  const int64_t G0 = s->G;
  std::vector<int32_t> new_of_old(G0, 0);
  for (int32_t t = 0; t < m; ++t) {
    auto it = std::lower_bound(s->ext.begin(), s->ext.end(), ids_host[t]);
    if (it == s->ext.end() || *it != ids_host[t])
      return sfail(s, GCR_ERR_INVALID, "id " + std::to_string(ids_host[t]) + " is not in the gallery");
    new_of_old[it - s->ext.begin()] = -1;
  }
  std::vector<int32_t> old_of_new;
  old_of_new.reserve(G0);
  for (int64_t i = 0; i < G0; ++i)
    if (new_of_old[i] == 0) {
      new_of_old[i] = (int32_t)old_of_new.size();
      old_of_new.push_back((int32_t)i);
    }
  if (old_of_new.size() < 2) return sfail(s, GCR_ERR_INVALID, "a gallery keeps at least 2 items");
  pause_and_drain(s);
  (void)hipSetDevice(s->device);
  const std::string e = remove_rows(s, new_of_old, old_of_new);
  if (e.empty()) {
    std::vector<int32_t> ext;
    ext.reserve(old_of_new.size());
    for (int32_t o : old_of_new) ext.push_back(s->ext[o]);
    s->ext.swap(ext);
  }
  resume(s);
  return e.empty() ? GCR_OK : sfail(s, GCR_ERR_HIP, e);
}

gcr_status gcr_server_gallery_ids(gcr_server* s, int32_t* ids_host, int64_t capacity, int64_t* count) {
  if (!s || !count) return GCR_ERR_INVALID;
  std::lock_guard<std::mutex> mg(s->mut_mu);
  *count = (int64_t)s->ext.size();
  if (ids_host) {
    if (capacity < *count) return sfail(s, GCR_ERR_INVALID, "ids buffer too small");
    memcpy(ids_host, s->ext.data(), s->ext.size() * sizeof(int32_t));
  }
  return GCR_OK;
}

gcr_status gcr_server_save(gcr_server* s, const char* path) {
  if (!s) return GCR_ERR_INVALID;
  if (!path) return sfail(s, GCR_ERR_INVALID, "path is NULL");
  std::lock_guard<std::mutex> mg(s->mut_mu);
  pause_and_drain(s);
  (void)hipSetDevice(s->device);
  const int64_t G = s->G;
  const int k = s->k, d = s->d;
  std::vector<float> X((size_t)G * d), dist((size_t)G * k);
  std::vector<int32_t> idx((size_t)G * k);
  hipError_t e = hipMemcpy(X.data(), s->X[0], X.size() * sizeof(float), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(idx.data(), s->g.idx, idx.size() * sizeof(int32_t), hipMemcpyDeviceToHost);
  if (e == hipSuccess) e = hipMemcpy(dist.data(), s->g.dist, dist.size() * sizeof(float), hipMemcpyDeviceToHost);
  resume(s);
  if (e != hipSuccess) return sfail(s, GCR_ERR_HIP, std::string("save: ") + hipGetErrorString(e));
  FILE* f = fopen(path, "wb");
  if (!f) return sfail(s, GCR_ERR_INVALID, std::string("cannot open ") + path + " for writing");
  const int32_t hdr[4] = {1, d, k, 0};
  const int64_t sizes[2] = {G, s->next_id};
  bool ok = fwrite(kMagic, 1, 8, f) == 8 && fwrite(hdr, sizeof hdr, 1, f) == 1 &&
            fwrite(sizes, sizeof sizes, 1, f) == 1 && fwrite(&s->p, sizeof s->p, 1, f) == 1 &&
            fwrite(s->ext.data(), sizeof(int32_t), (size_t)G, f) == (size_t)G &&
            fwrite(X.data(), sizeof(float), X.size(), f) == X.size() &&
            fwrite(idx.data(), sizeof(int32_t), idx.size(), f) == idx.size() &&
            fwrite(dist.data(), sizeof(float), dist.size(), f) == dist.size();
  ok = (fclose(f) == 0) && ok;
  return ok ? GCR_OK : sfail(s, GCR_ERR_INVALID, std::string("write to ") + path + " failed");
}

gcr_status gcr_server_load(gcr_ctx* ctx, const char* path, const gcr_server_config* cfg, gcr_server** out) {
  if (!ctx || !out) return GCR_ERR_INVALID;
  *out = nullptr;
  if (!path) return fail(ctx, GCR_ERR_INVALID, "path is NULL");
  FILE* f = fopen(path, "rb");
  if (!f) return fail(ctx, GCR_ERR_INVALID, "cannot open %s", path);
  char magic[8];
  int32_t hdr[4];
  int64_t sizes[2];
  gcr_params p;
  bool ok = fread(magic, 1, 8, f) == 8 && memcmp(magic, kMagic, 8) == 0 && fread(hdr, sizeof hdr, 1, f) == 1 &&
            hdr[0] == 1 && fread(sizes, sizeof sizes, 1, f) == 1 && fread(&p, sizeof p, 1, f) == 1;
  const int d = ok ? hdr[1] : 0, k = ok ? hdr[2] : 0;
  const int64_t G = ok ? sizes[0] : 0;
  ok = ok && d > 0 && d <= 2048 && k == p.k && G >= 2 && G <= ((int64_t)1 << 30) && sizes[1] >= G &&
       sizes[1] <= (int64_t)INT32_MAX;
  std::vector<int32_t> ext, idx;
  std::vector<float> X, dist;
  if (ok) {
    ext.resize((size_t)G);
    X.resize((size_t)G * d);
    idx.resize((size_t)G * k);
    dist.resize((size_t)G * k);
    ok = fread(ext.data(), sizeof(int32_t), ext.size(), f) == ext.size() &&
         fread(X.data(), sizeof(float), X.size(), f) == X.size() &&
         fread(idx.data(), sizeof(int32_t), idx.size(), f) == idx.size() &&
         fread(dist.data(), sizeof(float), dist.size(), f) == dist.size();
  }
  fclose(f);
  for (size_t i = 1; ok && i < ext.size(); ++i) ok = ext[i] > ext[i - 1];
  for (size_t i = 0; ok && i < idx.size(); ++i) ok = idx[i] >= -1 && idx[i] < G;
  if (!ok) return fail(ctx, GCR_ERR_INVALID, "%s is not a saved server state", path);
  gcr_server* s = nullptr;
  gcr_status st = server_new(ctx, &p, cfg, G, d, &s);
  if (st != GCR_OK) return st;
  s->ext = ext;
  s->next_id = sizes[1];
  hipError_t e = hipMemcpy(s->X[0], X.data(), X.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->g.idx, idx.data(), idx.size() * sizeof(int32_t), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(s->g.dist, dist.data(), dist.size() * sizeof(float), hipMemcpyHostToDevice);
  std::string err = e == hipSuccess ? "" : std::string("load: ") + hipGetErrorString(e);
  if (err.empty()) err = server_start(s);
  if (!err.empty()) {
    if (s->worker.joinable()) gcr_server_destroy(s);
    else release(s);
    return fail(ctx, GCR_ERR_HIP, "%s", err.c_str());
  }
  *out = s;
  return GCR_OK;
}

gcr_status gcr_server_submit(gcr_server* s, const float* q_host, int32_t b, uint64_t* ticket) {
  if (!s || !ticket) return GCR_ERR_INVALID;
  if (!q_host || b < 1) return sfail(s, GCR_ERR_INVALID, "queries must be a host array of b >= 1 rows");
  if (b > s->Rq)
    return sfail(s, GCR_ERR_INVALID, "request of " + std::to_string(b) + " queries exceeds the batch capacity of " +
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
  s->sched->push(r->ticket, b);
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
  out->gallery_size = s->G;
  out->gallery_capacity = s->Gcap;
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
  for (Lane& ln : s->lanes)
    if (ln.st) (void)hipStreamSynchronize(ln.st);
  release(s);
  return GCR_OK;
}

}  // extern "C"
