/*
 * gcr.h - C ABI of the GCR / GCRV re-ranking library for AMD MI355X (gfx950).
 *
 * Graph Convolution based Re-ranking updates retrieval features by parameter-
 * free graph convolution over a k-nearest-neighbour graph of the query and
 * gallery features, then ranks by distance between the updated features
 * (Sec. III-A, Eq. (2)-(3)).  This library runs every step on the GPU:
 *   gcr_normalize_rows  row L2 normalisation (input preparation)
 *   gcr_knn             all-pairs similarity + per-row k nearest neighbours
 *                       (Eq. (4) neighbour sets; Eq. (8) cross-camera sets)
 *   gcr_build_graph     kNN + exp affinities + symmetrisation + degrees
 *                       (Eq. (4)-(8))
 *   gcr_propagate       one synchronous propagation round (Eq. (2) / (9))
 *                       followed by row re-normalisation
 *   gcr_final_distances squared distances between query and gallery rows of
 *                       the updated features, dense or top-K per query
 *   gcr_rerank          the whole pipeline: T rounds (Eq. (3)), the graph
 *                       rebuilt from the current features before each round
 *                       (Sec. III-C) or fixed, then final distances
 *   gcr_profile_vectors tracklet profile vectors for video (Eq. (10), (16);
 *                       Alg. 2 step 1)
 *   gcr_dsfp            decentralised synchronous feature propagation
 *                       (DSFP, Alg. 1): every node propagates on its own
 *                       local neighbourhood graph
 *   gcr_rerank_local    the GCR_Local pipeline: kNN once, DSFP, final
 *                       distances
 *
 * Conventions
 *   Memory: every array argument is a DEVICE pointer owned by the caller,
 *     contiguous and row-major, unless stated otherwise.  The library owns
 *     only the workspace inside a gcr_ctx: one device block sized at
 *     gcr_create (gcr_workspace_size gives the bytes for a problem size) and
 *     grown only by gcr_reserve.  No other call allocates, frees or
 *     synchronises the device (except those that say so: statistics, timing,
 *     profile vectors, servers), so the batch calls can be captured into a
 *     HIP graph on their first use; a call whose workspace is too small
 *     fails with GCR_ERR_NOMEM and names the size it needs.
 *   Streams: `stream` is a hipStream_t passed as void*; NULL means the
 *     default stream.  Calls enqueue work on that stream and return without
 *     synchronising, except where a function says it synchronises.
 *   Errors: functions return gcr_status; a negative value is an error and
 *     gcr_last_error(ctx) returns its message.  Nothing throws across the ABI.
 *     Argument checks happen on the host before anything is enqueued.
 *   Threads: a gcr_ctx must be used by one host thread at a time.
 *   Feature width: d <= 2048 for every entry point that takes features
 *     (GCR_ERR_UNSUPPORTED above), d <= 8192 for gcr_profile_vectors.
 *   Neighbour lists: row i lists its k nearest other rows j != i, ordered by
 *     (squared distance, j) ascending; rows with fewer than k eligible
 *     neighbours are padded with index -1 and distance +inf.
 */
#ifndef GCR_H
#define GCR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  GCR_OK = 0,
  GCR_ERR_INVALID = -1,     /* bad argument (shape, NULL, range)            */
  GCR_ERR_NOMEM = -2,       /* device allocation failed                     */
  GCR_ERR_HIP = -3,         /* a HIP runtime call failed                    */
  GCR_ERR_UNSUPPORTED = -4, /* valid but not supported by the library      */
  GCR_ERR_TIMEOUT = -5      /* gcr_server_wait: the request is not done yet */
} gcr_status;

/* Precision of the similarity screening (Eq. (4) neighbour sets are ranked
 * by squared distance).  The refine modes re-score every screened candidate
 * within the screening margin of the k-th key exactly (float64 sums of
 * squared float64 differences of the float32 rows), so their neighbour lists
 * and distances equal the float32 mode's; only speed differs.  The raw modes
 * keep the k smallest screened distances n2_i + n2_j - 2 s~ (float32 norms,
 * screened inner product s~) with no re-score: faster, not exact; they exist
 * to measure what the re-score buys.  With GCR_FP8 the final top-K output
 * (gcr_final_distances, gcr_rerank, servers) is screened in BF16: FP8's
 * margin, about 0.13 in squared distance for unit rows, spans thousands of
 * unrelated items once K exceeds the natural neighbourhood size and would
 * send queries to the exhaustive path; the kNN graph keeps FP8. */
typedef enum {
  GCR_FP32 = 0,     /* float32 MFMA screening + exact re-score               */
  GCR_BF16 = 1,     /* bfloat16 (RNE) MFMA screening, float32 accumulation,
                       + exact re-score                                      */
  GCR_FP8 = 2,      /* OCP E4M3 with per-row scale, float32 accumulation,
                       + exact re-score                                      */
  GCR_BF16_RAW = 3, /* bfloat16 screening only (lists by screened key)       */
  GCR_FP8_RAW = 4   /* FP8 E4M3 screening only (lists by screened key)       */
} gcr_precision;

typedef struct {
  int32_t k;                  /* neighbours per node, Eq. (4); 0 <= k <= 120  */
  int32_t cross_k;            /* cross-camera neighbours, Eq. (8); <0: = k    */
  int32_t rounds;             /* T, Eq. (3)                                    */
  int32_t rebuild_each_round; /* 1: rebuild the graph from X_{t-1} each round  */
  int32_t normalize_input;    /* 1: L2-normalise input rows first              */
  int32_t precision;          /* gcr_precision of the similarity screening     */
  int32_t topk_out;           /* K of gcr_rerank's per-query output list       */
  int32_t symmetric;          /* 1: A = (A~ + A~^T)/2, Eq. (7) + (2); 0: the
                                 asymmetric D_r^-1/2 A~ D_c^-1/2 of Eq. (6)     */
  float gamma;                /* temperature of Eq. (4), > 0                   */
  float alpha;                /* blend of Eq. (9) in [0, 1]; 1: global only    */
  float beta_same;            /* factor on global-graph edges, same camera     */
  float beta_cross;           /* factor on global-graph edges, other camera    */
  float lambda;               /* regulariser of Eq. (16), > 0                  */
} gcr_params;

/* Paper defaults: gamma 0.2, k 15, T 3, lambda 10 (Sec. IV-B), alpha 1,
 * graph rebuilt each round, inputs normalised, FP32 screening, K 100. */
void gcr_params_default(gcr_params* p);

typedef struct gcr_ctx gcr_ctx;

/* Create a context on HIP device `device` (made current for the calls that
 * use this context) with a workspace of workspace_bytes (0: none yet).
 * *out receives the handle.  Errors: INVALID (bad device / NULL out), NOMEM
 * (the workspace allocation failed), HIP. */
gcr_status gcr_create(gcr_ctx** out, int device, size_t workspace_bytes);
/* Grow the workspace to at least workspace_bytes (never shrinks).  This is
 * the one call after gcr_create that allocates: it synchronises the device
 * and frees the old block, so work enqueued earlier must not be relied on
 * to keep using it (the synchronisation finishes that work first).  Not
 * capturable.  Errors: INVALID, NOMEM, HIP. */
gcr_status gcr_reserve(gcr_ctx* ctx, size_t workspace_bytes);
/* Bytes of workspace the context holds. */
size_t gcr_workspace_bytes(const gcr_ctx* ctx);
/* Workspace bytes that every batch entry point (gcr_knn, gcr_build_graph,
 * gcr_propagate, gcr_final_distances with dense and top-K output,
 * gcr_rerank, gcr_dsfp, gcr_rerank_local) needs for nq queries and ng
 * gallery rows of width d with parameters p (precision, k, cross_k,
 * topk_out), with the cross-camera lists when with_cameras != 0; entry
 * points that take n rows use n = nq + ng (nq may be 0).  Computed on the
 * host for the current HIP device (the similarity schedule depends on its
 * compute-unit count).  Returns 0 for invalid or unsupported sizes: d
 * outside 1..2048, invalid parameters, or a screening operand above 4 GiB
 * (about 1M rows of BF16 or 524k rows of float32 at d = 2048). */
size_t gcr_workspace_size(const gcr_params* p, int64_t nq, int64_t ng, int32_t d, int32_t with_cameras);
/* Workspace bytes gcr_profile_vectors needs for nt tracklets with nf frames
 * in all of width d (mode as there); 0 for invalid sizes. */
size_t gcr_profile_workspace_size(int32_t nt, int64_t nf, int32_t d, int32_t mode);
/* Free the context and its workspace (synchronises the device). */
gcr_status gcr_destroy(gcr_ctx* ctx);
/* Message of the last error on ctx (never NULL; "" if none). */
const char* gcr_last_error(const gcr_ctx* ctx);

/* Run statistics.  Synchronises the device to read counters. */
typedef struct {
  int64_t knn_rows;           /* rows whose neighbour lists were built         */
  int64_t knn_candidates;     /* screened candidates re-scored exactly         */
  int64_t knn_fallback_rows;  /* (row, list) pairs re-swept in float32 because
                                 a truncated buffer did not reach the cut      */
  int64_t splits;             /* column splits of the last similarity sweep    */
  int64_t knn_exhaustive_rows;/* (row, list) pairs whose float32 band exceeded
                                 2,048 items, scored exactly over all columns */
  int64_t tile_rows;          /* rows per workgroup tile of the last similarity
                                 sweep: 128, or 256 for sweeps of one list over
                                 many row blocks in float32 or BF16 */
} gcr_stats;
gcr_status gcr_get_stats(gcr_ctx* ctx, gcr_stats* out);
gcr_status gcr_reset_stats(gcr_ctx* ctx);

/* Per-kernel-class timing with HIP events recorded on the launch stream
 * around every launch of that class while timing is on (off by default).
 * Classes: 0 similarity + top-k screening of the kNN graph, 1 its exact
 * refine (with the exhaustive fallback and threshold seeding), 2 graph
 * build (weights, reverse lists, degrees, normalised values), 3
 * propagation (global rounds, or the DSFP kernel), 4 dense final
 * distances, 5 input preparation (normalisation and screening operands),
 * 6 screening sweep of the final top-K (queries against the gallery), 7
 * its exact refine.
 * gcr_get_timing synchronises the device, returns the totals since the last
 * reset (milliseconds and launch counts) and resets them. */
#define GCR_NUM_TIMERS 8
typedef struct {
  double ms[GCR_NUM_TIMERS];
  int64_t launches[GCR_NUM_TIMERS];
} gcr_timing;
gcr_status gcr_set_timing(gcr_ctx* ctx, int32_t on);
gcr_status gcr_get_timing(gcr_ctx* ctx, gcr_timing* out);

/* Row L2 normalisation: Y[i] = X[i] / max(||X[i]||, 1e-12).
 * X, Y: float32 [n, d] (may alias).  Errors: INVALID. */
gcr_status gcr_normalize_rows(gcr_ctx* ctx, const float* X, float* Y,
                              int64_t n, int32_t d, void* stream);

/* k nearest neighbours of every row of X among the other rows (Eq. (4)),
 * and, when cam != NULL and cr_idx != NULL, the cross_k nearest rows with a
 * different camera label (Eq. (8)).
 *   X: float32 [n, d]; used as given (no normalisation).
 *   cam: int32 [n] camera labels or NULL.
 *   idx: int32 [n, k] out; dist: float32 [n, k] out, squared distances.
 *   cr_idx / cr_dist: int32 / float32 [n, cross_k] out, or NULL.
 * Uses p->k, p->cross_k, p->precision.  Errors: INVALID, UNSUPPORTED
 * (k > 120), NOMEM, HIP. */
gcr_status gcr_knn(gcr_ctx* ctx, const float* X, int64_t n, int32_t d,
                   const int32_t* cam, const gcr_params* p,
                   int32_t* idx, float* dist, int32_t* cr_idx, float* cr_dist,
                   void* stream);

/* Sparse propagation graph (Eq. (4)-(9)), in caller memory.
 * For each of the global graph and (if has_cross) the cross-camera graph:
 *   idx [n,k] int32, dist [n,k] float32   forward kNN lists
 *   w   [n,k] float32   beta * exp(-dist / gamma)   (0 for padding)
 *   rev_ptr [n+1], rev_src [n*k] int32, rev_w [n*k] float32: the transposed
 *       edges j -> i stored at row i, sorted by source index
 *   deg [n] float32: D_i of A = (A~ + A~^T)/2, i.e. 1 + sum(w)/2 over the
 *       forward and reverse edges of row i
 *   pf [n,k], pr [n*k] float32: normalised values c * w / (2 sqrt(D_i D_j))
 *       of the forward and reverse entries, with c = alpha for the global
 *       graph and 1 - alpha for the cross graph
 *   Asymmetric graphs (built with p->symmetric = 0, Eq. (5), (6)): deg holds
 *   the row degrees D_r(i) = 1 + sum of the forward w, pf = c * w /
 *   sqrt(D_r(i) D_c(j)) with the column degrees D_c(j) = 1 + sum of the
 *   reverse w, pr is unused and self = c / sqrt(D_r(i) D_c(i)) summed over
 *   the graphs
 * and self[n] float32 = alpha / D_i + (1 - alpha) / D^cr_i (diagonal of the
 * blended operator).  gcr_graph_bytes gives the size of one device buffer
 * holding all of it; gcr_graph_bind carves that buffer into the fields. */
typedef struct {
  int64_t n;
  int32_t k, cross_k, has_cross;
  int32_t asymmetric; /* set by gcr_build_graph: 0 symmetric (Eq. (7)),
                         1 asymmetric (Eq. (6)): deg holds the row degrees
                         and the reverse lists are not propagated */
  int32_t *idx, *rev_ptr, *rev_src;
  float *dist, *w, *rev_w, *deg, *pf, *pr;
  int32_t *cr_idx, *cr_rev_ptr, *cr_rev_src;
  float *cr_dist, *cr_w, *cr_rev_w, *cr_deg, *cr_pf, *cr_pr;
  float* self;
} gcr_graph;

size_t gcr_graph_bytes(int64_t n, int32_t k, int32_t cross_k, int32_t has_cross);
gcr_status gcr_graph_bind(gcr_graph* g, void* dev_buf, int64_t n, int32_t k,
                          int32_t cross_k, int32_t has_cross);

/* Build the propagation graph of X (float32 [n, d], used as given).  cam may
 * be NULL; the cross graph is built when g->has_cross (requires cam).
 * Edge factor beta_same / beta_cross applies to the global graph when cam is
 * given.  Errors: INVALID, UNSUPPORTED, NOMEM, HIP. */
gcr_status gcr_build_graph(gcr_ctx* ctx, const float* X, int64_t n, int32_t d,
                           const int32_t* cam, const gcr_params* p,
                           gcr_graph* g, void* stream);

/* One propagation round over graph g:
 *   y_i = self_i x_i + sum_fwd pf x_j + sum_rev pr x_j (+ cross graph terms)
 *   X_out[i] = y_i / max(||y_i||, 1e-12)
 * X_in, X_out: float32 [n, d], distinct buffers (in-place is INVALID). */
gcr_status gcr_propagate(gcr_ctx* ctx, const gcr_graph* g, const float* X_in,
                         float* X_out, int64_t n, int32_t d, void* stream);

/* One propagation round exactly as gcr_propagate (same kernels, bitwise the
 * same output), for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation.
 * It uses neither the context workspace nor any allocation: its scratch (the
 * locality order of the round, 24 bytes per node) lives in a fixed 32 MiB
 * device array of the library, one per GPU, obtained once per device in
 * gcr_create and held until the process ends.  n is limited to
 * gcr_propagate_noalloc_max_nodes() (about 1.39M nodes); larger n returns
 * UNSUPPORTED.  All calls on one GPU share that array: calls that overlap in
 * time on one GPU (other streams, other contexts, other threads) race and
 * must be ordered by the caller.  Arguments and errors as gcr_propagate. */
gcr_status gcr_propagate_noalloc(gcr_ctx* ctx, const gcr_graph* g,
                                 const float* X_in, float* X_out, int64_t n,
                                 int32_t d, void* stream);
size_t gcr_propagate_noalloc_max_nodes(void);

/* Distances between the first nq rows (queries) and the next ng rows
 * (gallery) of X (float32 [nq+ng, d]):
 *   dist_out: float32 [nq, ng] dense squared distances, or NULL (inner
 *     products from a 16-bit-mantissa split of every feature, hi + lo in
 *     bfloat16, |x - hi - lo| <= 2^-16 |x|, accumulated in float32);
 *   topk_idx / topk_dist: int32 / float32 [nq, K] with K = p->topk_out: the
 *     K nearest gallery items (gallery index 0..ng-1) by (distance, index),
 *     or NULL.
 * Errors: INVALID, UNSUPPORTED, NOMEM, HIP. */
gcr_status gcr_final_distances(gcr_ctx* ctx, const float* X, int64_t nq,
                               int64_t ng, int32_t d, const gcr_params* p,
                               float* dist_out, int32_t* topk_idx,
                               float* topk_dist, void* stream);

/* Whole re-ranking of X = [queries; gallery] (float32 [nq+ng, d]):
 * normalise (if asked), T = p->rounds propagation rounds with the graph
 * rebuilt each round (or built once), then final distances as in
 * gcr_final_distances.  X_final (float32 [nq+ng, d]) receives X_T if not
 * NULL.  cam (int32 [nq+ng]) may be NULL; with cam and alpha < 1 the
 * cross-camera graph and the blend of Eq. (9) are used.
 * last_graph: NULL, or a graph bound by gcr_graph_bind for n = nq + ng,
 * k = p->k and, with cameras and alpha < 1, has_cross = 1 and cross_k as in
 * p (else has_cross = 0); the rounds then build into it, so it holds the
 * graph of the last round afterwards (untouched when p->rounds = 0).
 * Errors: INVALID, UNSUPPORTED, NOMEM (workspace too small), HIP. */
gcr_status gcr_rerank(gcr_ctx* ctx, const float* X, int64_t nq, int64_t ng,
                      int32_t d, const int32_t* cam, const gcr_params* p,
                      float* dist_out, int32_t* topk_idx, float* topk_dist,
                      float* X_final, gcr_graph* last_graph, void* stream);

/* Decentralised synchronous feature propagation, DSFP (Alg. 1).  For every
 * node i independently: the local set L_i = {i} plus the entries of row i
 * of idx; the local affinity A_uv = exp(-||x_u - x_v||^2 / gamma) over all
 * pairs u, v of L_i (1 on the diagonal); the local degrees D_u = sum_v A_uv
 * for every member u (Alg. 1 prints the degree of node i only; the
 * normalisation needs every member's); then `rounds` local rounds
 *   X_L <- rownorm(D^-1/2 A D^-1/2 X_L),  rownorm(y) = y / max(||y||, 1e-12),
 * starting from the rows of X, as a global round does; Y[i] = node i's row
 * of the local X_L after the last round.  Nodes never see each other's
 * local updates (synchronous: every node starts from X).
 *   X: float32 [n, d], used as given (no normalisation).
 *   idx: int32 [n, k] neighbour lists (as gcr_knn writes them); entries < 0
 *     or >= n, equal to i, or repeating an earlier entry of the row are
 *     ignored; may be NULL when k = 0.
 *   Y: float32 [n, d] out; must not overlap X.  rounds = 0 copies X to Y.
 * Errors: INVALID (NULL or overlapping buffers, n < 1, d < 1, k < 0,
 * rounds < 0, gamma not finite and > 0), UNSUPPORTED (k > 59: the local
 * matrices must fit one workgroup's LDS; d > 2048), NOMEM, HIP. */
gcr_status gcr_dsfp(gcr_ctx* ctx, const float* X, const int32_t* idx,
                    int64_t n, int32_t d, int32_t k, float gamma,
                    int32_t rounds, float* Y, void* stream);

/* GCR_Local re-ranking (DSFP in place of the global rounds, Alg. 1) of
 * X = [queries; gallery] (float32 [nq+ng, d]): normalise (if
 * p->normalize_input), the p->k nearest neighbours of every row once (with
 * p->precision screening; no camera lists), gcr_dsfp with p->gamma and
 * p->rounds, then final distances as in gcr_final_distances.  X_final
 * (float32 [nq+ng, d]) receives the DSFP features if not NULL.  p->alpha,
 * cross_k, beta_*, rebuild_each_round and symmetric do not apply.
 * Errors: INVALID, UNSUPPORTED (as gcr_dsfp; K above 120), NOMEM, HIP. */
gcr_status gcr_rerank_local(gcr_ctx* ctx, const float* X, int64_t nq,
                            int64_t ng, int32_t d, const gcr_params* p,
                            float* dist_out, int32_t* topk_idx,
                            float* topk_dist, float* X_final, void* stream);

/* Tracklet profile vectors (video re-ID, Alg. 2 step 1).
 *   frames: float32 [nf, d]; offsets: int32 [nt+1] (frames of tracklet c are
 *   rows offsets[c] .. offsets[c+1]-1, nonempty, contiguous, increasing);
 *   group: int32 [nt] camera group per tracklet or NULL (one group);
 *   mode 0: PVG, Eq. (16) per group: w_c = (F^T F + lambda n I)^-1 (mu_c - mu)
 *           where F holds the group's n frames and mu their mean;
 *   mode 1: mean profile, Eq. (10);
 *   W_out: float32 [nt, d], each row L2-normalised.
 * Host-side reads of offsets/group: offsets_host and group_host are HOST
 * copies of the same arrays (the solver plans per-group work on the host).
 * Mode 0 synchronises the stream once per group, to read the trace of the
 * group's Gram (it fixes the Chebyshev iteration count); the last group's
 * solve is left running on the stream.  Mode 1 does not synchronise.
 * Errors: INVALID, NOMEM, HIP. */
gcr_status gcr_profile_vectors(gcr_ctx* ctx, const float* frames,
                               const int32_t* offsets, const int32_t* group,
                               const int32_t* offsets_host,
                               const int32_t* group_host, int32_t nt, int32_t d,
                               int32_t mode, float lambda, float* W_out,
                               void* stream);

/* ---------------------------------------------------------------------
 * Serving: a resident gallery and continuous batching of requests.
 *
 * The paper notes that the kNN graph of the database can be computed in
 * advance, leaving only the queries' part per request (Sec. IV-F).  A server
 * keeps the gallery's features, its kNN lists and degrees (built on the
 * gallery alone and then frozen) and its gallery-only propagated features of
 * every round resident in HBM.  One request with queries Q is computed over
 * the node set gallery + Q: a query row lists its k nearest gallery items
 * (Eq. (4)); gallery rows keep their frozen lists; A = (A~ + A~^T)/2 with self
 * weight 1, D and P = D^-1/2 A D^-1/2 (Eq. (5)-(7)) over that node set;
 * p->rounds rounds of x <- P x with row renormalisation (Eq. (2), (3)) on
 * the fixed graph; the result is each query's top-K gallery items
 * (K = p->topk_out) by squared distance over the propagated features,
 * ordered by (distance, gallery index).  Requests do not see each other:
 * a result is the same whether the request ran alone or among others.
 *
 * Only gallery rows within `rounds` hops of the gallery items the queries
 * touch change; the server recomputes exactly those rows (up to
 * cfg.max_recomputed per round and request) and reads the rest from the
 * resident copy.
 *
 * Continuous batching: a worker thread keeps cfg.lanes batches on the
 * device (one HIP stream each).  Whenever a lane is free it forms a batch
 * from the queued requests in order, while their queries fit the lane's
 * cfg.max_batch query rows, the batch holds at most cfg.max_requests
 * requests, and a request scratch slot is free: admission is by memory (a
 * 1-query request takes one row and one slot; the number of slots comes
 * from cfg.mem_budget).  A batch shares its two gallery sweeps among all its
 * queries (their kNN over the gallery, and the final top-K over the
 * gallery's round-L rows, where each query leaves out the rows its own
 * request recomputed); each request's propagation and recomputed rows use
 * its own slot.  Cameras (Eq. (8), (9)) are not used in serving.
 * ------------------------------------------------------------------- */
typedef struct gcr_server gcr_server;

typedef struct {
  int32_t lanes;            /* batches on the device at once, 1..8 (default 2) */
  int32_t max_batch;        /* query rows of one batch, which also bounds one
                               request (default 512; capped so that
                               max_batch * k <= 16384)                       */
  int32_t max_requests;     /* requests co-batched into one batch, 1..256
                               (default 16)                                  */
  int32_t max_recomputed;   /* gallery rows recomputed per round and request
                               (default 65536)                               */
  int32_t gallery_capacity; /* gallery rows reserved for inserts; 0: the
                               initial gallery size (default 0)              */
  int32_t reserved;         /* 0                                              */
  uint64_t mem_budget;      /* device bytes for request scratch slots (the
                               per-request hop sets and recomputed rows); 0:
                               lanes x max_requests slots (default 0)        */
} gcr_server_config;
void gcr_server_config_default(gcr_server_config* cfg);

typedef struct {
  int64_t requests_done;       /* requests finished (any status)             */
  int64_t queries_done;
  int64_t batches_done;        /* batches finished                           */
  int64_t max_batch_requests;  /* most requests seen in one batch            */
  int64_t max_batch_rows;      /* most query rows seen in one batch          */
  int64_t max_recomputed_rows; /* largest per-round recomputed set seen      */
  int64_t lanes, max_batch, max_requests, request_slots, max_recomputed;
  int64_t device_bytes;        /* device memory held by the server           */
  int64_t slot_bytes;          /* device memory of one request slot          */
  int64_t gallery_size;        /* live gallery items                          */
  int64_t gallery_capacity;    /* gallery rows reserved                       */
  int64_t enqueue_us;          /* host time spent enqueuing batches, in all   */
} gcr_server_stats;

/* Build a server on ctx's device.
 *   gallery: DEVICE array [ng, d], float32 (gallery_dtype 0) or BF16 bit
 *   patterns (gallery_dtype 1, widened exactly); rows are used as given
 *   (queries are normalised when p->normalize_input).  The array is copied;
 *   the caller may free it afterwards.
 *   p: k >= 1, rounds, gamma, precision (screening), topk_out (1..120),
 *   normalize_input; rebuild_each_round must be 0 (the gallery graph is
 *   fixed); alpha / beta / cross_k are ignored.
 *   cfg: NULL for the defaults.
 * Synchronous: first synchronises the device, so work the caller enqueued
 * on any stream (for example a kernel still writing the gallery) completes
 * before the gallery is read; then builds the gallery graph and the
 * resident propagated copies and starts the worker thread.
 * Errors: INVALID, UNSUPPORTED, NOMEM, HIP (message in gcr_last_error(ctx)). */
gcr_status gcr_server_create(gcr_ctx* ctx, const void* gallery,
                             int32_t gallery_dtype, int64_t ng, int32_t d,
                             const gcr_params* p, const gcr_server_config* cfg,
                             gcr_server** out);
/* Queue one request: q_host is a HOST array [b, d] float32, copied before
 * the call returns; 1 <= b <= cfg.max_batch.  *ticket identifies the
 * request.
 * Thread-safe.  Errors: INVALID. */
gcr_status gcr_server_submit(gcr_server* srv, const float* q_host, int32_t b,
                             uint64_t* ticket);
/* Wait for a request (timeout_ms < 0: no limit; 0: poll).  On success the
 * HOST arrays idx_host [b, K] int32 (external gallery ids, -1 padding) and
 * dist_host [b, K] float32 receive the result (either may be NULL) and the
 * ticket is released.  Returns TIMEOUT (ticket kept) if not done in time;
 * UNSUPPORTED if the request needed more than max_recomputed rows in a
 * round; INVALID for an unknown ticket.  Thread-safe. */
gcr_status gcr_server_wait(gcr_server* srv, uint64_t ticket, int32_t* idx_host,
                           float* dist_host, int32_t timeout_ms);
gcr_status gcr_server_get_stats(gcr_server* srv, gcr_server_stats* out);
/* Message of the last failed server call (never NULL). */
const char* gcr_server_last_error(const gcr_server* srv);
/* Mutable gallery.  Every gallery item has an external id: the initial
 * items get 0..ng-1 and inserted items the next unused ids, in order.
 * Results of gcr_server_wait are external ids.  A mutation waits for the
 * requests on the device, holds back new ones while it runs, and leaves the
 * server exactly as a server created on the resulting gallery (items in id
 * order) would be: the gallery's kNN lists are maintained exactly (inserted
 * rows are searched against the whole gallery and merged into the lists they
 * enter; lists that lose a removed item are searched again), and the graph,
 * degrees, gallery-only rounds and screening operands are recomputed from
 * the lists.  The precomputed database graph of Sec. IV-F thereby follows a
 * changing database without a full rebuild.  Requests submitted before a
 * mutation call returns may run before or after it.  After a HIP error the
 * server must be destroyed.
 *
 * gcr_server_insert: rows_host is a HOST array [m, d] float32, used as
 *   supplied (as the gallery at creation); ids_out (HOST [m] or NULL)
 *   receives the new ids.  Errors: INVALID, UNSUPPORTED (beyond
 *   cfg.gallery_capacity), HIP.
 * gcr_server_remove: ids_host is a HOST array [m] of external ids (repeats
 *   allowed).  Errors: INVALID (an id not in the gallery, or fewer than 2
 *   items would remain; nothing is changed), HIP.
 * gcr_server_gallery_ids: the live ids in increasing order (the gallery's
 *   row order) into ids_host (HOST, capacity entries; NULL: count only);
 *   *count receives their number.
 * gcr_server_save / gcr_server_load: the resident state that is expensive to
 *   rebuild (parameters, ids, level-0 features, kNN lists) to / from a file;
 *   load recomputes the rest and starts a server with configuration cfg.
 *   Errors: INVALID (unreadable file or not a saved state), NOMEM, HIP. */
gcr_status gcr_server_insert(gcr_server* srv, const float* rows_host, int32_t m,
                             int32_t* ids_out);
gcr_status gcr_server_remove(gcr_server* srv, const int32_t* ids_host,
                             int32_t m);
gcr_status gcr_server_gallery_ids(gcr_server* srv, int32_t* ids_host,
                                  int64_t capacity, int64_t* count);
gcr_status gcr_server_save(gcr_server* srv, const char* path);
gcr_status gcr_server_load(gcr_ctx* ctx, const char* path,
                           const gcr_server_config* cfg, gcr_server** out);

/* Finish the requests in flight, fail the queued ones, free everything. */
gcr_status gcr_server_destroy(gcr_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* GCR_H */
