"""Serving (resident gallery + request loop) against the FP64 oracle's
serving semantics: node set = gallery + the request's queries, gallery lists
frozen, query rows over the gallery only, fixed-graph rounds, top-K by
squared distance over the propagated features."""
import numpy as np
import pytest
import torch

from oracle import gcr_oracle as O
from paper_2306_08792_amd import datagen
from paper_2306_08792_amd.gcr import BF16, FP8, FP32, Context, GcrError, Params, Server

from parity import DIST_ATOL, DIST_RTOL

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def gallery_and_queries(seed=3, n_ids=150, per=20, d=64, sigma=0.6, nreq=6, sizes=(1, 5, 17, 64, 3, 40)):
    X, ids = datagen.clustered(n_ids, per, d, sigma, seed)
    rng = np.random.default_rng(seed + 100)
    centres = np.random.default_rng(seed).standard_normal((n_ids, d))  # same centres as `clustered`
    reqs = []
    for b in sizes[:nreq]:
        cid = rng.integers(0, n_ids, size=b)
        reqs.append(datagen._unit_rows_f32(centres[cid] + sigma * rng.standard_normal((b, d))))
    return X, reqs


def oracle_gallery_lists(XG, k):
    Dm = O.sq_dists(np.asarray(XG, np.float64))
    return O.knn_lists(Dm, k)


def check_request(gi, gd, XG, g_idx, g_dist, Q, op, K):
    """GPU top-K of one request vs the oracle: sorted distances position by
    position within the distance tolerance; every oracle item clearly inside
    the top-K (by more than two tolerances) is returned; every returned item
    is among the oracle's top-(K + 10) with a matching distance."""
    oi, od = O.serve_request(XG, g_idx, g_dist, Q, op, K + 10)
    for r in range(len(Q)):
        lim = DIST_RTOL * np.abs(od[r, :K]) + DIST_ATOL
        assert np.all(np.abs(gd[r].astype(np.float64) - od[r, :K]) <= lim), (r, gd[r][:5], od[r, :5])
        band = 2 * (DIST_RTOL * od[r, K - 1] + DIST_ATOL)
        must = set(oi[r, :K][od[r, :K] < od[r, K - 1] - band].tolist())
        got = gi[r].tolist()
        assert must <= set(got), (r, sorted(must - set(got))[:5])
        pos = {int(j): t for t, j in enumerate(oi[r])}
        for t, j in enumerate(got):
            assert j in pos, (r, j)
            o = od[r, pos[j]]
            assert abs(float(gd[r, t]) - o) <= DIST_RTOL * abs(o) + DIST_ATOL


@pytest.mark.parametrize("prec", [FP32, BF16, FP8])
def test_serving_matches_oracle(ctx, prec):
    print(f"serving parity prec={prec}", flush=True)
    X, reqs = gallery_and_queries()
    k, K = 8, 10
    p = Params(k=k, rounds=2, gamma=0.2, topk_out=K, precision=prec, rebuild_each_round=False)
    op = O.Params(k=k, gamma=0.2, rounds=2, alpha=1.0, rebuild_each_round=False)
    g_idx, g_dist = oracle_gallery_lists(X, k)
    srv = Server(ctx, torch.from_numpy(X).cuda(), p, lanes=3, max_batch=64, max_recomputed=3000)
    try:
        for Q in reqs:
            gi, gd = srv.query(Q)
            check_request(gi, gd, X, g_idx, g_dist, Q, op, K)
        st = srv.stats()
        assert st["requests_done"] == len(reqs)
        assert 0 < st["max_recomputed_rows"] <= 3000
    finally:
        srv.close()


def test_serving_one_round_and_zero_rounds(ctx):
    print("serving rounds 1 and 0", flush=True)
    X, reqs = gallery_and_queries(seed=4, nreq=3)
    k, K = 6, 12
    g_idx, g_dist = oracle_gallery_lists(X, k)
    for rounds in (1, 0):
        p = Params(k=k, rounds=rounds, topk_out=K, precision=BF16, rebuild_each_round=False)
        op = O.Params(k=k, gamma=0.2, rounds=rounds, alpha=1.0, rebuild_each_round=False)
        srv = Server(ctx, torch.from_numpy(X).cuda(), p, lanes=2, max_batch=64, max_recomputed=3000)
        try:
            for Q in reqs:
                gi, gd = srv.query(Q)
                check_request(gi, gd, X, g_idx, g_dist, Q, op, K)
        finally:
            srv.close()


def test_serving_alone_equals_mix(ctx):
    """Each request's result is bitwise the same when it runs alone and when
    it is co-batched with others (12 requests queued at once on 2 lanes:
    batches of up to 64 query rows share their gallery sweeps)."""
    print("serving alone vs mix", flush=True)
    sizes = (1, 64, 7, 33, 2, 50, 16, 5, 64, 9, 21, 3)
    X, reqs = gallery_and_queries(seed=5, nreq=len(sizes), sizes=sizes)
    p = Params(k=8, rounds=2, topk_out=10, precision=BF16, rebuild_each_round=False)
    op = O.Params(k=8, gamma=0.2, rounds=2, alpha=1.0, rebuild_each_round=False)
    g_idx, g_dist = oracle_gallery_lists(X, 8)
    srv = Server(ctx, torch.from_numpy(X).cuda(), p, lanes=2, max_batch=64, max_recomputed=3000)
    try:
        alone = [srv.query(Q) for Q in reqs]
        assert srv.stats()["max_batch_requests"] == 1
        tickets = [srv.submit(Q) for Q in reqs]
        mixed = [srv.wait(t) for t in reversed(tickets)][::-1]
        st = srv.stats()
        assert st["max_batch_requests"] > 1, st  # the queued requests were co-batched
        assert st["max_batch_rows"] <= 64, st
        for (ai, ad), (mi, md), Q in zip(alone, mixed, reqs):
            assert np.array_equal(ai, mi)
            assert np.array_equal(ad.view(np.uint32), md.view(np.uint32))
            check_request(mi, md, X, g_idx, g_dist, Q, op, 10)
    finally:
        srv.close()


def test_serving_memory_based_admission(ctx):
    """The request scratch comes from the memory budget: with room for two
    request slots, batches hold at most two requests, every result still
    equals the request run alone, and a budget below one slot is refused."""
    print("serving memory budget", flush=True)
    sizes = (3, 1, 20, 8, 2, 40, 5, 11)
    X, reqs = gallery_and_queries(seed=7, nreq=len(sizes), sizes=sizes)
    p = Params(k=8, rounds=2, topk_out=10, precision=BF16, rebuild_each_round=False)
    ref = Server(ctx, torch.from_numpy(X).cuda(), p, lanes=1, max_batch=64, max_recomputed=3000)
    slot = ref.stats()["slot_bytes"]
    try:
        alone = [ref.query(Q) for Q in reqs]
    finally:
        ref.close()
    srv = Server(ctx, torch.from_numpy(X).cuda(), p, lanes=2, max_batch=64, max_requests=16, max_recomputed=3000,
                 mem_budget=2 * slot + slot // 2)
    try:
        st = srv.stats()
        assert st["request_slots"] == 2, st
        tickets = [srv.submit(Q) for Q in reqs]
        mixed = [srv.wait(t) for t in tickets]
        st = srv.stats()
        assert 1 <= st["max_batch_requests"] <= 2, st
        for (ai, ad), (mi, md) in zip(alone, mixed):
            assert np.array_equal(ai, mi)
            assert np.array_equal(ad.view(np.uint32), md.view(np.uint32))
    finally:
        srv.close()
    with pytest.raises(GcrError, match="NOMEM"):
        Server(ctx, torch.from_numpy(X).cuda(), p, lanes=1, max_batch=64, max_recomputed=3000, mem_budget=slot // 2)


def test_serving_bf16_gallery(ctx):
    """A BF16 gallery (bit patterns) serves the same results as the float32
    gallery holding the same values."""
    print("serving bf16 gallery", flush=True)
    bits, vals, centres = datagen.serving_gallery(seed=2, ng=3000, d=64, n_ids=150)
    trace = datagen.serving_trace(centres, 4, 1000.0, seed=3, max_b=64)
    p = Params(k=8, rounds=2, topk_out=10, precision=BF16, rebuild_each_round=False)
    op = O.Params(k=8, gamma=0.2, rounds=2, alpha=1.0, rebuild_each_round=False)
    g_idx, g_dist = oracle_gallery_lists(vals, 8)
    s16 = Server(ctx, torch.from_numpy(bits.view(np.int16)).cuda(), p, lanes=2, max_batch=64, max_recomputed=3000)
    s32 = Server(ctx, torch.from_numpy(vals).cuda(), p, lanes=2, max_batch=64, max_recomputed=3000)
    try:
        for _, Q, _ in trace:
            a = s16.query(Q)
            b = s32.query(Q)
            assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
            check_request(a[0], a[1], vals, g_idx, g_dist, Q, op, 10)
    finally:
        s16.close()
        s32.close()


def test_serving_errors(ctx):
    print("serving errors", flush=True)
    X, reqs = gallery_and_queries(seed=6, nreq=2, sizes=(5, 40))
    p = Params(k=8, rounds=2, topk_out=10, precision=BF16, rebuild_each_round=False)
    with pytest.raises(GcrError):
        Server(ctx, torch.from_numpy(X).cuda(), Params(k=8, rebuild_each_round=True))
    with pytest.raises(GcrError):
        Server(ctx, torch.from_numpy(X).cuda(), p, lanes=0)
    srv = Server(ctx, torch.from_numpy(X).cuda(), p, lanes=2, max_batch=16, max_recomputed=20)
    try:
        with pytest.raises(GcrError):
            srv.submit(reqs[1])  # 40 queries > 16
        t = srv.submit(reqs[0])
        with pytest.raises(GcrError, match="per-request capacity"):
            srv.wait(t)  # five queries touch more than 20 rows
    finally:
        srv.close()


def test_serving_gallery_smaller_than_k(ctx):
    """Six gallery items with k = 8: every list (gallery and query) holds all
    eligible items and -1 padding."""
    print("serving tiny gallery", flush=True)
    X, reqs = gallery_and_queries(seed=12, n_ids=3, per=2, nreq=2, sizes=(1, 4))
    k, K = 8, 5
    p = Params(k=k, rounds=2, gamma=0.2, topk_out=K, precision=BF16, rebuild_each_round=False)
    op = O.Params(k=k, gamma=0.2, rounds=2, alpha=1.0, rebuild_each_round=False)
    g_idx, g_dist = oracle_gallery_lists(X, k)
    srv = Server(ctx, torch.from_numpy(X).cuda(), p, lanes=1, max_batch=8, max_recomputed=6)
    try:
        for Q in reqs:
            gi, gd = srv.query(Q)
            check_request(gi, gd, X, g_idx, g_dist, Q, op, K)
    finally:
        srv.close()
