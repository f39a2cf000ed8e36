"""Parity at the full workload sizes, in the launch configurations the
benchmark uses, on outputs the FP64 oracle can compute one by one (sampled
rows), plus the cross-precision identity that holds at any size."""
import numpy as np
import pytest
import torch

from oracle import gcr_oracle as O
from paper_2306_08792_amd import datagen
from paper_2306_08792_amd.gcr import BF16, FP8, FP32, Context, Params

from parity import check_distances, check_features, check_knn_rows, oracle_round_from_lists

pytestmark = pytest.mark.gpu


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def sample(n, m, seed):
    return np.sort(np.random.default_rng(seed).choice(n, size=m, replace=False))


def test_cross_camera_full_size():
    """3,368 + 15,913 x 2,048, 6 cameras, k = 20, alpha = 0.5, L = 3, BF16
    screening: sampled neighbour lists of the first graph, one whole
    propagation round, and sampled final distance rows."""
    print("cross-camera full size", flush=True)
    ctx = Context(0)
    w = datagen.cross_camera_reid()
    n = w.X.shape[0]
    cam = dev(w.cams, torch.int32)
    p = Params(k=20, gamma=0.2, rounds=3, alpha=0.5, precision=BF16, rebuild_each_round=True)
    Xn = ctx.normalize_rows(dev(w.X))
    Xh = host(Xn).astype(np.float64)
    idx, dist, cidx, cdist = ctx.knn(Xn, p, cam, cross=True)
    rows = sample(n, 48, 1)
    check_knn_rows(host(idx)[rows], host(dist)[rows], Xh, rows, 20)
    check_knn_rows(host(cidx)[rows], host(cdist)[rows], Xh, rows, 20, cam=w.cams, cross=True, what="cross")
    g = ctx.build_graph(Xn, p, cam)
    Y = ctx.propagate(g, Xn)
    Yo, _, _ = oracle_round_from_lists(Xh, O.Params(k=20, gamma=0.2, rounds=1, alpha=0.5),
                                       host(g.field("idx")), host(g.field("cr_idx")), w.cams)
    check_features(host(Y), Yo, what="round 1")
    out = ctx.rerank(dev(w.X), w.nq, p, cam, dense=True, keep_features=True)
    XL = host(out["X"]).astype(np.float64)
    q = sample(w.nq, 32, 2)
    G = XL[w.nq:]
    Do = np.maximum(np.sum(XL[q] ** 2, 1)[:, None] + np.sum(G ** 2, 1)[None, :] - 2.0 * XL[q] @ G.T, 0.0)
    check_distances(host(out["dist"])[q], Do, what="final distances")
    ctx.close()


def test_video_full_size():
    """1,980 + 6,000 tracklets of 4-32 frames, d = 2,048: profile vectors
    (Eq. (16), lambda = 10) against np.linalg.solve, then GCRV (k = 15,
    L = 2) with sampled neighbour lists and final distances."""
    print("video full size", flush=True)
    ctx = Context(0)
    w = datagen.video_tracklets()
    offs = torch.from_numpy(w.offsets)
    W = ctx.profile_vectors(dev(w.frames), offs, None, mode="pvg", lam=10.0)
    Wo = O.profile_vectors(w.frames, w.offsets, None, lam=10.0, mode="pvg")
    check_features(host(W), Wo, what="profiles")
    p = Params(k=15, gamma=0.2, rounds=2, precision=BF16, lam=10.0)
    Wh = host(W).astype(np.float64)
    idx, dist = ctx.knn(W, p)
    rows = sample(Wh.shape[0], 48, 3)
    check_knn_rows(host(idx)[rows], host(dist)[rows], Wh, rows, 15)
    out = ctx.rerank(W, w.nq, p, dense=True, keep_features=True)
    XL = host(out["X"]).astype(np.float64)
    q = sample(w.nq, 32, 4)
    G = XL[w.nq:]
    Do = np.maximum(np.sum(XL[q] ** 2, 1)[:, None] + np.sum(G ** 2, 1)[None, :] - 2.0 * XL[q] @ G.T, 0.0)
    check_distances(host(out["dist"])[q], Do, what="final distances")
    ctx.close()


def test_large_retrieval_full_size_precisions():
    """20,000 + 200,000 x 512, k = 20, L = 2, top-100 output: FP32, BF16 and
    FP8 screening give bitwise the same features and top-100 lists (exact
    re-scoring), sampled first-graph lists and sampled top-100 rows match
    FP64 brute force."""
    print("large retrieval full size", flush=True)
    ctx = Context(0)
    w = datagen.large_retrieval()
    X = dev(w.X)
    res = {}
    for prec in (BF16, FP8, FP32):
        p = Params(k=20, gamma=0.2, rounds=2, precision=prec, topk_out=100, rebuild_each_round=True)
        out = ctx.rerank(X, w.nq, p, dense=False, topk=True, keep_features=True)
        res[prec] = (host(out["topk_idx"]), host(out["topk_dist"]), host(out["X"]))
        del out
        torch.cuda.empty_cache()
    for prec in (BF16, FP8):
        np.testing.assert_array_equal(res[prec][0], res[FP32][0])
        np.testing.assert_array_equal(res[prec][2].view(np.uint32), res[FP32][2].view(np.uint32))
    Xn = ctx.normalize_rows(X)
    Xh = host(Xn).astype(np.float64)
    idx, dist = ctx.knn(Xn, Params(k=20, precision=BF16))
    rows = sample(Xh.shape[0], 32, 5)
    check_knn_rows(host(idx)[rows], host(dist)[rows], Xh, rows, 20)
    XL = res[BF16][2].astype(np.float64)
    q = sample(w.nq, 24, 6)
    check_knn_rows(res[BF16][0][q], res[BF16][1][q], XL, q, 100, cols=np.arange(w.nq, XL.shape[0]),
                   exclude_self=False, what="final top-100")
    ctx.close()


def test_serving_full_size():
    """Resident 500,000 x 512 BF16 gallery, k = 20, L = 2, K = 100: sampled
    gallery lists against FP64 brute force, then three requests against the
    oracle's serving semantics evaluated over the whole gallery (with the
    library's gallery lists, which the sample checks)."""
    print("serving full size", flush=True)
    from paper_2306_08792_amd.gcr import Server

    from test_gpu_serving import check_request

    ctx = Context(0)
    bits, vals, centres = datagen.serving_gallery()
    g = dev(bits.view(np.int16), torch.int16)
    p = Params(k=20, rounds=2, gamma=0.2, topk_out=100, precision=BF16, rebuild_each_round=False)
    gidx, gdist = ctx.knn(dev(vals), Params(k=20, precision=BF16))
    gi, gd = host(gidx), host(gdist)
    rows = sample(vals.shape[0], 16, 7)
    check_knn_rows(gi[rows], gd[rows], vals, rows, 20)
    srv = Server(ctx, g, p, slots=2, max_batch=512, max_recomputed=65536, gallery_capacity=vals.shape[0] + 500)
    trace = datagen.serving_trace(centres, 3, 1000.0, seed=11)
    op = O.Params(k=20, gamma=0.2, rounds=2, alpha=1.0, rebuild_each_round=False)
    try:
        for _, Q, _ in trace:
            ri, rd = srv.query(Q)
            check_request(ri, rd, vals, gi.astype(np.int64), gd.astype(np.float64), Q, op, 100)
        # 500 items in, 500 out: the same answers as a server built on the
        # resulting gallery
        rng = np.random.default_rng(12)
        new = datagen._unit_rows_f32(centres[rng.integers(0, len(centres), 500)]
                                     + 0.6 * rng.standard_normal((500, vals.shape[1])))
        srv.insert(new)
        srv.remove(rng.choice(vals.shape[0], 500, replace=False))
        live = srv.ids()
        Xlive = np.concatenate([vals, new])[live]
        fresh = Server(ctx, dev(Xlive), p, slots=1, max_batch=512, max_recomputed=65536)
        try:
            for _, Q, _ in trace[:2]:
                a_i, a_d = srv.query(Q)
                b_i, b_d = fresh.query(Q)
                assert np.array_equal(a_i, np.where(b_i >= 0, live[np.maximum(b_i, 0)], -1))
                assert np.array_equal(a_d.view(np.uint32), b_d.view(np.uint32))
        finally:
            fresh.close()
    finally:
        srv.close()
    ctx.close()
