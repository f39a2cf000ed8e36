"""Parity of the HIP library (through its C ABI) with the FP64 oracle.

Small shapes span several 128-row tiles, ragged tails, tiny and odd feature
widths, k = 0 / 1 / large, all three screening precisions and camera lists.
"""
import math

import numpy as np
import pytest
import torch

from oracle import gcr_oracle as O
from paper_2306_08792_amd import datagen
from paper_2306_08792_amd.gcr import BF16, BF16_RAW, FP8, FP8_RAW, FP32, Context, Params

from parity import (check_distances, check_features, check_knn_rows,
                    oracle_round_from_lists)

pytestmark = pytest.mark.gpu

PRECS = [FP32, BF16, FP8]


@pytest.fixture(scope="module")
def ctx():
    c = Context(0)
    yield c
    c.close()


def dev(a, dtype=torch.float32):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(t):
    torch.cuda.synchronize()
    return t.cpu().numpy()


def case(n, d, seed, clustered=True):
    if clustered and n >= 8:
        per = max(2, n // max(1, n // 12))
        nc = (n + per - 1) // per
        X, _ = datagen.clustered(nc, per, d, 0.5, seed)
        return X[:n]
    return datagen.random_unit(n, d, seed)


@pytest.mark.parametrize("prec", PRECS)
@pytest.mark.parametrize("n,d,k,seed", [
    (7, 3, 2, 0), (9, 1, 8, 1), (40, 16, 7, 2), (129, 64, 20, 3), (300, 300, 15, 4),
    (517, 256, 20, 5), (260, 33, 1, 6), (200, 128, 120, 7),
])
def test_knn_matches_exhaustive(ctx, prec, n, d, k, seed):
    print(f"knn prec={prec} n={n} d={d} k={k} seed={seed}", flush=True)
    X = case(n, d, seed)
    p = Params(k=k, precision=prec)
    idx, dist = ctx.knn(dev(X), p)
    check_knn_rows(host(idx), host(dist), X, np.arange(n), k)


@pytest.mark.parametrize("prec,eps", [(BF16_RAW, 0.0080), (FP8_RAW, 0.14)])
@pytest.mark.parametrize("n,d", [(517, 256), (300, 512)])
def test_knn_raw_modes(ctx, prec, eps, n, d):
    """Screening-only modes: errors are reported, not gated, so this checks
    what holds for any screened selection.  With |s~ - s| <= eps for unit
    rows, every reported distance is within 2 eps of the exact one, the list
    is ordered by (reported distance, index), and every member's exact
    distance is at most the exact k-th distance + 4 eps."""
    print(f"raw knn prec={prec} n={n} d={d}", flush=True)
    X = case(n, d, 5).astype(np.float64)
    k = 20
    idx, dist = ctx.knn(dev(X), Params(k=k, precision=prec))
    gi, gd = host(idx), host(dist).astype(np.float64)
    D = O.sq_dists(X)
    ref, _ = O.knn_lists(D, k)
    agree = 0
    for i in range(n):
        assert np.all(gi[i] >= 0) and len(set(gi[i].tolist())) == k and i not in gi[i]
        ex = D[i, gi[i]]
        assert np.all(np.abs(gd[i] - ex) <= 2 * eps), f"row {i}: reported distance off by more than 2 eps"
        assert all((gd[i, t], gi[i, t]) <= (gd[i, t + 1], gi[i, t + 1]) for t in range(k - 1)), f"row {i}: order"
        kth = D[i, ref[i, -1]]
        assert np.all(ex <= kth + 4 * eps), f"row {i}: member beyond the k-th distance + 4 eps"
        agree += int(set(gi[i].tolist()) == set(ref[i].tolist()))
    print(f"raw mode {prec}: {agree}/{n} lists equal the exact ones", flush=True)


@pytest.mark.parametrize("prec", PRECS)
def test_knn_cross_camera(ctx, prec):
    print(f"knn cross prec={prec}", flush=True)
    rng = np.random.default_rng(11)
    n, d = 390, 96
    X = case(n, d, 12)
    cam = rng.integers(0, 4, size=n).astype(np.int32)
    p = Params(k=10, cross_k=6, precision=prec, alpha=0.5)
    idx, dist, cidx, cdist = ctx.knn(dev(X), p, dev(cam, torch.int32), cross=True)
    check_knn_rows(host(idx), host(dist), X, np.arange(n), 10)
    check_knn_rows(host(cidx), host(cdist), X, np.arange(n), 6, cam=cam, cross=True, what="cross")


def test_knn_duplicates_force_fallback(ctx):
    # 3,000 identical points: every screened key ties, the candidate buffers
    # (512 entries) overflow and the exhaustive path must still return
    # (distance, index) order, i.e. the lowest indices
    print("knn duplicates", flush=True)
    n = 3000  # four column splits of 768 columns: more ties than a buffer holds
    X = np.tile(datagen.random_unit(1, 64, 3), (n, 1))
    ctx.reset_stats()
    idx, dist = ctx.knn(dev(X), Params(k=20, precision=BF16))
    st = ctx.stats()
    I = host(idx)
    for i in list(range(0, n, 37)) + [n - 1]:
        exp = [j for j in range(n) if j != i][:20]
        assert I[i].tolist() == exp
    assert np.all(host(dist) == 0.0)
    assert st["knn_fallback_rows"] > 0
    # 2,999 ties per row exceed the float32 band (2,048 items)
    assert st["knn_exhaustive_rows"] > 0


def shell_workload(hubs=12, shell=1500, d=64, seed=5, shuffle=True):
    """Hubs with a shell of points whose squared distances to the hub are
    spread over [0.5, 0.51]: a hub's k-th neighbour sits inside a band of
    1,500 items narrower than the BF16 screening margin, more than one
    candidate buffer (256-512 entries) keeps.  Without shuffling, each hub's
    shell is a contiguous index range, so it lands in one or two column
    splits whatever the number of splits.  Returns (X, hub row indices)."""
    rng = np.random.default_rng(seed)
    H = datagen.random_unit(hubs, d, seed + 1).astype(np.float64)
    pts = []
    for h in H:
        U = rng.standard_normal((shell, d))
        U -= np.outer(U @ h, h)
        U /= np.linalg.norm(U, axis=1, keepdims=True)
        rho = np.sqrt(rng.uniform(0.5, 0.51, shell))
        pts.append(np.vstack([h[None], h[None] + rho[:, None] * U]))
    X = np.vstack(pts).astype(np.float32)
    perm = rng.permutation(len(X)) if shuffle else np.arange(len(X))
    inv = np.empty_like(perm)
    inv[perm] = np.arange(len(X))
    return X[perm], np.sort(inv[np.arange(hubs) * (shell + 1)])


@pytest.mark.parametrize("prec", [BF16, FP8])
def test_knn_band_resweep(ctx, prec):
    """Rows whose screening band overflows the candidate buffer are re-swept
    in float32 against every column; their lists stay exact, and a band
    within the re-sweep capacity (2,048 items) needs no exhaustive pass."""
    print(f"knn band re-sweep prec={prec}", flush=True)
    X, hub_rows = shell_workload(shuffle=False)
    n = len(X)
    ctx.reset_stats()
    idx, dist = ctx.knn(dev(X), Params(k=20, precision=prec))
    st = ctx.stats()
    rows = np.union1d(hub_rows, np.arange(0, n, 211))
    check_knn_rows(host(idx)[rows], host(dist)[rows], X, rows, 20)
    assert st["knn_fallback_rows"] >= len(hub_rows), st
    assert st["knn_exhaustive_rows"] <= max(0, st["knn_fallback_rows"] - 2048), st


def test_knn_k0_and_empty_cross(ctx):
    X = case(50, 8, 4)
    idx, dist = ctx.knn(dev(X), Params(k=0))
    assert idx.shape == (50, 0)
    cam = np.zeros(50, dtype=np.int32)
    i1, d1, ci, cd = ctx.knn(dev(X), Params(k=3, cross_k=3, alpha=0.5), dev(cam, torch.int32), cross=True)
    assert np.all(host(ci) == -1) and np.all(np.isinf(host(cd)))


def _oracle_graph_values(X, p, idx, cam=None, cr_idx=None):
    n = len(X)
    X = np.asarray(X, np.float64)
    def dist_of(ix):
        d = np.full(ix.shape, np.inf)
        for i in range(n):
            for s in range(ix.shape[1]):
                j = ix[i, s]
                if j >= 0:
                    d[i, s] = np.sum((X[i] - X[j]) ** 2)
        return d
    At = O.affinity_dense(n, idx, dist_of(idx), p.gamma, O._edge_scale(idx, cam, p))
    P, A, Dg = O.sym_propagation_matrix(At)
    return P, Dg


@pytest.mark.parametrize("d", [3, 101, 256, 2048, 2052, 3000])
def test_normalize_rows_widths(ctx, d):
    """Row normalisation on every path: scalar (d % 4 != 0), 16-byte with the
    row held in registers (d <= 2048), 16-byte two-pass (d > 2048); a zero
    row stays zero; in place gives the same result."""
    print(f"normalize d={d}", flush=True)
    rng = np.random.default_rng(d)
    X = (rng.standard_normal((37, d)) * rng.uniform(0.01, 50.0, (37, 1))).astype(np.float32)
    X[5] = 0.0
    Y = host(ctx.normalize_rows(dev(X)))
    X64 = X.astype(np.float64)
    ref = X64 / np.maximum(np.linalg.norm(X64, axis=1, keepdims=True), 1e-12)
    np.testing.assert_allclose(Y, ref, rtol=0, atol=2e-6)
    assert np.all(Y[5] == 0.0)
    Xd = dev(X)
    Z = host(ctx.normalize_rows(Xd, out=Xd))
    assert np.array_equal(Z.view(np.uint32), Y.view(np.uint32))


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_build_graph_values(ctx, prec):
    print(f"graph prec={prec}", flush=True)
    n, d = 333, 48
    X = case(n, d, 21)
    p = Params(k=9, gamma=0.3, precision=prec)
    g = ctx.build_graph(dev(X), p)
    idx = host(g.field("idx")).astype(np.int64)
    check_knn_rows(idx, host(g.field("dist")), X, np.arange(n), 9)
    P, Dg = _oracle_graph_values(X, O.Params(k=9, gamma=0.3), idx)
    np.testing.assert_allclose(host(g.field("deg")), Dg, rtol=2e-6)
    pf = host(g.field("pf"))
    for i in range(n):
        for s in range(9):
            j = idx[i, s]
            # forward value = half of A_ij's forward part / sqrt(D_i D_j)
            wij = math.exp(-np.sum((X[i].astype(np.float64) - X[j]) ** 2) / 0.3)
            assert abs(pf[i, s] - 0.5 * wij / math.sqrt(Dg[i] * Dg[j])) < 2e-6 * max(1.0, pf[i, s])
    rp, rs, pr = host(g.field("rev_ptr")), host(g.field("rev_src")), host(g.field("pr"))
    dense = np.zeros((n, n))
    for i in range(n):
        dense[i, idx[i]] += pf[i]
        for q in range(rp[i], rp[i + 1]):
            dense[i, rs[q]] += pr[q]
        assert np.all(np.diff(rs[rp[i]:rp[i + 1]]) > 0), "reverse row not sorted by source"
        dense[i, i] += host(g.field("self"))[i]
    np.testing.assert_allclose(dense, P, atol=2e-6)
    assert rp[-1] == n * 9


def test_build_graph_hub_rows(ctx):
    """A hub that nearly every row lists as a neighbour: its reverse row holds
    more than the 512 entries the wave-per-row sort stages in LDS, so the
    one-lane path sorts it; degrees, sorted reverse rows and the normalised
    matrix against the oracle."""
    print("graph hub rows", flush=True)
    rng = np.random.default_rng(77)
    d, m = 32, 1100
    S = rng.standard_normal((m, d))
    S /= np.linalg.norm(S, axis=1, keepdims=True)
    far = 5.0 + rng.standard_normal((99, d))
    X = np.concatenate([np.zeros((1, d)), S, far]).astype(np.float32)
    n, k = X.shape[0], 9
    g = ctx.build_graph(dev(X), Params(k=k, gamma=0.5, precision=FP32))
    idx = host(g.field("idx")).astype(np.int64)
    check_knn_rows(idx, host(g.field("dist")), X, np.arange(n), k)
    rp, rs, pr = host(g.field("rev_ptr")), host(g.field("rev_src")), host(g.field("pr"))
    assert rp[1] - rp[0] > 512, "the hub's reverse row should exceed the LDS-staged size"
    P, Dg = _oracle_graph_values(X, O.Params(k=k, gamma=0.5), idx)
    np.testing.assert_allclose(host(g.field("deg")), Dg, rtol=2e-6)
    pf, selfv = host(g.field("pf")), host(g.field("self"))
    dense = np.zeros((n, n))
    for i in range(n):
        dense[i, idx[i]] += pf[i]
        assert np.all(np.diff(rs[rp[i]:rp[i + 1]]) > 0), "reverse row not sorted by source"
        dense[i, rs[rp[i]:rp[i + 1]]] += pr[rp[i]:rp[i + 1]]
        dense[i, i] += selfv[i]
    np.testing.assert_allclose(dense, P, atol=2e-6)


@pytest.mark.parametrize("d", [3, 64, 256, 512, 700])
def test_propagate_one_round(ctx, d):
    print(f"propagate d={d}", flush=True)
    n = 290
    X = case(n, d, 30 + d)
    p = Params(k=7, gamma=0.2)
    Xd = dev(X)
    g = ctx.build_graph(Xd, p)
    Y = ctx.propagate(g, Xd)
    Yo, _, _ = oracle_round_from_lists(X, O.Params(k=7, gamma=0.2), host(g.field("idx")))
    check_features(host(Y), Yo)


@pytest.mark.parametrize("d,k", [(256, 20), (512, 20), (512, 3)])
def test_propagate_larger_graphs(ctx, d, k):
    """One round on 6,001 clustered nodes (many workgroups, a ragged last
    one, reverse lists of every length) against the oracle's sparse round,
    and bitwise the same on a second run."""
    print(f"propagate n=6001 d={d} k={k}", flush=True)
    n = 6001
    X = case(n, d, 40 + d + k)
    p = Params(k=k, gamma=0.2)
    Xd = dev(X)
    g = ctx.build_graph(Xd, p)
    Y = ctx.propagate(g, Xd)
    Yo, _, _ = oracle_round_from_lists(X, O.Params(k=k, gamma=0.2), host(g.field("idx")))
    check_features(host(Y), Yo)
    Y2 = ctx.propagate(g, Xd)
    assert np.array_equal(host(Y).view(np.uint32), host(Y2).view(np.uint32))


def test_propagate_rejects_in_place(ctx):
    X = dev(case(40, 8, 1))
    g = ctx.build_graph(X, Params(k=3))
    with pytest.raises(Exception):
        ctx.propagate(g, X, out=X)


@pytest.mark.parametrize("prec", PRECS)
def test_final_distances_dense_and_topk(ctx, prec):
    print(f"final prec={prec}", flush=True)
    nq, ng, d = 150, 700, 72
    X = case(nq + ng, d, 40)
    p = Params(topk_out=25, precision=prec)
    D, ti, td = ctx.final_distances(dev(X), nq, p, dense=True, topk=True)
    Do = O.final_distances(X, nq)
    check_distances(host(D), Do)
    check_knn_rows(host(ti), host(td), X, np.arange(nq), 25, cols=np.arange(nq, nq + ng),
                   exclude_self=False, what="final top-K")


@pytest.mark.parametrize("d,scale", [(2048, 1e-3), (512, 1e-5), (100, 0.0)])
def test_final_distances_near_duplicates(ctx, d, scale):
    """Gallery rows that are the queries plus tiny perturbations (and exact
    copies): distances near zero, where the absolute tolerance binds and the
    split-bfloat16 inner products must cancel against the float32 norms."""
    print(f"final near-duplicates d={d} scale={scale}", flush=True)
    rng = np.random.default_rng(d)
    nq = 130
    Q = rng.standard_normal((nq, d))
    Q /= np.linalg.norm(Q, axis=1, keepdims=True)
    G = np.concatenate([Q + scale * rng.standard_normal((nq, d)), Q, rng.standard_normal((200, d)) * 0.05])
    X = np.concatenate([Q, G]).astype(np.float32)
    D, _, _ = ctx.final_distances(dev(X), nq, Params(), dense=True)
    Dg, Do = host(D), O.final_distances(X, nq)
    check_distances(Dg, Do, what="near-duplicate distances")
    # exact copies: the distance of a row to itself
    np.testing.assert_allclose(Dg[np.arange(nq), nq + np.arange(nq)], 0.0, atol=1e-5)


def _stagewise_rerank(ctx, X, nq, p, op, cam=None, prec=FP32):
    """Run the rounds one at a time through the C ABI and check each stage
    against the oracle fed with the GPU's previous features."""
    Xd = ctx.normalize_rows(dev(X))
    Xh = host(Xd)
    np.testing.assert_allclose(Xh, O.row_normalize(X), atol=3e-7)
    camd = None if cam is None else dev(cam, torch.int32)
    g = None
    for t in range(p.rounds):
        if g is None or p.rebuild_each_round:
            g = ctx.build_graph(Xd, p, camd)
            Xgraph = Xh
            n = Xh.shape[0]
            check_knn_rows(host(g.field("idx")), host(g.field("dist")), Xh, np.arange(n), p.k)
            if g.has_cross:
                check_knn_rows(host(g.field("cr_idx")), host(g.field("cr_dist")), Xh, np.arange(n),
                               g.cross_k, cam=cam, cross=True, what="cross")
        Yd = ctx.propagate(g, Xd)
        Yo, _, _ = oracle_round_from_lists(Xh, op, host(g.field("idx")),
                                           host(g.field("cr_idx")) if g.has_cross else None, cam,
                                           X_graph=Xgraph)
        check_features(host(Yd), Yo, what=f"round {t + 1}")
        Xd, Xh = Yd, host(Yd)
    return Xd


@pytest.mark.parametrize("prec", [FP32, BF16])
@pytest.mark.parametrize("rebuild", [True, False])
def test_rerank_small_plain(ctx, prec, rebuild):
    print(f"rerank small prec={prec} rebuild={rebuild}", flush=True)
    X, _ = datagen.clustered(40, 9, 64, 0.5, 50)
    nq = 90
    p = Params(k=8, gamma=0.2, rounds=3, rebuild_each_round=rebuild, precision=prec)
    op = O.Params(k=8, gamma=0.2, rounds=3, rebuild_each_round=rebuild)
    XT = _stagewise_rerank(ctx, X, nq, p, op)
    out = ctx.rerank(dev(X), nq, p, dense=True, topk=True, keep_features=True)
    # the fused entry point must equal the step-by-step calls bit for bit
    np.testing.assert_array_equal(host(out["X"]), host(XT))
    check_distances(host(out["dist"]), O.final_distances(host(XT), nq))
    # and the independent FP64 run from X_0
    ref = O.gcr(X, op)
    check_features(host(out["X"]), ref["X"][-1], what="end-to-end features")
    check_distances(host(out["dist"]), O.final_distances(ref["X"][-1], nq), what="end-to-end distances")


def test_rerank_seeded_lists_longer_than_a_wave(ctx):
    """k = 70 > 64: from the second round on the screening thresholds are
    seeded from the previous lists, which the seeding reads 64 entries at a
    time.  BF16 (seeded from the BF16 operand) and FP32 screening give the
    same features bit for bit, and both match the FP64 oracle."""
    print("rerank k=70 seeded", flush=True)
    X, _ = datagen.clustered(30, 14, 512, 0.6, 61)
    nq = 60
    outs = {}
    for prec in (BF16, FP32):
        p = Params(k=70, gamma=0.3, rounds=3, precision=prec)
        outs[prec] = host(ctx.rerank(dev(X), nq, p, dense=True, keep_features=True)["X"])
    assert np.array_equal(outs[BF16].view(np.uint32), outs[FP32].view(np.uint32))
    ref = O.gcr(X, O.Params(k=70, gamma=0.3, rounds=3))
    check_features(outs[BF16], ref["X"][-1], what="k = 70 features")


@pytest.mark.parametrize("alpha,beta", [(0.5, (1.0, 1.0)), (0.7, (1.0, 1.0)), (1.0, (0.5, 1.0))])
def test_rerank_cross_camera(ctx, alpha, beta):
    print(f"rerank cross alpha={alpha} beta={beta}", flush=True)
    w = datagen.cross_camera_reid(seed=3, nq=120, ng=500, d=128, n_ids=60, n_cams=4)
    p = Params(k=10, gamma=0.2, rounds=3, alpha=alpha, beta_same=beta[0], beta_cross=beta[1])
    op = O.Params(k=10, gamma=0.2, rounds=3, alpha=alpha, beta_same=beta[0], beta_cross=beta[1])
    XT = _stagewise_rerank(ctx, w.X, w.nq, p, op, cam=w.cams)
    out = ctx.rerank(dev(w.X), w.nq, p, dev(w.cams, torch.int32), dense=True, keep_features=True)
    np.testing.assert_array_equal(host(out["X"]), host(XT))
    ref = O.gcr(w.X, op, w.cams)
    check_features(host(out["X"]), ref["X"][-1], what="end-to-end features")
    check_distances(host(out["dist"]), O.final_distances(ref["X"][-1], w.nq), what="end-to-end distances")


def test_rerank_k0_is_normalisation(ctx):
    X = case(70, 20, 5)
    out = ctx.rerank(dev(X), 10, Params(k=0, rounds=2), keep_features=True)
    np.testing.assert_allclose(host(out["X"]), O.row_normalize(X), atol=3e-7)


@pytest.mark.parametrize("mode", ["pvg", "mean"])
@pytest.mark.parametrize("groups", [False, True])
def test_profile_vectors(ctx, mode, groups):
    print(f"pvg mode={mode} groups={groups}", flush=True)
    w = datagen.video_tracklets(seed=2, nq=30, ng=90, d=200, n_ids=25)
    nt = len(w.offsets) - 1
    grp = (np.arange(nt) % 3).astype(np.int32) if groups else None
    W = ctx.profile_vectors(dev(w.frames), torch.from_numpy(w.offsets), None if grp is None else torch.from_numpy(grp),
                            mode=mode, lam=10.0)
    Wo = O.profile_vectors(w.frames, w.offsets, grp, lam=10.0, mode=mode)
    check_features(host(W), Wo, what="profiles")


@pytest.mark.parametrize("d", [3, 130, 132, 260])
def test_profile_vectors_widths(ctx, d):
    """Feature widths off the 16-byte path (3, 130: the scalar Gram and GEMM)
    and on it with a ragged last 128-column tile (132, 260), three groups."""
    print(f"pvg d={d}", flush=True)
    w = datagen.video_tracklets(seed=6, nq=20, ng=60, d=d, n_ids=20)
    nt = len(w.offsets) - 1
    grp = (np.arange(nt) % 3).astype(np.int32)
    W = ctx.profile_vectors(dev(w.frames), torch.from_numpy(w.offsets), torch.from_numpy(grp), mode="pvg", lam=10.0)
    Wo = O.profile_vectors(w.frames, w.offsets, grp, lam=10.0, mode="pvg")
    check_features(host(W), Wo, what="profiles")


def test_profile_vectors_small_lambda(ctx):
    w = datagen.video_tracklets(seed=4, nq=10, ng=30, d=64, n_ids=10)
    W = ctx.profile_vectors(dev(w.frames), torch.from_numpy(w.offsets), None, mode="pvg", lam=0.05)
    Wo = O.profile_vectors(w.frames, w.offsets, None, lam=0.05)
    check_features(host(W), Wo, what="profiles")


def test_gcrv_small(ctx):
    w = datagen.video_tracklets(seed=5, nq=40, ng=120, d=128, n_ids=30)
    p = Params(k=6, gamma=0.2, rounds=2, lam=10.0)
    out = ctx.gcrv(dev(w.frames), torch.from_numpy(w.offsets), 40, p, dense=True)
    ref = O.gcrv(w.frames, w.offsets, None, 40, O.Params(k=6, gamma=0.2, rounds=2, lam=10.0))
    check_features(host(out["W"]), ref["W"], what="profiles")
    check_features(host(out["X"]), ref["X"][-1], what="gcrv features")
    check_distances(host(out["dist"]), O.final_distances(ref["X"][-1], 40))


def test_plain_gcr_small_workload(ctx):
    """The 500 + 1,500 x 256 workload end to end (k 20, gamma 0.1, 2 rounds)."""
    w = datagen.plain_gcr_small()
    p = Params(k=20, gamma=0.1, rounds=2)
    op = O.Params(k=20, gamma=0.1, rounds=2)
    XT = _stagewise_rerank(ctx, w.X, w.nq, p, op)
    out = ctx.rerank(dev(w.X), w.nq, p, dense=True, topk=True, keep_features=True)
    np.testing.assert_array_equal(host(out["X"]), host(XT))
    check_distances(host(out["dist"]), O.final_distances(host(XT), w.nq))
    from oracle.metrics import mean_average_precision
    m = mean_average_precision(host(out["dist"]), w.ids[:w.nq], w.ids[w.nq:])
    assert m >= 0.99


@pytest.mark.parametrize("prec", PRECS)
def test_knn_truncated_splits(ctx, prec):
    """Identities interleaved over 3,000 rows: each column split holds only a
    few members of a row's cluster, so its local k-th neighbour lies among
    unrelated items and the split buffers truncate.  The lists must stay
    exact, and no row should need the exhaustive path."""
    print(f"knn truncated splits prec={prec}", flush=True)
    w = datagen.cross_camera_reid(seed=9, nq=600, ng=2400, d=128, n_ids=150, n_cams=5)
    p = Params(k=15, precision=prec, alpha=0.5)
    ctx.reset_stats()
    idx, dist, cidx, cdist = ctx.knn(dev(w.X), p, dev(w.cams, torch.int32), cross=True)
    st = ctx.stats()
    rows = np.arange(0, 3000, 7)
    check_knn_rows(host(idx)[rows], host(dist)[rows], w.X, rows, 15)
    check_knn_rows(host(cidx)[rows], host(cdist)[rows], w.X, rows, 15, cam=w.cams, cross=True, what="cross")
    if prec != FP8:
        assert st["knn_fallback_rows"] == 0, st


@pytest.mark.parametrize("prec", [FP32, BF16])
@pytest.mark.parametrize("npts", [5, 1])
def test_knn_exact_ties_exhaustive_paths(ctx, prec, npts):
    """9,000 rows that are `npts` distinct points repeated: every neighbour
    is at distance 0 and a column split holds more ties than a candidate
    buffer keeps.  A buffer cannot keep part of a tie, so it truncates below
    the tied key, the row has no bound on its k-th distance and every row
    takes the exhaustive paths (column-chunked, then one block per row past
    its capacity).  The lists must be the lowest indices of the same point
    in (distance, index) order."""
    print(f"knn exact ties prec={prec} points={npts}", flush=True)
    n, d, k = 9000, 16, 20
    base = datagen.random_unit(npts, d, 21)
    X = base[np.arange(n) % npts]
    ctx.reset_stats()
    idx, dist = ctx.knn(dev(X), Params(k=k, precision=prec))
    st = ctx.stats()
    I = host(idx)
    for i in list(range(0, n, 97)) + [n - 1]:
        exp = [j for j in range(i % npts, n, npts) if j != i][:k]
        assert I[i].tolist() == exp, i
    assert np.all(host(dist) == 0.0)
    assert st["knn_fallback_rows"] == n
    assert st["knn_exhaustive_rows"] == n, st


@pytest.mark.parametrize("prec", [FP32, BF16, FP8])
def test_knn_fewer_eligible_than_k(ctx, prec):
    """Rows with fewer eligible items than k: 9 rows with k = 12 (global
    lists), and a cross-camera list where 35 of 40 rows share a camera
    (those rows have 5 other-camera items for cross_k = 8).  The lists hold
    every eligible item and -1 padding, never a column outside the set."""
    print(f"knn fewer eligible than k prec={prec}", flush=True)
    X = datagen.random_unit(9, 40, seed=41)
    idx, dist = ctx.knn(dev(X), Params(k=12, precision=prec))
    check_knn_rows(host(idx), host(dist), X.astype(np.float64), np.arange(9), 12)
    X2 = datagen.random_unit(40, 72, seed=42)
    cams = np.zeros(40, dtype=np.int32)
    cams[35:] = np.arange(1, 6)
    p = Params(k=6, cross_k=8, alpha=0.5, precision=prec)
    i0, d0, i1, d1 = ctx.knn(dev(X2), p, dev(cams, torch.int32), cross=True)
    X2d = X2.astype(np.float64)
    check_knn_rows(host(i0), host(d0), X2d, np.arange(40), 6)
    check_knn_rows(host(i1), host(d1), X2d, np.arange(40), 8, cam=cams, cross=True, what="cross")


@pytest.mark.parametrize("prec", PRECS)
def test_short_lists_in_final_topk_and_rerank(ctx, prec):
    """Top-K with K above the gallery size (padding), and a whole re-ranking
    of 1 query + 2 gallery items with k above n - 1."""
    print(f"short lists prec={prec}", flush=True)
    nq, ng, d = 5, 10, 24
    X = case(nq + ng, d, 43)
    p = Params(topk_out=25, precision=prec)
    D, ti, td = ctx.final_distances(dev(X), nq, p, dense=True, topk=True)
    check_distances(host(D), O.final_distances(X, nq))
    check_knn_rows(host(ti), host(td), X, np.arange(nq), 25, cols=np.arange(nq, nq + ng),
                   exclude_self=False, what="final top-K")
    X3 = case(3, 16, 44, clustered=False)
    p3 = Params(k=5, gamma=0.5, rounds=2, precision=prec, topk_out=4)
    out = ctx.rerank(dev(X3), 1, p3, dense=True, topk=True, keep_features=True)
    ref = O.gcr(X3, O.Params(k=5, gamma=0.5, rounds=2))
    check_features(host(out["X"]), ref["X"][-1], what="tiny rerank")
    check_distances(host(out["dist"]), O.final_distances(ref["X"][-1], 1), what="tiny rerank distances")
    ti = host(out["topk_idx"])
    assert np.all(ti[0, 2:] == -1) and sorted(ti[0, :2].tolist()) == [0, 1]
