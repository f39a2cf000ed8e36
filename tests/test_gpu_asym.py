"""Asymmetric normalisation, Eq. (5)-(6): P = D_r^-1/2 A~ D_c^-1/2 with row
degrees D_r and column degrees D_c of the (non-symmetric) kNN affinity, in
the plain and the cross-camera (Eq. (9)) forms, against the FP64 oracle."""
import numpy as np
import pytest
import torch

from oracle import gcr_oracle as O
from paper_2306_08792_amd import datagen
from paper_2306_08792_amd.gcr import BF16, FP32, Context, Params

from parity import check_distances, check_features, check_knn_rows

pytestmark = pytest.mark.gpu


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


def oracle_asym_round(X, Xg, idx, gamma, cr_idx=None, alpha=1.0):
    """One round of Eq. (6) (blended as Eq. (9) when a cross list is given)
    from given lists; affinities from FP64 distances on Xg."""
    X = np.asarray(X, np.float64)
    Xg = np.asarray(Xg, np.float64)
    n = X.shape[0]

    def P_of(ix):
        ix = np.asarray(ix, np.int64)
        dist = np.full(ix.shape, np.inf)
        for i in range(n):
            for s in range(ix.shape[1]):
                j = ix[i, s]
                if j >= 0:
                    dist[i, s] = np.sum((Xg[i] - Xg[j]) ** 2)
        return O.asym_propagation_matrix(O.affinity_dense(n, ix, dist, gamma))

    P, Dr, Dc = P_of(idx)
    Y = P @ X
    if cr_idx is not None:
        Pc, _, _ = P_of(cr_idx)
        Y = alpha * Y + (1.0 - alpha) * (Pc @ X)
    return O.row_normalize(Y), Dr


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_asym_graph_and_round(ctx, prec):
    print(f"asym graph prec={prec}", flush=True)
    X, _ = datagen.clustered(30, 10, 48, 0.6, 11)
    n = len(X)
    p = Params(k=9, gamma=0.3, precision=prec, symmetric=False)
    Xd = dev(X)
    g = ctx.build_graph(Xd, p)
    assert g.g.asymmetric == 1
    idx = host(g.field("idx")).astype(np.int64)
    check_knn_rows(idx, host(g.field("dist")), X, np.arange(n), 9)
    Y = ctx.propagate(g, Xd)
    Yo, Dr = oracle_asym_round(X, X, idx, 0.3)
    np.testing.assert_allclose(host(g.field("deg")), Dr, rtol=2e-6)
    check_features(host(Y), Yo, what="asymmetric round")


def test_asym_cross_camera_rerank(ctx):
    """Two rebuilt rounds of Eq. (9) with asymmetric graphs, stage by stage,
    then the whole re-ranking call against the stages and the oracle's final
    distances."""
    print("asym cross camera rerank", flush=True)
    w = datagen.cross_camera_reid(seed=4, nq=100, ng=380, d=96, n_ids=60, n_cams=4)
    n = w.X.shape[0]
    cam = dev(w.cams, torch.int32)
    p = Params(k=8, gamma=0.2, rounds=2, alpha=0.7, precision=BF16, rebuild_each_round=True, symmetric=False)
    Xd = ctx.normalize_rows(dev(w.X))
    for t in range(p.rounds):
        Xh = host(Xd)
        g = ctx.build_graph(Xd, p, cam)
        assert g.g.asymmetric == 1 and g.has_cross
        check_knn_rows(host(g.field("idx")), host(g.field("dist")), Xh, np.arange(n), 8)
        check_knn_rows(host(g.field("cr_idx")), host(g.field("cr_dist")), Xh, np.arange(n), 8, cam=w.cams,
                       cross=True, what="cross")
        Yd = ctx.propagate(g, Xd)
        Yo, _ = oracle_asym_round(Xh, Xh, host(g.field("idx")), 0.2, host(g.field("cr_idx")), 0.7)
        check_features(host(Yd), Yo, what=f"round {t + 1}")
        Xd = Yd
    out = ctx.rerank(dev(w.X), w.nq, p, cam, dense=True, keep_features=True)
    np.testing.assert_array_equal(host(out["X"]), host(Xd))
    check_distances(host(out["dist"]), O.final_distances(host(Xd), w.nq))


def test_asym_end_to_end_matches_oracle(ctx):
    """Plain GCR with asymmetric graphs against the oracle's own rounds (its
    own exhaustive kNN), on well-separated clusters where the lists agree."""
    print("asym end to end", flush=True)
    X, _ = datagen.clustered(40, 8, 64, 0.4, 12)
    nq = 80
    p = Params(k=6, gamma=0.2, rounds=2, precision=FP32, rebuild_each_round=True, symmetric=False)
    out = ctx.rerank(dev(X), nq, p, dense=True, keep_features=True)
    ref = O.gcr(X, O.Params(k=6, gamma=0.2, rounds=2, symmetric=False))
    check_features(host(out["X"]), ref["X"][-1], what="asymmetric gcr")
    check_distances(host(out["dist"]), O.final_distances(ref["X"][-1], nq))


def test_serving_rejects_asym(ctx):
    from paper_2306_08792_amd.gcr import GcrError, Server
    X, _ = datagen.clustered(20, 10, 16, 0.5, 3)
    with pytest.raises(GcrError):
        Server(ctx, dev(X), Params(k=5, rebuild_each_round=False, symmetric=False))
