"""DSFP (Alg. 1, GCR_Local) against the FP64 oracle: the kernel over given
lists (all list sizes up to the maximum, widths with and without the vector
path, 0-3 rounds, padded / repeated / self / out-of-range entries), the
whole GCR_Local pipeline, and sampled rows at the full cross-camera size."""
import numpy as np
import pytest
import torch

from oracle import gcr_oracle as O
from paper_2306_08792_amd import datagen
from paper_2306_08792_amd.gcr import BF16, FP32, Context, GcrError, Params

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


def oracle_lists(X, k):
    idx, _ = O.knn_lists(O.sq_dists(np.asarray(X, np.float64)), k)
    return idx


def oracle_rows(X, idx, rows, gamma, rounds):
    """Oracle DSFP output of the given nodes only (each node is independent)."""
    X = np.asarray(X, np.float64)
    return np.stack([O.dsfp_node(X, O.local_set(int(i), idx[i]), gamma, rounds) for i in rows])


@pytest.mark.parametrize("k", [0, 1, 5, 20, 37, 59])
def test_dsfp_list_sizes(ctx, k):
    """Every local-set size class (one to fifteen 4 x 4 Gram blocks per side),
    d = 200 (vector path, four staged chunks with a ragged tail)."""
    print(f"dsfp k={k}", flush=True)
    X, _ = datagen.clustered(40, 12, 200, 0.6, seed=k + 1)
    idx = oracle_lists(X, k).astype(np.int32)
    p = Params(k=k, gamma=0.3, rounds=2)
    Y = ctx.dsfp(dev(X), dev(idx, torch.int32) if k else None, p)
    Yo = O.dsfp(X, O.Params(k=k, gamma=0.3, rounds=2, normalize_input=False), idx)
    check_features(host(Y), Yo, what=f"dsfp k={k}")


@pytest.mark.parametrize("d,rounds", [(64, 1), (101, 3), (2048, 2), (7, 2), (1, 1), (2048, 3)])
def test_dsfp_widths_and_rounds(ctx, d, rounds):
    """Vector (d % 4 == 0) and scalar widths, one to three rounds."""
    print(f"dsfp d={d} rounds={rounds}", flush=True)
    X, _ = datagen.clustered(30, 10, d, 0.5, seed=d + rounds)
    k = 12 if d > 1 else 4
    idx = oracle_lists(X, k).astype(np.int32)
    Y = ctx.dsfp(dev(X), dev(idx, torch.int32), Params(k=k, gamma=0.2, rounds=rounds))
    Yo = O.dsfp(X, O.Params(k=k, gamma=0.2, rounds=rounds, normalize_input=False), idx)
    check_features(host(Y), Yo, what=f"dsfp d={d} T={rounds}")


def test_dsfp_zero_rounds_copies(ctx):
    X = np.random.default_rng(5).standard_normal((50, 32)).astype(np.float32)
    idx = oracle_lists(X, 4).astype(np.int32)
    Y = ctx.dsfp(dev(X), dev(idx, torch.int32), Params(k=4, rounds=0))
    assert np.array_equal(host(Y), X)


def test_dsfp_irregular_lists(ctx):
    """-1 padding, repeats, the node itself and out-of-range entries add
    nothing to the local set (the oracle sees the out-of-range entries as
    padding)."""
    print("dsfp irregular lists", flush=True)
    rng = np.random.default_rng(7)
    n, d, k = 300, 48, 10
    X = datagen.random_unit(n, d, seed=8)
    idx = np.stack([rng.choice(n, size=k, replace=False) for _ in range(n)]).astype(np.int32)
    idx[::3, 2] = -1
    idx[1::4, 4] = idx[1::4, 1]
    idx[::5, 0] = np.arange(0, n, 5)
    idx[2::7, 6] = n + 5
    idx[3::11, 9] = -7
    idx[10, :] = -1
    Y = ctx.dsfp(dev(X), dev(idx, torch.int32), Params(k=k, gamma=0.5, rounds=3))
    io = np.where(idx >= n, -1, idx)
    Yo = O.dsfp(X, O.Params(k=k, gamma=0.5, rounds=3, normalize_input=False), io)
    check_features(host(Y), Yo, what="irregular lists")
    np.testing.assert_allclose(host(Y)[10], X[10] / np.linalg.norm(X[10]), rtol=0, atol=1e-6)


def test_dsfp_deterministic(ctx):
    X, _ = datagen.clustered(50, 20, 256, 0.6, seed=9)
    idx = dev(oracle_lists(X, 20).astype(np.int32), torch.int32)
    p = Params(k=20, gamma=0.2, rounds=3)
    a = host(ctx.dsfp(dev(X), idx, p))
    b = host(ctx.dsfp(dev(X), idx, p))
    assert np.array_equal(a.view(np.uint32), b.view(np.uint32))


@pytest.mark.parametrize("prec", [FP32, BF16])
def test_rerank_local_matches_oracle(ctx, prec):
    """GCR_Local end to end (normalise, kNN once, DSFP, final distances and
    top-K) on the small image re-ID workload: 500 + 1,500 x 256, k = 20."""
    print(f"rerank_local prec={prec}", flush=True)
    w = datagen.plain_gcr_small()
    p = Params(k=20, gamma=0.1, rounds=2, precision=prec, topk_out=50)
    out = ctx.rerank_local(dev(w.X), w.nq, p, dense=True, topk=True, keep_features=True)
    Do, XTo = O.gcr_local(w.X, w.nq, O.Params(k=20, gamma=0.1, rounds=2))
    check_features(host(out["X"]), XTo, what="GCR_Local features")
    check_distances(host(out["dist"]), Do, what="GCR_Local distances")
    ti, td = host(out["topk_idx"]), host(out["topk_dist"])
    XL = host(out["X"]).astype(np.float64)
    q = np.arange(0, w.nq, 17)
    check_knn_rows(ti[q], td[q], XL, q, 50, cols=np.arange(w.nq, XL.shape[0]), exclude_self=False,
                   what="GCR_Local top-50")


def test_rerank_local_full_size(ctx):
    """3,368 + 15,913 x 2,048, k = 20, gamma = 0.2, T = 3, BF16 screening:
    sampled neighbour lists, sampled DSFP rows (each from the library's lists,
    which the sample checks) and sampled final distance rows."""
    print("rerank_local full size", flush=True)
    w = datagen.cross_camera_reid()
    n = w.X.shape[0]
    p = Params(k=20, gamma=0.2, rounds=3, precision=BF16)
    Xd = dev(w.X)
    out = ctx.rerank_local(Xd, w.nq, p, dense=True, keep_features=True)
    Xn = ctx.normalize_rows(Xd)
    Xh = host(Xn).astype(np.float64)
    idx, dist = ctx.knn(Xn, Params(k=20, precision=BF16))
    gi = host(idx)
    rows = np.sort(np.random.default_rng(12).choice(n, size=48, replace=False))
    check_knn_rows(gi[rows], host(dist)[rows], Xh, rows, 20)
    XL = host(out["X"])
    check_features(XL[rows], oracle_rows(Xh, gi, rows, 0.2, 3), what="DSFP rows")
    XL = XL.astype(np.float64)
    q = np.sort(np.random.default_rng(13).choice(w.nq, size=24, replace=False))
    G = XL[w.nq:]
    Do = np.maximum(np.sum(XL[q] ** 2, 1)[:, None] + np.sum(G ** 2, 1)[None, :] - 2.0 * XL[q] @ G.T, 0.0)
    check_distances(host(out["dist"])[q], Do, what="GCR_Local final distances")


def test_dsfp_errors(ctx):
    X = dev(datagen.random_unit(20, 16, seed=1))
    idx = dev(np.zeros((20, 60), np.int32), torch.int32)
    with pytest.raises(GcrError, match="UNSUPPORTED"):
        ctx.dsfp(X, idx, Params(k=60))
    with pytest.raises(GcrError, match="INVALID"):
        ctx.dsfp(X, idx[:, :4].contiguous(), Params(k=4, gamma=0.0))
    with pytest.raises(GcrError, match="INVALID"):
        ctx.dsfp(X, idx[:, :4].contiguous(), Params(k=4), out=X)
    with pytest.raises(GcrError, match="UNSUPPORTED"):
        ctx.rerank_local(X, 5, Params(k=60))


def test_dsfp_on_padded_library_lists(ctx):
    """Fewer rows than k + 1: the library's lists carry -1 padding, which adds
    nothing to the local sets (every node's local set is the whole set)."""
    print("dsfp padded lists", flush=True)
    X = datagen.random_unit(9, 40, seed=31)
    p = Params(k=12, gamma=0.4, rounds=2, precision=FP32)
    Xd = dev(X)
    idx, _ = ctx.knn(Xd, p)
    assert np.all(host(idx)[:, 8:] == -1)
    Y = ctx.dsfp(Xd, idx, p)
    Yo = O.dsfp(X, O.Params(k=12, gamma=0.4, rounds=2, normalize_input=False), host(idx))
    check_features(host(Y), Yo, what="padded lists")
    # every local set is the complete set: global GCR with a fixed graph
    ref = O.gcr(X, O.Params(k=8, gamma=0.4, rounds=2, rebuild_each_round=False))["X"][-1]
    check_features(host(Y), ref, what="complete local sets")


def test_rerank_local_single_query(ctx):
    print("rerank_local single query", flush=True)
    X, _ = datagen.clustered(20, 10, 96, 0.5, seed=32)
    p = Params(k=6, gamma=0.3, rounds=1, precision=BF16, topk_out=5)
    out = ctx.rerank_local(dev(X), 1, p, dense=True, topk=True, keep_features=True)
    Do, XTo = O.gcr_local(X, 1, O.Params(k=6, gamma=0.3, rounds=1))
    check_distances(host(out["dist"]), Do, what="single query")
    assert host(out["topk_idx"]).shape == (1, 5)
