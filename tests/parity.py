"""Comparison helpers between the GPU library and the FP64 oracle.

Tolerances (fixed by the method's parity criteria):
  * neighbour indices: equal sets, except that a member may differ when its
    exact distance is within TIE = 1e-6 of the k-th neighbour's;
  * features: ||x_gpu - x_oracle|| / ||x_oracle|| <= 1e-4 per row;
  * distances: |d_gpu - d_oracle| <= 1e-4 |d_oracle| + 1e-5.
"""
from __future__ import annotations

import numpy as np

from oracle import gcr_oracle as O

TIE = 1e-6
FEAT_RTOL = 1e-4
DIST_RTOL, DIST_ATOL = 1e-4, 1e-5


def check_knn_rows(idx_gpu, dist_gpu, X, rows, k, cam=None, cross=False, col_offset=0, cols=None,
                   exclude_self=True, tie=TIE, what="knn"):
    """Validate GPU neighbour lists of `rows` against exhaustive FP64 kNN.

    idx_gpu / dist_gpu: arrays [len(rows), k] (column indices relative to
    col_offset).  X: features (float32 values as float64).  cols: the
    candidate column range (default: all rows of X).
    Returns the number of rows whose set differs only inside the tie band.
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if cols is None:
        cols = np.arange(n)
    Xc = X[cols]
    nc = np.sum(Xc * Xc, axis=1)
    tie_rows = 0
    for t, i in enumerate(rows):
        i = int(i)
        dr = np.maximum(np.sum(X[i] * X[i]) + nc - 2.0 * (Xc @ X[i]), 0.0)
        ok = np.ones(len(cols), dtype=bool)
        if exclude_self:
            ok &= cols != i
        if cross:
            ok &= cam[cols] != cam[i]
        cand = np.nonzero(ok)[0]
        order = cand[np.argsort(dr[cand], kind="stable")]
        kk = min(k, len(order))
        ref = order[:kk]
        g = np.asarray(idx_gpu[t])
        gv = g[g >= 0]
        assert len(gv) == kk, f"{what}: row {i}: {len(gv)} valid neighbours, expected {kk}"
        assert np.all(g[kk:] == -1), f"{what}: row {i}: padding not -1"
        assert len(set(gv.tolist())) == kk, f"{what}: row {i}: duplicate neighbours"
        assert np.all(ok[gv]), f"{what}: row {i}: ineligible neighbour"
        if kk == 0:
            continue
        dk = dr[ref[-1]]
        gd = dr[gv]
        assert np.all(gd <= dk + tie), f"{what}: row {i}: neighbour beyond the k-th distance + tie"
        must = ref[dr[ref] < dk - tie]
        missing = set(must.tolist()) - set(gv.tolist())
        assert not missing, f"{what}: row {i}: missing neighbours {sorted(missing)[:5]}"
        assert np.all(np.diff(gd) >= -tie), f"{what}: row {i}: not ordered by distance"
        if set(gv.tolist()) != set(ref.tolist()):
            tie_rows += 1
        dg = np.asarray(dist_gpu[t])[:kk].astype(np.float64)
        np.testing.assert_allclose(dg, gd, rtol=2e-6, atol=1e-7, err_msg=f"{what}: row {i}: distances")
    return tie_rows


def check_features(Xg, Xo, rtol=FEAT_RTOL, what="features"):
    Xg = np.asarray(Xg, dtype=np.float64)
    Xo = np.asarray(Xo, dtype=np.float64)
    num = np.linalg.norm(Xg - Xo, axis=1)
    den = np.maximum(np.linalg.norm(Xo, axis=1), 1e-30)
    rel = num / den
    worst = int(np.argmax(rel))
    assert rel[worst] <= rtol, f"{what}: row {worst} relative error {rel[worst]:.3e} > {rtol}"
    return float(rel.max())


def check_distances(Dg, Do, what="distances"):
    Dg = np.asarray(Dg, dtype=np.float64)
    Do = np.asarray(Do, dtype=np.float64)
    err = np.abs(Dg - Do)
    lim = DIST_RTOL * np.abs(Do) + DIST_ATOL
    bad = err > lim
    if bad.any():
        q, g = np.argwhere(bad)[0]
        raise AssertionError(f"{what}: ({q},{g}) gpu {Dg[q, g]:.9g} oracle {Do[q, g]:.9g}; "
                             f"{int(bad.sum())} entries out of tolerance")
    return float((err / np.maximum(lim, 1e-30)).max())


def oracle_round_from_lists(X, p, idx, cr_idx=None, cam=None, X_graph=None):
    """Oracle one round driven by given (GPU) neighbour lists: distances are
    recomputed in FP64 for the listed pairs, from X_graph (the features the
    graph was built on; default X)."""
    X = np.asarray(X, dtype=np.float64)
    Xg = X if X_graph is None else np.asarray(X_graph, dtype=np.float64)
    n = X.shape[0]

    def dist_of(ix):
        ix = np.asarray(ix, dtype=np.int64)
        d = np.full(ix.shape, np.inf)
        ok = ix >= 0
        r = np.broadcast_to(np.arange(n)[:, None], ix.shape)[ok]
        c = ix[ok]
        d[ok] = np.maximum(np.sum((Xg[r] - Xg[c]) ** 2, axis=1), 0.0)
        return d

    dist = dist_of(idx)
    cdist = dist_of(cr_idx) if cr_idx is not None else None
    Y, Dg, Dc = O.sparse_round_from_lists(X, p, np.asarray(idx, np.int64), dist, cam,
                                          None if cr_idx is None else np.asarray(cr_idx, np.int64), cdist)
    return Y, Dg, Dc


def oracle_chain(X0, p, cam=None, rounds=None, tie=TIE):
    """The oracle's rounds at sizes where N x N does not fit: lists by the
    blocked exhaustive FP64 kNN (k + 1 per row, to see the gap at the cut),
    then one sparse FP64 round with exactly those nonzeros, the graph
    rebuilt from each round's features.  Returns per round t = 1..T the
    dict(idx, dist, cr_idx, cr_dist, X, ties) where `ties` are the rows whose
    k-th and (k+1)-th oracle distances are within `tie` (either list): rows
    whose neighbour sets are not unique within the parity tie band."""
    X = O.row_normalize(X0) if p.normalize_input else np.asarray(X0, np.float64)
    k = p.k
    kc = p.k if p.cross_k is None else p.cross_k
    use_cr = cam is not None and p.alpha < 1.0
    out = []
    for _ in range(p.rounds if rounds is None else rounds):
        gi, gd = O.knn_blocked(X, k + 1)
        ties = np.abs(gd[:, k] - gd[:, k - 1]) <= tie
        idx, dist = gi[:, :k], gd[:, :k]
        cidx = cdist = None
        if use_cr:
            ci, cd = O.knn_blocked(X, kc + 1, cam=cam, cross=True)
            ties |= np.abs(cd[:, kc] - cd[:, kc - 1]) <= tie
            cidx, cdist = ci[:, :kc], cd[:, :kc]
        Xn, _, _ = O.sparse_round_from_lists(X, p, idx, dist, cam, cidx, cdist)
        out.append(dict(idx=idx, dist=dist, cr_idx=cidx, cr_dist=cdist, X=Xn, ties=np.nonzero(ties)[0]))
        X = Xn
    return out


def expand_hops(rows, lists, hops):
    """rows plus every node within `hops` edges of them in the symmetric
    graph of the given forward lists (each an int array [n, k], -1 padded)."""
    n = lists[0].shape[0]
    adj_r, adj_c = [], []
    for ix in lists:
        ok = ix >= 0
        r = np.broadcast_to(np.arange(n)[:, None], ix.shape)[ok]
        adj_r += [r, ix[ok]]
        adj_c += [ix[ok], r]
    import scipy.sparse as sp
    A = sp.coo_matrix((np.ones(sum(len(a) for a in adj_r)), (np.concatenate(adj_r), np.concatenate(adj_c))),
                      shape=(n, n)).tocsr()
    mark = np.zeros(n, dtype=bool)
    mark[np.asarray(rows, dtype=np.int64)] = True
    for _ in range(hops):
        mark |= (A @ mark.astype(np.float64)) > 0
    return np.nonzero(mark)[0]


def closed_neighbourhood_round(X, ids, k, gamma, rows):
    """One oracle round at `rows` of a graph too large to build whole, made
    exact by closing the neighbourhood.  Every row's k-th distance is at most
    U = the largest, over all rows, k-th distance to the row's own identity
    group (any k other items bound it), so m lists j only if
    ||x_m - x_j||^2 <= U.  The lists of `rows`, of their neighbours and of
    every row within U of those are computed exactly (knn_blocked); rows
    outside that closure get empty lists, which changes no degree or value
    the round at `rows` reads.  Returns (X1[rows], exact lists of rows)."""
    n = X.shape[0]
    nr = np.sum(X * X, axis=1)
    U = 0.0
    for g in np.unique(ids):
        M = np.nonzero(ids == g)[0]
        if len(M) <= k:
            return None  # no bound from this group
        D = np.maximum(nr[M][:, None] + nr[M][None, :] - 2.0 * X[M] @ X[M].T, 0.0)
        np.fill_diagonal(D, np.inf)
        U = max(U, float(np.partition(D, k - 1, axis=1)[:, k - 1].max()))
    U += 1e-9

    def within_U(S):
        out = set()
        for a in range(0, len(S), 512):
            b = S[a:a + 512]
            D = nr[b][:, None] + nr[None, :] - 2.0 * (X[b] @ X.T)
            out.update(np.nonzero(D <= U)[1].tolist())
        return out

    lists = {}

    def ensure(S):
        S = np.array(sorted(set(S) - set(lists)), dtype=np.int64)
        if len(S):
            li, ld = O.knn_blocked(X, k, rows=S)
            for t, r in enumerate(S):
                lists[int(r)] = (li[t], ld[t])

    rows = np.asarray(rows, dtype=np.int64)
    ensure(within_U(rows) | set(rows.tolist()))
    S1 = set(rows.tolist())
    for r in rows:
        S1.update(int(j) for j in lists[int(r)][0] if j >= 0)
    S1.update(m for m in list(lists) if set(lists[m][0].tolist()) & set(rows.tolist()))
    ensure(within_U(np.array(sorted(S1))) | S1)
    idx = np.full((n, k), -1, dtype=np.int64)
    dist = np.full((n, k), np.inf)
    for m, (li, ld) in lists.items():
        idx[m], dist[m] = li, ld
    Y, _, _ = O.sparse_round_from_lists(X, O.Params(k=k, gamma=gamma, rounds=1), idx, dist, rows=rows)
    return Y, idx, sorted(lists)


def chain_compare(ctx, w, p, op, cam_d, what, dense_last=True):
    """GPU features of every round t = 1..T (each a whole re-ranking with t
    rounds, its last graph kept) against the oracle chain.  Where the
    library's neighbour set of a row differs from the oracle's, the row must
    sit in the oracle's tie band (or next to a row already set aside), and
    the rows within two hops of it are set aside from then on: a legitimate
    tie choice changes the weights there.  Every other row is compared.
    Returns (oracle chain, rows compared at round T, last GPU output)."""
    import torch

    def host(t):
        torch.cuda.synchronize()
        return t.cpu().numpy()

    n = w.X.shape[0]
    cross = cam_d is not None and op.alpha < 1.0
    chain = oracle_chain(w.X, op, w.cams if cam_d is not None else None)
    excl = np.zeros(0, dtype=np.int64)
    Xd = torch.from_numpy(np.ascontiguousarray(w.X)).to("cuda", torch.float32)
    out = None
    for t in range(1, op.rounds + 1):
        pt = type(p)(**{**p.__dict__, "rounds": t})
        g = ctx.new_graph(n, pt, has_cross=cross)
        out = ctx.rerank(Xd, w.nq, pt, cam_d, dense=dense_last and t == op.rounds, keep_features=True,
                         last_graph=g)
        ch = chain[t - 1]
        gi = host(g.field("idx"))
        diff = np.array([r for r in range(n) if set(gi[r].tolist()) != set(ch["idx"][r].tolist())], dtype=np.int64)
        lists = [ch["idx"]]
        if cross:
            gc = host(g.field("cr_idx"))
            dc = [r for r in range(n) if set(gc[r].tolist()) != set(ch["cr_idx"][r].tolist())]
            diff = np.union1d(diff, np.array(dc, dtype=np.int64))
            lists.append(ch["cr_idx"])
        allowed = np.union1d(ch["ties"], expand_hops(excl, lists, 1) if len(excl) else excl)
        stray = np.setdiff1d(diff, allowed)
        assert len(stray) == 0, f"{what} round {t}: lists differ outside the tie band at rows {stray[:8]}"
        excl = expand_hops(np.union1d(excl, diff), lists, 2) if len(diff) or len(excl) else excl
        assert len(excl) <= 0.02 * n, f"{what}: {len(excl)} rows set aside by round {t}"
        keep = np.setdiff1d(np.arange(n), excl)
        check_features(host(out["X"])[keep], ch["X"][keep], what=f"{what} round {t}")
        print(f"{what}: round {t}: {len(diff)} tie-band list differences, features equal on {len(keep)} of {n}",
              flush=True)
    return chain, np.setdiff1d(np.arange(n), excl), out
