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
