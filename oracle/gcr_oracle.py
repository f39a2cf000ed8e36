"""FP64 CPU oracle for Graph Convolution based Re-ranking (GCR / GCRV).

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow, obviously correct
statement of what the re-ranking computes.  It exists so that tests, the smoke
check and the benchmark's CPU baseline can compare the GPU library against it.
The product path never imports, calls or falls back to anything here.

Everything runs in float64 NumPy on the canonical float32 inputs (upcast is
exact).  Where the method reaches a result that has a plain definition, that
definition is written out directly: a full N x N distance matrix, a full
stable sort of every row, dense N x N affinity and propagation matrices.

Paper references (Graph Convolution Based Efficient Re-Ranking for Visual
Retrieval, Sec. III):
  * Eq. (2)  parameter-free propagation  X~ = D^-1/2 A D^-1/2 X
  * Eq. (3)  iteration  X_t = G(X_{t-1}),  t = 1..T
  * Eq. (4)  kNN affinity  A~_ij = exp(-||x_i - x_j||^2 / gamma) for j in N_i,
             1 on the diagonal, 0 elsewhere
  * Eq. (5)  row / column degrees
  * Eq. (6)  asymmetric propagation  D_r^-1/2 A~ D_c^-1/2 X
  * Eq. (7)  symmetrisation  A = (A~ + A~^T) / 2
  * Eq. (8)  cross-camera kNN affinity (neighbours restricted to other cameras)
  * Eq. (9)  blend  alpha P X + (1 - alpha) P^cr X (symmetric form)
  * Sec. III-C text: the neighbour graphs change between iterations, so the
    graph is rebuilt from the current features before every round
  * Eq. (10) mean tracklet profile; Eq. (16) profile vector closed form
  * Alg. 1   DSFP ("GCR_Local"): per node, a dense local affinity over the
             node and its k neighbours, local degrees, T local rounds
  * Alg. 2   GCRV: profile vectors, then T rounds on the profile vectors
  * Sec. IV-F (experimental analysis, efficiency): gallery graphs may be
    computed in advance (used by the serving reading)

Readings where the paper is silent or ambiguous (each is implemented here and
listed with its reason in the design notes):
  * distances are squared Euclidean, as in Eq. (4);
  * N_i excludes i itself; the diagonal weight is 1 (Eq. (4) third case);
  * neighbours are ordered by (distance, index) ascending; a row with fewer
    than k eligible nodes takes all of them;
  * every propagation round ends with a row re-normalisation
    x <- y / max(||y||, 1e-12); the paper's derivations assume unit rows;
  * a cross-camera list and the alpha blend are used only when camera labels
    are given and alpha < 1; the global list includes all cameras;
  * optional per-edge camera factor beta(cam_i, cam_j) multiplies the global
    graph's off-diagonal weights (1.0 unless asked otherwise);
  * Eq. (16) is used as printed with X^T X (d x d, the covariance the text
    names) in place of the garbled X X^T, per camera group;
  * final ranking distances are squared Euclidean on X_T only;
  * DSFP (Alg. 1): the local degree is the row sum of A^i for every member
    of the local set (the printed degree names only node i's own entry);
    A^i covers all pairs of the local set with 1 on its diagonal; the local
    rounds run t = 1..T and each ends with the same row re-normalisation as
    a global round; node i's row of the local X_T is its output; the kNN
    lists come once from the (normalised) input features and are not
    rebuilt; cameras and the blend of Eq. (9) do not apply.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Params",
    "row_normalize",
    "sq_dists",
    "knn_lists",
    "affinity_dense",
    "sym_propagation_matrix",
    "asym_propagation_matrix",
    "propagation_round",
    "gcr",
    "final_distances",
    "profile_vectors",
    "sparse_round_from_lists",
    "degrees_from_lists",
    "knn_rows",
    "knn_blocked",
    "serve_request",
    "local_set",
    "dsfp",
    "gcr_local",
]

NORM_FLOOR = 1e-12


@dataclasses.dataclass
class Params:
    """Hyper-parameters.  Paper defaults: gamma 0.2, k 15, T 3, lambda 10
    (Sec. IV-B) and alpha 0.7 (Sec. IV-F, ablation study)."""

    k: int = 15
    gamma: float = 0.2
    rounds: int = 3
    alpha: float = 1.0
    beta_same: float = 1.0
    beta_cross: float = 1.0
    rebuild_each_round: bool = True
    normalize_input: bool = True
    symmetric: bool = True
    cross_k: Optional[int] = None  # defaults to k
    lam: float = 10.0


# ----------------------------------------------------------------------------
# elementary steps


def row_normalize(X: np.ndarray) -> np.ndarray:
    """x_i / max(||x_i||, 1e-12); zero rows stay zero."""
    X = np.asarray(X, dtype=np.float64)
    nrm = np.sqrt(np.sum(X * X, axis=1))
    return X / np.maximum(nrm, NORM_FLOOR)[:, None]


def sq_dists(X: np.ndarray, rows: Optional[np.ndarray] = None) -> np.ndarray:
    """Squared Euclidean distances ||x_i - x_j||^2 (Eq. (4) exponent).

    Returns the [len(rows), N] block (all rows if ``rows`` is None).  Uses
    ||x_i||^2 + ||x_j||^2 - 2 x_i.x_j in float64, clamped at 0, with the
    exact zero on the diagonal.
    """
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    if rows is None:
        rows = np.arange(n)
    rows = np.asarray(rows)
    nr = np.sum(X * X, axis=1)
    G = X[rows] @ X.T
    Dm = nr[rows][:, None] + nr[None, :] - 2.0 * G
    np.maximum(Dm, 0.0, out=Dm)
    Dm[np.arange(len(rows)), rows] = 0.0
    return Dm


def knn_rows(Drow_block: np.ndarray, rows: np.ndarray, k: int,
             cam: Optional[np.ndarray] = None, cross: bool = False):
    """k nearest neighbours of each listed row, from its distance row.

    N_i = the first min(k, |C_i|) members of C_i = {j != i} (and, for the
    cross-camera list of Eq. (8), cam_j != cam_i), ordered by (distance,
    index) ascending via a full stable sort.  Missing slots hold index -1
    and distance +inf.
    """
    nr, n = Drow_block.shape
    idx = np.full((nr, k), -1, dtype=np.int64)
    dist = np.full((nr, k), np.inf, dtype=np.float64)
    allj = np.arange(n)
    for t in range(nr):
        i = int(rows[t])
        ok = allj != i
        if cross:
            ok &= cam != cam[i]
        cand = allj[ok]  # ascending index order
        order = np.argsort(Drow_block[t, cand], kind="stable")
        take = cand[order[:k]]
        idx[t, : len(take)] = take
        dist[t, : len(take)] = Drow_block[t, take]
    return idx, dist


def knn_blocked(X: np.ndarray, k: int, rows: Optional[np.ndarray] = None,
                cam: Optional[np.ndarray] = None, cross: bool = False,
                block: int = 1024, threads: int = 0):
    """The same lists as knn_rows (first min(k, |C_i|) of C_i by (distance,
    index)) for inputs where the N x N matrix does not fit: distance rows
    are formed a block at a time (the sq_dists arithmetic), the k-th smallest
    eligible distance is found by a partition, every eligible item at or
    below it is kept (so ties at the cut are all present) and those are
    stably sorted by distance, index order breaking ties.  Blocks run on a
    thread pool (NumPy's BLAS and partition release the interpreter lock).
    Returns (idx int64 [len(rows), k], dist float64), -1 / +inf padded."""
    from concurrent.futures import ThreadPoolExecutor
    import os

    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    rows = np.arange(n) if rows is None else np.asarray(rows)
    nr_all = np.sum(X * X, axis=1)
    idx = np.full((len(rows), k), -1, dtype=np.int64)
    dist = np.full((len(rows), k), np.inf, dtype=np.float64)

    def one_block(a):
        r = rows[a:a + block]
        D = nr_all[r][:, None] + nr_all[None, :] - 2.0 * (X[r] @ X.T)
        np.maximum(D, 0.0, out=D)
        D[np.arange(len(r)), r] = 0.0
        # ineligible entries (the row itself, same-camera items for Eq. (8))
        D[np.arange(len(r)), r] = np.inf
        if cross:
            D[cam[r][:, None] == cam[None, :]] = np.inf
        m = min(k, n - 1)
        if m <= 0:
            return
        kth = np.partition(D, m - 1, axis=1)[:, m - 1]
        for t in range(len(r)):
            cand = np.nonzero(D[t] <= kth[t])[0]  # ascending index order
            cand = cand[np.isfinite(D[t, cand])]
            order = np.argsort(D[t, cand], kind="stable")
            take = cand[order[:k]]
            idx[a + t, :len(take)] = take
            dist[a + t, :len(take)] = D[t, take]

    # each block's distance rows stay within 256 MB
    block = max(16, min(block, (1 << 28) // (8 * max(n, 1))))
    nt = threads or max(1, min(16, len(os.sched_getaffinity(0))))
    with ThreadPoolExecutor(nt) as ex:
        list(ex.map(one_block, range(0, len(rows), block)))
    return idx, dist


def knn_lists(Dm: np.ndarray, k: int, cam: Optional[np.ndarray] = None,
              cross: bool = False):
    """kNN lists for every row of a full distance matrix (see knn_rows)."""
    n = Dm.shape[0]
    return knn_rows(Dm, np.arange(n), k, cam, cross)


def affinity_dense(n: int, idx: np.ndarray, dist: np.ndarray, gamma: float,
                   edge_scale: Optional[np.ndarray] = None) -> np.ndarray:
    """A~ of Eq. (4) / Eq. (8): 1 on the diagonal, exp(-d/gamma) (times an
    optional per-edge factor) at (i, j) for j in N_i, 0 elsewhere."""
    At = np.zeros((n, n), dtype=np.float64)
    for i in range(n):
        for s in range(idx.shape[1]):
            j = int(idx[i, s])
            if j < 0:
                continue
            w = math.exp(-float(dist[i, s]) / gamma)
            if edge_scale is not None:
                w *= float(edge_scale[i, s])
            At[i, j] = w
        At[i, i] = 1.0
    return At


def sym_propagation_matrix(At: np.ndarray):
    """Eq. (7) then Eq. (2): A = (A~ + A~^T)/2, D_ii = sum_j A_ij,
    P = D^-1/2 A D^-1/2.  Returns (P, A, D)."""
    A = 0.5 * (At + At.T)
    Dg = A.sum(axis=1)
    s = 1.0 / np.sqrt(Dg)
    P = s[:, None] * A * s[None, :]
    return P, A, Dg


def asym_propagation_matrix(At: np.ndarray):
    """Eq. (5) and Eq. (6): D_r = row sums, D_c = column sums of A~,
    P = D_r^-1/2 A~ D_c^-1/2.  Returns (P, D_r, D_c)."""
    Dr = At.sum(axis=1)
    Dc = At.sum(axis=0)
    P = (1.0 / np.sqrt(Dr))[:, None] * At * (1.0 / np.sqrt(Dc))[None, :]
    return P, Dr, Dc


def _edge_scale(idx: np.ndarray, cam: Optional[np.ndarray], p: Params):
    if cam is None or (p.beta_same == 1.0 and p.beta_cross == 1.0):
        return None
    n, k = idx.shape
    sc = np.ones((n, k), dtype=np.float64)
    for i in range(n):
        for s in range(k):
            j = int(idx[i, s])
            if j >= 0:
                sc[i, s] = p.beta_same if cam[j] == cam[i] else p.beta_cross
    return sc


def _uses_cross(cam, p: Params) -> bool:
    return cam is not None and p.alpha < 1.0


def build_graphs(X: np.ndarray, p: Params, cam: Optional[np.ndarray] = None):
    """kNN lists, affinities and propagation matrices of one round
    (Eq. (4)-(8)).  Returns a dict of dense float64 matrices and lists."""
    n = X.shape[0]
    Dm = sq_dists(X)
    idx, dist = knn_lists(Dm, p.k)
    At = affinity_dense(n, idx, dist, p.gamma, _edge_scale(idx, cam, p))
    out = dict(dist_matrix=Dm, idx=idx, dist=dist, At=At)
    if p.symmetric:
        P, A, Dg = sym_propagation_matrix(At)
        out.update(P=P, A=A, deg=Dg)
    else:
        P, Dr, Dc = asym_propagation_matrix(At)
        out.update(P=P, deg_r=Dr, deg_c=Dc)
    if _uses_cross(cam, p):
        kc = p.k if p.cross_k is None else p.cross_k
        cidx, cdist = knn_lists(Dm, kc, cam, cross=True)
        Atc = affinity_dense(n, cidx, cdist, p.gamma)
        if p.symmetric:
            Pc, Ac, Dc_ = sym_propagation_matrix(Atc)
            out.update(cr_P=Pc, cr_A=Ac, cr_deg=Dc_)
        else:
            Pc, Drc, Dcc = asym_propagation_matrix(Atc)
            out.update(cr_P=Pc, cr_deg_r=Drc, cr_deg_c=Dcc)
        out.update(cr_idx=cidx, cr_dist=cdist, cr_At=Atc)
    return out


def propagation_round(X: np.ndarray, graphs: dict, p: Params,
                      cam: Optional[np.ndarray] = None) -> np.ndarray:
    """One round: Y = alpha P X + (1 - alpha) P^cr X (Eq. (2) / Eq. (9)),
    then x_i <- y_i / max(||y_i||, 1e-12)."""
    Y = graphs["P"] @ X
    if _uses_cross(cam, p):
        Y = p.alpha * Y + (1.0 - p.alpha) * (graphs["cr_P"] @ X)
    return row_normalize(Y)


def gcr(X0: np.ndarray, p: Params, cam: Optional[np.ndarray] = None,
        keep_graphs: bool = True) -> dict:
    """Plain or cross-camera GCR on the stacked features X0 (queries first).

    Eq. (3): X_t = G(X_{t-1}) for t = 1..T.  With rebuild_each_round the
    kNN graph and affinities are recomputed from X_{t-1} before each round
    (Sec. III-C, Alg. 2); otherwise the graph of X_0 is reused.
    Returns {"X": [X_0, ..., X_T], "graphs": [per-round dicts]}.
    """
    X = np.asarray(X0, dtype=np.float64)
    if p.normalize_input:
        X = row_normalize(X)
    xs = [X]
    graphs = []
    g = None
    for t in range(p.rounds):
        if g is None or p.rebuild_each_round:
            g = build_graphs(X, p, cam)
        X = propagation_round(X, g, p, cam)
        xs.append(X)
        if keep_graphs:
            graphs.append(g)
    return dict(X=xs, graphs=graphs)


def final_distances(X: np.ndarray, nq: int) -> np.ndarray:
    """Re-ranked distances ||x_q - x_g||^2 between the nq query rows and the
    gallery rows of the final features (the ranking is read off the
    updated features, Sec. III-A)."""
    X = np.asarray(X, dtype=np.float64)
    return sq_dists(X, np.arange(nq))[:, nq:]


# ----------------------------------------------------------------------------
# sparse evaluation of one round from given kNN lists (same nonzeros as the
# dense matrices above; used where N x N does not fit)


def degrees_from_lists(n: int, idx: np.ndarray, w: np.ndarray) -> np.ndarray:
    """D_i of A = (A~ + A~^T)/2 from forward lists: 1 + half the forward
    weights of row i + half the weights of edges j -> i."""
    Dg = np.ones(n, dtype=np.float64)
    ok = idx >= 0
    rows = np.broadcast_to(np.arange(n)[:, None], idx.shape)[ok]
    np.add.at(Dg, rows, 0.5 * w[ok])
    np.add.at(Dg, idx[ok], 0.5 * w[ok])
    return Dg


def _sparse_sym_P(n, idx, dist, gamma, edge_scale=None):
    import scipy.sparse as sp

    ok = idx >= 0
    rr = np.broadcast_to(np.arange(n)[:, None], idx.shape)[ok]
    cc = idx[ok]
    vv = np.exp(-np.asarray(dist, dtype=np.float64)[ok] / gamma)
    if edge_scale is not None:
        vv = vv * edge_scale[ok]
    # duplicate (i, j) pairs cannot occur: a list holds distinct j
    At = sp.coo_matrix((vv, (rr, cc)), shape=(n, n)).tocsr()
    At = At + sp.identity(n, format="csr")
    A = 0.5 * (At + At.T)
    Dg = np.asarray(A.sum(axis=1)).ravel()
    s = sp.diags(1.0 / np.sqrt(Dg))
    return (s @ A @ s).tocsr(), Dg


def sparse_round_from_lists(X: np.ndarray, p: Params, idx: np.ndarray,
                            dist: np.ndarray, cam: Optional[np.ndarray] = None,
                            cr_idx: Optional[np.ndarray] = None,
                            cr_dist: Optional[np.ndarray] = None,
                            rows: Optional[np.ndarray] = None):
    """One symmetric propagation round from given neighbour lists, with
    scipy.sparse float64 matrices that have exactly the nonzeros of the
    dense A of Eq. (7).  Returns (X_next rows, D, D_cr)."""
    X = np.asarray(X, dtype=np.float64)
    n = X.shape[0]
    P, Dg = _sparse_sym_P(n, idx, dist, p.gamma, _edge_scale(idx, cam, p))
    Pr = P if rows is None else P[rows]
    Y = Pr @ X
    Dc = None
    if _uses_cross(cam, p):
        Pc, Dc = _sparse_sym_P(n, cr_idx, cr_dist, p.gamma)
        Pcr = Pc if rows is None else Pc[rows]
        Y = p.alpha * Y + (1.0 - p.alpha) * (Pcr @ X)
    return row_normalize(Y), Dg, Dc


# ----------------------------------------------------------------------------
# video: profile vectors


def profile_vectors(frames: np.ndarray, offsets: np.ndarray,
                    groups: Optional[np.ndarray] = None, lam: float = 10.0,
                    mode: str = "pvg", normalize: bool = True) -> np.ndarray:
    """Tracklet profile vectors.

    mode "mean": Eq. (10), w_c = mean of tracklet c's frames.
    mode "pvg":  Eq. (16) within each camera group g:
        F = the group's frames (n of them), mu = mean(F),
        M = F^T F + lambda n I  (d x d),
        w_c = M^-1 (mu_c - mu)  for every tracklet c of the group.
    Each w_c is then L2-normalised (if ``normalize``).
    """
    frames = np.asarray(frames, dtype=np.float64)
    offsets = np.asarray(offsets, dtype=np.int64)
    nt = len(offsets) - 1
    d = frames.shape[1]
    if groups is None:
        groups = np.zeros(nt, dtype=np.int64)
    groups = np.asarray(groups)
    W = np.zeros((nt, d), dtype=np.float64)
    mu_c = np.zeros((nt, d), dtype=np.float64)
    for c in range(nt):
        a, b = int(offsets[c]), int(offsets[c + 1])
        mu_c[c] = frames[a:b].mean(axis=0)
    if mode == "mean":
        W = mu_c
    elif mode == "pvg":
        for g in np.unique(groups):
            members = np.nonzero(groups == g)[0]
            rows = np.concatenate([np.arange(offsets[c], offsets[c + 1]) for c in members])
            F = frames[rows]
            n = F.shape[0]
            mu = F.mean(axis=0)
            M = F.T @ F + lam * n * np.eye(d)
            B = (mu_c[members] - mu[None, :]).T  # d x m
            W[members] = np.linalg.solve(M, B).T
    else:
        raise ValueError(mode)
    return row_normalize(W) if normalize else W


def gcrv(frames, offsets, groups, nq: int, p: Params, mode: str = "pvg",
         cam: Optional[np.ndarray] = None) -> dict:
    """Alg. 2: profile vectors of all tracklets (queries first), then GCR
    rounds on the profile vectors.  Returns the gcr() dict plus "W"."""
    W = profile_vectors(frames, offsets, groups, p.lam, mode)
    out = gcr(W, p, cam)
    out["W"] = W
    return out


# ----------------------------------------------------------------------------
# serving reading: precomputed gallery graph, queries attached to it


def serve_request(XG0: np.ndarray, g_idx: np.ndarray, g_dist: np.ndarray,
                  Q: np.ndarray, p: Params, topk: int):
    """One request against a resident gallery (precomputed graphs, Sec.
    IV-F, efficiency analysis).

    Node set = gallery then the request's queries.  Gallery rows keep their
    precomputed kNN lists (built on the gallery alone, frozen); query rows
    take their k nearest gallery items.  The symmetric normalisation, the
    rounds (fixed graph) and the renormalisation are those of gcr().
    Returns (top-k gallery indices [b, topk], their distances).
    """
    XG0 = np.asarray(XG0, dtype=np.float64)
    Q = row_normalize(np.asarray(Q, dtype=np.float64)) if p.normalize_input else np.asarray(Q, np.float64)
    ng = XG0.shape[0]
    b = Q.shape[0]
    X = np.concatenate([XG0, Q], axis=0)
    # query rows: exhaustive kNN over the gallery only
    nr = np.sum(XG0 * XG0, axis=1)
    qn = np.sum(Q * Q, axis=1)
    Dq = np.maximum(qn[:, None] + nr[None, :] - 2.0 * (Q @ XG0.T), 0.0)
    q_idx = np.full((b, p.k), -1, dtype=np.int64)
    q_dist = np.full((b, p.k), np.inf)
    for t in range(b):
        order = np.argsort(Dq[t], kind="stable")[: p.k]  # all of them if the gallery is smaller than k
        q_idx[t, : len(order)] = order
        q_dist[t, : len(order)] = Dq[t, order]
    idx = np.concatenate([g_idx, q_idx], axis=0)
    dist = np.concatenate([g_dist, q_dist], axis=0)
    for _ in range(p.rounds):
        X, _, _ = sparse_round_from_lists(X, p, idx, dist)
    Xq, Xg = X[ng:], X[:ng]
    dfin = np.maximum(np.sum(Xq * Xq, 1)[:, None] + np.sum(Xg * Xg, 1)[None, :] - 2.0 * (Xq @ Xg.T), 0.0)
    order = np.argsort(dfin, axis=1, kind="stable")[:, :topk]
    return order, np.take_along_axis(dfin, order, axis=1)


# ----------------------------------------------------------------------------
# Alg. 1: decentralised and synchronous feature propagation (DSFP, GCR_Local)


def local_set(i: int, idx_row) -> list:
    """The local node set N_i plus i itself (Alg. 1, first two steps), node i
    first and then the listed neighbours in list order.  Padding (-1), i
    itself and repeated entries add nothing: the set is a set."""
    nodes = [int(i)]
    for j in np.asarray(idx_row).tolist():
        if j >= 0 and j not in nodes:
            nodes.append(int(j))
    return nodes


def dsfp_node(X: np.ndarray, nodes: list, gamma: float, rounds: int) -> np.ndarray:
    """Alg. 1 for one node (nodes[0]): local affinity A over every pair of the
    local set (exp(-||x_u - x_v||^2 / gamma), 1 on the diagonal), local
    degrees D = row sums of A, then T rounds X <- D^-1/2 A D^-1/2 X, each
    followed by the row re-normalisation of a global round.  Returns the
    node's own row of the local X_T."""
    Xl = np.asarray(X, dtype=np.float64)[nodes]
    A = np.exp(-sq_dists(Xl) / gamma)
    deg = A.sum(axis=1)
    P = A / np.sqrt(deg)[:, None] / np.sqrt(deg)[None, :]
    for _ in range(rounds):
        Xl = row_normalize(P @ Xl)
    return Xl[0]


def dsfp(X0: np.ndarray, p: Params, idx: Optional[np.ndarray] = None) -> np.ndarray:
    """DSFP over all nodes (Alg. 1).  X0: input features (normalised first if
    p.normalize_input).  idx: neighbour lists [n, k] (-1 padding allowed);
    default: the exact k nearest other rows of the normalised input.
    Every node is updated from the input features only (the rounds are
    local and synchronous), so nodes are independent."""
    X = np.asarray(X0, dtype=np.float64)
    if p.normalize_input:
        X = row_normalize(X)
    n = X.shape[0]
    if idx is None:
        idx, _ = knn_lists(sq_dists(X), p.k)
    out = np.empty_like(X)
    for i in range(n):
        out[i] = dsfp_node(X, local_set(i, idx[i]), p.gamma, p.rounds)
    return out


def gcr_local(X0: np.ndarray, nq: int, p: Params, idx: Optional[np.ndarray] = None):
    """GCR_Local re-ranking: DSFP features, then the squared distances between
    the first nq rows (queries) and the rest (gallery).  Returns (dist
    [nq, ng], X_T)."""
    XT = dsfp(X0, p, idx)
    return final_distances(XT, nq), XT
