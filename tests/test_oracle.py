"""Pins for the FP64 oracle: hand-derived worked examples, brute force on tiny
inputs, closed forms and invariants of the method.  None of the expected
values here comes from the oracle itself or from the GPU library.
"""
import itertools
import math

import numpy as np
import pytest

from oracle import gcr_oracle as O
from oracle.metrics import mean_average_precision
from paper_2306_08792_amd import datagen

E = math.exp


def unit_at(deg):
    r = math.radians(deg)
    return (math.cos(r), math.sin(r))


def d_angle(a, b):
    """||u(a) - u(b)||^2 = 2 - 2 cos(a - b) for unit vectors at angles a, b."""
    return 2.0 - 2.0 * math.cos(math.radians(a - b))


# ---------------------------------------------------------------------------
# worked example: four unit vectors in the plane at 0, 60, 90, 200 degrees,
# k = 2, gamma = 1.  Every expected number below is derived by hand from the
# definitions (Eq. (4), (7), (5), (2)) for this instance.

ANG = [0.0, 60.0, 90.0, 200.0]


@pytest.fixture(scope="module")
def wx():
    return np.array([unit_at(a) for a in ANG])


def _hand_graph():
    d01, d02, d03 = d_angle(0, 60), d_angle(0, 90), d_angle(0, 200)
    d12, d13, d23 = d_angle(60, 90), d_angle(60, 200), d_angle(90, 200)
    assert abs(d01 - 1.0) < 1e-15 and abs(d12 - (2 - math.sqrt(3))) < 1e-15
    # kNN (k = 2) read off the distances:
    #   row 0: d01=1 < d02=2 < d03   -> {1, 2}
    #   row 1: d12 < d01 < d13       -> {2, 0}
    #   row 2: d12 < d02 < d23       -> {1, 0}
    #   row 3: d23 < d13 < d03       -> {2, 1}
    knn = [[1, 2], [2, 0], [1, 0], [2, 1]]
    # symmetric A: mutual pairs (0,1), (0,2), (1,2) keep exp(-d); the
    # one-sided edges 3->1, 3->2 carry half their weight
    A = np.zeros((4, 4))
    A[0, 1] = A[1, 0] = E(-d01)
    A[0, 2] = A[2, 0] = E(-d02)
    A[1, 2] = A[2, 1] = E(-d12)
    A[1, 3] = A[3, 1] = 0.5 * E(-d13)
    A[2, 3] = A[3, 2] = 0.5 * E(-d23)
    for i in range(4):
        A[i, i] = 1.0
    D = [1 + E(-d01) + E(-d02),
         1 + E(-d01) + E(-d12) + 0.5 * E(-d13),
         1 + E(-d02) + E(-d12) + 0.5 * E(-d23),
         1 + 0.5 * E(-d13) + 0.5 * E(-d23)]
    return knn, A, D, (d01, d02, d03, d12, d13, d23)


def _hand_round(X, A, D):
    """y_i = sum_j A_ij x_j / sqrt(D_i D_j), then y_i / ||y_i||, entry by entry."""
    out = []
    for i in range(4):
        y0 = y1 = 0.0
        for j in range(4):
            c = A[i][j] / math.sqrt(D[i] * D[j])
            y0 += c * X[j][0]
            y1 += c * X[j][1]
        nrm = math.hypot(y0, y1)
        out.append((y0 / nrm, y1 / nrm))
    return out


def test_worked_example_graph(wx):
    knn, A, D, _ = _hand_graph()
    p = O.Params(k=2, gamma=1.0, rounds=1, alpha=1.0)
    g = O.build_graphs(wx, p)
    assert g["idx"].tolist() == knn
    np.testing.assert_allclose(g["A"], A, rtol=0, atol=1e-14)
    np.testing.assert_allclose(g["deg"], D, rtol=1e-14)
    # P row 0 and P_33 (Eq. (2)): A_0j / sqrt(D_0 D_j), 1 / D_3
    P0 = [A[0][j] / math.sqrt(D[0] * D[j]) for j in range(4)]
    np.testing.assert_allclose(g["P"][0], P0, rtol=1e-13, atol=1e-15)
    assert abs(g["P"][3, 3] - 1.0 / D[3]) < 1e-14
    # independently spelled-out numbers for the first row of P
    np.testing.assert_allclose(g["P"][0, :3], [0.6652409558, 0.2047546071, 0.0793641824], atol=1e-9)


def test_worked_example_rounds_fixed_and_rebuilt(wx):
    knn, A, D, dd = _hand_graph()
    X0 = [tuple(r) for r in wx]
    X1 = _hand_round(X0, A, D)
    X2_fixed = _hand_round(X1, A, D)
    p = O.Params(k=2, gamma=1.0, rounds=2, alpha=1.0, rebuild_each_round=False)
    out = O.gcr(wx, p)
    np.testing.assert_allclose(out["X"][1], X1, atol=1e-13)
    np.testing.assert_allclose(out["X"][2], X2_fixed, atol=1e-13)
    # rebuilt graph: kNN lists of X1 are the same sets here, weights change
    ang1 = [math.degrees(math.atan2(y, x)) for x, y in X1]
    D1 = {(i, j): d_angle(ang1[i], ang1[j]) for i in range(4) for j in range(4)}
    for i, nb in enumerate(knn):
        others = sorted((D1[i, j], j) for j in range(4) if j != i)
        assert [j for _, j in others[:2]] == nb
    A1 = np.zeros((4, 4))
    for i, nb in enumerate(knn):
        for j in nb:
            A1[i, j] += 0.5 * E(-D1[i, j])
            A1[j, i] += 0.5 * E(-D1[i, j])
        A1[i, i] = 1.0
    Dg1 = A1.sum(axis=1)
    X2_rebuilt = _hand_round(X1, A1, Dg1)
    pr = O.Params(k=2, gamma=1.0, rounds=2, alpha=1.0, rebuild_each_round=True)
    outr = O.gcr(wx, pr)
    np.testing.assert_allclose(outr["X"][2], X2_rebuilt, atol=1e-13)
    # final distances, queries {0, 3} vs gallery {1, 2} (rows reordered so
    # that the queries come first)
    for X2 in (X2_fixed, X2_rebuilt):
        Xo = np.array([X2[0], X2[3], X2[1], X2[2]])
        dq = O.final_distances(Xo, 2)
        for a, qi in enumerate((0, 3)):
            for b, gi in enumerate((1, 2)):
                ref = (X2[qi][0] - X2[gi][0]) ** 2 + (X2[qi][1] - X2[gi][1]) ** 2
                assert abs(dq[a, b] - ref) < 1e-13


def test_worked_example_cross_camera(wx):
    _, A, D, (d01, d02, d03, d12, d13, d23) = _hand_graph()
    cam = np.array([0, 0, 1, 1])
    # cross-camera lists with k = 1: 0 -> 2, 1 -> 2, 2 -> 1, 3 -> 1
    Ac = np.eye(4)
    Ac[0, 2] = Ac[2, 0] = 0.5 * E(-d02)
    Ac[1, 2] = Ac[2, 1] = E(-d12)  # mutual
    Ac[1, 3] = Ac[3, 1] = 0.5 * E(-d13)
    Dc = Ac.sum(axis=1)
    p = O.Params(k=2, gamma=1.0, rounds=1, alpha=0.7, cross_k=1)
    g = O.build_graphs(wx, p, cam)
    assert g["cr_idx"].ravel().tolist() == [2, 2, 1, 1]
    Pc1 = [Ac[1, j] / math.sqrt(Dc[1] * Dc[j]) for j in range(4)]
    np.testing.assert_allclose(g["cr_P"][1], Pc1, atol=1e-14)
    # Eq. (9), row 0: 0.7 * P x + 0.3 * P^cr x, renormalised
    y = np.zeros(2)
    for j in range(4):
        y += 0.7 * A[0][j] / math.sqrt(D[0] * D[j]) * wx[j]
        y += 0.3 * Ac[0, j] / math.sqrt(Dc[0] * Dc[j]) * wx[j]
    out = O.gcr(wx, p, cam)
    np.testing.assert_allclose(out["X"][1][0], y / np.linalg.norm(y), atol=1e-13)


def test_tie_break_by_index():
    # x3 at 180 degrees: d(2,0) = d(2,3) = 2 exactly in exact arithmetic
    X = np.array([[1.0, 0.0], [0.5, math.sqrt(3) / 2], [0.0, 1.0], [-1.0, 0.0]])
    Dm = O.sq_dists(X)
    assert Dm[2, 0] == Dm[2, 3]
    idx, _ = O.knn_lists(Dm, 2)
    assert idx[2].tolist() == [1, 0]


# ---------------------------------------------------------------------------
# brute force on tiny inputs


def _brute_knn(X, k, cam=None, cross=False):
    n = len(X)
    out = []
    for i in range(n):
        cands = []
        for j in range(n):
            if j == i or (cross and cam[j] == cam[i]):
                continue
            d = math.fsum((float(a) - float(b)) ** 2 for a, b in zip(X[i], X[j]))
            cands.append((d, j))
        cands.sort()
        out.append([j for _, j in cands[:k]] + [-1] * max(0, k - len(cands)))
    return out


@pytest.mark.parametrize("n,d,k,seed", [(7, 3, 2, 0), (23, 5, 4, 1), (40, 16, 7, 2), (9, 1, 8, 3), (12, 4, 20, 4)])
def test_knn_matches_bruteforce(n, d, k, seed):
    X = datagen.random_unit(n, d, seed).astype(np.float64)
    idx, dist = O.knn_lists(O.sq_dists(X), k)
    assert idx.tolist() == _brute_knn(X, k)
    for i in range(n):
        for s in range(k):
            j = idx[i, s]
            if j >= 0:
                ref = math.fsum((a - b) ** 2 for a, b in zip(X[i], X[j]))
                assert abs(dist[i, s] - ref) < 1e-13


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_cross_knn_matches_bruteforce(seed):
    rng = np.random.default_rng(100 + seed)
    X = datagen.random_unit(30, 6, seed).astype(np.float64)
    cam = rng.integers(0, 3, size=30)
    idx, _ = O.knn_lists(O.sq_dists(X), 5, cam, cross=True)
    assert idx.tolist() == _brute_knn(X, 5, cam, cross=True)


def test_final_distances_bruteforce():
    X = datagen.random_unit(11, 4, 5).astype(np.float64)
    dq = O.final_distances(X, 3)
    for q in range(3):
        for g in range(8):
            ref = math.fsum((a - b) ** 2 for a, b in zip(X[q], X[3 + g]))
            assert abs(dq[q, g] - ref) < 1e-14


# ---------------------------------------------------------------------------
# invariants and closed forms


def _small(seed=0, n_c=6, per=9, d=12, sigma=0.4):
    X, ids = datagen.clustered(n_c, per, d, sigma, seed)
    return O.row_normalize(X), ids


def test_symmetry_degree_and_stationary_vector():
    X, _ = _small()
    p = O.Params(k=5, gamma=0.2, rounds=1)
    g = O.build_graphs(X, p)
    A, P, Dg = g["A"], g["P"], g["deg"]
    assert np.array_equal(A, A.T)
    assert np.all(Dg >= 1.0)
    np.testing.assert_allclose(Dg, A @ np.ones(len(A)), rtol=1e-15)
    # sqrt(D) is an eigenvector of D^-1/2 A D^-1/2 with eigenvalue 1
    s = np.sqrt(Dg)
    np.testing.assert_allclose(P @ s, s, rtol=1e-12)
    # every off-diagonal nonzero of A comes from a kNN edge in one direction
    nz = (A > 0) & ~np.eye(len(A), dtype=bool)
    E_ = np.zeros_like(nz)
    for i in range(len(A)):
        E_[i, g["idx"][i]] = True
    assert np.array_equal(nz, E_ | E_.T)


def test_unit_rows_after_every_round():
    X, _ = _small(1)
    out = O.gcr(X, O.Params(k=6, gamma=0.2, rounds=4))
    for Xt in out["X"]:
        np.testing.assert_allclose(np.linalg.norm(Xt, axis=1), 1.0, atol=1e-14)


def test_k0_leaves_features_unchanged():
    X, _ = _small(2)
    out = O.gcr(X, O.Params(k=0, gamma=0.2, rounds=3))
    np.testing.assert_allclose(out["X"][-1], O.row_normalize(X), atol=1e-15)


def test_complete_graph_flat_weights_gives_normalised_mean():
    X, _ = _small(3, n_c=3, per=5, d=7)
    n = len(X)
    out = O.gcr(X, O.Params(k=n - 1, gamma=1e300, rounds=1))
    m = X.mean(axis=0)
    np.testing.assert_allclose(out["X"][1], np.tile(m / np.linalg.norm(m), (n, 1)), atol=1e-13)


def test_single_camera_cross_graph_is_identity():
    X, _ = _small(4)
    cam = np.zeros(len(X), dtype=np.int64)
    p = O.Params(k=5, gamma=0.2, rounds=1, alpha=0.6)
    g = O.build_graphs(X, p, cam)
    assert np.all(g["cr_idx"] == -1)
    np.testing.assert_array_equal(g["cr_P"], np.eye(len(X)))
    Y = 0.6 * g["P"] @ X + 0.4 * X
    out = O.gcr(X, p, cam)
    np.testing.assert_allclose(out["X"][1], O.row_normalize(Y), atol=1e-14)


def test_alpha_one_is_plain_gcr():
    X, _ = _small(5)
    cam = np.arange(len(X)) % 3
    a = O.gcr(X, O.Params(k=5, rounds=2, alpha=1.0), cam)
    b = O.gcr(X, O.Params(k=5, rounds=2, alpha=1.0), None)
    np.testing.assert_array_equal(a["X"][-1], b["X"][-1])


def test_asymmetric_equals_symmetric_on_symmetric_affinity():
    # when A~ is already symmetric (all lists mutual), Eq. (6) equals Eq. (2)
    X, _ = _small(6, n_c=2, per=4, d=5, sigma=0.05)
    n = len(X)
    ps = O.Params(k=n - 1, rounds=1, symmetric=True)
    pa = O.Params(k=n - 1, rounds=1, symmetric=False)
    np.testing.assert_allclose(O.gcr(X, ps)["X"][1], O.gcr(X, pa)["X"][1], atol=1e-14)


def test_far_clusters_stay_separated():
    rng = np.random.default_rng(7)
    a = rng.standard_normal((8, 5)) * 0.05 + np.array([10, 0, 0, 0, 0])
    b = rng.standard_normal((8, 5)) * 0.05 + np.array([0, 10, 0, 0, 0])
    X = O.row_normalize(np.concatenate([a, b]))
    out = O.gcr(X, O.Params(k=5, rounds=3))
    Xt = out["X"][-1]
    assert np.all(Xt[:8, 1] < 0.1) and np.all(Xt[8:, 0] < 0.1)


def test_sparse_round_matches_dense():
    X, _ = _small(8)
    cam = np.arange(len(X)) % 4
    p = O.Params(k=6, gamma=0.3, rounds=1, alpha=0.7)
    g = O.build_graphs(X, p, cam)
    dense = O.propagation_round(X, g, p, cam)
    sp, Dg, Dc = O.sparse_round_from_lists(X, p, g["idx"], g["dist"], cam, g["cr_idx"], g["cr_dist"])
    np.testing.assert_allclose(sp, dense, atol=1e-14)
    np.testing.assert_allclose(Dg, g["deg"], rtol=1e-14)
    w = np.exp(-g["dist"] / p.gamma)
    np.testing.assert_allclose(O.degrees_from_lists(len(X), g["idx"], w), g["deg"], rtol=1e-14)


def test_beta_edge_factors():
    # beta_same = beta_cross = b scales every off-diagonal weight by b
    X, _ = _small(9)
    cam = np.arange(len(X)) % 2
    g1 = O.build_graphs(X, O.Params(k=4, alpha=1.0), cam)
    g2 = O.build_graphs(X, O.Params(k=4, alpha=1.0, beta_same=0.5, beta_cross=0.5), cam)
    off = ~np.eye(len(X), dtype=bool)
    np.testing.assert_allclose(g2["At"][off], 0.5 * g1["At"][off], rtol=1e-15)


# ---------------------------------------------------------------------------
# profile vectors (Eq. (10), Eq. (16))


def _det3(m):
    return (m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1])
            - m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0])
            + m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]))


def _cramer3(m, b):
    dm = _det3(m)
    out = []
    for c in range(3):
        mc = [[(b[r] if cc == c else m[r][cc]) for cc in range(3)] for r in range(3)]
        out.append(_det3(mc) / dm)
    return out


def test_pvg_worked_example():
    F = np.array([[1, 0, 0], [.8, .6, 0], [0, 1, 0], [0, .6, .8], [0, 0, 1]], dtype=np.float64)
    offs = np.array([0, 2, 5])
    # by hand: F^T F + lambda n I with lambda = 1, n = 5
    M = [[6.64, 0.48, 0.0], [0.48, 6.72, 0.48], [0.0, 0.48, 6.64]]
    mu = [0.36, 0.44, 0.36]
    mu0 = [0.9, 0.3, 0.0]
    mu1 = [0.0, 1.6 / 3, 0.6]
    w0 = _cramer3(M, [a - b for a, b in zip(mu0, mu)])
    w1 = _cramer3(M, [a - b for a, b in zip(mu1, mu)])
    W = O.profile_vectors(F, offs, None, lam=1.0)
    np.testing.assert_allclose(W[0], np.array(w0) / np.linalg.norm(w0), atol=1e-14)
    np.testing.assert_allclose(W[1], np.array(w1) / np.linalg.norm(w1), atol=1e-14)
    # two tracklets: m0 w0 + m1 w1 = 0, so the profiles are opposite
    np.testing.assert_allclose(W[0], -W[1], atol=1e-14)
    np.testing.assert_allclose(W[0], [0.8225833722, -0.2280482701, -0.5209132196], atol=1e-9)


def test_pvg_orthonormal_frames():
    # frames e1 | e2: F^T F = I, n = 2, M = (1 + 2 lambda) I, mu = (.5, .5)
    F = np.eye(2)
    W = O.profile_vectors(F, np.array([0, 1, 2]), None, lam=3.0)
    np.testing.assert_allclose(W, [[1 / math.sqrt(2), -1 / math.sqrt(2)], [-1 / math.sqrt(2), 1 / math.sqrt(2)]], atol=1e-15)


def test_pvg_weighted_sum_zero_and_residual():
    rng = np.random.default_rng(3)
    lens = rng.integers(2, 6, size=7)
    offs = np.concatenate([[0], np.cumsum(lens)])
    F = O.row_normalize(rng.standard_normal((offs[-1], 9)))
    lam = 0.7
    Wu = O.profile_vectors(F, offs, None, lam=lam, normalize=False)
    np.testing.assert_allclose((lens[:, None] * Wu).sum(axis=0), 0.0, atol=1e-14)
    n = offs[-1]
    M = sum(np.outer(f, f) for f in F) + lam * n * np.eye(9)
    mu = F.sum(axis=0) / n
    for c in range(7):
        muc = F[offs[c]:offs[c + 1]].sum(axis=0) / lens[c]
        np.testing.assert_allclose(M @ Wu[c], muc - mu, atol=1e-13)


def test_pvg_large_lambda_tends_to_centred_mean():
    rng = np.random.default_rng(4)
    offs = np.array([0, 3, 5, 9])
    F = O.row_normalize(rng.standard_normal((9, 4)))
    W = O.profile_vectors(F, offs, None, lam=1e9)
    mu = F.mean(axis=0)
    for c in range(3):
        v = F[offs[c]:offs[c + 1]].mean(axis=0) - mu
        np.testing.assert_allclose(W[c], v / np.linalg.norm(v), atol=1e-8)


def test_pvg_groups_are_independent():
    rng = np.random.default_rng(5)
    offs = np.array([0, 2, 5, 7, 10])
    F = O.row_normalize(rng.standard_normal((10, 4)))
    groups = np.array([0, 1, 0, 1])
    W = O.profile_vectors(F, offs, groups, lam=2.0)
    Wa = O.profile_vectors(np.concatenate([F[0:2], F[5:7]]), np.array([0, 2, 4]), None, lam=2.0)
    np.testing.assert_allclose(W[[0, 2]], Wa, atol=1e-14)


def test_mean_profile():
    F = np.array([[1.0, 0], [0, 1.0], [3.0, 4.0]])
    W = O.profile_vectors(F, np.array([0, 2, 3]), None, mode="mean")
    np.testing.assert_allclose(W, [[2 ** -0.5, 2 ** -0.5], [0.6, 0.8]], atol=1e-15)


# ---------------------------------------------------------------------------
# serving reading


def test_serve_request_equals_dense_construction():
    rng = np.random.default_rng(11)
    XG = O.row_normalize(rng.standard_normal((25, 6)))
    Q = O.row_normalize(rng.standard_normal((3, 6)))
    p = O.Params(k=4, gamma=0.5, rounds=2, rebuild_each_round=False)
    gi, gd = O.knn_lists(O.sq_dists(XG), 4)
    top, dist = O.serve_request(XG, gi, gd, Q, p, topk=5)
    # dense construction by hand: node order gallery then queries
    n = 28
    At = np.eye(n)
    for i in range(25):
        for s in range(4):
            At[i, gi[i, s]] = math.exp(-gd[i, s] / 0.5)
    for q in range(3):
        dq = [(math.fsum((a - b) ** 2 for a, b in zip(Q[q], XG[j])), j) for j in range(25)]
        dq.sort()
        for d_, j in dq[:4]:
            At[25 + q, j] = math.exp(-d_ / 0.5)
    A = (At + At.T) / 2
    Dg = A.sum(1)
    P = A / np.sqrt(np.outer(Dg, Dg))
    X = np.concatenate([XG, Q])
    for _ in range(2):
        X = P @ X
        X /= np.linalg.norm(X, axis=1, keepdims=True)
    for q in range(3):
        ref = sorted((math.fsum((a - b) ** 2 for a, b in zip(X[25 + q], X[j])), j) for j in range(25))
        assert [j for _, j in ref[:5]] == top[q].tolist()
        np.testing.assert_allclose(dist[q], [d_ for d_, _ in ref[:5]], atol=1e-13)


# ---------------------------------------------------------------------------
# the small plain-GCR workload: near-perfect retrieval before and after


@pytest.mark.slow
def test_plain_gcr_small_map():
    w = datagen.plain_gcr_small()
    p = O.Params(k=20, gamma=0.1, rounds=2, alpha=1.0)
    out = O.gcr(w.X, p)
    qid, gid = w.ids[:w.nq], w.ids[w.nq:]
    before = mean_average_precision(O.final_distances(out["X"][0], w.nq), qid, gid)
    after = mean_average_precision(O.final_distances(out["X"][-1], w.nq), qid, gid)
    assert before >= 0.99 and after >= 0.99


def test_asymmetric_closed_form_two_nodes():
    # Eq. (5)-(6) by hand: A~ = [[1, a], [0, 1]] (node 1 is node 0's only
    # neighbour, not the reverse): D_r = (1 + a, 1), D_c = (1, 1 + a), so
    # P = [[1/sqrt(1+a), a/(1+a)], [0, 1/sqrt(1+a)]]
    a = math.exp(-0.3 / 0.2)
    At = np.array([[1.0, a], [0.0, 1.0]])
    P, Dr, Dc = O.asym_propagation_matrix(At)
    np.testing.assert_allclose(Dr, [1 + a, 1.0], rtol=0, atol=1e-15)
    np.testing.assert_allclose(Dc, [1.0, 1 + a], rtol=0, atol=1e-15)
    s = 1.0 / math.sqrt(1 + a)
    np.testing.assert_allclose(P, [[s, a / (1 + a)], [0.0, s]], rtol=0, atol=1e-15)
    # the symmetric form of the same pair averages the edge: A_01 = a / 2
    Ps, As, Ds = O.sym_propagation_matrix(At)
    np.testing.assert_allclose(As, [[1.0, a / 2], [a / 2, 1.0]], rtol=0, atol=1e-15)
    np.testing.assert_allclose(Ps[0, 1], (a / 2) / (1 + a / 2), rtol=1e-15)


# ---------------------------------------------------------------------------
# DSFP (Alg. 1): closed forms, special cases and locality


def test_dsfp_three_nodes_closed_form():
    """x0 = (1,0), x1 = (0,1), x2 = (-1,0), gamma = 1, k = 2: the local set of
    every node is all three.  Squared distances 2, 4, 2, so A has a = e^-2
    next to the diagonal and b = e^-4 in the corners; degrees s0 = s2 =
    1 + a + b, s1 = 1 + 2a.  By hand, with P_uv = A_uv / sqrt(s_u s_v):
      round 1: y0 = ((1-b)/s0, a/sqrt(s0 s1)), y1 = (0, 1/s1),
               y2 = (-(1-b)/s0, a/sqrt(s0 s1)); rows re-normalised;
      round 2: w0 = z0/s0 + a z1/sqrt(s0 s1) + b z2/s0, re-normalised.
    The degree of every member (not only node i's) and the per-round
    re-normalisation both change these numbers."""
    X = np.array([[1.0, 0.0], [0.0, 1.0], [-1.0, 0.0]])
    idx = np.array([[1, 2], [0, 2], [1, 0]])
    a, b = E(-2.0), E(-4.0)
    s0, s1 = 1 + a + b, 1 + 2 * a
    y0 = np.array([(1 - b) / s0, a / math.sqrt(s0 * s1)])
    y2 = np.array([-(1 - b) / s0, a / math.sqrt(s0 * s1)])
    z0, z1, z2 = y0 / np.linalg.norm(y0), np.array([0.0, 1.0]), y2 / np.linalg.norm(y2)
    w0 = z0 / s0 + a * z1 / math.sqrt(s0 * s1) + b * z2 / s0
    p1 = O.Params(k=2, gamma=1.0, rounds=1)
    np.testing.assert_allclose(O.dsfp(X, p1, idx)[0], y0 / np.linalg.norm(y0), rtol=0, atol=1e-14)
    np.testing.assert_allclose(O.dsfp(X, p1, idx)[1], [0.0, 1.0], rtol=0, atol=1e-14)
    p2 = O.Params(k=2, gamma=1.0, rounds=2)
    np.testing.assert_allclose(O.dsfp(X, p2, idx)[0], w0 / np.linalg.norm(w0), rtol=0, atol=1e-14)


def test_dsfp_two_nodes_closed_form():
    """Two orthogonal unit vectors, gamma = 1, w = e^-2: after T rounds node
    0's direction is that of (1, w) for T = 1 and (1 + w^2, 2w) for T = 2."""
    X = np.array([[1.0, 0.0], [0.0, 1.0]])
    w = E(-2.0)
    for T, v in ((1, (1.0, w)), (2, (1.0 + w * w, 2.0 * w))):
        got = O.dsfp(X, O.Params(k=1, gamma=1.0, rounds=T))
        v = np.array(v) / math.hypot(*v)
        np.testing.assert_allclose(got[0], v, rtol=0, atol=1e-14)
        np.testing.assert_allclose(got[1], v[::-1], rtol=0, atol=1e-14)


def test_dsfp_flat_affinity_gives_local_mean():
    """gamma -> infinity makes A all ones: for any T >= 1 node i becomes the
    normalised mean of its local set (i and its listed neighbours), for any
    lists, including -1 padding and repeats."""
    rng = np.random.default_rng(21)
    n, d, k = 14, 6, 4
    X = O.row_normalize(rng.standard_normal((n, d)))
    idx = np.array([rng.choice(np.delete(np.arange(n), i), size=k, replace=False) for i in range(n)])
    idx[3, 1] = -1
    idx[5, 2] = idx[5, 0]
    for T in (1, 3):
        got = O.dsfp(X, O.Params(k=k, gamma=1e13, rounds=T), idx)
        for i in range(n):
            nodes = {i} | {int(j) for j in idx[i] if j >= 0}
            m = X[sorted(nodes)].mean(axis=0)
            np.testing.assert_allclose(got[i], m / np.linalg.norm(m), rtol=0, atol=1e-9)


def test_dsfp_zero_rounds_is_identity():
    rng = np.random.default_rng(22)
    X = rng.standard_normal((7, 5))
    got = O.dsfp(X, O.Params(k=3, rounds=0))
    np.testing.assert_allclose(got, X / np.linalg.norm(X, axis=1, keepdims=True), rtol=0, atol=1e-15)


def test_dsfp_complete_graph_equals_global():
    """k = N - 1: every local set is the whole node set and A^i is the global
    affinity of the complete graph, so DSFP equals global GCR with the graph
    built once (alpha = 1)."""
    rng = np.random.default_rng(23)
    n, d = 9, 4
    X = rng.standard_normal((n, d))
    for T in (1, 3):
        got = O.dsfp(X, O.Params(k=n - 1, gamma=0.7, rounds=T))
        ref = O.gcr(X, O.Params(k=n - 1, gamma=0.7, rounds=T, rebuild_each_round=False))["X"][-1]
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12)


def test_dsfp_node_depends_on_its_local_set_only():
    """Node i's output is node i's row of global GCR run on the local set
    alone as a complete graph (the local rounds never look outside it)."""
    rng = np.random.default_rng(24)
    n, d, k = 30, 8, 5
    X = O.row_normalize(rng.standard_normal((n, d)))
    p = O.Params(k=k, gamma=0.5, rounds=2)
    got = O.dsfp(X, p)
    idx, _ = O.knn_lists(O.sq_dists(X), k)
    for i in range(n):
        sub = X[[i] + [int(j) for j in idx[i]]]
        ref = O.gcr(sub, O.Params(k=k, gamma=0.5, rounds=2, rebuild_each_round=False))["X"][-1][0]
        np.testing.assert_allclose(got[i], ref, rtol=0, atol=1e-12)


# ---------------------------------------------------------------------------
# pins for the camera factors, the profile mode of GCRV, the zero-row floor,
# the serving tie order and the retrieval metric


def _fsum_d(a, b):
    return math.fsum((float(x) - float(y)) ** 2 for x, y in zip(a, b))


def _hand_sym_round(X, lists, weights):
    """One symmetric round by hand: A~ from explicit (i, j, w) edges plus the
    unit diagonal, A = (A~ + A~^T) / 2, D = row sums, y_i = sum_j A_ij x_j /
    sqrt(D_i D_j), then y_i / ||y_i||.  Pure Python scalars."""
    n = len(X)
    At = [[1.0 if i == j else 0.0 for j in range(n)] for i in range(n)]
    for i in range(n):
        for j, w in zip(lists[i], weights[i]):
            At[i][j] = w
    A = [[0.5 * (At[i][j] + At[j][i]) for j in range(n)] for i in range(n)]
    D = [math.fsum(A[i]) for i in range(n)]
    out = []
    for i in range(n):
        y = [math.fsum(A[i][j] * X[j][c] / math.sqrt(D[i] * D[j]) for j in range(n)) for c in range(len(X[0]))]
        nrm = math.sqrt(math.fsum(v * v for v in y))
        out.append([v / nrm for v in y])
    return out


def _hand_knn(X, k):
    lists, dists = [], []
    for i in range(len(X)):
        c = sorted((_fsum_d(X[i], X[j]), j) for j in range(len(X)) if j != i)[:k]
        lists.append([j for _, j in c])
        dists.append([d for d, _ in c])
    return lists, dists


def test_beta_same_and_cross_are_not_interchangeable():
    # three unit vectors at 0, 30 and 100 degrees; cameras (0, 0, 1); k = 2
    # makes both other points neighbours of every point.  Same-camera edges
    # (0-1) carry beta_same, the others beta_cross; the factors differ, so a
    # swapped assignment changes every off-diagonal entry.
    X = np.array([unit_at(0.0), unit_at(30.0), unit_at(100.0)])
    cam = np.array([0, 0, 1])
    bs, bc = 0.25, 3.0
    p = O.Params(k=2, gamma=1.0, rounds=1, alpha=1.0, beta_same=bs, beta_cross=bc)
    g = O.build_graphs(X, p, cam)
    ang = [0.0, 30.0, 100.0]
    for i in range(3):
        for j in range(3):
            if i == j:
                assert g["At"][i, j] == 1.0
                continue
            f = bs if cam[i] == cam[j] else bc
            assert abs(g["At"][i, j] - f * E(-d_angle(ang[i], ang[j]))) < 1e-15
    # the round that follows uses these weights (dense and sparse forms)
    lists, dists = _hand_knn(X.tolist(), 2)
    wts = [[(bs if cam[i] == cam[j] else bc) * E(-d) for j, d in zip(lists[i], dists[i])] for i in range(3)]
    ref = _hand_sym_round(X.tolist(), lists, wts)
    np.testing.assert_allclose(O.gcr(X, p, cam)["X"][1], ref, rtol=0, atol=1e-14)
    sp, _, _ = O.sparse_round_from_lists(X, p, g["idx"], g["dist"], cam)
    np.testing.assert_allclose(sp, ref, rtol=0, atol=1e-14)


def _pvg_case():
    # three tracklets of two unit frames each in R^3
    F = [[1.0, 0.0, 0.0], [0.8, 0.6, 0.0],
         [0.0, 1.0, 0.0], [0.0, 0.6, 0.8],
         [0.0, 0.0, 1.0], [0.6, 0.0, 0.8]]
    return F, [0, 2, 4, 6]


def test_gcrv_uses_the_requested_profile_mode():
    """Alg. 2 on the three-tracklet case: W by Cramer's rule from Eq. (16)
    (lambda = 2, one group, n = 6) or the mean profile of Eq. (10), then one
    fixed-graph round with k = 1 worked by hand.  A GCRV that ignored its
    mode would give the other profile."""
    F, offs = _pvg_case()
    lam, n = 2.0, 6
    M = [[math.fsum(f[a] * f[b] for f in F) + (lam * n if a == b else 0.0) for b in range(3)] for a in range(3)]
    mu = [math.fsum(f[a] for f in F) / n for a in range(3)]
    w_pvg, w_mean = [], []
    for c in range(3):
        muc = [math.fsum(F[r][a] for r in range(offs[c], offs[c + 1])) / 2.0 for a in range(3)]
        w = _cramer3(M, [muc[a] - mu[a] for a in range(3)])
        nw, nm = math.sqrt(math.fsum(v * v for v in w)), math.sqrt(math.fsum(v * v for v in muc))
        w_pvg.append([v / nw for v in w])
        w_mean.append([v / nm for v in muc])
    p = O.Params(k=1, gamma=1.0, rounds=1, lam=lam, rebuild_each_round=False)
    for mode, W in (("pvg", w_pvg), ("mean", w_mean)):
        out = O.gcrv(np.array(F), np.array(offs), None, 1, p, mode=mode)
        np.testing.assert_allclose(out["W"], W, rtol=0, atol=1e-14)
        lists, dists = _hand_knn(W, 1)
        ref = _hand_sym_round(W, lists, [[E(-d) for d in ds] for ds in dists])
        np.testing.assert_allclose(out["X"][1], ref, rtol=0, atol=1e-13)
    # the two profiles really differ here
    assert np.abs(np.array(w_pvg) - np.array(w_mean)).max() > 0.1


def test_row_normalize_zero_row_stays_zero():
    Y = O.row_normalize(np.array([[0.0, 0.0, 0.0], [3.0, 0.0, 4.0], [0.0, 0.0, 0.0]]))
    assert np.all(np.isfinite(Y))
    np.testing.assert_array_equal(Y[0], 0.0)
    np.testing.assert_array_equal(Y[2], 0.0)
    np.testing.assert_allclose(Y[1], [0.6, 0.0, 0.8], rtol=0, atol=1e-16)
    # a round whose blended row vanishes keeps it at zero (the 1e-12 floor)
    tiny = O.row_normalize(np.array([[1e-13, 0.0]]))
    np.testing.assert_allclose(tiny, [[0.1, 0.0]], rtol=1e-12)


def _hand_serve(XG, gi, gd, Q, k, gamma, rounds, topk):
    """S1 by hand: node order gallery then queries; query rows list their k
    nearest gallery items by (distance, index); fixed graph, `rounds` rounds."""
    ng, b = len(XG), len(Q)
    X = [list(map(float, r)) for r in XG] + [list(map(float, r)) for r in Q]
    lists = [list(map(int, gi[i])) for i in range(ng)]
    wts = [[E(-float(d) / gamma) for d in gd[i]] for i in range(ng)]
    for q in range(b):
        c = sorted((_fsum_d(Q[q], XG[j]), j) for j in range(ng))[:k]
        lists.append([j for _, j in c])
        wts.append([E(-d / gamma) for d, _ in c])
    for _ in range(rounds):
        X = _hand_sym_round(X, lists, wts)
    res = []
    for q in range(b):
        res.append(sorted((_fsum_d(X[ng + q], X[j]), j) for j in range(ng))[:topk])
    return res


def test_serve_request_ties_resolve_by_gallery_index():
    rng = np.random.default_rng(12)
    XG = O.row_normalize(rng.standard_normal((12, 5)))
    XG[7] = XG[3]   # exact copies: equal distances to every query
    XG[10] = XG[1]
    # each query sits next to one copied pair, so with k = 1 its only
    # neighbour is decided by the index tie-break
    Q = O.row_normalize(np.array([XG[3] + 0.05 * rng.standard_normal(5), XG[1] + 0.05 * rng.standard_normal(5)]))
    gi, gd = O.knn_lists(O.sq_dists(XG), 1)
    assert gi[3, 0] == 7 and gi[7, 0] == 3
    for rounds in (0, 1, 2):
        p = O.Params(k=1, gamma=0.5, rounds=rounds, rebuild_each_round=False)
        top, dist = O.serve_request(XG, gi, gd, Q, p, topk=6)
        ref = _hand_serve(XG, gi, gd, Q, 1, 0.5, rounds, 6)
        for q in range(2):
            assert top[q].tolist() == [j for _, j in ref[q]], (rounds, q)
            np.testing.assert_allclose(dist[q], [d for d, _ in ref[q]], rtol=0, atol=1e-13)
    # with no rounds the copies tie exactly and appear in index order
    top0, d0 = O.serve_request(XG, gi, gd, Q, O.Params(k=1, rounds=0, rebuild_each_round=False), topk=2)
    assert top0[0].tolist() == [3, 7] and d0[0, 0] == d0[0, 1]
    assert top0[1].tolist() == [1, 10] and d0[1, 0] == d0[1, 1]


def test_mean_average_precision_hand_computed():
    # query 0 (id 5): ranking by distance is g2, g0, g3, g1 (g0 and g3 tie at
    # 0.4 and keep index order); relevant g0, g1 -> hits at ranks 2 and 4:
    #   AP = (1/2 + 2/4) / 2 = 0.5
    # query 1 (id 7): ranking g3, g1, g0, g2; relevant g3, g2 -> ranks 1, 4:
    #   AP = (1/1 + 2/4) / 2 = 0.75
    # query 2 (id 9): no relevant item, skipped
    dq = np.array([[0.4, 0.9, 0.1, 0.4],
                   [0.5, 0.3, 0.8, 0.2],
                   [0.1, 0.2, 0.3, 0.4]])
    qids = np.array([5, 7, 9])
    gids = np.array([5, 5, 7, 7])
    gids_q0 = np.array([5, 5, 6, 6])
    assert mean_average_precision(dq[:1], qids[:1], gids_q0) == pytest.approx(0.5, abs=1e-15)
    gids_q1 = np.array([6, 6, 7, 7])
    assert mean_average_precision(dq[1:2], qids[1:2], gids_q1) == pytest.approx(0.75, abs=1e-15)
    # together, with the per-query gallery ids folded into one labelling
    dq2 = np.array([[0.4, 0.9, 0.1, 0.4, 0.95, 0.96], [0.97, 0.98, 0.8, 0.2, 0.5, 0.3]])
    gids2 = np.array([5, 5, 6, 7, 6, 6])
    # q0 (5): order g2, g0, g3, g1, g4, g5 -> hits at 2, 4: (1/2 + 2/4)/2 = 0.5
    # q1 (7): order g3, g5, g4, g2, g0, g1 -> hit at 1: 1.0
    assert mean_average_precision(dq2, np.array([5, 7]), gids2) == pytest.approx(0.75, abs=1e-15)
    assert mean_average_precision(dq[2:], qids[2:], gids) == 0.0


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_knn_blocked_equals_full_sort(seed):
    """The blocked large-N kNN against brute force (math.fsum distances,
    Python sort by (distance, index)), with exact ties planted at the cut
    (duplicated rows), blocks smaller than the input, and the cross-camera
    lists."""
    rng = np.random.default_rng(seed)
    n, d, k = 97, 6, 7
    X = rng.standard_normal((n, d))
    X[10] = X[3]
    X[11] = X[3]
    X[50] = X[40]
    cam = rng.integers(0, 3, size=n)
    gi, gd = O.knn_blocked(X, k, block=16, threads=3)
    assert gi.tolist() == _brute_knn(X, k)
    ci, _ = O.knn_blocked(X, k, cam=cam, cross=True, block=16, threads=3)
    assert ci.tolist() == _brute_knn(X, k, cam=cam, cross=True)
    rows = np.array([3, 10, 96, 0])
    ri, rd = O.knn_blocked(X, k, rows=rows, block=2)
    assert ri.tolist() == [_brute_knn(X, k)[r] for r in rows]
    for t, r in enumerate(rows):
        for s_, j in enumerate(ri[t]):
            assert abs(rd[t, s_] - math.fsum((a - b) ** 2 for a, b in zip(X[r], X[j]))) < 1e-12
    # fewer eligible items than k: padding
    small = X[:5]
    pi, pd = O.knn_blocked(small, k)
    assert np.all(pi[:, 4:] == -1) and np.all(np.isinf(pd[:, 4:]))


def test_closed_neighbourhood_round_equals_whole_graph():
    """The closed-neighbourhood evaluation used at sizes where the whole
    graph does not fit gives the whole-graph round at the chosen rows."""
    import sys, os
    sys.path.insert(0, os.path.dirname(__file__))
    from parity import closed_neighbourhood_round

    X, ids = datagen.clustered(40, 30, 24, 0.6, seed=9)
    X = O.row_normalize(X)
    whole = O.gcr(X, O.Params(k=8, gamma=0.3, rounds=1, normalize_input=False))["X"][1]
    rows = np.nonzero(np.isin(ids, [3, 17, 29]))[0]
    Y, _, closure = closed_neighbourhood_round(X, ids, 8, 0.3, rows)
    assert len(closure) < len(X)
    np.testing.assert_allclose(Y, whole[rows], rtol=0, atol=1e-13)
