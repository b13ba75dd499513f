"""Pins of the CPU oracle and of the seeded input chain (no GPU).

Every check compares against something other than the code under test:
closed forms, textbook special cases, invariants the paper's equations imply,
an independent brute-force implementation (oracle.refchain) or a library
routine.  Citations name the paper's section / equation.
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csgraph

from oracle import eig as oeig
from oracle import mds as omds
from oracle import refchain as ref
from synth import _geodesic, configs, meshes
from synth import operator as op


# ---------------------------------------------------------------- fixtures
@pytest.fixture(scope="module")
def small_torus():
    return meshes.torus_grid(12, 8, 1.0, 0.4, jitter=0.01, seed=7)


@pytest.fixture(scope="module")
def small_sphere():
    return meshes.deformed_icosphere(2, seed=5)


def _dense(A):
    return A.toarray() if sp.issparse(A) else np.asarray(A)


# ------------------------------------------- cotangent operator (Section 2.2)
def test_cotan_weights_match_bruteforce(small_torus, small_sphere):
    for V, F in (small_torus, small_sphere):
        A = _dense(op.cotan_weights(V, F))
        Aref = ref.cot_adjacency_dense(V, F)
        np.testing.assert_allclose(A, Aref, rtol=1e-11, atol=1e-12)
        np.testing.assert_allclose(A, A.T, atol=1e-14)


def test_mass_matches_heron_and_total_area(small_torus, small_sphere):
    for V, F in (small_torus, small_sphere):
        d = op.lumped_mass(V, F)
        np.testing.assert_allclose(d, ref.mass_dense(V, F), rtol=1e-11)
    # a fine regular torus approaches the analytic area 4 pi^2 R r
    V, F = meshes.torus_grid(128, 64, 1.0, 0.4)
    total = op.lumped_mass(V, F).sum()
    assert abs(total - 4 * math.pi ** 2 * 0.4) / (4 * math.pi ** 2 * 0.4) < 2e-3


def test_equilateral_interior_weight_is_inverse_sqrt3():
    # two equilateral triangles on an interior edge: (cot 60 + cot 60)/2 = 1/sqrt(3)
    V, F = meshes.equilateral_patch(rings=3)
    A = _dense(op.cotan_weights(V, F))
    r = np.linalg.norm(V[:, :2], axis=1)
    interior = np.flatnonzero(r < 1.5)
    for i in interior:
        nb = np.flatnonzero(A[i])
        assert len(nb) == 6
        np.testing.assert_allclose(A[i, nb], 1 / math.sqrt(3), rtol=1e-12)


def test_laplacian_linear_precision_and_null_space():
    # the cotangent Laplacian is exact on linear functions of a flat mesh
    V, F = meshes.flat_grid(9, 7, h=0.3, seed=3, jitter=0.05)
    L = _dense(op.laplacian(op.cotan_weights(V, F)))
    nx, ny = 9, 7
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    interior = ((i > 0) & (i < nx - 1) & (j > 0) & (j < ny - 1)).ravel()
    for c in (0, 1):
        np.testing.assert_allclose((L @ V[:, c])[interior], 0.0, atol=1e-12)
    np.testing.assert_allclose(L @ np.ones(len(V)), 0.0, atol=1e-12)
    assert np.linalg.eigvalsh(0.5 * (L + L.T)).min() > -1e-10


def test_biharmonic_operator(small_torus, small_sphere):
    for V, F in (small_torus, small_sphere):
        M = _dense(op.biharmonic(V, F))
        Mref, L, d = ref.biharmonic_dense(V, F)
        np.testing.assert_allclose(M, Mref, rtol=1e-10, atol=1e-9 * np.abs(Mref).max())
        np.testing.assert_allclose(M, M.T, atol=1e-10 * np.abs(M).max())
        np.testing.assert_allclose(M @ np.ones(len(V)), 0.0, atol=1e-9 * np.abs(M).max())
        assert np.linalg.eigvalsh(M).min() > -1e-8 * np.abs(M).max()


def test_graph_variant_operator(small_torus):
    V, F = small_torus
    M = _dense(op.biharmonic(V, F, graph=True))
    np.testing.assert_allclose(M, ref.graph_biharmonic_dense(len(V), F), atol=1e-12)


# ---------------------------------- interpolation operator (Eq. PDefinition)
@pytest.fixture(scope="module")
def torus_chain(small_torus):
    V, F = small_torus
    M = op.biharmonic(V, F)
    G = op.edge_graph(V, F)
    lm = op.farthest_point_landmarks(G, 10, seed=11)
    return V, F, M, lm


def test_dense_p_identity_rows_and_unit_row_sums(torus_chain):
    V, F, M, lm = torus_chain
    P, _ = op.interpolation_operator(M, lm, None)
    Pd = P.toarray()
    np.testing.assert_array_equal(Pd[lm], np.eye(len(lm)))
    # M 1 = 0 implies -M_uu^-1 M_ub 1 = 1: every row of P sums to one
    np.testing.assert_allclose(Pd.sum(axis=1), 1.0, atol=1e-9)
    # residual of the defining linear system
    n = len(V)
    u = np.setdiff1d(np.arange(n), lm)
    Md = M.toarray()
    R = Md[np.ix_(u, u)] @ Pd[u] + Md[np.ix_(u, lm)]
    assert np.abs(R).max() <= 1e-9 * np.abs(Md[np.ix_(u, lm)]).max()
    # brute-force dense solve from the independent reference chain
    Mref, _, _ = ref.biharmonic_dense(V, F)
    np.testing.assert_allclose(Pd, ref.interp_dense(Mref, lm), atol=1e-9)


def test_p_invariant_to_scale_and_rigid_motion(torus_chain):
    V, F, M, lm = torus_chain
    P0 = op.interpolation_operator(M, lm, None)[0].toarray()
    rng = np.random.default_rng(0)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    for V2 in (3.7 * V, V @ Q.T + np.array([1.0, -2.0, 0.5])):
        P2 = op.interpolation_operator(op.biharmonic(V2, F), lm, None)[0].toarray()
        np.testing.assert_allclose(P2, P0, atol=1e-9)


def test_threshold_rule_matches_full_sort():
    rng = np.random.default_rng(1)
    for trial in range(200):
        m = int(rng.integers(1, 40))
        x = rng.choice([-2.0, -1.0, -0.5, 0.0, 0.5, 1.0, 2.0], size=m) * rng.integers(1, 3, size=m)
        if trial % 3 == 0:
            x = rng.standard_normal(m)
        p = int(rng.integers(1, m + 2))
        np.testing.assert_array_equal(op.threshold_column(x, p), ref.threshold_sorted(x, p))


def test_thresholded_p(torus_chain):
    V, F, M, lm = torus_chain
    n, l = len(V), len(lm)
    Pdense = op.interpolation_operator(M, lm, None)[0].toarray()
    p = 7
    P, info = op.interpolation_operator(M, lm, p)
    Pd = P.toarray()
    u = np.setdiff1d(np.arange(n), lm)
    for j in range(l):
        keep = ref.threshold_sorted(Pdense[u, j], p)
        col = np.zeros(len(u))
        col[keep] = Pdense[u[keep], j]
        np.testing.assert_allclose(Pd[u, j], col, atol=1e-12)
        assert np.count_nonzero(Pd[u, j]) == min(p, np.count_nonzero(Pdense[u, j]))
    np.testing.assert_array_equal(Pd[lm], np.eye(l))
    # p = n - l keeps everything
    Pall = op.interpolation_operator(M, lm, n - l)[0].toarray()
    np.testing.assert_array_equal(Pall, Pdense)


def test_p_from_prow_values():
    assert op.p_from_prow(2048, 64, 10) == 310
    assert op.p_from_prow(163842, 2000, 10) == 809
    assert op.p_from_prow(524288, 10000, 10) == 514
    assert op.p_from_prow(1_800_000, 50_000, 10) == 350
    assert op.p_from_prow(10, 9, 10) == 1


# ------------------------------------------ geodesics and FPS (Eq. FarthestPoint)
def test_dijkstra_matches_floyd_warshall_and_heap(small_sphere):
    V, F = small_sphere
    G = op.edge_graph(V, F)
    Dfw = ref.floyd_warshall(V, F)
    src = np.array([0, 5, 17])
    D = _geodesic.sssp_to(G, src, np.arange(len(V)), threads=2)
    np.testing.assert_allclose(D, Dfw[src], rtol=1e-12)
    edges = [(int(a), int(b), float(np.linalg.norm(V[a] - V[b]))) for a, b in zip(*sp.triu(G).nonzero())]
    np.testing.assert_allclose(D[1], ref.dijkstra_heap(len(V), edges, 5), rtol=1e-12)
    np.testing.assert_allclose(D[2], csgraph.dijkstra(G, directed=False, indices=17), rtol=1e-12)


def test_dijkstra_torus_grid_closed_form():
    # unit-weight periodic grid graph: distance = wrap-around Manhattan
    nu, nv = 9, 6
    idx = lambda i, j: (i % nu) * nv + (j % nv)
    rows, cols = [], []
    for i in range(nu):
        for j in range(nv):
            for a, b in ((1, 0), (0, 1)):
                rows += [idx(i, j), idx(i + a, j + b)]
                cols += [idx(i + a, j + b), idx(i, j)]
    G = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(nu * nv, nu * nv))
    G.sum_duplicates()
    G.data[:] = 1.0
    D = _geodesic.sssp_to(G, np.array([0, 13]), np.arange(nu * nv), threads=1)
    for s, (si, sj) in zip(range(2), [(0, 0), (13 // nv, 13 % nv)]):
        for i in range(nu):
            for j in range(nv):
                di = min(abs(i - si), nu - abs(i - si))
                dj = min(abs(j - sj), nv - abs(j - sj))
                assert D[s, idx(i, j)] == di + dj


def test_fps_matches_literal_definition(small_sphere):
    V, F = small_sphere
    G = op.edge_graph(V, F)
    D = ref.floyd_warshall(V, F)
    for first in (0, 33, 101):
        lm = op.farthest_point_landmarks(G, 25, first=first)
        np.testing.assert_array_equal(lm, ref.fps_literal(D, 25, first))
    lm = op.farthest_point_landmarks(G, 10, seed=4)
    assert lm[0] == np.random.default_rng(4).integers(len(V))


def test_w_is_squared_landmark_distances(small_sphere):
    V, F = small_sphere
    G = op.edge_graph(V, F)
    lm = op.farthest_point_landmarks(G, 12, seed=2)
    W = op.landmark_sq_distances(G, lm)
    D = ref.floyd_warshall(V, F)
    np.testing.assert_allclose(W, D[np.ix_(lm, lm)] ** 2, rtol=1e-12)
    np.testing.assert_array_equal(W, W.T)
    np.testing.assert_array_equal(np.diag(W), 0.0)


# --------------------------------------------- the embedding (Sections 2.3, 3.3)
def _chain_problem(V, F, l, p_row, landmarks=None, seed=0):
    return configs.build_problem(V, F, l, p_row, seed, np.float64, landmarks=landmarks)


def test_b_double_centred_symmetric_and_interpolates_w(small_torus):
    V, F = small_torus
    prob = _chain_problem(V, F, 12, 5, seed=3)
    P = prob["P64"]
    B = oeig.b_matrix(P, prob["W64"])
    nrm = np.abs(B).max()
    np.testing.assert_allclose(B @ np.ones(len(V)), 0.0, atol=1e-12 * nrm * len(V))
    np.testing.assert_allclose(B, B.T, atol=1e-13 * nrm)
    # exact interpolation at the landmarks: (P W P^T)[b, b] = W
    K = P.toarray() @ prob["W64"] @ P.toarray().T
    lm = prob["landmarks"]
    np.testing.assert_array_equal(K[np.ix_(lm, lm)], prob["W64"])


def test_routes_agree_on_torus64x32():
    prob = configs.torus64x32(use_cache=False)
    P = configs.operator_rounded(prob)
    W = prob["W"]
    for k in (3, 10):
        ld, vd, zd = oeig.top_k(P, W, k, route="dense")
        lr, vr, zr = oeig.top_k(P, W, k, route="reduction")
        la, va, za = oeig.top_k(P, W, k, route="arpack")
        np.testing.assert_allclose(lr, ld, rtol=1e-10)
        np.testing.assert_allclose(la, ld, rtol=1e-10)
        # eigenvectors of simple eigenvalues agree once signs are canonical
        gaps = np.abs(np.diff(ld)) / np.abs(ld[:-1])
        for i in range(k):
            left = i == 0 or gaps[i - 1] > 1e-3
            right = i == k - 1 or gaps[i] > 1e-3
            if left and right:
                np.testing.assert_allclose(vr[:, i], vd[:, i], atol=1e-8)
                np.testing.assert_allclose(va[:, i], vd[:, i], atol=1e-8)


def test_stored_coefficients_reproduce_eigenpairs():
    # the coefficient form the full-size expected values are stored in:
    # V = J P C must be orthonormal, centred and satisfy B V = V diag(lambda)
    # against the dense B (a dropped centering term or a wrong scaling of C
    # fails one of these)
    prob = configs.torus64x32(use_cache=False)
    P = configs.operator_rounded(prob)
    W = prob["W"]
    lam, C = oeig.reduction_coefficients(P, W, 5)
    V = oeig.vectors_from_coefficients(P, C)
    np.testing.assert_allclose(V.T @ V, np.eye(5), atol=1e-10)
    np.testing.assert_allclose(V.sum(axis=0), 0.0, atol=1e-10)
    B = oeig.b_matrix(P, W)
    for i in range(5):
        assert np.linalg.norm(B @ V[:, i] - lam[i] * V[:, i]) <= 1e-9 * abs(lam[0])
    ld, _, _ = oeig.top_k(P, W, 5, route="dense")
    np.testing.assert_allclose(lam, ld, rtol=1e-10)


def test_blockwise_operator_matches_dense_b():
    # the blockwise float64 application of B used for residual checks at
    # sizes where B (and W in float64) cannot be held: equal to the dense B
    # on a torus and on random vectors, for a block size that leaves a ragged
    # last block
    prob = configs.torus64x32(use_cache=False)
    P = configs.operator_rounded(prob)
    W = prob["W"].astype(np.float32)
    X = np.random.default_rng(3).standard_normal((P.shape[0], 4))
    B = oeig.b_matrix(P, W)
    got = oeig.apply_b(P, W, X, chunk_rows=10)
    np.testing.assert_allclose(got, B @ X, rtol=0, atol=1e-11 * np.abs(B @ X).max())


def test_arpack_residuals():
    prob = configs.torus64x32(use_cache=False)
    P = configs.operator_rounded(prob)
    lam, vec, _ = oeig.top_k(P, prob["W"], 3, route="arpack")
    B = oeig.b_matrix(P, prob["W"])
    for i in range(3):
        r = np.linalg.norm(B @ vec[:, i] - lam[i] * vec[:, i])
        assert r <= 1e-10 * abs(lam[0])


def test_landmarks_everywhere_is_classical_mds(small_sphere):
    # l = n gives P = I and B = -1/2 J E J: the textbook classical MDS
    V, F = small_sphere
    n = len(V)
    prob = _chain_problem(V, F, n, None, seed=1)
    P = prob["P64"]
    np.testing.assert_array_equal(P.toarray()[np.ix_(prob["landmarks"], np.arange(n))], np.eye(n))
    E = np.zeros((n, n))
    lm = prob["landmarks"]
    E[np.ix_(lm, lm)] = prob["W64"]
    lam_mds, Z_mds = omds.classical_mds(E, 5)
    for route in ("dense", "reduction", "arpack"):
        lam, _, Z = oeig.top_k(P, prob["W64"], 5, route=route)
        np.testing.assert_allclose(lam, lam_mds, rtol=1e-10)
        np.testing.assert_allclose(np.abs(Z), np.abs(Z_mds), atol=1e-8)


@pytest.mark.parametrize("route", ["dense", "reduction", "arpack"])
def test_euclidean_closed_form(route):
    # W = squared Euclidean distances of landmark points Yl and P with unit
    # row sums give B = J (P Yl)(P Yl)^T J exactly: three positive eigenvalues
    # equal to those of the 3 x 3 Gram (J P Yl)^T (J P Yl), and Z Z^T = that
    # rank-3 matrix.
    rng = np.random.default_rng(3)
    n, l = 300, 40
    Yl = rng.standard_normal((l, 3)) * np.array([3.0, 2.0, 1.0])
    W = ((Yl[:, None, :] - Yl[None, :, :]) ** 2).sum(-1)
    rows, cols, vals = [], [], []
    for i in range(n):
        c = rng.choice(l, size=4, replace=False)
        w = rng.random(4) + 0.1
        w /= w.sum()
        rows += [i] * 4
        cols += list(c)
        vals += list(w)
    P = sp.csr_matrix((vals, (rows, cols)), shape=(n, l))
    X = P @ Yl
    Xc = X - X.mean(axis=0)
    expect = np.sort(np.linalg.eigvalsh(Xc.T @ Xc))[::-1]
    lam, _, Z = oeig.top_k(P, W, 3, route=route)
    np.testing.assert_allclose(lam, expect, rtol=1e-10)
    np.testing.assert_allclose(Z @ Z.T, Xc @ Xc.T, atol=1e-9 * np.abs(Xc).max() ** 2)


def test_vertex_order_invariance(small_sphere):
    V, F = small_sphere
    n = len(V)
    base = _chain_problem(V, F, 20, 6, seed=9)
    rng = np.random.default_rng(12)
    perm = rng.permutation(n)          # new id -> old id
    inv = np.empty(n, dtype=np.int64)
    inv[perm] = np.arange(n)           # old id -> new id
    V2 = V[perm]
    F2 = inv[F]
    prob2 = _chain_problem(V2, F2, 20, 6, landmarks=inv[base["landmarks"]])
    lam1 = oeig.top_k(base["P64"], base["W64"], 6, route="dense")[0]
    lam2 = oeig.top_k(prob2["P64"], prob2["W64"], 6, route="dense")[0]
    np.testing.assert_allclose(lam2, lam1, rtol=1e-9)


def test_rigid_motion_and_scale(small_torus):
    V, F = small_torus
    base = _chain_problem(V, F, 14, 6, seed=21)
    lm = base["landmarks"]
    lam = oeig.top_k(base["P64"], base["W64"], 4, route="dense")[0]
    rng = np.random.default_rng(5)
    Q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    moved = _chain_problem(V @ Q.T + 2.0, F, 14, 6, landmarks=lm)
    np.testing.assert_allclose(oeig.top_k(moved["P64"], moved["W64"], 4, route="dense")[0], lam, rtol=1e-9)
    s = 2.5
    scaled = _chain_problem(s * V, F, 14, 6, landmarks=lm)
    np.testing.assert_allclose(oeig.top_k(scaled["P64"], scaled["W64"], 4, route="dense")[0], lam * s * s,
                               rtol=1e-9)


def test_centering_and_sign_pins():
    # a dropped J or a flipped -1/2 changes the spectrum of this pinned case
    rng = np.random.default_rng(8)
    pts = rng.standard_normal((50, 2)) + np.array([5.0, -3.0])
    E = ((pts[:, None] - pts[None]) ** 2).sum(-1)
    lam, Z = omds.classical_mds(E, 2)
    c = pts - pts.mean(0)
    np.testing.assert_allclose(lam, np.sort(np.linalg.eigvalsh(c.T @ c))[::-1], rtol=1e-10)
    assert omds.strain(Z, E) < 1e-9 * np.abs(E).max()
    # for Euclidean points -1/2 J E J is the Gram matrix of the centred points,
    # whose nonzero eigenvalues are those of c^T c: the empty embedding has
    # stress sqrt(l1^2 + l2^2), the one-dimensional one has stress l2
    g = np.sort(np.linalg.eigvalsh(c.T @ c))[::-1]
    assert abs(omds.strain(np.zeros((50, 1)), E) - np.hypot(g[0], g[1])) <= 1e-9 * g[0]
    assert abs(omds.strain(Z[:, :1], E) - g[1]) <= 1e-9 * g[0]


def test_sphere_spectrum_funk_hecke():
    # Own derivation (not in the paper): for squared geodesic distances on
    # the unit sphere, -1/2 J E J has eigenvalues mu_l = -(n/4) int
    # arccos(t)^2 P_l(t) dt; mu_1 / mu_3 = 16 and mu_1 / |mu_2| = 5.55 with
    # multiplicities 3, 5, 7.  Graph distances on a level-3 icosphere land
    # within 10%.
    V, F = meshes.icosphere(3)
    G = op.edge_graph(V, F)
    D = csgraph.dijkstra(G, directed=False)
    lam, _ = omds.classical_mds(D ** 2, 20)
    full = np.linalg.eigvalsh(-0.5 * (omds.centering(len(V)) @ (D ** 2) @ omds.centering(len(V))))
    mu1 = lam[:3].mean()
    mu3 = lam[3:10].mean()
    neg = np.sort(full)[:5].mean()
    assert abs(mu1 / mu3 - 16.0) / 16.0 < 0.1
    assert abs(mu1 / abs(neg) - 5.55) / 5.55 < 0.1
    np.testing.assert_allclose(lam[:3], mu1, rtol=1e-2)


def test_approximation_improves_with_landmarks():
    # sBHA approximates the full squared-distance matrix better as l grows
    # (Section 4.1); the paper's curves are stripped, so only the trend and
    # p_row = 50 ~ dense are gated (tolerance unpinned by the paper).
    V, F = meshes.torus_grid(24, 12, 1.0, 0.4, jitter=0.01, seed=2)
    G = op.edge_graph(V, F)
    D = csgraph.dijkstra(G, directed=False)
    E = D ** 2
    errs = []
    for l in (10, 25, 60):
        pr = _chain_problem(V, F, l, None, seed=4)
        Pd = pr["P64"].toarray()
        errs.append(omds.approx_error(Pd @ pr["W64"] @ Pd.T, E))
    assert errs[0] > errs[1] > errs[2]
    pr50 = _chain_problem(V, F, 25, 50, seed=4)
    Pd = pr50["P64"].toarray()
    e50 = omds.approx_error(Pd @ pr50["W64"] @ Pd.T, E)
    assert e50 < 1.2 * errs[1]


def test_synthetic_grid_torus_operator_structure():
    # the large synthetic operators: identity rows at the landmarks, every
    # other row its nbr nearest grid landmarks with weights summing to 1 and
    # increasing column ids, W exactly symmetric with a zero diagonal; the
    # batch recipe's sizes and landmark counts
    from synth import large
    p = large.grid_torus_operator(nu=90, nv=60, lu=12, lv=10, nbr=10, seed=3)
    n, l = p["n"], p["l"]
    assert (n, l) == (5400, 120)
    P = sp.csr_matrix((p["val"].astype(np.float64), p["col"], p["rowptr"]), shape=(n, l))
    np.testing.assert_allclose(np.asarray(P.sum(axis=1)).ravel(), 1.0, atol=1e-6)
    lm = p["landmarks"]
    assert len(np.unique(lm)) == l
    np.testing.assert_array_equal(P[lm].toarray(), np.eye(l))
    lens = np.diff(p["rowptr"])
    others = np.setdiff1d(np.arange(n), lm)
    assert np.all(lens[others] == 10) and np.all(lens[lm] == 1)
    for i in others[::37]:
        c = p["col"][p["rowptr"][i]:p["rowptr"][i + 1]]
        assert np.all(np.diff(c) > 0)
    W = p["W"]
    assert W.dtype == np.float32 and np.array_equal(W, W.T) and np.all(np.diag(W) == 0) and np.all(W >= 0)
    batch = large.grid_torus_batch(count=6, nmin=2000, nmax=6000, seed0=11)
    for q in batch:
        assert 2000 * 0.9 <= q["n"] <= 6000 * 1.1 and 25 <= q["l"] and abs(q["l"] - q["n"] / 50) <= 0.35 * q["n"] / 50


# ------------------------------------------- sign convention and error measure
def test_canonical_signs_hand_built():
    # the entry of largest magnitude ends up positive; on a tie of magnitudes
    # the lowest index decides; columns are independent; values are kept
    V = np.array([[0.1, -0.5, 0.3, 2.0],
                  [-0.9, 0.5, -0.3, -1.0],
                  [0.2, 0.1, 0.1, 0.5]])
    got = oeig.canonical_signs(V)
    want = np.array([[-0.1, 0.5, 0.3, 2.0],      # col 0: -0.9 largest -> flipped
                     [0.9, -0.5, -0.3, -1.0],    # col 1: |-0.5| = |0.5|, row 0 first -> flipped
                     [-0.2, -0.1, 0.1, 0.5]])    # col 2: |0.3| tie, row 0 (+) first -> kept
    np.testing.assert_array_equal(got, want)     # col 3: 2.0 largest and positive -> kept
    assert np.array_equal(V[:, 0], [0.1, -0.9, 0.2])  # input untouched
    # idempotent, and the same for v and -v
    np.testing.assert_array_equal(oeig.canonical_signs(got), got)
    np.testing.assert_array_equal(oeig.canonical_signs(-V), want)


def test_approx_error_hand_computed():
    # eps = ||K~ - K||_F^2 / ||K||_F^2 (Section 4.1) on a 3 x 3 case by hand:
    # K has squared entries 0,1,4 / 1,0,9 / 4,9,0 -> ||K||^2 = 2(1 + 16 + 81) = 196;
    # K~ differs by +1 at (0,1), (1,0) and by -2 at (2,2) -> ||diff||^2 = 1 + 1 + 4 = 6
    K = np.array([[0.0, 1.0, 4.0], [1.0, 0.0, 9.0], [4.0, 9.0, 0.0]])
    Kt = K.copy()
    Kt[0, 1] += 1.0
    Kt[1, 0] += 1.0
    Kt[2, 2] -= 2.0
    assert omds.approx_error(Kt, K) == pytest.approx(6.0 / 196.0, rel=1e-15)
    assert omds.approx_error(K, K) == 0.0
    # scale invariant in the pair, quadratic in the perturbation
    assert omds.approx_error(3 * Kt, 3 * K) == pytest.approx(6.0 / 196.0, rel=1e-14)
    assert omds.approx_error(K + 2 * (Kt - K), K) == pytest.approx(24.0 / 196.0, rel=1e-14)


def test_coefficients_from_vectors_dense_route():
    # every eigenvector of B with a non-zero eigenvalue lies in range(J P):
    # v = J P c with c = -1/2 W P^T J v / lambda (Section 3.3's factored B);
    # checked against the dense route's eigenvectors
    rng = np.random.default_rng(8)
    n, l = 60, 9
    P = sp.random(n, l, density=0.4, random_state=3, format="csr") + sp.csr_matrix(
        (np.ones(l), (rng.choice(n, l, replace=False), np.arange(l))), shape=(n, l))
    pts = rng.standard_normal((l, 3))
    W = ((pts[:, None] - pts[None]) ** 2).sum(-1)
    W = W + 0.3 * np.sqrt(W)
    lam, V, _ = oeig.top_k(P, W, 4, route="dense")
    C = oeig.coefficients_from_vectors(P, W, lam, V)
    np.testing.assert_allclose(oeig.vectors_from_coefficients(P, C), V, atol=1e-12)
    B = oeig.b_matrix(P, W)
    np.testing.assert_allclose(B @ V, V * lam[None, :], atol=1e-10 * abs(lam).max())


def test_approx_rows_special_cases():
    # rows of K~ = P L P^T: with l = n and P = I (Section 3.1's limit) K~ = L
    # exactly and eps = 0; a landmark's row of K~ interpolates row j of L
    # (its P row is e_j, Eq. (PDefinition)); the row-subset error over all
    # rows is the full-matrix error
    rng = np.random.default_rng(4)
    n = 30
    pts = rng.standard_normal((n, 3))
    K = np.sqrt(((pts[:, None] - pts[None]) ** 2).sum(-1))
    rows = np.array([0, 7, 29])
    np.testing.assert_array_equal(omds.approx_rows(sp.identity(n, format="csr"), K, rows), K[rows])
    assert omds.approx_error_rows(sp.identity(n, format="csr"), K, rows, K[rows]) == 0.0
    V, F = meshes.torus_grid(12, 8, 1.0, 0.4, jitter=0.01, seed=3)
    pr = _chain_problem(V, F, 10, None, seed=2)
    P = pr["P64"]
    G = op.edge_graph(V, F)
    D = csgraph.dijkstra(G, directed=False)
    lm = pr["landmarks"]
    Kll = D[np.ix_(lm, lm)]
    Kt = omds.approx_rows(P, Kll, lm[:3])
    np.testing.assert_allclose(Kt, (P @ Kll.T).T[:3], atol=1e-12)
    full = omds.approx_error(P.toarray() @ Kll @ P.toarray().T, D)
    np.testing.assert_allclose(omds.approx_error_rows(P, Kll, np.arange(V.shape[0]), D), full, rtol=1e-12)
