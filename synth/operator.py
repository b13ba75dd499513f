"""The inputs of the eigensolve: sparse interpolation operator P and W = D^2_ll.

This is the input chain of the method (the paper's Sections 2.2, 3 and 3.1),
written for speed on the CPU with SciPy sparse routines.  It produces the two
arrays the embedding path consumes, and nothing of the path itself (no
centering, no products with P or W, no eigensolve).

* cotangent weights and lumped mass (Section 2.2): A_ij = (cot a_ij + cot b_ij)/2,
  D_ii = one third of the area of the triangles around vertex i,
  V_ii = sum_j A_ij;
* discrete biharmonic operator M = (V - A)^T D^-1 (V - A) (Section 2.2);
* farthest-point landmarks, Eq. (FarthestPoint), with geodesics taken as
  Dijkstra shortest paths over mesh edges (Euclidean edge lengths);
* W = squared landmark-to-landmark geodesic distance (the matrix classical
  scaling needs, Section 3.3), symmetrised in float64 with a zero diagonal;
* P = [I; -M_uu^-1 M_ub] of Eq. (PDefinition), thresholded per column to the
  p entries of largest magnitude (Section 3.1), with p = (n - l) p_row / l.

Readings of points the paper leaves open (each also listed in the design
notes of the repository):
  p is rounded half up and clamped to [1, n - l]; ties in magnitude go to the
  lower vertex id; exact zeros are never stored; rows are not renormalised
  after thresholding; P is returned in original vertex order with identity
  rows at the landmark vertices; the first landmark is
  ``default_rng(seed).integers(n)`` and argmax ties go to the lowest id.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = [
    "cotan_weights",
    "lumped_mass",
    "laplacian",
    "biharmonic",
    "edge_graph",
    "farthest_point_landmarks",
    "landmark_sq_distances",
    "p_from_prow",
    "interpolation_operator",
    "threshold_column",
]


def _n_workers() -> int:
    env = os.environ.get("SBMDS_GEN_THREADS")
    if env:
        return max(1, int(env))
    return max(1, min(16, os.cpu_count() or 1))


def cotan_weights(V: np.ndarray, F: np.ndarray) -> sp.csr_matrix:
    """Symmetric weighted adjacency A with A_ij = (cot alpha_ij + cot beta_ij)/2.

    Each triangle contributes half the cotangent of its angle at the vertex
    opposite an edge to that edge's weight.  Obtuse angles give negative
    cotangents; they are kept (no intrinsic-Delaunay flip).
    """
    n = V.shape[0]
    rows, cols, vals = [], [], []
    for k in range(3):
        i = F[:, (k + 1) % 3]
        j = F[:, (k + 2) % 3]
        o = F[:, k]
        e1 = V[i] - V[o]
        e2 = V[j] - V[o]
        dot = np.einsum("ij,ij->i", e1, e2)
        crs = np.linalg.norm(np.cross(e1, e2), axis=1)
        cot = dot / crs
        rows += [i, j]
        cols += [j, i]
        vals += [0.5 * cot, 0.5 * cot]
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(n, n)).tocsr()
    A.sum_duplicates()
    return A


def lumped_mass(V: np.ndarray, F: np.ndarray) -> np.ndarray:
    """Diagonal of D: one third of the total area of the incident triangles."""
    n = V.shape[0]
    area = 0.5 * np.linalg.norm(np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]]), axis=1)
    d = np.zeros(n)
    for k in range(3):
        np.add.at(d, F[:, k], area / 3.0)
    return d


def laplacian(A: sp.csr_matrix) -> sp.csr_matrix:
    """L = V - A with V_ii = sum_j A_ij."""
    deg = np.asarray(A.sum(axis=1)).ravel()
    return (sp.diags(deg) - A).tocsr()


def biharmonic(V: np.ndarray, F: np.ndarray, graph: bool = False) -> sp.csr_matrix:
    """M = (V - A)^T D^-1 (V - A).

    With ``graph=True`` the generic-graph variant is used: D = I and A the
    0/1 adjacency of the mesh edges.
    """
    if graph:
        n = V.shape[0]
        e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], 0)
        A = sp.coo_matrix((np.ones(2 * len(e)),
                           (np.concatenate([e[:, 0], e[:, 1]]), np.concatenate([e[:, 1], e[:, 0]]))),
                          shape=(n, n)).tocsr()
        A.data[:] = 1.0
        d = np.ones(n)
    else:
        A = cotan_weights(V, F)
        d = lumped_mass(V, F)
    L = laplacian(A)
    M = (L.T @ sp.diags(1.0 / d) @ L).tocsr()
    M.sum_duplicates()
    M.sort_indices()
    return M


def edge_graph(V: np.ndarray, F: np.ndarray) -> sp.csr_matrix:
    """Symmetric sparse graph of mesh edges weighted by Euclidean length."""
    n = V.shape[0]
    e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], 0)
    e = np.unique(np.sort(e, axis=1), axis=0)
    w = np.linalg.norm(V[e[:, 0]] - V[e[:, 1]], axis=1)
    G = sp.coo_matrix((np.concatenate([w, w]), (np.concatenate([e[:, 0], e[:, 1]]),
                                                np.concatenate([e[:, 1], e[:, 0]]))),
                      shape=(n, n)).tocsr()
    return G


def farthest_point_landmarks(G: sp.csr_matrix, l: int, seed: int | None = None,
                             first: int | None = None) -> np.ndarray:
    """Eq. (FarthestPoint): first landmark at random, then repeatedly the
    vertex with the largest minimum geodesic distance to those chosen
    (lowest vertex id on ties).  Runs in the native helper."""
    from . import _geodesic

    n = G.shape[0]
    if first is None:
        first = int(np.random.default_rng(seed).integers(n))
    return _geodesic.fps(G, l, first)


def landmark_sq_distances(G: sp.csr_matrix, landmarks: np.ndarray) -> np.ndarray:
    """W_ij = d(b_i, b_j)^2 by Dijkstra, symmetrised in float64, zero diagonal."""
    from . import _geodesic

    D = _geodesic.sssp_to(G, landmarks, landmarks, _n_workers())
    W = D * D
    W = 0.5 * (W + W.T)
    np.fill_diagonal(W, 0.0)
    return W


def p_from_prow(n: int, l: int, p_row: float) -> int:
    """p = (n - l) p_row / l rounded half up, clamped to [1, n - l]."""
    p = math.floor((n - l) * p_row / l + 0.5)
    return int(min(max(p, 1), n - l))


def threshold_column(x: np.ndarray, p: int) -> np.ndarray:
    """Indices (ascending) of the p entries of largest magnitude.

    Ties at the cut go to the lower index; exact zeros are never kept.
    """
    a = np.abs(x)
    nz = np.count_nonzero(a)
    if p >= nz:
        return np.flatnonzero(a)
    thr = np.partition(a, a.size - p)[a.size - p]
    above = np.flatnonzero(a > thr)
    ties = np.flatnonzero(a == thr)
    keep = np.concatenate([above, ties[: p - above.size]])
    keep.sort()
    return keep


def interpolation_operator(M: sp.csr_matrix, landmarks: np.ndarray, p: int | None,
                           block: int = 64):
    """Sparse P (n x l CSR, float64) of Eq. (PDefinition) thresholded per column.

    Rows are in original vertex order; row landmarks[j] is e_j.  With
    ``p=None`` the dense (unthresholded) P_u is kept in full.
    Returns (P csr_matrix, info dict).
    """
    n = M.shape[0]
    l = len(landmarks)
    is_lm = np.zeros(n, dtype=bool)
    is_lm[landmarks] = True
    u = np.flatnonzero(~is_lm)
    Mc = M.tocsc()
    Muu = Mc[u][:, u].tocsc()
    Mub = Mc[u][:, landmarks].tocsc()
    lu = spla.splu(Muu, permc_spec="COLAMD")
    m = len(u)
    keep_all = p is None or p >= m

    starts = list(range(0, l, block))

    def solve(s):
        e = min(s + block, l)
        rhs = -Mub[:, s:e].toarray()
        X = lu.solve(rhs)
        out = []
        for c in range(e - s):
            x = X[:, c]
            idx = np.flatnonzero(x) if keep_all else threshold_column(x, p)
            out.append((idx, x[idx]))
        return out

    col_rows, col_vals = [], []
    with ThreadPoolExecutor(_n_workers()) as ex:
        for res in ex.map(solve, starts):
            for idx, vals in res:
                col_rows.append(u[idx])
                col_vals.append(vals)
    counts = np.array([len(r) for r in col_rows], dtype=np.int64)
    rows = np.concatenate([np.concatenate(col_rows), landmarks])
    cols = np.concatenate([np.repeat(np.arange(l), counts), np.arange(l)])
    vals = np.concatenate([np.concatenate(col_vals), np.ones(l)])
    P = sp.csr_matrix((vals, (rows, cols)), shape=(n, l))
    P.sort_indices()
    info = {"p": p, "col_counts": counts, "nnz": P.nnz}
    return P, info
