"""Brute-force CPU reference of the input chain, for tiny meshes only.

TEST INFRASTRUCTURE ONLY (see the package docstring).  These functions are
slow, dense and written independently of the generator they are used to
check: per-triangle Python loops, Heron's formula for areas, angles from
atan2, a dense linear solve for P, full sorting for the threshold, an
all-pairs Floyd-Warshall for geodesics and a literal farthest-point loop.

* cotangent weights, lumped mass, V and M = (V-A)^T D^-1 (V-A): Section 2.2
* interpolation operator P = [I; -M_uu^-1 M_ub]: Eq. (PDefinition)
* per-column thresholding to the p largest magnitudes: Section 3.1
* farthest-point landmarks: Eq. (FarthestPoint)
"""
from __future__ import annotations

import heapq
import math

import numpy as np

__all__ = [
    "cot_adjacency_dense",
    "mass_dense",
    "biharmonic_dense",
    "graph_biharmonic_dense",
    "floyd_warshall",
    "dijkstra_heap",
    "fps_literal",
    "interp_dense",
    "threshold_sorted",
]


def _angle(a, b, c):
    """Interior angle at vertex a of triangle (a, b, c)."""
    u = [b[i] - a[i] for i in range(3)]
    v = [c[i] - a[i] for i in range(3)]
    cx = (u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0])
    s = math.sqrt(cx[0] ** 2 + cx[1] ** 2 + cx[2] ** 2)
    d = u[0] * v[0] + u[1] * v[1] + u[2] * v[2]
    return math.atan2(s, d)


def cot_adjacency_dense(V, F) -> np.ndarray:
    """A_ij = (cot alpha_ij + cot beta_ij) / 2 summed over the triangles on
    edge ij (one triangle on a boundary edge)."""
    n = len(V)
    A = np.zeros((n, n))
    for tri in F:
        for k in range(3):
            o, i, j = int(tri[k]), int(tri[(k + 1) % 3]), int(tri[(k + 2) % 3])
            ang = _angle(V[o], V[i], V[j])
            w = 0.5 / math.tan(ang)
            A[i, j] += w
            A[j, i] += w
    return A


def mass_dense(V, F) -> np.ndarray:
    """D_ii = (1/3) * sum of the areas (Heron) of the triangles at vertex i."""
    n = len(V)
    d = np.zeros(n)
    for tri in F:
        p = [np.asarray(V[int(t)], dtype=np.float64) for t in tri]
        a = float(np.linalg.norm(p[1] - p[2]))
        b = float(np.linalg.norm(p[0] - p[2]))
        c = float(np.linalg.norm(p[0] - p[1]))
        # Kahan's numerically stable form of Heron's formula
        x, y, z = sorted([a, b, c], reverse=True)
        area = 0.25 * math.sqrt(max((x + (y + z)) * (z - (x - y)) * (z + (x - y)) * (x + (y - z)), 0.0))
        for t in tri:
            d[int(t)] += area / 3.0
    return d


def biharmonic_dense(V, F):
    """Returns (M, L, d) with L = V - A and M = L^T D^-1 L, all dense."""
    A = cot_adjacency_dense(V, F)
    L = np.diag(A.sum(axis=1)) - A
    d = mass_dense(V, F)
    M = L.T @ np.diag(1.0 / d) @ L
    return M, L, d


def graph_biharmonic_dense(n, F):
    """Generic-graph variant: D = I, A = 0/1 edge adjacency."""
    A = np.zeros((n, n))
    for tri in F:
        for k in range(3):
            i, j = int(tri[k]), int(tri[(k + 1) % 3])
            A[i, j] = 1.0
            A[j, i] = 1.0
    L = np.diag(A.sum(axis=1)) - A
    return L.T @ L


def floyd_warshall(V, F) -> np.ndarray:
    """All-pairs shortest path lengths over mesh edges (Euclidean weights)."""
    n = len(V)
    D = np.full((n, n), np.inf)
    np.fill_diagonal(D, 0.0)
    for tri in F:
        for k in range(3):
            i, j = int(tri[k]), int(tri[(k + 1) % 3])
            w = float(np.linalg.norm(np.asarray(V[i]) - np.asarray(V[j])))
            D[i, j] = min(D[i, j], w)
            D[j, i] = min(D[j, i], w)
    for m in range(n):
        D = np.minimum(D, D[:, m:m + 1] + D[m:m + 1, :])
    return D


def dijkstra_heap(n, edges, src):
    """Textbook Dijkstra with a binary heap; edges = list of (i, j, w)."""
    adj = [[] for _ in range(n)]
    for i, j, w in edges:
        adj[i].append((j, w))
        adj[j].append((i, w))
    dist = [math.inf] * n
    dist[src] = 0.0
    pq = [(0.0, src)]
    while pq:
        d, v = heapq.heappop(pq)
        if d > dist[v]:
            continue
        for u, w in adj[v]:
            nd = d + w
            if nd < dist[u]:
                dist[u] = nd
                heapq.heappush(pq, (nd, u))
    return np.array(dist)


def fps_literal(D: np.ndarray, l: int, first: int) -> np.ndarray:
    """Eq. (FarthestPoint) on a full distance matrix: each new landmark is
    argmax_x min_t D[b_t, x] (lowest index on ties)."""
    lm = [first]
    for _ in range(1, l):
        mind = D[lm, :].min(axis=0)
        lm.append(int(np.argmax(mind)))
    return np.array(lm)


def threshold_sorted(x: np.ndarray, p: int) -> np.ndarray:
    """Indices of the p largest |x_i| by a full sort on (-|x_i|, i); exact
    zeros are dropped.  Returned ascending."""
    order = sorted(range(len(x)), key=lambda i: (-abs(x[i]), i))
    keep = [i for i in order[:p] if x[i] != 0.0]
    return np.array(sorted(keep), dtype=np.int64)


def interp_dense(M: np.ndarray, landmarks, p: int | None = None) -> np.ndarray:
    """Dense n x l P of Eq. (PDefinition) in original vertex order, with
    optional per-column thresholding of the non-landmark block."""
    n = M.shape[0]
    landmarks = np.asarray(landmarks)
    l = len(landmarks)
    u = np.array([i for i in range(n) if i not in set(landmarks.tolist())])
    Pu = -np.linalg.solve(M[np.ix_(u, u)], M[np.ix_(u, landmarks)])
    if p is not None:
        for j in range(l):
            keep = threshold_sorted(Pu[:, j], p)
            col = np.zeros(len(u))
            col[keep] = Pu[keep, j]
            Pu[:, j] = col
    P = np.zeros((n, l))
    P[landmarks, np.arange(l)] = 1.0
    P[u, :] = Pu
    return P
