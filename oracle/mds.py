"""Classical MDS and quality measures on full matrices (small n only).

TEST INFRASTRUCTURE ONLY (see the package docstring).

* classical MDS, Section 2.3: eigendecomposition of -1/2 J E J, keep the
  largest eigenvalues, Z = V_m Lambda_m^{1/2};
* the objective of Eq. (MDS_problem), ||Z Z^T + 1/2 J E J||_F, which the
  experiments call stress (Section 4.2);
* relative approximation error eps(K~) = ||K~ - K||_F^2 / ||K||_F^2
  (Section 4.1), also on a subset of rows of the sparse biharmonic
  approximation K~ = P L P^T (L the landmark block of the matrix being
  approximated: distances for Section 4.1's geodesic distance matrix).
"""
from __future__ import annotations

import numpy as np

__all__ = ["centering", "classical_mds", "strain", "approx_error", "approx_rows", "approx_error_rows"]


def centering(n: int) -> np.ndarray:
    return np.eye(n) - np.full((n, n), 1.0 / n)


def classical_mds(E: np.ndarray, m: int):
    """Returns (eigenvalues [m] descending, Z [n,m]) of classical MDS on the
    squared-distance matrix E."""
    n = E.shape[0]
    J = centering(n)
    Bf = -0.5 * (J @ E @ J)
    lam, vec = np.linalg.eigh(0.5 * (Bf + Bf.T))
    order = np.argsort(-lam, kind="stable")[:m]
    lam = lam[order]
    vec = vec[:, order]
    return lam, vec * np.sqrt(np.clip(lam, 0.0, None))[None, :]


def strain(Z: np.ndarray, E: np.ndarray) -> float:
    n = E.shape[0]
    J = centering(n)
    return float(np.linalg.norm(Z @ Z.T + 0.5 * (J @ E @ J), "fro"))


def approx_error(K_approx: np.ndarray, K: np.ndarray) -> float:
    return float(np.linalg.norm(K_approx - K, "fro") ** 2 / np.linalg.norm(K, "fro") ** 2)


def approx_rows(P, L, rows) -> np.ndarray:
    """Rows `rows` of K~ = P L P^T (dense |rows| x n, float64): row s is
    P[s, :] L P^T, i.e. the landmark block interpolated to every vertex."""
    import scipy.sparse as sp
    P = sp.csr_matrix(P, dtype=np.float64)
    L = np.asarray(L, dtype=np.float64)
    Ps = P[np.asarray(rows)].toarray()
    return (P @ (L @ Ps.T)).T


def approx_error_rows(P, L, rows, K_rows) -> float:
    """eps(K~) restricted to the rows `rows`: ||K~_S - K_S||_F^2 / ||K_S||_F^2."""
    return approx_error(approx_rows(P, L, rows), np.asarray(K_rows, dtype=np.float64))
