"""CPU oracle of the embedding path: top-k classical scaling of B = -1/2 J P W P^T J.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package; only
the tests, the smoke check and the CPU-baseline leg of the benchmark do.

What it computes (Sections 2.3 and 3.3 of the paper): with J = I - 11^T/n the
centering matrix, the classical-scaling matrix built from the sparse
biharmonic approximation of the squared distances is
        B = -1/2 * J * P * W * P^T * J           (n x n, symmetric)
and the embedding keeps its k algebraically largest eigenpairs
(lambda_i, v_i):  Z = V_k * Lambda_k^{1/2}  (Section 2.3, classical MDS).
Coordinates whose eigenvalue is not positive are set to zero.

Everything is float64.  Three routes reach the same eigenpairs:

* ``dense``     forms B explicitly and calls numpy.linalg.eigh (n <= ~4096);
* ``reduction`` uses the Gram matrix of A = J P (l x l) -- the paper's BMDS
                reduction of Section 3.3 written with an eigendecomposition of
                A^T A in place of the QR of J P (so a rank-deficient J P does
                not break it);
* ``arpack``    runs scipy.sparse.linalg.eigsh on the implicit operator
                v -> -1/2 J (P (W (P^T (J v)))), the matrix-vector form the
                paper proposes for sBMDS (Section 3.3).

Eigenvector signs are made canonical: the entry of largest magnitude
(lowest index on ties) is positive.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

__all__ = ["b_matrix", "top_k", "embed", "canonical_signs", "centered_gram", "reduction_coefficients",
           "vectors_from_coefficients", "coefficients_from_vectors", "apply_b"]


def _as_csr64(P) -> sp.csr_matrix:
    P = sp.csr_matrix(P)
    return sp.csr_matrix((P.data.astype(np.float64), P.indices, P.indptr), shape=P.shape)


def b_matrix(P, W) -> np.ndarray:
    """Dense B = -1/2 J P W P^T J (float64).  For small n only."""
    P = _as_csr64(P)
    n = P.shape[0]
    Pd = P.toarray()
    K = Pd @ np.asarray(W, dtype=np.float64) @ Pd.T
    J = np.eye(n) - np.full((n, n), 1.0 / n)
    return -0.5 * (J @ K @ J)


def canonical_signs(Vk: np.ndarray) -> np.ndarray:
    """Flip each column so that its largest-magnitude entry is positive."""
    Vk = np.array(Vk, dtype=np.float64, copy=True)
    for j in range(Vk.shape[1]):
        i = int(np.argmax(np.abs(Vk[:, j])))
        if Vk[i, j] < 0:
            Vk[:, j] = -Vk[:, j]
    return Vk


def _finish(lam: np.ndarray, vec: np.ndarray, k: int):
    order = np.argsort(-lam, kind="stable")[:k]
    lam = lam[order]
    vec = canonical_signs(vec[:, order])
    Z = vec * np.sqrt(np.clip(lam, 0.0, None))[None, :]
    return lam, vec, Z


def _top_dense(P, W, k):
    B = b_matrix(P, W)
    lam, vec = np.linalg.eigh(B)
    return _finish(lam, vec, k)


def centered_gram(P) -> np.ndarray:
    """A^T A for A = J P:  P^T P - c c^T / n with c = P^T 1 (dense l x l)."""
    P = _as_csr64(P)
    n = P.shape[0]
    c = np.asarray(P.sum(axis=0)).ravel()
    G = (P.T @ P).toarray()
    return G - np.outer(c, c) / n


def reduction_coefficients(P, W, k, rank_tol=1e-12):
    """The reduction route's k largest eigenvalues of B and coefficients C
    (l x k) with eigenvectors V = J P C (orthonormal columns)."""
    P = _as_csr64(P)
    W = np.asarray(W, dtype=np.float64)
    G = centered_gram(P)
    sig, Ug = np.linalg.eigh(G)
    keep = sig > rank_tol * max(sig.max(), 0.0)
    sig = sig[keep]
    Ug = Ug[:, keep]
    sh = np.sqrt(sig)
    # Columns of A U Sigma^{-1/2} are orthonormal and span range(J P), which
    # holds every eigenvector of B with a non-zero eigenvalue.
    S = -0.5 * (sh[:, None] * (Ug.T @ W @ Ug) * sh[None, :])
    S = 0.5 * (S + S.T)
    lam, Yr = np.linalg.eigh(S)
    order = np.argsort(-lam, kind="stable")[:k]
    return lam[order], Ug @ (Yr[:, order] / sh[:, None])


def vectors_from_coefficients(P, coef) -> np.ndarray:
    """V = J P C (n x k) for coefficients from reduction_coefficients."""
    P = _as_csr64(P)
    n = P.shape[0]
    coef = np.asarray(coef, dtype=np.float64)
    c = np.asarray(P.sum(axis=0)).ravel()
    return P @ coef - np.outer(np.ones(n), c @ coef) / n


def coefficients_from_vectors(P, W, lam, V) -> np.ndarray:
    """Coefficients C (l x k) with V = J P C for eigenpairs (lam, V) of B with
    non-zero eigenvalues: B v = lam v gives v = J P (-1/2 W P^T J v / lam),
    so every such eigenvector lies in range(J P) (Section 3.3's factored B).
    W may be float32; it is widened a block of rows at a time."""
    P = _as_csr64(P)
    V = np.asarray(V, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    T = P.T @ (V - V.mean(axis=0, keepdims=True))
    l = T.shape[0]
    U = np.empty_like(T)
    for r0 in range(0, l, 1024):
        r1 = min(l, r0 + 1024)
        U[r0:r1] = np.asarray(W[r0:r1], dtype=np.float64) @ T
    return -0.5 * U / lam[None, :]


def apply_b(P, W, X, chunk_rows=1024) -> np.ndarray:
    """B X = -1/2 J P W P^T J X in float64 for X (n x k), taking W a block of
    rows at a time (widened to float64 per block), so that a W too large to
    hold in float64 (l = 50,000: 10 GB in float32) can still be applied."""
    P = _as_csr64(P)
    X = np.asarray(X, dtype=np.float64)
    Xc = X - X.mean(axis=0, keepdims=True)
    T = P.T @ Xc
    l = T.shape[0]
    U = np.empty_like(T)
    for r0 in range(0, l, chunk_rows):
        r1 = min(l, r0 + chunk_rows)
        U[r0:r1] = np.asarray(W[r0:r1], dtype=np.float64) @ T
    Y = P @ U
    Y -= Y.mean(axis=0, keepdims=True)
    return -0.5 * Y


def _top_reduction(P, W, k, rank_tol=1e-12):
    lam, coef = reduction_coefficients(P, W, k, rank_tol)
    return _finish(lam, vectors_from_coefficients(P, coef), k)


def _top_arpack(P, W, k, tol=1e-12, ncv=None, v0_seed=0):
    P = _as_csr64(P)
    n, l = P.shape
    W = np.asarray(W, dtype=np.float64)
    PT = P.T.tocsr()

    def mv(x):
        x = np.asarray(x, dtype=np.float64).reshape(n, -1)
        xc = x - x.mean(axis=0, keepdims=True)
        y = P @ (W @ (PT @ xc))
        y = y - y.mean(axis=0, keepdims=True)
        return -0.5 * y

    op = spla.LinearOperator((n, n), matvec=mv, matmat=mv, dtype=np.float64)
    if ncv is None:
        ncv = min(n - 1, max(2 * k + 20, 40))
    v0 = np.random.default_rng(v0_seed).standard_normal(n)
    lam, vec = spla.eigsh(op, k=k, which="LA", tol=tol, ncv=ncv, v0=v0)
    return _finish(lam, vec, k)


def top_k(P, W, k: int, route: str = "auto", **kw):
    """k algebraically largest eigenpairs of B and the embedding.

    Returns (eigenvalues [k] descending, eigenvectors [n,k] canonical signs,
    Z [n,k]).  ``route`` is 'dense', 'reduction', 'arpack' or 'auto'
    (dense for n <= 4096, reduction for l <= 12000, arpack otherwise).
    """
    P = _as_csr64(P)
    n, l = P.shape
    if route == "auto":
        route = "dense" if n <= 4096 else ("reduction" if l <= 12000 else "arpack")
    if route == "dense":
        return _top_dense(P, W, k)
    if route == "reduction":
        return _top_reduction(P, W, k, **kw)
    if route == "arpack":
        return _top_arpack(P, W, k, **kw)
    raise ValueError(f"unknown route {route!r}")


def embed(P, W, k: int, route: str = "auto", **kw) -> np.ndarray:
    """Z = V_k Lambda_k^{1/2} (n x k), non-positive eigenvalues clamped to 0."""
    return top_k(P, W, k, route=route, **kw)[2]
