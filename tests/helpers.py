"""Comparison helpers shared by the GPU parity tests."""
import numpy as np
import scipy.sparse as sp

from oracle import eig as oeig
from synth import configs


def rel_eig_err(got, ref):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.max(np.abs(got - ref) / np.abs(ref)))


def gap_closed_sets(lam, k, rel=1e-3):
    """Index sets that cover the wanted k values, closed under near-ties."""
    sets, i = [], 0
    while i < k:
        j = i
        while j + 1 < len(lam) and abs(lam[j] - lam[j + 1]) <= rel * max(abs(lam[j]), abs(lam[j + 1])):
            j += 1
        sets.append(list(range(i, j + 1)))
        i = j + 1
    return sets


def subspace_angle(Z, V_ref, lam_ref, k, tol=None):
    """Largest principal angle between span(Z[:, S]) and span(V_ref[:, S]) over
    the gap-separated clusters S of the k wanted eigenvalues.  A cluster that
    straddles the cut at k has no unique wanted subspace and is skipped (its
    eigenvalues are still gated).

    With ``tol`` (the relative eigenvalue accuracy the solve certified) the
    angle is returned relative to what that accuracy implies: a Ritz pair
    with |theta - lambda| <= tol |lambda| from the quadratic residual bound
    has residual r <= sqrt(tol |lambda| gap) and angle <= r / gap, so the
    value returned is max over clusters of angle / (sqrt(tol |lambda| / gap)).
    """
    worst = 0.0
    for S in gap_closed_sets(lam_ref, k):
        if S[-1] >= k or lam_ref[S[-1]] <= 0:
            continue
        A = np.asarray(Z[:, S], dtype=np.float64)
        A = A - A.mean(axis=0, keepdims=True)
        Qa, _ = np.linalg.qr(A)
        Qb, _ = np.linalg.qr(V_ref[:, S])
        s = np.linalg.svd(Qa.T @ Qb, compute_uv=False)
        ang = float(np.arccos(np.clip(s.min(), -1.0, 1.0)))
        if tol is not None:
            gaps = []
            if S[0] > 0:
                gaps.append(lam_ref[S[0] - 1] - lam_ref[S[0]])
            if S[-1] + 1 < len(lam_ref):
                gaps.append(lam_ref[S[-1]] - lam_ref[S[-1] + 1])
            gap = min(gaps) if gaps else abs(lam_ref[S[0]])
            ang = ang / np.sqrt(tol * abs(lam_ref[S[0]]) / gap)
        worst = max(worst, ang)
    return worst


def oracle_for(prob, k, route="auto"):
    P = configs.operator_rounded(prob)
    W = prob["W"].astype(np.float64)
    m = min(k + 2, prob["l"] - 1)
    lam, V, Z = oeig.top_k(P, W, m, route=route)
    return lam, V, Z


def random_problem(n, l, row_len_max, seed, dtype=np.float32, empty_rows=0.0, long_rows=0):
    """Synthetic CSR with ragged rows (some empty, a few very long) and a
    W of squared distances between random points; B is then low-rank-ish
    with a clear top of the spectrum."""
    rng = np.random.default_rng(seed)
    lm = rng.choice(n, size=l, replace=False)
    rows = []
    for i in range(n):
        r = int(rng.integers(0, row_len_max + 1))
        if rng.random() < empty_rows:
            r = 0
        rows.append(np.sort(rng.choice(l, size=min(r, l), replace=False)))
    for i in rng.choice(n, size=long_rows, replace=False):
        rows[i] = np.arange(l)
    for j, v in enumerate(lm):
        rows[v] = np.array([j])
    rp = np.cumsum([0] + [len(r) for r in rows]).astype(np.int32)
    ci = np.concatenate(rows).astype(np.int32) if rp[-1] else np.zeros(0, np.int32)
    val = (rng.random(len(ci)) * 0.6 + 0.05).astype(dtype)
    for j, v in enumerate(lm):
        val[rp[v]] = 1.0
    pts = rng.standard_normal((l, 3)) * np.array([3.0, 1.5, 1.0])
    W = np.sqrt(((pts[:, None] - pts[None]) ** 2).sum(-1))
    W = (W ** 2 + 0.3 * W).astype(dtype)  # not exactly Euclidean: indefinite B
    W = 0.5 * (W + W.T)
    np.fill_diagonal(W, 0)
    return {"n": n, "l": l, "rowptr": rp, "col": ci, "val": val, "W": W.astype(dtype)}


def as_csr(prob):
    return sp.csr_matrix((prob["val"].astype(np.float64), prob["col"], prob["rowptr"]),
                         shape=(prob["n"], prob["l"]))


def device_chain(sb, torch, m):
    """The input chain of one mesh on the device: farthest-point landmarks
    from m["first"] and W (sbmds_landmarks_geodesic on the edge graph), then
    P (sbmds_interpolation); W and P's values rounded to float32 as the
    host generator stores them."""
    from synth import operator as op

    G = op.edge_graph(m["V"], m["F"]).tocsr()
    G.sort_indices()
    arrs = [torch.from_numpy(a).cuda() for a in (G.indptr.astype(np.int32), G.indices.astype(np.int32), G.data)]
    lm, W = sb.landmarks_geodesic(*arrs, m["l"], m["first"], batch=256)
    lmh = lm.cpu().numpy()
    rp, col, val = sb.interpolation(m["V"], m["F"], lmh, p=m["p"])
    return {"n": m["n"], "l": m["l"], "p": m["p"], "landmarks": lmh, "rowptr": rp, "col": col,
            "val": val.astype(np.float32), "val64": val, "W": W.float().cpu().numpy()}
