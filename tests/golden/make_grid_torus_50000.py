"""Writes the oracle's expected eigenpairs for the largest workload's shape:
the seeded synthetic grid-torus operator of synth.large (n = 1,800,000,
l = 50,000, 17.55M stored entries, float32 P and W), k = 3 plus two more
pairs for the spectral gaps.

Calls only the seeded input generator and oracle/: the oracle's ARPACK route
(scipy's eigsh on the implicit float64 operator v -> -1/2 J P W P^T J v, the
matrix-vector form of Section 3.3) on exactly the float32-rounded operator
the GPU path receives, W widened to float64 (20 GB of host memory).  The
eigenvectors are stored as coefficients C (l x m) with V = J P C, recovered
from B v = lambda v, together with the eigenvalues, the residuals of the
pairs and the sha1 of the input arrays.

    python tests/golden/make_grid_torus_50000.py     # ~10-30 min, ~32 GB RAM
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import eig as oeig  # noqa: E402
from synth import configs, large  # noqa: E402

M = 5
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid_torus_1800x1000_l50000.npz")


def main():
    t0 = time.time()
    prob = large.grid_torus_operator()
    digest = configs.input_digest(prob)
    P = configs.operator_rounded(prob)
    W = prob.pop("W").astype(np.float64)
    print(f"input {digest} ready after {time.time() - t0:.1f} s", flush=True)
    t1 = time.time()
    lam, V, _ = oeig.top_k(P, W, M, route="arpack", tol=1e-12)
    t_arpack = time.time() - t1
    coef = oeig.coefficients_from_vectors(P, W, lam, V)
    back = oeig.vectors_from_coefficients(P, coef)
    BV = oeig.apply_b(P, W, V)
    resid = np.linalg.norm(BV - V * lam[None, :], axis=0) / np.abs(lam)
    meta = {"n": int(prob["n"]), "l": int(prob["l"]), "nnz": int(len(prob["col"])), "m": M,
            "input_sha1": digest, "route": "arpack", "arpack_tol": 1e-12,
            "rel_residuals": [float(r) for r in resid],
            "coef_roundtrip": float(np.abs(back - V).max()),
            "seconds": round(t_arpack, 1)}
    np.savez(OUT, meta=json.dumps(meta), lam=lam, coef=coef)
    print(json.dumps(meta), lam.tolist(), flush=True)


if __name__ == "__main__":
    main()
