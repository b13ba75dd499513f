"""Writes the oracle's expected eigenpairs for the full-size precision
workload: the 1024 x 512 bumpy torus (n = 524,288, l = 10,000 farthest-point
landmarks, p_row = 10, float32 operator and W), k = 3 plus two more pairs for
the spectral gaps.

Calls only the seeded input generator and oracle/: the oracle's reduction
route (the l x l problem of Section 3.3) in float64 on exactly the
float32-rounded operator the GPU path receives.  Stores the eigenvalues, the
coefficients C (l x m) of the eigenvectors V = J P C, and the sha1 of the
input arrays, so a test can check that its input is the one these values
belong to.

    python tests/golden/make_bumpy_torus1024x512.py     # minutes; needs the cached input
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import eig as oeig  # noqa: E402
from synth import configs  # noqa: E402

M = 5  # eigenpairs kept: k = 3 and two below it
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bumpy_torus1024x512_l10000.npz")


def main():
    prob = configs.bumpy_torus(1024, 512, l=10000, generate=False)
    if prob is None:
        sys.exit("the 1024 x 512 torus input is not generated (synth.configs.bumpy_torus(1024, 512, l=10000))")
    t0 = time.time()
    P = configs.operator_rounded(prob)
    W = prob["W"].astype(np.float64)
    lam, coef = oeig.reduction_coefficients(P, W, M)
    meta = {"n": int(prob["n"]), "l": int(prob["l"]), "nnz": int(len(prob["col"])), "p": int(prob["p"]),
            "m": M, "input_sha1": configs.input_digest(prob), "route": "reduction",
            "seconds": round(time.time() - t0, 1)}
    np.savez(OUT, meta=json.dumps(meta), lam=lam, coef=coef)
    print(json.dumps(meta), lam.tolist())


if __name__ == "__main__":
    main()
