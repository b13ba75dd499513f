"""Writes the oracle's expected eigenpairs for the batched workload's full
shape: the 256 seeded synthetic grid-torus meshes of synth.large (n from
about 2,000 to 200,000, l ~ n / 50, float32 P and W), k = 3 plus two more
eigenvalues per mesh for the spectral gaps.

Calls only the seeded input generator and oracle/: the reduction route (the
l x l problem of Section 3.3) in float64 on exactly the float32-rounded
operator of each mesh.  Stores per mesh the five largest eigenvalues, the
coefficients C (l x 3, float32) of the wanted eigenvectors V = J P C, and
the sha1 of the input arrays.

    python tests/golden/make_grid_torus_batch256.py     # ~20-40 min on 8 cores
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

M, K = 5, 3
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "grid_torus_batch256.npz")


def main():
    t0 = time.time()
    lams, coefs, digests, ls = [], [], [], []
    for i, shape in enumerate(large.grid_torus_batch_shapes()):
        prob = large.grid_torus_batch_mesh(shape)
        P = configs.operator_rounded(prob)
        lam, coef = oeig.reduction_coefficients(P, prob["W"].astype(np.float64), M)
        lams.append(lam)
        coefs.append(coef[:, :K].astype(np.float32))
        digests.append(configs.input_digest(prob))
        ls.append(int(prob["l"]))
        print(f"[{time.time() - t0:7.1f}s] mesh {i} n={prob['n']} l={prob['l']} lam={lam[:3]}", flush=True)
    offs = np.zeros(len(ls) + 1, dtype=np.int64)
    np.cumsum(ls, out=offs[1:])
    meta = {"count": len(ls), "m": M, "k": K, "route": "reduction", "input_sha1": digests,
            "seconds": round(time.time() - t0, 1)}
    np.savez_compressed(OUT, meta=json.dumps(meta), lam=np.array(lams), coef=np.concatenate(coefs),
                        offsets=offs)
    print(json.dumps({k: v for k, v in meta.items() if k != "input_sha1"}), flush=True)


if __name__ == "__main__":
    main()
