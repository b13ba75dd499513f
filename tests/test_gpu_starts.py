"""Start blocks other than the random one (needs a gfx950 GPU).

Landmark MDS start: the top eigenvectors of -1/2 J W J on the landmarks (the
same iteration run with P = I), lifted through P.  Whatever the start, the
certified result must match the float64 oracle; the start only changes how
many iterations the solve needs.
"""
import numpy as np
import pytest

from synth import configs
from tests import helpers as H
from tests.test_gpu_batch import problems, split_rows
from tests.test_gpu_parity import check, run

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["FP32", "BF16_FP32"])
def test_lmds_start_sphere7(gpu, prec):
    sb = gpu
    prob = configs.sphere7()
    Z, eig, rep, rc, _ = run(sb, prob, 3, 16, getattr(sb, prec), start=sb.START_LMDS)
    assert rc == 0 and rep["certified"]
    assert rep["start_iters"] >= 1
    check(prob, Z, eig, rep, 3, 1e-6)
    _, _, rep_r, _, _ = run(sb, prob, 3, 16, getattr(sb, prec))
    it = lambda r: r["iters_bf16"] + r["iters_fp32"] + r["iters_fp64"]
    print(f"{prec}: iterations lmds {it(rep)} (+{rep['start_iters']} landmark) random {it(rep_r)}", flush=True)


def test_lmds_start_fp64_torus(gpu):
    sb = gpu
    prob = configs.torus64x32()
    Z, eig, rep, rc, _ = run(sb, prob, 3, 16, sb.FP64, start=sb.START_LMDS, tol=1e-10)
    assert rc == 0 and rep["certified"]
    check(prob, Z, eig, rep, 3, 1e-10)


def test_lmds_start_batch(gpu):
    sb = gpu
    probs = problems()
    ps = [sb.Problem.from_arrays(p["rowptr"], p["col"], p["val"], p["W"]) for p in probs]
    with sb.Context(ps, k=3, block=16, prec=sb.FP32, start=sb.START_LMDS) as ctx:
        for call in range(2):  # the second call reuses the landmark buffers
            Z, eig, reps, rc = ctx.embed()
            assert rc == 0
            for i, (p, Zi) in enumerate(zip(probs, split_rows(Z, probs))):
                lam, V, _ = H.oracle_for(p, 3)
                assert reps[i]["certified"] and reps[i]["start_iters"] >= 1, (call, i, reps[i])
                assert H.rel_eig_err(eig[i], lam[:3]) <= 1e-6, (call, i)
                assert H.subspace_angle(Zi, V, lam, 3, tol=1e-6) <= 3.0, (call, i)
