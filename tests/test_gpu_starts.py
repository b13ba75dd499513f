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


@pytest.mark.parametrize("defect", ["zero", "repeated"])
def test_user_start_rank_deficient(gpu, defect):
    # a start block of width 8 whose columns leave fewer live ones than k
    # (six zero columns, or seven copies of one column) loses rank in its
    # first CholQR; the dropped columns are refilled with fresh Gaussian
    # ones, so the block regains its width and the solve certifies the
    # oracle's answer (with the dropped columns left out it could never hold
    # three Ritz pairs).  Two calls on one context: the second starts from
    # the same defective block.
    sb = gpu
    prob = H.random_problem(n=8000, l=400, row_len_max=10, seed=5)
    rng = np.random.default_rng(3)
    X0 = rng.standard_normal((prob["n"], 8)).astype(np.float32)
    if defect == "zero":
        X0[:, 2:] = 0.0
    else:
        X0[:, 1:] = X0[:, :1]
    p = sb.Problem.from_arrays(prob["rowptr"], prob["col"], prob["val"], prob["W"], X0=X0)
    lam, V, _ = H.oracle_for(prob, 3)
    with sb.Context([p], k=3, block=8, prec=sb.FP32, start=sb.START_USER, max_iter=300) as ctx:
        for call in range(2):
            Z, eig, reps, rc = ctx.embed()
            rep = reps[0]
            print(f"{defect} call {call}: iters {rep['iters_fp32']}+{rep['iters_fp64']} eig {eig[0]}", flush=True)
            assert rc == 0 and rep["certified"], (call, rep)
            assert H.rel_eig_err(eig[0], lam[:3]) <= 1e-6, call
            assert H.subspace_angle(Z, V, lam, 3, tol=1e-6) <= 3.0, call


def test_learned_start_zero_prediction_column(gpu, tmp_path):
    # a network whose first output is identically zero predicts a start block
    # with a zero column (the other five columns of the block are Gaussian);
    # the solve refills it and certifies the oracle's answer
    from paper_1705_10887_amd import mlp
    sb = gpu
    prob = dict(configs.torus64x32())
    prob["val"] = prob["val"].astype(np.float32)
    prob["W"] = prob["W"].astype(np.float32)
    k = 3
    with mlp.Net(k=k, seed=4) as net:
        theta = net.get_params()
        nh = 128
        w3 = len(theta) - (nh * k + k)      # W3 [128][k] then b3 [k]
        W3 = theta[w3:w3 + nh * k].reshape(nh, k)
        W3[:, 0] = 0.0
        theta[w3:w3 + nh * k] = W3.ravel()
        theta[-k] = 0.0
        net.set_params(theta)
        path = str(tmp_path / "zero_col.bin")
        net.save(path)
    p = sb.Problem.from_arrays(prob["rowptr"], prob["col"], prob["val"], prob["W"], xyz=prob["V"].astype(np.float32),
                               landmark_vertex=prob["landmarks"].astype(np.int32))
    with sb.Context([p], k=k, block=8, prec=sb.FP32, start=sb.START_LEARNED, mlp_weights=path,
                    max_iter=500) as ctx:
        Z, eig, reps, rc = ctx.embed()
    rep = reps[0]
    print(f"learned zero column: iters {rep['iters_fp32']}+{rep['iters_fp64']}", flush=True)
    assert rc == 0 and rep["certified"], rep
    check(prob, Z, eig[0], rep, k, 1e-6)
