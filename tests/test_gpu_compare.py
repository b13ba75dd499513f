"""The paper's other eigen routes (Section 3.3) on the GPU through the C ABI:
(block) Lanczos on the implicit operator -1/2 J P W P^T J (block 1 is the
paper's sBMDS) and BMDS (QR of the dense J P, eigendecomposition of
-1/2 R W R^T), against the float64 oracle on the same rounded values
(needs a gfx950 GPU)."""
import numpy as np
import pytest

from synth import configs
from tests import helpers as H

pytestmark = pytest.mark.gpu


def context(sb, probs, prec, k=3, **kw):
    ps = [sb.Problem.from_arrays(p["rowptr"], p["col"], p["val"], p["W"]) for p in probs]
    return sb.Context(ps, k=k, block=16, prec=prec, **kw)


def check(prob, Z, eig, rep, k, tol, angle_tol=3.0):
    lam, V, _ = H.oracle_for(prob, k)
    err = H.rel_eig_err(eig, lam[:k])
    ang = H.subspace_angle(Z, V, lam, k, tol=tol)
    print(f"n={prob['n']} l={prob['l']} err={err:.3e} angle={ang:.3e} steps={rep['steps']} "
          f"basis={rep['basis']} bound={max(rep['err_bound'][:k]):.2e}", flush=True)
    assert err <= tol, (eig, lam[:k])
    assert ang <= angle_tol
    return err


def fp32(prob):
    q = dict(prob)
    q["val"] = q["val"].astype(np.float32)
    q["W"] = q["W"].astype(np.float32)
    return q


@pytest.mark.parametrize("block", [1, 2, 4])
def test_lanczos_torus_fp64(gpu, block):
    # the 64 x 32 torus (n = 2048, l = 64): float64 operator, tol 1e-10
    sb = gpu
    prob = configs.torus64x32()
    with context(sb, [prob], sb.FP64, tol=1e-10) as ctx:
        Z, eig, reps, rc = ctx.embed_lanczos(block=block, max_steps=200)
    rep = reps[0]
    assert rc == 0 and rep["status"] == 0
    assert max(rep["err_bound"][:3]) <= 1e-10
    check(prob, Z, eig[0], rep, 3, 1e-10)


@pytest.mark.parametrize("block", [1, 8])
def test_lanczos_random_ragged_fp32(gpu, block):
    # ragged operator (empty rows, a few long rows), float32 values: the
    # eigenvalues of that rounded operator within tol 1e-6
    sb = gpu
    prob = H.random_problem(n=6000, l=200, row_len_max=9, seed=23, empty_rows=0.05, long_rows=3)
    with context(sb, [prob], sb.FP32) as ctx:
        Z, eig, reps, rc = ctx.embed_lanczos(block=block, max_steps=150)
    assert rc == 0
    check(prob, Z, eig[0], reps[0], 3, 1e-6)


def test_lanczos_step_cap_and_two_problems(gpu):
    # two problems in one context: Z concatenated as sbmds_embed writes it;
    # a step cap too small to converge returns SBMDS_ENOCONV with finite
    # best-effort Ritz values
    sb = gpu
    import torch
    a = configs.torus64x32()
    b = configs.torus64x32(seed=1002)
    with context(sb, [a, b], sb.FP64, tol=1e-10) as ctx:
        Zd = torch.zeros((a["n"] + b["n"], 3), dtype=torch.float64, device="cuda")
        _, eig, reps, rc = ctx.embed_lanczos(block=2, max_steps=200, Z_out=Zd)
        torch.cuda.synchronize()
        Z = Zd.cpu().numpy()
        assert rc == 0
        check(a, Z[:a["n"]], eig[0], reps[0], 3, 1e-10)
        check(b, Z[a["n"]:], eig[1], reps[1], 3, 1e-10)
        _, eig2, reps2, rc2 = ctx.embed_lanczos(block=2, max_steps=3)
    assert rc2 == 1 and reps2[0]["status"] == 1
    assert np.all(np.isfinite(eig2))
    assert reps2[0]["steps"] == 3 and reps2[0]["basis"] == 6


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_bmds_torus(gpu, prec):
    # the dense route: eigenvalues of -1/2 R W R^T equal the oracle's, the
    # measured residuals are at rounding level
    sb = gpu
    prob = configs.torus64x32()
    if prec == "fp32":
        prob = fp32(prob)
    with context(sb, [prob], sb.FP64 if prec == "fp64" else sb.FP32) as ctx:
        Z, eig, reps, rc = ctx.embed_bmds()
    rep = reps[0]
    assert rc == 0
    assert max(rep["resid"][:3]) <= 1e-10
    check(prob, Z, eig[0], rep, 3, 1e-12)


def test_bmds_random_ragged_fp32(gpu):
    sb = gpu
    prob = H.random_problem(n=6000, l=200, row_len_max=9, seed=23, empty_rows=0.05, long_rows=3)
    with context(sb, [prob], sb.FP32) as ctx:
        Z, eig, reps, rc = ctx.embed_bmds()
    assert rc == 0
    check(prob, Z, eig[0], reps[0], 3, 1e-12)
