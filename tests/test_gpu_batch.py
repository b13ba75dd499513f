"""Many meshes in one context: every launch covers all problems (needs a gfx950 GPU).

Each problem of a batch follows its own precision schedule and stops on its
own certified bound, so each must agree with the float64 oracle exactly as a
single-problem solve does, and the trajectory of a problem must not depend on
the other problems it shares launches with.
"""
import json
import os

import numpy as np
import pytest

from tests import helpers as H

pytestmark = pytest.mark.gpu

# (n, l, row_len_max, seed): ragged sizes, all with 64..256 stored entries per
# landmark column on average, so batch and single solves pick the same launch
# shape of the transposed product
SHAPES = [(5000, 300, 12, 31), (8000, 400, 10, 32), (3001, 150, 8, 33), (6500, 333, 11, 34), (2048, 100, 9, 35)]


def problems(dtype=np.float32):
    return [H.random_problem(n=n, l=l, row_len_max=r, seed=s, dtype=dtype, empty_rows=0.05, long_rows=2)
            for n, l, r, s in SHAPES]


def solve(sb, probs, prec, k=3, block=16, **kw):
    ps = [sb.Problem.from_arrays(p["rowptr"], p["col"], p["val"], p["W"]) for p in probs]
    with sb.Context(ps, k=k, block=block, prec=prec, **kw) as ctx:
        Z, eig, reps, rc = ctx.embed()
        blocks = [ctx.get_block(i) for i in range(len(probs))]
    return Z, eig, reps, rc, blocks


def split_rows(Z, probs):
    out, r = [], 0
    for p in probs:
        out.append(Z[r:r + p["n"]])
        r += p["n"]
    return out


@pytest.mark.parametrize("prec,tol", [("FP32", 1e-6), ("BF16_FP32", 1e-6), ("FP64", 1e-10)])
def test_batch_each_problem_matches_oracle(gpu, prec, tol):
    sb = gpu
    dtype = np.float64 if prec == "FP64" else np.float32
    probs = problems(dtype)
    Z, eig, reps, rc, _ = solve(sb, probs, getattr(sb, prec), tol=tol)
    assert rc == 0
    for i, (p, Zi) in enumerate(zip(probs, split_rows(Z, probs))):
        lam, V, _ = H.oracle_for(p, 3)
        err = H.rel_eig_err(eig[i], lam[:3])
        ang = H.subspace_angle(Zi, V, lam, 3, tol=tol)
        print(f"problem {i} n={p['n']} l={p['l']} err={err:.2e} angle={ang:.2e} "
              f"iters={reps[i]['iters_bf16']},{reps[i]['iters_fp32']},{reps[i]['iters_fp64']}", flush=True)
        assert reps[i]["status"] == 0 and reps[i]["certified"], (i, reps[i])
        assert err <= tol, (i, eig[i], lam[:3])
        assert ang <= 3.0, i
        assert max(reps[i]["err_bound"][:3]) <= tol


def test_batch_problem_independent_of_companions(gpu):
    # problem 0 draws the same start block alone or in a batch, and the
    # kernels take the same per-problem launch shape, so its solve is the same
    # to the bit
    sb = gpu
    probs = problems()
    Zb, eb, rb, _, Xb = solve(sb, probs, sb.FP32)
    Zs, es, rs, _, Xs = solve(sb, probs[:1], sb.FP32)
    np.testing.assert_array_equal(eb[0], es[0])
    np.testing.assert_array_equal(split_rows(Zb, probs)[0], Zs)
    np.testing.assert_array_equal(Xb[0], Xs[0])
    assert (rb[0]["iters_fp32"], rb[0]["iters_fp64"]) == (rs[0]["iters_fp32"], rs[0]["iters_fp64"])


def test_batch_resume_one_problem(gpu):
    # the block of problem 2 of a batch resumes a single-problem solve
    sb = gpu
    probs = problems()
    _, eb, rb, _, Xb = solve(sb, probs, sb.FP32)
    p = probs[2]
    prob = sb.Problem.from_arrays(p["rowptr"], p["col"], p["val"], p["W"], X0=Xb[2])
    with sb.Context([prob], k=3, block=16, prec=sb.FP32, start=sb.START_USER) as ctx:
        _, e2, r2, rc = ctx.embed()
    assert rc == 0
    assert r2[0]["iters_fp32"] + r2[0]["iters_fp64"] <= rb[2]["iters_fp32"] + rb[2]["iters_fp64"]
    np.testing.assert_allclose(e2[0], eb[2], rtol=1e-7)


def test_batch_device_output(gpu):
    import torch
    sb = gpu
    probs = problems()
    Zh, eh, _, _, _ = solve(sb, probs, sb.FP32)
    ps = [sb.Problem.from_arrays(p["rowptr"], p["col"], p["val"], p["W"]) for p in probs]
    Zd = torch.full((sum(p["n"] for p in probs), 3), float("nan"), dtype=torch.float32, device="cuda")
    with sb.Context(ps, k=3, block=16, prec=sb.FP32) as ctx:
        _, ed, _, rc = ctx.embed(Z_out=Zd)
    torch.cuda.synchronize()
    assert rc == 0
    np.testing.assert_array_equal(ed, eh)
    np.testing.assert_array_equal(Zd.cpu().numpy(), Zh)


@pytest.mark.parametrize("prec", ["FP32", "BF16_FP32"])
def test_mesh_batch_matches_oracle(gpu, prec):
    # the batched workload's recipe at reduced scale: 16 bumpy tori and
    # deformed geodesic spheres of 2k-20k vertices, l = n/50, in one context
    from synth import configs
    sb = gpu
    probs = configs.mesh_batch()
    Z, eig, reps, rc, _ = solve(sb, probs, getattr(sb, prec))
    assert rc == 0
    worst = 0.0
    for i, (p, Zi) in enumerate(zip(probs, split_rows(Z, probs))):
        lam, V, _ = H.oracle_for(p, 3)
        err = H.rel_eig_err(eig[i], lam[:3])
        worst = max(worst, err)
        assert reps[i]["certified"], (i, reps[i])
        assert err <= 1e-6, (i, p["n"], eig[i], lam[:3])
        assert H.subspace_angle(Zi, V, lam, 3, tol=1e-6) <= 3.0, i
    print(f"{prec}: 16 meshes, worst rel eig err {worst:.2e}", flush=True)


def test_device_chain_batch_matches_host_chain(gpu):
    # the same 16 meshes with their inputs built on the device (landmarks,
    # geodesic W, P by the blocked route for n > 4096): landmarks and W equal
    # the host chain's bit for bit, P's pattern equal and its float32 values
    # within one rounding; the batched solve on the device inputs matches
    # the oracle on them
    import torch

    from synth import configs
    sb = gpu
    host = configs.mesh_batch()
    dev = [H.device_chain(sb, torch, m) for m in configs.batch_meshes()]
    for i, (d, h) in enumerate(zip(dev, host)):
        assert np.array_equal(d["landmarks"], h["landmarks"]), i
        assert np.array_equal(d["W"], h["W"]), i
        assert np.array_equal(d["rowptr"], h["rowptr"]) and np.array_equal(d["col"], h["col"]), i
        hv = h["val"].astype(np.float64)
        assert np.all(np.abs(d["val"] - hv) <= 2.0 ** -23 * np.abs(hv) + 1e-12), i
    Z, eig, reps, rc, _ = solve(sb, dev, sb.FP32)
    assert rc == 0
    worst = 0.0
    for i, (p, Zi) in enumerate(zip(dev, split_rows(Z, dev))):
        lam, V, _ = H.oracle_for(p, 3)
        err = H.rel_eig_err(eig[i], lam[:3])
        worst = max(worst, err)
        assert reps[i]["certified"] and err <= 1e-6, (i, p["n"], eig[i], lam[:3])
        assert H.subspace_angle(Zi, V, lam, 3, tol=1e-6) <= 3.0, i
    print(f"device chain: 16 meshes, worst rel eig err {worst:.2e}", flush=True)


GOLDEN_256 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grid_torus_batch256.npz")


def test_batch_256_meshes_full_scale(gpu):
    # the batched workload's full shape: 256 grid-torus meshes with n from
    # about 2,000 to 200,000 (24.9M vertices, 499k landmarks, 245M stored
    # entries, 5.2 GB of W, so W is packed) in one context; every mesh
    # against the float64 oracle's eigenpairs (reduction route, stored with
    # each input's sha1 by tests/golden/make_grid_torus_batch256.py):
    # eigenvalues within 1e-6, eigenvector clusters within the angle that
    # accuracy implies
    from oracle import eig as oeig
    from synth import configs, large
    sb = gpu
    g = np.load(GOLDEN_256, allow_pickle=False)
    meta = json.loads(str(g["meta"]))
    probs = large.grid_torus_batch()
    assert len(probs) == meta["count"]
    for i, p in enumerate(probs):
        assert meta["input_sha1"][i] == configs.input_digest(p), f"mesh {i} differs from its stored values"
    Z, eig, reps, rc, _ = solve(sb, probs, sb.FP32)
    assert rc == 0
    assert all(r["status"] == 0 and r["certified"] for r in reps)
    Zs = split_rows(Z, probs)
    offs = g["offsets"]
    worst_err = worst_ang = 0.0
    for i, p in enumerate(probs):
        lam = g["lam"][i]
        coef = g["coef"][offs[i]:offs[i + 1]].astype(np.float64)
        V = oeig.vectors_from_coefficients(configs.operator_rounded(p), coef)
        err = H.rel_eig_err(eig[i], lam[:3])
        ang = H.subspace_angle(Zs[i], V, lam, 3, tol=1e-6)
        worst_err, worst_ang = max(worst_err, err), max(worst_ang, ang)
        assert err <= 1e-6, (i, p["n"], eig[i], lam[:3])
        assert ang <= 3.0, (i, p["n"], ang)
    print(f"256 meshes: worst rel eig err {worst_err:.2e}, worst relative subspace angle {worst_ang:.2e}", flush=True)


def test_batch_push_form_mixed(gpu):
    # with SBMDS_FLAG_PUSH_T the chain meshes take the push form and the
    # random ragged ones (too many block-landmark pairs) keep the gathering
    # form, in the same launches; every problem still matches the oracle and
    # solves the same as alone
    sb = gpu
    from synth import configs
    torus = dict(configs.torus64x32())
    torus["val"] = torus["val"].astype(np.float32)
    torus["W"] = torus["W"].astype(np.float32)
    probs = [torus] + problems()[:2]
    Z, eig, reps, rc, _ = solve(sb, probs, sb.FP32, flags=sb.FLAG_PUSH_T)
    assert rc == 0
    for i, (p, Zi) in enumerate(zip(probs, split_rows(Z, probs))):
        lam, V, _ = H.oracle_for(p, 3)
        assert H.rel_eig_err(eig[i], lam[:3]) <= 1e-6, i
        assert H.subspace_angle(Zi, V, lam, 3, tol=1e-6) <= 3.0, i
    Zs, es, _, _, _ = solve(sb, probs[:1], sb.FP32, flags=sb.FLAG_PUSH_T)
    np.testing.assert_array_equal(eig[0], es[0])
