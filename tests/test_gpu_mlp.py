"""Learned warm start on the GPU against the float64 reference (oracle/mlp.py):
features, forward pass, loss and gradient, Adam, weights files, and what a
trained network gains over the random start (needs a gfx950 GPU)."""
import os

import numpy as np
import pytest

from oracle import mlp as om
from synth import configs

pytestmark = pytest.mark.gpu


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def random_case(k=3, rows=(57, 130, 41, 1), seed=5):
    rng = np.random.default_rng(seed)
    n = sum(rows)
    F = rng.standard_normal((n, om.N_FEAT)).astype(np.float32) * 0.7 + 0.2
    T = rng.standard_normal((n, k)).astype(np.float32)
    seg = np.concatenate([[0], np.cumsum(rows)]).astype(np.int64)
    mean = rng.standard_normal(om.N_FEAT).astype(np.float32) * 0.1
    std = (0.5 + rng.random(om.N_FEAT)).astype(np.float32)
    return F, T, seg, mean, std


def test_features_match_oracle(gpu):
    from paper_1705_10887_amd import mlp
    prob = configs.torus64x32()  # float64 W
    lm = prob["landmarks"].astype(np.int32)
    xyz = prob["V"].astype(np.float32)
    F = mlp.features(xyz, lm, prob["W"])
    ref = om.features(xyz.astype(np.float64), lm, prob["W"])
    np.testing.assert_allclose(F, ref, rtol=2e-6, atol=2e-7)
    # float32 W, with repeated distances (ties at bin edges are decided in float64 on both sides)
    rng = np.random.default_rng(1)
    pts = rng.integers(0, 5, size=(300, 3)).astype(np.float32)
    W = ((pts[:, None] - pts[None]) ** 2).sum(-1).astype(np.float32)
    lm2 = np.arange(300, dtype=np.int32)
    F2 = mlp.features(pts, lm2, W)
    ref2 = om.features(pts.astype(np.float64), lm2, W.astype(np.float64))
    np.testing.assert_allclose(F2, ref2, rtol=2e-6, atol=2e-7)


def test_features_device_inputs(gpu):
    import torch
    from paper_1705_10887_amd import mlp
    prob = configs.torus64x32()
    lm = prob["landmarks"].astype(np.int32)
    xyz = prob["V"].astype(np.float32)
    Fh = mlp.features(xyz, lm, prob["W"])
    Fd = mlp.features(torch.from_numpy(xyz).cuda(), torch.from_numpy(lm).cuda(), torch.from_numpy(prob["W"]).cuda())
    torch.cuda.synchronize()
    np.testing.assert_array_equal(Fd.cpu().numpy(), Fh)


def test_forward_loss_gradient_match_oracle(gpu):
    from paper_1705_10887_amd import mlp
    k = 3
    F, T, seg, mean, std = random_case(k)
    with mlp.Net(k=k, seed=11) as net:
        net.set_norm(mean, std)
        theta = net.get_params().astype(np.float64)
        X = om.standardise(F, mean.astype(np.float64), std.astype(np.float64))
        y_ref, _ = om.forward(theta, X, k)
        assert rel(net.forward(F), y_ref) <= 1e-5
        loss, g = net.loss_grad(F, T, seg)
        L_ref, g_ref = om.loss_and_grad(theta, X, T.astype(np.float64), seg, k)
        print(f"loss {loss:.8e} ref {L_ref:.8e} grad rel err {rel(g, g_ref):.2e}", flush=True)
        assert loss == pytest.approx(L_ref, rel=1e-5)
        assert rel(g, g_ref) <= 1e-4
        # each parameter block on its own (a dropped term in a small block
        # would hide in the norm of the whole vector)
        o = 0
        for name, shape in om.param_shapes(k):
            size = int(np.prod(shape))
            assert rel(g[o:o + size], g_ref[o:o + size]) <= 1e-4, name
            o += size


@pytest.mark.parametrize("k", [1, 2, 8])
def test_gradient_other_widths(gpu, k):
    from paper_1705_10887_amd import mlp
    F, T, seg, mean, std = random_case(k, rows=(300, 9, 77), seed=k)
    with mlp.Net(k=k, seed=k) as net:
        net.set_norm(mean, std)
        theta = net.get_params().astype(np.float64)
        X = om.standardise(F, mean.astype(np.float64), std.astype(np.float64))
        loss, g = net.loss_grad(F, T, seg)
        L_ref, g_ref = om.loss_and_grad(theta, X, T.astype(np.float64), seg, k)
        assert loss == pytest.approx(L_ref, rel=1e-5)
        assert rel(g, g_ref) <= 1e-4


def test_adam_step_matches_oracle(gpu):
    from paper_1705_10887_amd import mlp
    k = 3
    F, T, seg, mean, std = random_case(k)
    with mlp.Net(k=k, seed=3) as net:
        net.set_norm(mean, std)
        th = net.get_params().astype(np.float64)
        m = np.zeros_like(th)
        v = np.zeros_like(th)
        for t in (1, 2, 3):
            _, g = net.loss_grad(F, T, seg)
            net.adam_step(1e-3)
            th, m, v = om.adam_step(th, g.astype(np.float64), m, v, t, lr=1e-3)
            got = net.get_params()
            assert np.max(np.abs(got - th)) <= 1e-6 + 1e-5 * np.max(np.abs(th)), t
            th = got.astype(np.float64)  # follow the device trajectory


def test_weights_file_roundtrip(gpu, tmp_path):
    from paper_1705_10887_amd import mlp
    F, _, _, mean, std = random_case(3)
    path = str(tmp_path / "net.bin")
    with mlp.Net(k=3, seed=7) as net:
        net.set_norm(mean, std)
        net.save(path)
        y1 = net.forward(F)
        th = net.get_params()
    with mlp.Net.load(path) as net2:
        assert net2.k == 3
        np.testing.assert_array_equal(net2.get_params(), th)
        np.testing.assert_array_equal(net2.forward(F), y1)


# ---------------------------------------------------------------------------
# training on solver-converged embeddings and the gain over the random start
# ---------------------------------------------------------------------------
TRAIN = configs.TORUS_FAMILY
HELD_OUT = (96, 48, 4199)


def torus(nu, nv, seed):
    prob = configs.bumpy_torus(nu, nv, seed=seed)
    prob["landmarks"] = prob["landmarks"].astype(np.int32)
    prob["xyz"] = prob["V"].astype(np.float32)
    return prob


def test_training_and_gain_over_random_start(gpu, tmp_path):
    import paper_1705_10887_amd as sb
    from paper_1705_10887_amd import mlp
    k = 3
    meshes = [torus(*t) for t in TRAIN]
    targets = mlp.solve_targets(meshes, k=k)
    feats = [mlp.features(m["xyz"], m["landmarks"], m["W"]) for m in meshes]
    net, losses = mlp.train(feats, targets, k=k, steps=500, lr=3e-3, seed=0)
    print(f"training loss {losses[0]:.3e} -> {losses[-1]:.3e}", flush=True)
    assert losses[-1] < 0.5 * losses[0]
    path = str(tmp_path / "warm.bin")
    net.save(path)
    net.close()

    held = torus(*HELD_OUT)

    def run(start, max_iter, flags=0):
        p = sb.Problem.from_arrays(held["rowptr"], held["col"], held["val"], held["W"], xyz=held["xyz"],
                                   landmark_vertex=held["landmarks"])
        with sb.Context([p], k=k, block=16, prec=sb.FP32, start=start, mlp_weights=path, max_iter=max_iter,
                        flags=flags) as ctx:
            Z, eig, reps, rc = ctx.embed()
        return Z, eig[0], reps[0], rc

    # the residual after one iteration: how far each start is from the answer
    res = {}
    for name, st in (("random", sb.START_RANDOM), ("lmds", sb.START_LMDS), ("learned", sb.START_LEARNED)):
        _, _, rep, _ = run(st, 1, sb.FLAG_NO_CERTIFY)
        res[name] = max(rep["resid"][:k])
    print("residual after one iteration: " + ", ".join(f"{a} {b:.3e}" for a, b in res.items()), flush=True)
    assert res["learned"] < res["random"]

    # full solves: the learned start certifies the same answer, in no more iterations
    from tests import helpers as H
    Zl, el, rl, rc = run(sb.START_LEARNED, 500)
    Zr, er, rr, _ = run(sb.START_RANDOM, 500)
    assert rc == 0 and rl["certified"]
    lam, V, _ = H.oracle_for(held, k)
    assert H.rel_eig_err(el, lam[:k]) <= 1e-6
    assert H.subspace_angle(Zl, V, lam, k, tol=1e-6) <= 3.0
    it = lambda r: r["iters_fp32"] + r["iters_fp64"]
    print(f"iterations: learned {it(rl)} random {it(rr)}", flush=True)
    assert it(rl) < it(rr)  # measured: learned 4, random 5


def test_learned_start_sphere7_block8(gpu, tmp_path):
    # the benchmark's learned form: a network trained on level-6 spheres of
    # the same family starts the level-7 solve at block 8
    import paper_1705_10887_amd as sb
    from paper_1705_10887_amd import mlp
    from tests import helpers as H
    k = 3
    meshes = configs.sphere_family(level=6)
    for m in meshes:
        m["landmarks"] = m["landmarks"].astype(np.int32)
        m["xyz"] = m["V"].astype(np.float32)
    targets = mlp.solve_targets(meshes, k=k, block=8)
    feats = [mlp.features(m["xyz"], m["landmarks"], m["W"]) for m in meshes]
    net, losses = mlp.train(feats, targets, k=k, steps=600, lr=3e-3, seed=0)
    assert losses[-1] < 0.05 * losses[0]
    path = str(tmp_path / "sphere.bin")
    net.save(path)
    net.close()
    prob = configs.sphere7()
    xyz = prob["V"].astype(np.float32)
    lm = prob["landmarks"].astype(np.int32)

    def run(start):
        p = sb.Problem.from_arrays(prob["rowptr"], prob["col"], prob["val"], prob["W"], xyz=xyz, landmark_vertex=lm)
        with sb.Context([p], k=k, block=8, prec=sb.FP32, start=start, mlp_weights=path) as ctx:
            Z, eig, reps, rc = ctx.embed()
        return Z, eig[0], reps[0], rc

    Zl, el, rl, rc = run(sb.START_LEARNED)
    _, _, rr, _ = run(sb.START_RANDOM)
    assert rc == 0 and rl["certified"]
    lam, V, _ = H.oracle_for(prob, k)
    assert H.rel_eig_err(el, lam[:k]) <= 1e-6
    assert H.subspace_angle(Zl, V, lam, k, tol=1e-6) <= 3.0
    it = lambda r: r["iters_fp32"] + r["iters_fp64"]
    print(f"sphere7 block 8: iterations learned {it(rl)} random {it(rr)}", flush=True)
    assert it(rl) < it(rr)
