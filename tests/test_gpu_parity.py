"""HIP path vs the float64 CPU oracle, through the C ABI (needs a gfx950 GPU).

Tolerances: 1e-6 relative eigenvalue error for float32 / bf16+fp32 solves
(the target of the method's measurement), 1e-10 for the FP64 solve.  The
oracle sees exactly the float32-rounded operator handed to the GPU.
"""
import json
import os

import numpy as np
import pytest

from oracle import eig as oeig
from synth import configs
from tests import helpers as H

pytestmark = pytest.mark.gpu


def run(sb, prob, k, block, prec, **kw):
    p = sb.Problem.from_arrays(prob["rowptr"], prob["col"], prob["val"], prob["W"], X0=kw.pop("X0", None))
    with sb.Context([p], k=k, block=block, prec=prec, **kw) as ctx:
        Z, eig, reps, rc = ctx.embed()
        X = ctx.get_block(0)
    return Z, eig[0], reps[0], rc, X


def check(prob, Z, eig, rep, k, tol, angle_tol=3.0):
    """Eigenvalues within `tol`; eigenvector clusters within `angle_tol` times
    the angle that a `tol`-accurate Ritz value implies (see helpers)."""
    lam, V, _ = H.oracle_for(prob, k)
    return check_against(prob, lam, V, Z, eig, rep, k, tol, angle_tol)


def check_against(prob, lam, V, Z, eig, rep, k, tol, angle_tol=3.0):
    err = H.rel_eig_err(eig, lam[:k])
    ang = H.subspace_angle(Z, V, lam, k, tol=tol)
    print(f"n={prob['n']} l={prob['l']} k={k} err={err:.3e} angle={ang:.3e} rep={rep['iters_bf16']},"
          f"{rep['iters_fp32']},{rep['iters_fp64']} bound={max(rep['err_bound'][:k]):.2e}", flush=True)
    assert err <= tol, (eig, lam[:k])
    assert ang <= angle_tol
    assert all(b <= tol for b in rep["err_bound"][:k]) or not rep["certified"]
    return err, ang


def test_torus64x32_fp64(gpu):
    sb = gpu
    prob = configs.torus64x32()
    Z, eig, rep, rc, _ = run(sb, prob, 3, 16, sb.FP64, tol=1e-10)
    assert rc == 0 and rep["certified"]
    check(prob, Z, eig, rep, 3, 1e-10)


def test_torus64x32_fp32(gpu):
    sb = gpu
    prob = dict(configs.torus64x32())
    prob["val"] = prob["val"].astype(np.float32)
    prob["W"] = prob["W"].astype(np.float32)
    Z, eig, rep, rc, _ = run(sb, prob, 3, 16, sb.FP32)
    assert rc == 0 and rep["certified"]
    check(prob, Z, eig, rep, 3, 1e-6)


@pytest.mark.parametrize("block", [4, 8, 16, 32, 64])
def test_random_operator_all_widths(gpu, block):
    sb = gpu
    prob = H.random_problem(n=5000, l=300, row_len_max=12, seed=block, empty_rows=0.05, long_rows=3)
    k = min(3, block)
    Z, eig, rep, rc, _ = run(sb, prob, k, block, sb.FP32, max_iter=300)
    assert rc == 0
    check(prob, Z, eig, rep, k, 1e-6)


@pytest.mark.parametrize("prec", ["FP32", "BF16_FP32"])
def test_block8_u_past_lds_copy(gpu, prec):
    # l x 8 x 4 bytes above 64 KB: the SpMM gathers U from global memory
    # instead of its LDS copy (the other width-8 tests use the copy)
    sb = gpu
    prob = H.random_problem(n=6000, l=2100, row_len_max=12, seed=81, empty_rows=0.05, long_rows=2)
    Z, eig, rep, rc, _ = run(sb, prob, 3, 8, getattr(sb, prec), max_iter=300)
    assert rc == 0 and rep["certified"]
    check(prob, Z, eig, rep, 3, 1e-6)


def test_random_operator_fp64_ragged(gpu):
    sb = gpu
    prob = H.random_problem(n=3001, l=130, row_len_max=20, seed=7, dtype=np.float64, empty_rows=0.1,
                            long_rows=2)
    Z, eig, rep, rc, _ = run(sb, prob, 4, 16, sb.FP64, tol=1e-11)
    assert rc == 0
    check(prob, Z, eig, rep, 4, 1e-10)


@pytest.mark.parametrize("block", [16, 8])
def test_sphere7_fp32_k3(gpu, block):
    # block 8 holds the three wanted eigenvalues and the five negative ones
    # of larger magnitude than the rest of the spectrum
    sb = gpu
    prob = configs.sphere7()
    Z, eig, rep, rc, _ = run(sb, prob, 3, block, sb.FP32)
    assert rc == 0 and rep["certified"]
    check(prob, Z, eig, rep, 3, 1e-6)


def test_sphere7_fp32_k10(gpu):
    sb = gpu
    prob = configs.sphere7()
    Z, eig, rep, rc, _ = run(sb, prob, 10, 48, sb.FP32)
    assert rc == 0 and rep["certified"]
    check(prob, Z, eig, rep, 10, 1e-6)


@pytest.mark.parametrize("block", [16, 8])
def test_sphere7_bf16_fp32(gpu, block):
    sb = gpu
    prob = configs.sphere7()
    Z, eig, rep, rc, _ = run(sb, prob, 3, block, sb.BF16_FP32)
    assert rc == 0 and rep["certified"]
    assert rep["iters_bf16"] >= 1
    check(prob, Z, eig, rep, 3, 1e-6)


GOLDEN_TORUS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                            "bumpy_torus1024x512_l10000.npz")


@pytest.mark.parametrize("prec", ["BF16_FP32", "FP32"])
def test_bumpy_torus1024x512_l10000(gpu, prec):
    # the precision workload at full size: n = 524,288, l = 10,000, W 400 MB
    # in float32; the oracle's eigenpairs (reduction route, float64) are
    # stored, since its two l x l eigendecompositions take minutes
    sb = gpu
    prob = configs.bumpy_torus(1024, 512, l=10000, generate=False)
    if prob is None:
        pytest.skip("the 1024 x 512 torus input is not generated (about an hour of host time)")
    if not os.path.exists(GOLDEN_TORUS):
        pytest.skip("stored oracle values missing (tests/golden/make_bumpy_torus1024x512.py writes them)")
    g = np.load(GOLDEN_TORUS, allow_pickle=False)
    meta = json.loads(str(g["meta"]))
    assert meta["input_sha1"] == configs.input_digest(prob), "input differs from the one the stored values are for"
    Z, eig, rep, rc, _ = run(sb, prob, 3, 16, getattr(sb, prec))
    assert rc == 0 and rep["certified"]
    if prec == "BF16_FP32":
        assert rep["iters_bf16"] >= 1
    V = oeig.canonical_signs(oeig.vectors_from_coefficients(configs.operator_rounded(prob), g["coef"]))
    check_against(prob, g["lam"], V, Z, eig, rep, 3, 1e-6)


GOLDEN_50K = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "grid_torus_1800x1000_l50000.npz")


@pytest.fixture(scope="module")
def grid_torus_50000():
    from synth import large
    prob = large.grid_torus_operator()
    g = np.load(GOLDEN_50K, allow_pickle=False)
    meta = json.loads(str(g["meta"]))
    assert meta["input_sha1"] == configs.input_digest(prob), "input differs from the one the stored values are for"
    V = oeig.canonical_signs(oeig.vectors_from_coefficients(configs.operator_rounded(prob), g["coef"]))
    return prob, g["lam"], V


@pytest.mark.parametrize("prec", ["FP32", "BF16_FP32"])
def test_grid_torus_50000_landmarks(gpu, grid_torus_50000, prec):
    # the largest workload's shape (n = 1.8M, l = 50,000, W 10 GB in float32)
    # on the seeded synthetic operator of synth.large, against the float64
    # oracle's eigenpairs (ARPACK route on the implicit operator, stored with
    # the sha1 of the input by tests/golden/make_grid_torus_50000.py):
    # eigenvalues within 1e-6, eigenvector clusters within the angle that
    # accuracy implies; the reported residuals agree with B applied on the host
    sb = gpu
    prob, lam, V = grid_torus_50000
    Z, eig, rep, rc, _ = run(sb, prob, 3, 16, getattr(sb, prec))
    assert rc == 0 and rep["certified"]
    if prec == "BF16_FP32":
        assert rep["iters_bf16"] >= 1
    check_against(prob, lam, V, Z, eig, rep, 3, 1e-6)
    Vg = np.asarray(Z, dtype=np.float64) / np.sqrt(np.asarray(eig[:3], dtype=np.float64))
    BV = oeig.apply_b(configs.operator_rounded(prob), prob["W"], Vg)
    for i in range(3):
        v = Vg[:, i]
        r = np.linalg.norm(BV[:, i] - eig[i] * v) / np.linalg.norm(v) / abs(eig[i])
        # Z comes back in float32: its rounding (unit 2^-24 per entry) adds up
        # to about 2^-24 |lambda_max| / |theta_i| to the host residual
        round_term = 4.0 * 2.0 ** -24 * max(abs(e) for e in eig[:3]) / abs(eig[i])
        print(f"  pair {i}: residual host {r:.3e} reported {rep['resid'][i]:.3e}", flush=True)
        assert r <= 1.2 * rep["resid"][i] + round_term


def test_tiny_landmark_count(gpu):
    sb = gpu
    prob = H.random_problem(n=50, l=3, row_len_max=3, seed=3)
    Z, eig, rep, rc, _ = run(sb, prob, 1, 2, sb.FP32)
    check(prob, Z, eig, rep, 1, 1e-6)


def test_bitwise_repeatable(gpu):
    sb = gpu
    prob = H.random_problem(n=20000, l=500, row_len_max=10, seed=11)
    Z1, e1, _, _, _ = run(sb, prob, 3, 16, sb.FP32)
    Z2, e2, _, _, _ = run(sb, prob, 3, 16, sb.FP32)
    np.testing.assert_array_equal(e1, e2)
    np.testing.assert_array_equal(Z1, Z2)


def test_resume_from_block(gpu):
    sb = gpu
    prob = H.random_problem(n=8000, l=400, row_len_max=10, seed=5)
    Z1, e1, rep1, _, X = run(sb, prob, 3, 16, sb.FP32)
    Z2, e2, rep2, rc, _ = run(sb, prob, 3, 16, sb.FP32, start=sb.START_USER, X0=X)
    assert rc == 0
    assert rep2["iters_fp32"] + rep2["iters_fp64"] <= rep1["iters_fp32"] + rep1["iters_fp64"]
    np.testing.assert_allclose(e2, e1, rtol=1e-7)


def test_device_inputs_match_host_inputs(gpu):
    sb = gpu
    import torch
    prob = H.random_problem(n=6000, l=200, row_len_max=8, seed=9)
    Zh, eh, _, _, _ = run(sb, prob, 3, 16, sb.FP32)
    dev = {k: (torch.from_numpy(v).cuda() if isinstance(v, np.ndarray) else v) for k, v in prob.items()}
    p = sb.Problem.from_arrays(dev["rowptr"], dev["col"], dev["val"], dev["W"])
    Zd = torch.zeros((prob["n"], 3), dtype=torch.float32, device="cuda")
    with sb.Context([p], k=3, block=16, prec=sb.FP32) as ctx:
        _, ed, _, _ = ctx.embed(Z_out=Zd)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(ed[0], eh)
    np.testing.assert_array_equal(Zd.cpu().numpy(), Zh)


@pytest.mark.parametrize("prec", ["FP32", "BF16_FP32"])
def test_repeated_calls_same_context(gpu, prec):
    # a context is reused across calls; buffers left by a previous call (in
    # another storage precision) must not leak into the next solve
    sb = gpu
    prob = H.random_problem(n=12000, l=700, row_len_max=10, seed=21)
    p = sb.Problem.from_arrays(prob["rowptr"], prob["col"], prob["val"], prob["W"])
    lam, _, _ = H.oracle_for(prob, 3)
    with sb.Context([p], k=3, block=16, prec=getattr(sb, prec)) as ctx:
        for call in range(3):
            Z, eig, reps, rc = ctx.embed()
            assert rc == 0 and reps[0]["certified"], (call, reps[0])
            assert H.rel_eig_err(eig[0], lam[:3]) <= 1e-6, call


def test_graph_replay_matches_eager_launches(gpu):
    # rounds of iterations replayed from captured graphs do the same work as
    # eager launches: same results to the bit, on every call of a context
    sb = gpu
    prob = H.random_problem(n=15000, l=600, row_len_max=10, seed=23)
    out = {}
    for flags in (0, sb.FLAG_NO_GRAPH):
        p = sb.Problem.from_arrays(prob["rowptr"], prob["col"], prob["val"], prob["W"])
        with sb.Context([p], k=3, block=16, prec=sb.BF16_FP32, flags=flags) as ctx:
            out[flags] = [ctx.embed() for _ in range(3)]
    for call in range(3):
        Zg, eg, rg, _ = out[0][call]
        Ze, ee, re_, _ = out[sb.FLAG_NO_GRAPH][call]
        np.testing.assert_array_equal(eg, ee)
        np.testing.assert_array_equal(Zg, Ze)
        assert rg[0]["certified"] and re_[0]["certified"]


@pytest.mark.parametrize("prec,block", [("FP32", 8), ("BF16_FP32", 16), ("FP32", 32), ("FP64", 16)])
def test_two_block_spmm_form(gpu, tmp_path, prec, block):
    # the row-split SpMM in its two-blocks-per-CU form, with the
    # Rayleigh-Ritz step in a launch of its own (what the tuner picks for
    # launches that move many bytes), forced through the tuning cache on an
    # operator the oracle solves in seconds; ragged rows, some empty
    sb = gpu
    fp64 = prec == "FP64"
    prob = H.random_problem(n=40000, l=700, row_len_max=14, seed=91 + block, empty_rows=0.05, long_rows=2,
                            dtype=np.float64 if fp64 else np.float32)
    modes = {"FP32": (1, 2), "BF16_FP32": (0, 1, 2), "FP64": (3,)}[prec]
    key = f"{prob['n']},{prob['l']},{len(prob['col'])}"
    path = tmp_path / "tune.txt"
    path.write_text("".join(f"v1;B={block};m={m};{key} 200 0 1024 4 8\n" for m in modes))
    tol = 1e-10 if fp64 else 1e-6
    Z, eig, rep, rc, _ = run(sb, prob, 3, block, getattr(sb, prec), tune_cache=str(path), max_iter=300, tol=tol)
    assert rc == 0 and rep["certified"]
    assert path.read_text().count(" 8\n") == len(modes)  # the forced entries were used, not retuned
    check(prob, Z, eig, rep, 3, tol)


def test_autotune_cache(gpu, tmp_path):
    # tuning at create writes one line per arithmetic of the schedule; a second
    # context with the same cache reuses the choices (same launch shapes, so
    # the same result to the bit), and the tuned solve still matches the oracle
    sb = gpu
    prob = H.random_problem(n=30000, l=900, row_len_max=10, seed=31)
    path = str(tmp_path / "tune.txt")
    p = sb.Problem.from_arrays(prob["rowptr"], prob["col"], prob["val"], prob["W"])
    with sb.Context([p], k=3, block=16, prec=sb.BF16_FP32, tune_cache=path) as ctx:
        Z1, e1, r1, rc = ctx.embed()
    lines = open(path).read().splitlines()
    print("\n".join(lines), flush=True)
    assert len(lines) == 3  # bf16, fp32 and the float64 certification
    for ln in lines:
        key, *vals = ln.split()
        assert len(vals) == 7 and int(vals[3]) in (1, 2, 4) and int(vals[4]) in (4, 8)
        assert int(vals[5]) in (0, 1) and int(vals[6]) in (8, 16, 32)
    assert rc == 0 and r1[0]["certified"]
    lam, _, _ = H.oracle_for(prob, 3)
    assert H.rel_eig_err(e1[0], lam[:3]) <= 1e-6
    p = sb.Problem.from_arrays(prob["rowptr"], prob["col"], prob["val"], prob["W"])
    with sb.Context([p], k=3, block=16, prec=sb.BF16_FP32, tune_cache=path) as ctx:
        Z2, e2, _, _ = ctx.embed()
    assert open(path).read().splitlines() == lines
    np.testing.assert_array_equal(e1, e2)
    np.testing.assert_array_equal(Z1, Z2)


@pytest.mark.parametrize("prec,block", [("FP32", 16), ("FP32", 8), ("FP32", 32), ("BF16_FP32", 16)])
def test_packed_w_matches_oracle(gpu, prec, block):
    # the dense product from the packed upper triangle of W (each stored
    # 64 x 64 tile applied to both U_i and U_j), forced at a size the oracle
    # solves in seconds; l = 1,500 leaves a partial last tile; the bf16 phase
    # keeps its full bf16 W, the float32 and certification phases read the
    # packed one.  Two solves: bitwise the same.
    sb = gpu
    prob = H.random_problem(n=20000, l=1500, row_len_max=10, seed=61 + block, empty_rows=0.05, long_rows=2)
    out = [run(sb, prob, 3, block, getattr(sb, prec), flags=sb.FLAG_PACK_W, max_iter=300) for _ in range(2)]
    Z, eig, rep, rc, _ = out[0]
    assert rc == 0 and rep["certified"]
    check(prob, Z, eig, rep, 3, 1e-6)
    np.testing.assert_array_equal(out[1][1], eig)
    np.testing.assert_array_equal(out[1][0], Z)


@pytest.mark.parametrize("cw", [8, 32])
def test_packed_w_region_widths(gpu, tmp_path, cw):
    # region widths of 8 and 32 tile columns forced through the tuning cache
    # (several region columns per region row at l = 2,100; float32 and the
    # float64-accumulated certification both packed)
    sb = gpu
    prob = H.random_problem(n=25000, l=2100, row_len_max=10, seed=71 + cw)
    key = f"{prob['n']},{prob['l']},{len(prob['col'])}"
    path = tmp_path / "tune.txt"
    path.write_text("".join(f"v1;B=16;m={m};{key} 256 1 512 1 4 1 {cw}\n" for m in (1, 2)))
    Z, eig, rep, rc, _ = run(sb, prob, 3, 16, sb.FP32, tune_cache=str(path), flags=sb.FLAG_PACK_W, max_iter=300)
    assert rc == 0 and rep["certified"]
    assert path.read_text().count(f" 1 {cw}\n") == 2  # the forced entries were used, not retuned
    check(prob, Z, eig, rep, 3, 1e-6)


@pytest.mark.parametrize("defect", ["w_asym", "w_nan", "p_nan", "col_order", "col_range", "rowptr"])
def test_device_inputs_validated_on_device(gpu, defect):
    # device-resident inputs are checked by kernels (they never reach the
    # host): every defect is refused with SBMDS_EINVAL and a message naming
    # it; the kernels clamp every index, so a malformed row pointer is read
    # safely
    sb = gpu
    import torch
    prob = H.random_problem(n=3000, l=120, row_len_max=8, seed=13)
    rp, col, val, W = (prob[x].copy() for x in ("rowptr", "col", "val", "W"))
    row = int(np.argmax(np.diff(rp) >= 2))  # a row with two entries or more
    if defect == "w_asym":
        W[5, 17] += 1.0
    elif defect == "w_nan":
        W[40, 3] = np.nan
        W[3, 40] = np.nan
    elif defect == "p_nan":
        val[rp[row]] = np.inf
    elif defect == "col_order":
        col[rp[row]], col[rp[row] + 1] = col[rp[row] + 1], col[rp[row]]
    elif defect == "col_range":
        col[rp[row]] = prob["l"] + 3
    else:
        rp[10] = rp[12] + 1  # decreasing at row 10 / 11
    dev = [torch.from_numpy(a).cuda() for a in (rp, col, val, W)]
    p = sb.Problem.from_arrays(*dev)
    with pytest.raises(sb.SbmdsError) as exc:
        sb.Context([p], k=3, block=16, prec=sb.FP32)
    want = {"w_asym": "not symmetric", "w_nan": "non-finite W", "p_nan": "non-finite P", "col_order": "strictly",
            "col_range": "out of range", "rowptr": "P_rowptr"}[defect]
    assert exc.value.code == -1 and want in str(exc.value), str(exc.value)
    torch.cuda.synchronize()


@pytest.mark.parametrize("prec", ["FP32", "BF16_FP32", "FP64"])
def test_push_form_transposed_product(gpu, prec):
    # the push form of P^T Y (SBMDS_FLAG_PUSH_T) on the 64 x 32 torus: the
    # oracle's eigenpairs, in each arithmetic (bf16 -> fp32 also reads the
    # previous phase's block in the push kernel)
    sb = gpu
    prob = dict(configs.torus64x32())
    tol = 1e-10 if prec == "FP64" else 1e-6
    if prec != "FP64":
        prob["val"] = prob["val"].astype(np.float32)
        prob["W"] = prob["W"].astype(np.float32)
    Z, eig, rep, rc, _ = run(sb, prob, 3, 16, getattr(sb, prec), tol=tol, flags=sb.FLAG_PUSH_T)
    assert rc == 0 and rep["certified"]
    check(prob, Z, eig, rep, 3, tol)
