"""Rows of the sparse biharmonic approximation K~ = P L P^T and their
relative error on a row subset (Section 4.1's eps), and the stress of an
embedding (Eq. (MDS_problem)), on the GPU through the C ABI, against the
float64 oracle (oracle.mds.approx_rows / approx_error_rows / strain) on the
same rounded values (needs a gfx950 GPU)."""
import numpy as np
import pytest
import scipy.sparse.csgraph as csgraph

from oracle import mds as omds
from synth import configs
from synth import operator as op
from tests import helpers as H

pytestmark = pytest.mark.gpu


def torus_case(dtype):
    prob = configs.torus64x32()  # float64 chain
    G = op.edge_graph(prob["V"], prob["F"])
    D = csgraph.dijkstra(G, directed=False)
    lm = np.asarray(prob["landmarks"])
    rng = np.random.default_rng(17)
    rows = np.concatenate([lm[:3], rng.choice(prob["n"], 61, replace=False)]).astype(np.int32)
    val = prob["val"].astype(dtype)
    Lll = D[np.ix_(lm, lm)]
    L = (0.5 * (Lll + Lll.T)).astype(dtype)  # Dijkstra's last-bit asymmetry removed (L must be symmetric)
    K = D[rows].astype(dtype)
    return prob, val, L, rows, K


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_torus_distance_rows_match_oracle(gpu, dtype):
    # the geodesic distance approximation of the 64 x 32 torus (64 landmarks,
    # p_row = 10): eps on 64 rows (3 landmark rows among them) and the rows
    # themselves, float64 arithmetic on both sides from the same values
    sb = gpu
    prob, val, L, rows, K = torus_case(dtype)
    P = configs.operator_rounded(dict(prob, val=val))
    eps, (num, den), Kt = sb.approx_rows(prob["rowptr"], prob["col"], val, L, rows, K_rows=K, want_rows=True)
    ref_rows = omds.approx_rows(P, L.astype(np.float64), rows)
    ref = omds.approx_error_rows(P, L.astype(np.float64), rows, K.astype(np.float64))
    print(f"{np.dtype(dtype).name}: eps {eps:.6e} oracle {ref:.6e}", flush=True)
    np.testing.assert_allclose(Kt, ref_rows, rtol=1e-12, atol=1e-12 * np.abs(ref_rows).max())
    assert abs(eps - ref) <= 1e-10 * ref
    # landmark rows interpolate their row of L (Eq. (PDefinition)'s identity rows)
    lmrow = np.asarray(prob["landmarks"])[:3]
    np.testing.assert_allclose(Kt[:3][:, lmrow], L[:3, :3].astype(np.float64), rtol=1e-12, atol=0)


def test_device_inputs_and_ragged_rows(gpu):
    # device-resident inputs give the host-input result bit for bit; a vertex
    # whose row of P is empty gets a zero row of K~; rows out of range are refused
    sb = gpu
    import torch
    prob = H.random_problem(n=4000, l=150, row_len_max=9, seed=41, empty_rows=0.1, long_rows=2)
    rp = prob["rowptr"]
    empty = np.flatnonzero(np.diff(rp) == 0)[:2]
    rows = np.concatenate([empty, np.arange(10)]).astype(np.int32)
    L = prob["W"]
    rng = np.random.default_rng(2)
    K = rng.random((len(rows), prob["n"])).astype(np.float32)
    eh, nh, Kh = sb.approx_rows(rp, prob["col"], prob["val"], L, rows, K_rows=K, want_rows=True)
    dev = [torch.from_numpy(a).cuda() for a in (rp, prob["col"], prob["val"], L, rows, K)]
    ed, nd, Kd = sb.approx_rows(*dev[:5], K_rows=dev[5], want_rows=True)
    torch.cuda.synchronize()
    assert nh == nd
    np.testing.assert_array_equal(Kd.cpu().numpy(), Kh)
    assert np.all(Kh[:len(empty)] == 0.0)
    ref = omds.approx_error_rows(configs.operator_rounded(prob), L.astype(np.float64), rows, K.astype(np.float64))
    assert abs(eh - ref) <= 1e-10 * ref
    bad = rows.copy()
    bad[1] = prob["n"]
    with pytest.raises(sb.SbmdsError) as exc:
        sb.approx_rows(rp, prob["col"], prob["val"], L, bad, K_rows=K)
    assert "out of range" in str(exc.value)


def distance_case(n_sub=None):
    prob = configs.torus64x32()
    G = op.edge_graph(prob["V"], prob["F"])
    D = csgraph.dijkstra(G, directed=False)
    D = 0.5 * (D + D.T)
    if n_sub is not None:
        D = D[:n_sub, :n_sub]
    return D


@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_stress_matches_oracle(gpu, dtype):
    # exact classical MDS of the torus distances (3-D) and a perturbed copy
    # of it: the stress and its scale against the oracle's dense
    # ||Z Z^T + 1/2 J E J||_F on the same rounded values; n = 2047 leaves a
    # ragged last block of rows and a ragged column step
    sb = gpu
    D = distance_case(2047)
    E = D * D
    _, Z = omds.classical_mds(E, 3)
    rng = np.random.default_rng(5)
    for Zc in (Z, Z + 0.05 * rng.standard_normal(Z.shape)):
        Kc = D.astype(dtype)
        Zr = Zc.astype(dtype)
        st, scale = sb.stress(Zr, Kc)
        E64 = Kc.astype(np.float64) ** 2
        ref = omds.strain(Zr.astype(np.float64), E64)
        ref_scale = omds.strain(np.zeros((D.shape[0], 1)), E64)
        print(f"{np.dtype(dtype).name}: stress {st:.9e} oracle {ref:.9e} scale {scale:.6e}", flush=True)
        assert abs(st - ref) <= 1e-9 * ref_scale
        assert abs(scale - ref_scale) <= 1e-10 * ref_scale


def test_stress_device_inputs_many_dims_and_tiny(gpu):
    # device inputs equal host inputs bit for bit; m = 16 (the largest
    # supported); n = 1..5 (a single partial row block)
    sb = gpu
    import torch
    D = distance_case(300)
    rng = np.random.default_rng(6)
    Z = rng.standard_normal((300, 16))
    h = sb.stress(Z, D)
    d = sb.stress(torch.from_numpy(Z).cuda(), torch.from_numpy(D).cuda())
    assert h == d
    ref = omds.strain(Z, D * D)
    assert abs(h[0] - ref) <= 1e-10 * ref
    for n in (1, 2, 5):
        Zs, Ds = Z[:n, :2].copy(), D[:n, :n].copy()
        st, scale = sb.stress(Zs, Ds)
        ref = omds.strain(Zs, Ds * Ds)
        assert abs(st - ref) <= 1e-10 * max(ref, 1e-300) + 1e-12 * max(scale, 1.0)
    with pytest.raises(sb.SbmdsError):
        sb.stress(rng.standard_normal((10, 17)), D[:10, :10])
