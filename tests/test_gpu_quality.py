"""Rows of the sparse biharmonic approximation K~ = P L P^T and their
relative error on a row subset (Section 4.1's eps), on the GPU through the C
ABI, against the float64 oracle (oracle.mds.approx_rows / approx_error_rows)
on the same rounded values (needs a gfx950 GPU)."""
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
