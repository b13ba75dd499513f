"""The interpolation operator P of Eq. (PDefinition) built on the GPU
(cotangent assembly, M = L^T D^-1 L, dense Cholesky solve, per-column
thresholding of Section 3.1) through the C ABI, against the oracle's dense
brute-force chain (oracle.refchain) on small meshes and the generator's P
on the 64 x 32 torus: the kept index sets equal, values within 1e-10 of
the largest entry (needs a gfx950 GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import refchain as ref
from synth import configs, meshes

pytestmark = pytest.mark.gpu


def dense(rp, col, val, n, l):
    return sp.csr_matrix((val, col, rp), shape=(n, l)).toarray()


def compare(P, Pref, rtol=1e-10):
    np.testing.assert_array_equal(P != 0, Pref != 0)
    assert np.max(np.abs(P - Pref)) <= rtol * np.max(np.abs(Pref))


@pytest.mark.parametrize("p", [None, 6, 20])
def test_cotan_chain_matches_oracle(gpu, p):
    # jittered 12 x 8 torus (n = 96), 9 landmarks: the dense oracle chain
    sb = gpu
    V, F = meshes.torus_grid(12, 8, 1.0, 0.4, jitter=0.05, seed=7)
    lm = np.array([0, 13, 27, 40, 52, 61, 75, 83, 90])
    rp, col, val = sb.interpolation(V, F, lm, p=p)
    Mref, _, _ = ref.biharmonic_dense(V, F)
    Pref = ref.interp_dense(Mref, lm, p)
    P = dense(rp, col, val, V.shape[0], len(lm))
    compare(P, Pref)
    np.testing.assert_array_equal(P[lm], np.eye(len(lm)))  # identity rows of the landmarks
    assert np.all(np.diff(rp) >= 0) and rp[-1] == len(col)


def test_graph_variant_matches_oracle(gpu):
    sb = gpu
    V, F = meshes.deformed_icosphere(2, 3)
    lm = np.arange(0, V.shape[0], 9)
    rp, col, val = sb.interpolation(V, F, lm, p=12, graph=True)
    Mref = ref.graph_biharmonic_dense(V.shape[0], F)
    compare(dense(rp, col, val, V.shape[0], len(lm)), ref.interp_dense(Mref, lm, 12))


def test_torus64x32_matches_generator(gpu):
    # the 64 x 32 torus of the small configuration (n = 2048, 64 FPS
    # landmarks, p = 310): the generator's sparse-LU P (pinned to the oracle
    # chain at small sizes) is reproduced
    sb = gpu
    prob = configs.torus64x32()
    rp, col, val = sb.interpolation(prob["V"], prob["F"], prob["landmarks"], p=prob["p"])
    np.testing.assert_array_equal(rp, prob["rowptr"])
    np.testing.assert_array_equal(col, prob["col"])
    ref_val = np.asarray(prob["val"], dtype=np.float64)
    assert np.max(np.abs(val - ref_val)) <= 1e-10 * np.max(np.abs(ref_val))


def test_bad_inputs(gpu):
    sb = gpu
    V, F = meshes.torus_grid(6, 4, 1.0, 0.4, jitter=0.05, seed=1)
    with pytest.raises(sb.SbmdsError) as exc:
        sb.interpolation(V, F, np.array([1, 5, 1]), p=4)
    assert "repeated" in str(exc.value)
    bad = F.copy()
    bad[3, 1] = V.shape[0]
    with pytest.raises(sb.SbmdsError) as exc:
        sb.interpolation(V, bad, np.array([1, 5]), p=4)
    assert "face" in str(exc.value)
