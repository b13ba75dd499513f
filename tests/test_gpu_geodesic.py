"""Farthest-point landmarks and the landmark block W = D_ll o D_ll on the GPU
(Section 3, Eq. (FarthestPoint)) through the C ABI, against the oracle:
all-pairs textbook Dijkstra (oracle.refchain.dijkstra_heap), the literal
farthest-point loop (oracle.refchain.fps_literal) and W taken from those
distances.  Landmark ids and W are compared bit for bit (needs a gfx950
GPU)."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import refchain as ref
from synth import configs, meshes
from synth import operator as op

pytestmark = pytest.mark.gpu


def oracle_chain(G, l, first):
    n = G.shape[0]
    U = sp.triu(G).tocoo()
    edges = [(int(a), int(b), float(w)) for a, b, w in zip(U.row, U.col, U.data)]
    D = np.array([ref.dijkstra_heap(n, edges, s) for s in range(n)])
    lm = ref.fps_literal(D, l, first)
    Dl = D[np.ix_(lm, lm)]
    W = Dl * Dl
    W = 0.5 * (W + W.T)
    np.fill_diagonal(W, 0.0)
    return lm, W


def graph_arrays(G):
    G = sp.csr_matrix(G)
    G.sort_indices()
    return G.indptr.astype(np.int32), G.indices.astype(np.int32), G.data.astype(np.float64)


@pytest.mark.parametrize("l,first,batch", [(40, 0, 64), (40, 311, 7), (1, 5, 64)])
def test_fps_and_w_match_oracle(gpu, l, first, batch):
    # deformed icosphere of level 3 (n = 642): landmarks and W bit for bit;
    # batch 7 leaves a ragged last group of sources
    sb = gpu
    V, F = meshes.deformed_icosphere(3, 11)
    G = op.edge_graph(V, F)
    lm_ref, W_ref = oracle_chain(G, l, first)
    lm, W = sb.landmarks_geodesic(*graph_arrays(G), l, first, batch=batch)
    np.testing.assert_array_equal(lm, lm_ref)
    np.testing.assert_array_equal(W, W_ref)


def test_every_vertex_and_two_components(gpu):
    # l = n on a small torus; then two disjoint copies of it: the second
    # copy's vertices are infinitely far (+inf in W, and the farthest point
    # jumps there on the second step)
    sb = gpu
    V, F = meshes.torus_grid(8, 6, 1.0, 0.4, jitter=0.05, seed=3)
    G = op.edge_graph(V, F)
    n = G.shape[0]
    lm_ref, W_ref = oracle_chain(G, n, 7)
    lm, W = sb.landmarks_geodesic(*graph_arrays(G), n, 7)
    np.testing.assert_array_equal(lm, lm_ref)
    np.testing.assert_array_equal(W, W_ref)
    G2 = sp.block_diag([G, G]).tocsr()
    lm_ref, W_ref = oracle_chain(G2, 10, 0)
    lm, W = sb.landmarks_geodesic(*graph_arrays(G2), 10, 0)
    np.testing.assert_array_equal(lm, lm_ref)
    np.testing.assert_array_equal(W, W_ref)
    assert np.isinf(W).any()


def test_device_inputs_and_bad_graph(gpu):
    sb = gpu
    import torch
    V, F = meshes.deformed_icosphere(2, 5)
    G = op.edge_graph(V, F)
    arrs = graph_arrays(G)
    lm_h, W_h = sb.landmarks_geodesic(*arrs, 20, 3)
    lm_d, W_d = sb.landmarks_geodesic(*[torch.from_numpy(a).cuda() for a in arrs], 20, 3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(lm_d.cpu().numpy(), lm_h)
    np.testing.assert_array_equal(W_d.cpu().numpy(), W_h)
    lm_only, none = sb.landmarks_geodesic(*arrs, 20, 3, want_W=False)
    assert none is None
    np.testing.assert_array_equal(lm_only, lm_h)
    rp, ci, w = arrs
    bad = w.copy()
    bad[5] = -1.0
    with pytest.raises(sb.SbmdsError) as exc:
        sb.landmarks_geodesic(rp, ci, bad, 20, 3)
    assert "weight" in str(exc.value)


def test_sphere7_matches_generator(gpu):
    # the level-7 sphere of the sphere workload (n = 163,842, 2,000
    # landmarks): the device reproduces the generator's landmarks and its
    # float32 W exactly (the generator's farthest-point search and Dijkstra
    # are pinned to the oracle's definitions at small sizes)
    sb = gpu
    prob = configs.sphere7()
    G = op.edge_graph(prob["V"], prob["F"])
    lm, W = sb.landmarks_geodesic(*graph_arrays(G), prob["l"], int(prob["landmarks"][0]), batch=128)
    np.testing.assert_array_equal(lm, np.asarray(prob["landmarks"]))
    np.testing.assert_array_equal(W.astype(np.float32), prob["W"])
