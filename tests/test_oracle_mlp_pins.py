"""Pins of the float64 warm-start reference (oracle/mlp.py) against values
and properties fixed by the mathematics: hand-computed features, invariances,
the normal CDF, finite differences and the first Adam step."""
import math

import numpy as np
import pytest

from oracle import mlp as om


def test_gelu_values():
    # g(z) = z Phi(z); Phi(1) = 0.8413447460685429 (standard normal CDF)
    assert om.gelu(np.array([1.0]))[0] == pytest.approx(0.8413447460685429, rel=1e-15)
    assert om.gelu(np.array([0.0]))[0] == 0.0
    z = np.linspace(-4, 4, 17)
    np.testing.assert_allclose(om.gelu(z) - om.gelu(-z), z, atol=1e-15)  # Phi(z) + Phi(-z) = 1
    h = 1e-6
    fd = (om.gelu(z + h) - om.gelu(z - h)) / (2 * h)
    np.testing.assert_allclose(om.gelu_grad(z), fd, atol=1e-9)


def line_case():
    # four landmarks on a line at 0, 1, 2, 4 (mesh vertices 0..3)
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [2, 0, 0], [4, 0, 0]])
    x = xyz[:, 0]
    W = (x[:, None] - x[None, :]) ** 2
    return xyz, np.arange(4), W


def test_features_by_hand():
    xyz, lm, W = line_case()
    F = om.features(xyz, lm, W)
    # row 0: d = (1, 2, 4), max 4, u = (1/4, 1/2, 1)
    assert F[0, 3] == pytest.approx(1.75 / 3)
    assert F[0, 4] == pytest.approx(1.3125 / 3)
    assert F[0, 5] == pytest.approx((1 / 64 + 1 / 8 + 1) / 3)
    assert F[0, 7] == pytest.approx(math.sqrt(1.3125 / 3 - (1.75 / 3) ** 2))
    hist = np.zeros(10)
    hist[[2, 5, 9]] = 1 / 3
    np.testing.assert_allclose(F[0, 8:18], hist)
    # row 2: d = (2, 1, 2), max 2, u = (1, 1/2, 1)
    assert F[2, 3] == pytest.approx(2.5 / 3)
    hist = np.zeros(10)
    hist[5], hist[9] = 1 / 3, 2 / 3
    np.testing.assert_allclose(F[2, 8:18], hist)
    # row maxima 4, 3, 2, 4 over a global maximum of 4
    np.testing.assert_allclose(F[:, 18], [1.0, 0.75, 0.5, 1.0])
    # positions: centroid 1.75, rms distance sqrt(mean((x - 1.75)^2))
    x = np.array([0, 1, 2, 4.0])
    r = math.sqrt(np.mean((x - 1.75) ** 2))
    np.testing.assert_allclose(F[:, 0], (x - 1.75) / r)
    np.testing.assert_allclose(F[:, 1:3], 0.0)


def test_features_two_landmarks_and_equal_distances():
    xyz = np.array([[0.0, 0, 0], [0, 2, 0], [5, 5, 5]])
    F = om.features(xyz, np.array([0, 1]), np.array([[0.0, 4.0], [4.0, 0.0]]))
    np.testing.assert_allclose(F[:, 3:7], 1.0)
    np.testing.assert_allclose(F[:, 7], 0.0)
    np.testing.assert_allclose(F[:, 17], 1.0)      # u = 1 falls in the last bin
    np.testing.assert_allclose(F[:, 8:17], 0.0)
    np.testing.assert_allclose(F[:, 18], 1.0)
    np.testing.assert_allclose(F[:, 1], [-1.0, 1.0])


def test_features_invariances():
    rng = np.random.default_rng(0)
    l = 30
    pts = rng.standard_normal((l, 3))
    W = ((pts[:, None] - pts[None]) ** 2).sum(-1)
    lm = np.arange(l)
    F = om.features(pts, lm, W)
    # translation and scaling of the mesh; distances scaled consistently
    np.testing.assert_allclose(om.features(3.0 * pts + 7.0, lm, 9.0 * W), F, atol=1e-12)
    # relabelling the landmarks permutes the rows
    perm = rng.permutation(l)
    Fp = om.features(pts[perm], lm, W[np.ix_(perm, perm)])
    np.testing.assert_allclose(Fp, F[perm], atol=1e-12)
    np.testing.assert_allclose(F[:, 8:18].sum(axis=1), 1.0)
    assert F[:, 18].max() == 1.0


def small_net(k=2, hidden=6, rows=(5, 7, 6), seed=1):
    rng = np.random.default_rng(seed)
    n = sum(rows)
    X = rng.standard_normal((n, om.N_FEAT))
    T = rng.standard_normal((n, k))
    seg = np.concatenate([[0], np.cumsum(rows)])
    theta = 0.4 * rng.standard_normal(om.n_params(k, hidden))
    return theta, X, T, seg, k, hidden


def test_aligned_loss_span_invariance(monkeypatch):
    monkeypatch.setattr(om, "RIDGE", 0.0)
    rng = np.random.default_rng(2)
    Y = rng.standard_normal((20, 3))
    T = rng.standard_normal((20, 3))
    seg = np.array([0, 20])
    A = rng.standard_normal((3, 3)) + 3 * np.eye(3)
    L1, _ = om.aligned_loss(Y, T, seg)
    L2, _ = om.aligned_loss(Y @ A, T, seg)
    assert L1 == pytest.approx(L2, rel=1e-10)
    L0, g0 = om.aligned_loss(T @ A, T, seg)
    assert abs(L0) < 1e-20 and np.abs(g0).max() < 1e-12
    # a prediction orthogonal to the target explains nothing
    Q, _ = np.linalg.qr(rng.standard_normal((20, 6)))
    Lo, _ = om.aligned_loss(Q[:, :3], Q[:, 3:] * 2.0, seg)
    assert Lo == pytest.approx(1.0, abs=1e-12)


def test_aligned_loss_gradient_fd():
    rng = np.random.default_rng(3)
    Y = rng.standard_normal((13, 2))
    T = rng.standard_normal((13, 2))
    seg = np.array([0, 6, 13])
    _, g = om.aligned_loss(Y, T, seg)
    h = 1e-6
    fd = np.zeros_like(Y)
    for i in range(Y.shape[0]):
        for j in range(Y.shape[1]):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, j] += h
            Ym[i, j] -= h
            fd[i, j] = (om.aligned_loss(Yp, T, seg)[0] - om.aligned_loss(Ym, T, seg)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, atol=1e-8)


def test_network_gradient_fd():
    theta, X, T, seg, k, hidden = small_net()
    _, g = om.loss_and_grad(theta, X, T, seg, k, hidden)
    h = 1e-6
    fd = np.zeros_like(theta)
    for i in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[i] += h
        tm[i] -= h
        fd[i] = (om.loss_and_grad(tp, X, T, seg, k, hidden)[0] - om.loss_and_grad(tm, X, T, seg, k, hidden)[0]) / (2 * h)
    np.testing.assert_allclose(g, fd, atol=1e-8, rtol=1e-5)


def test_parameter_count_and_layout():
    assert om.n_params(3) == 19 * 128 + 128 + 128 * 128 + 128 + 128 * 3 + 3 == 19459
    theta = np.arange(om.n_params(3), dtype=np.float64)
    p = om.unpack(theta, 3)
    assert p["W1"][0, 1] == 1 and p["b1"][0] == 19 * 128 and p["b3"][-1] == theta[-1]
    np.testing.assert_array_equal(om.pack(p, 3), theta)


def test_adam_first_step():
    g = np.array([0.3, -2.0, 1e-3, 0.0])
    th, m, v = om.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01)
    # bias-corrected moments of the first step are g and g^2
    np.testing.assert_allclose(th, -0.01 * g / (np.abs(g) + 1e-8))
    np.testing.assert_allclose(m, 0.1 * g)
    np.testing.assert_allclose(v, 0.001 * g * g)
