"""Float64 reference of the learned warm start: landmark features, the MLP,
its alignment loss, gradients and the Adam update.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper has no learned component; this part only seeds the eigensolver
of Section 3.3, so every result it produces is judged by the certified
residual of the solve it starts.  The definitions below are this project's
own and are written out plainly:

features (19 per landmark j of a mesh)
  0..2   landmark position minus the centroid of all landmark positions,
         divided by their root-mean-square distance to that centroid
  3..6   mean of u, u^2, u^3, u^4 over the other landmarks i != j, where
         u_i = d_ji / max_i d_ji and d_ji = sqrt(W_ji) (W holds squared
         geodesic distances, as in Section 3.3)
  7      standard deviation of u
  8..17  fraction of the u_i in each of 10 equal bins of [0, 1]
         (bin index floor(10 u), u = 1 in the last bin)
  18     max_i d_ji divided by its maximum over all landmarks

network  y = W3^T g(W2^T g(W1^T x + b1) + b2) + b3 on standardised
         features x; g(z) = z Phi(z) (GELU with the normal CDF)

loss     per mesh m with predicted rows Y_m and target rows T_m (the
         landmark rows of a converged embedding):
           L_m = min_A ( ||Y_m A - T_m||_F^2 + delta_m ||A||_F^2 ) / ||T_m||_F^2,
         A any k x k matrix, delta_m = 1e-4 * rows_m; the loss is the mean of
         L_m.  Only the span of a start block matters to subspace iteration,
         so the loss is invariant (for delta -> 0) under Y -> Y A.  The
         minimiser is A* = (Y^T Y + delta I)^{-1} Y^T T, and because A is
         minimised out, dL_m/dY_m = 2 (Y_m A* - T_m) A*^T / ||T_m||^2.

Adam     Kingma & Ba (2015) with bias correction.
"""
from __future__ import annotations

import math

import numpy as np

N_FEAT = 19
N_HIST = 10
HIDDEN = 128
RIDGE = 1e-4


# ---------------------------------------------------------------------------
# features
# ---------------------------------------------------------------------------
def features(xyz: np.ndarray, landmarks: np.ndarray, W: np.ndarray) -> np.ndarray:
    """[l, 19] float64 features of one mesh (W: l x l squared distances)."""
    X = np.asarray(xyz, dtype=np.float64)[np.asarray(landmarks)]
    l = X.shape[0]
    W = np.asarray(W, dtype=np.float64)
    F = np.zeros((l, N_FEAT))
    c = X.mean(axis=0)
    r = math.sqrt(float(np.mean(np.sum((X - c) ** 2, axis=1))))
    F[:, 0:3] = (X - c) / (r if r > 0 else 1.0)
    rowmax = np.zeros(l)
    for j in range(l):
        w = np.delete(W[j], j)
        d = np.sqrt(np.maximum(w, 0.0))
        m = d.max() if d.size else 0.0
        rowmax[j] = m
        u = d / m if m > 0 else np.zeros_like(d)
        cnt = max(d.size, 1)
        mom = [float(np.sum(u ** p)) / cnt for p in (1, 2, 3, 4)]
        F[j, 3:7] = mom
        F[j, 7] = math.sqrt(max(mom[1] - mom[0] * mom[0], 0.0))
        bins = np.minimum(np.floor(u * N_HIST).astype(np.int64), N_HIST - 1)
        F[j, 8:8 + N_HIST] = np.bincount(bins, minlength=N_HIST) / cnt
    gmax = rowmax.max()
    F[:, 18] = rowmax / gmax if gmax > 0 else 0.0
    return F


# ---------------------------------------------------------------------------
# network
# ---------------------------------------------------------------------------
def gelu(z):
    z = np.asarray(z, dtype=np.float64)
    erf = np.vectorize(math.erf)
    return 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))


def gelu_grad(z):
    z = np.asarray(z, dtype=np.float64)
    erf = np.vectorize(math.erf)
    return 0.5 * (1.0 + erf(z / math.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)


def param_shapes(k: int, hidden: int = HIDDEN, n_in: int = N_FEAT):
    """Names and shapes in the order of the flat parameter vector."""
    return [("W1", (n_in, hidden)), ("b1", (hidden,)), ("W2", (hidden, hidden)), ("b2", (hidden,)),
            ("W3", (hidden, k)), ("b3", (k,))]


def n_params(k: int, hidden: int = HIDDEN, n_in: int = N_FEAT) -> int:
    return sum(int(np.prod(s)) for _, s in param_shapes(k, hidden, n_in))


def unpack(theta: np.ndarray, k: int, hidden: int = HIDDEN, n_in: int = N_FEAT) -> dict:
    out, o = {}, 0
    for name, shape in param_shapes(k, hidden, n_in):
        size = int(np.prod(shape))
        out[name] = np.asarray(theta[o:o + size], dtype=np.float64).reshape(shape)
        o += size
    return out


def pack(p: dict, k: int, hidden: int = HIDDEN, n_in: int = N_FEAT) -> np.ndarray:
    return np.concatenate([np.asarray(p[name], dtype=np.float64).ravel()
                           for name, _ in param_shapes(k, hidden, n_in)])


def standardise(F, mean, std):
    return (np.asarray(F, dtype=np.float64) - mean) / std


def forward(theta, X, k, hidden=HIDDEN):
    """Returns the output [rows, k] and the cache needed by backward."""
    p = unpack(theta, k, hidden, X.shape[1])
    z1 = X @ p["W1"] + p["b1"]
    h1 = gelu(z1)
    z2 = h1 @ p["W2"] + p["b2"]
    h2 = gelu(z2)
    y = h2 @ p["W3"] + p["b3"]
    return y, (X, z1, h1, z2, h2, p)


def backward(cache, dY, k, hidden=HIDDEN):
    """Gradient of a scalar with respect to the flat parameters, given dY."""
    X, z1, h1, z2, h2, p = cache
    g = {}
    g["W3"] = h2.T @ dY
    g["b3"] = dY.sum(axis=0)
    dz2 = (dY @ p["W3"].T) * gelu_grad(z2)
    g["W2"] = h1.T @ dz2
    g["b2"] = dz2.sum(axis=0)
    dz1 = (dz2 @ p["W2"].T) * gelu_grad(z1)
    g["W1"] = X.T @ dz1
    g["b1"] = dz1.sum(axis=0)
    return pack(g, k, hidden, X.shape[1])


# ---------------------------------------------------------------------------
# loss
# ---------------------------------------------------------------------------
def aligned_loss(Y, T, seg):
    """Mean over meshes of the alignment loss and its gradient dL/dY.
    seg: row offsets [nseg + 1] of the meshes in Y and T."""
    Y = np.asarray(Y, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    k = Y.shape[1]
    nseg = len(seg) - 1
    dY = np.zeros_like(Y)
    total = 0.0
    for m in range(nseg):
        a, b = int(seg[m]), int(seg[m + 1])
        Ym, Tm = Y[a:b], T[a:b]
        delta = RIDGE * (b - a)
        tt = float(np.sum(Tm * Tm))
        A = np.linalg.solve(Ym.T @ Ym + delta * np.eye(k), Ym.T @ Tm)
        R = Ym @ A - Tm
        total += (float(np.sum(R * R)) + delta * float(np.sum(A * A))) / tt
        dY[a:b] = 2.0 * (R @ A.T) / tt / nseg
    return total / nseg, dY


def loss_and_grad(theta, X, T, seg, k, hidden=HIDDEN):
    y, cache = forward(theta, X, k, hidden)
    L, dY = aligned_loss(y, T, seg)
    return L, backward(cache, dY, k, hidden)


# ---------------------------------------------------------------------------
# Adam
# ---------------------------------------------------------------------------
def adam_step(theta, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update (t counts from 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
