"""Seeded synthetic operator at the size of the paper's largest workload
(a 1.8M-vertex torus with 50,000 landmarks), built in seconds instead of the
hours that the cotangent biharmonic solve and the geodesics would take on
the host.

It keeps the shapes and structure the embedding path sees, not the exact
biharmonic values:

* vertices on a bumpy torus grid of nu x nv (vertex id i * nv + j, so rows
  of P are in spatial order along the grid), landmarks on a regular lu x lv
  sub-grid (landmark id a * lv + b);
* P: a landmark's row is the identity (Section 3.1 keeps landmark rows of
  P as unit rows); every other row holds its `nbr` nearest landmarks in the
  grid's parameter space (periodic), with Gaussian weights normalised to
  sum 1, which is what the unthresholded biharmonic rows sum to;
* W = D^2 + 0.3 D for D the Euclidean distances between the landmarks'
  positions: a squared-distance-like matrix that is not exactly Euclidean,
  so B has a full spectrum with negative eigenvalues, like squared geodesics.

Holds none of the embedding arithmetic.
"""
from __future__ import annotations

import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np


def _positions(i, j, nu, nv, phases):
    u = 2.0 * np.pi * i / nu
    v = 2.0 * np.pi * j / nv
    r = 0.4 + 0.02 * np.sin(3.0 * u + phases[0]) * np.sin(5.0 * v + phases[1])
    return np.stack([(1.0 + r * np.cos(v)) * np.cos(u), (1.0 + r * np.cos(v)) * np.sin(u), r * np.sin(v)], axis=-1)


def grid_torus_operator(nu=1800, nv=1000, lu=250, lv=200, nbr=10, seed=5005, chunk=200_000):
    """Returns {"n", "l", "rowptr", "col", "val", "W"} (int32 CSR, float32
    values and W) of the operator described in the module docstring."""
    assert nu >= 2 * lu and nv >= 2 * lv, "landmark spacing of at least two vertices"
    rng = np.random.default_rng(seed)
    phases = rng.uniform(0.0, 2.0 * np.pi, size=2)
    n, l = nu * nv, lu * lv
    # landmark (a, b) sits at vertex (round(a nu / lu), round(b nv / lv))
    ai = np.rint(np.arange(lu) * nu / lu).astype(np.int64)
    bj = np.rint(np.arange(lv) * nv / lv).astype(np.int64)
    lm_vertex = (ai[:, None] * nv + bj[None, :]).ravel()
    is_lm = np.full(n, -1, dtype=np.int64)
    is_lm[lm_vertex] = np.arange(l)
    # candidate landmarks: the 5 x 5 landmark cells around the vertex
    da, db = np.meshgrid(np.arange(-2, 3), np.arange(-2, 3), indexing="ij")
    da, db = da.ravel(), db.ravel()
    counts = np.empty(n, dtype=np.int64)
    cols, vals = [], []
    for v0 in range(0, n, chunk):
        vid = np.arange(v0, min(n, v0 + chunk))
        i, j = vid // nv, vid % nv
        x, y = i * lu / nu, j * lv / nv                   # position in landmark units
        ca = (np.floor(x)[:, None] + da[None, :]).astype(np.int64)
        cb = (np.floor(y)[:, None] + db[None, :]).astype(np.int64)
        dx = x[:, None] - ca
        dy = y[:, None] - cb
        d2 = dx * dx + dy * dy
        keep = np.argpartition(d2, nbr - 1, axis=1)[:, :nbr]
        d2k = np.take_along_axis(d2, keep, axis=1)
        cid = (np.take_along_axis(ca, keep, axis=1) % lu) * lv + np.take_along_axis(cb, keep, axis=1) % lv
        w = np.exp(-d2k)
        w /= w.sum(axis=1, keepdims=True)
        order = np.argsort(cid, axis=1, kind="stable")
        cid = np.take_along_axis(cid, order, axis=1)
        w = np.take_along_axis(w, order, axis=1)
        lmk = is_lm[vid]
        c = np.where(lmk[:, None] >= 0, np.where(np.arange(nbr)[None, :] == 0, lmk[:, None], -1), cid)
        wv = np.where(lmk[:, None] >= 0, np.where(np.arange(nbr)[None, :] == 0, 1.0, 0.0), w)
        m = c >= 0
        counts[vid] = m.sum(axis=1)
        cols.append(c[m].astype(np.int32))
        vals.append(wv[m].astype(np.float32))
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=rowptr[1:])
    assert rowptr[-1] < 2**31
    col = np.concatenate(cols)
    val = np.concatenate(vals)
    # W = D^2 + 0.3 D between landmark positions, symmetric with a zero
    # diagonal: every entry from the same float32 expression of the
    # coordinate differences (a negated difference squares to the same
    # value), so W is exactly symmetric; row blocks on worker threads
    pos = _positions(ai[:, None].repeat(lv, 1).ravel(), bj[None, :].repeat(lu, 0).ravel(), nu, nv,
                     phases).astype(np.float32)
    W = np.empty((l, l), dtype=np.float32)

    def rows(r0):
        r1 = min(l, r0 + 256)
        d2 = np.zeros((r1 - r0, l), dtype=np.float32)
        for c in range(3):
            t = pos[r0:r1, c, None] - pos[None, :, c]
            d2 += t * t
        d = np.sqrt(d2)
        W[r0:r1] = d * d + np.float32(0.3) * d

    with ThreadPoolExecutor(min(16, os.cpu_count() or 1)) as ex:
        list(ex.map(rows, range(0, l, 256)))
    np.fill_diagonal(W, 0.0)
    return {"n": n, "l": l, "rowptr": rowptr.astype(np.int32), "col": col, "val": val, "W": W,
            "landmarks": lm_vertex.astype(np.int32), "shape": (nu, nv, lu, lv), "phases": phases}


def grid_torus_positions(prob):
    """Vertex positions (n x 3, float32) of a grid-torus operator's mesh, in
    vertex order (the landmark rows of this array are the positions W was
    built from)."""
    nu, nv, _, _ = prob["shape"]
    out = np.empty((nu * nv, 3), dtype=np.float32)
    jj = np.arange(nv)
    for i0 in range(0, nu, 256):
        i1 = min(nu, i0 + 256)
        ii = np.arange(i0, i1)
        out[i0 * nv:i1 * nv] = _positions(np.repeat(ii, nv), np.tile(jj, i1 - i0), nu, nv,
                                          prob["phases"]).astype(np.float32)
    return out


def grid_torus_family(count=48, nmin=8000, nmax=60000, seed0=5100):
    """Smaller operators of the largest workload's recipe for training its
    start network: n_i uniform in [nmin, nmax] (default_rng(seed0)), the
    1800 x 1000 grid's aspect ratio and landmark spacing (n_u / n_v = 1.8,
    7.2 x 5 vertices per landmark), seeds seed0 + 1 + i."""
    rng = np.random.default_rng(seed0)
    out = []
    for i, ni in enumerate(rng.integers(nmin, nmax + 1, size=count)):
        nv = max(10, int(round(np.sqrt(ni / 1.8))))
        nu = max(10, int(round(1.8 * nv)))
        lu = max(5, int(round(nu / 7.2)))
        lv = max(5, int(round(nv / 5.0)))
        out.append(grid_torus_operator(nu, nv, lu, lv, seed=seed0 + 1 + i, chunk=1 << 20))
    return out


def grid_torus_batch_shapes(count=256, nmin=2000, nmax=200_000, seed0=6006):
    """Grid shapes and seeds of the batched workload's meshes (n_i uniform in
    [nmin, nmax] from default_rng(seed0), l_i ~ n_i / 50): per mesh the
    arguments (nu, nv, lu, lv, seed) of grid_torus_operator, with n_v =
    round(sqrt(n_i / 2)), n_u = round(n_i / n_v), a landmark grid about every
    sqrt(50) vertices (at least 5 x 5) and seed seed0 + 1 + i."""
    rng = np.random.default_rng(seed0)
    sizes = rng.integers(nmin, nmax + 1, size=count)
    out = []
    for i, ni in enumerate(sizes):
        nv = max(10, int(round(np.sqrt(ni / 2))))
        nu = max(10, int(round(ni / nv)))
        lu = max(5, int(round(nu / np.sqrt(50.0))))
        lv = max(5, int(round(nv / np.sqrt(50.0))))
        out.append((nu, nv, lu, lv, seed0 + 1 + i))
    return out


def grid_torus_batch_mesh(shape):
    nu, nv, lu, lv, seed = shape
    return grid_torus_operator(nu, nv, lu, lv, seed=seed, chunk=1 << 20)


def grid_torus_batch(count=256, nmin=2000, nmax=200_000, seed0=6006):
    """Many meshes of uneven size in the batched workload's recipe, each a
    grid torus of the kind above (shapes from grid_torus_batch_shapes)."""
    return [grid_torus_batch_mesh(s) for s in grid_torus_batch_shapes(count, nmin, nmax, seed0)]
