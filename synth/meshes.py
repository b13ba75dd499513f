"""Seeded synthetic triangle meshes standing in for the paper's scanned meshes.

The paper evaluates on scanned meshes (Brain, Bunny, Dragon at several
decimations, TOSCA; Section 4).  None of them is available here, so every
workload is a closed surface generated from a seed: tori on a regular grid
(optionally jittered or with sinusoidal radius bumps) and subdivided
icospheres deformed by random spherical harmonics.  Only geometry lives in
this module; nothing here touches the interpolation operator or the
eigensolve.

All randomness is drawn from ``numpy.random.default_rng(seed)``.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "torus_grid",
    "bumpy_torus",
    "icosphere",
    "deformed_icosphere",
    "geodesic_sphere",
    "flat_grid",
    "equilateral_patch",
    "real_sph_harm",
]


def _torus_faces(nu: int, nv: int) -> np.ndarray:
    """Faces of an nu x nv periodic grid, vertex (i, j) -> nv*i + j.

    Each quad (i,j),(i+1,j),(i+1,j+1),(i,j+1) is split along the
    (i,j)-(i+1,j+1) diagonal, both triangles with the same orientation.
    """
    i, j = np.meshgrid(np.arange(nu), np.arange(nv), indexing="ij")
    i = i.ravel()
    j = j.ravel()
    ip = (i + 1) % nu
    jp = (j + 1) % nv
    a = nv * i + j
    b = nv * ip + j
    c = nv * ip + jp
    d = nv * i + jp
    t1 = np.stack([a, b, c], axis=1)
    t2 = np.stack([a, c, d], axis=1)
    return np.concatenate([t1, t2], axis=0).astype(np.int64)


def torus_grid(nu: int, nv: int, R: float = 1.0, r: float = 0.4,
               jitter: float = 0.0, seed: int | None = None):
    """Torus from an nu (around the major circle) x nv (around the tube) grid.

    ``jitter`` is the standard deviation of isotropic Gaussian noise added to
    every coordinate.  Returns (V [n,3] float64, F [2*nu*nv,3] int64).
    """
    u = 2.0 * np.pi * np.arange(nu) / nu
    v = 2.0 * np.pi * np.arange(nv) / nv
    U, Vv = np.meshgrid(u, v, indexing="ij")
    x = (R + r * np.cos(Vv)) * np.cos(U)
    y = (R + r * np.cos(Vv)) * np.sin(U)
    z = r * np.sin(Vv)
    V = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        V = V + rng.normal(0.0, jitter, size=V.shape)
    return V, _torus_faces(nu, nv)


def bumpy_torus(nu: int, nv: int, seed: int, R: float = 1.0, r0: float = 0.4,
                amp: float = 0.05, nbumps: int = 4):
    """Torus whose tube radius carries seeded sinusoidal bumps.

    r(u, v) = r0 + amp * beta(u, v) / max|beta| with
    beta = sum_q sin(a_q u + phi_q) * sin(c_q v + psi_q), integer frequencies
    a_q in [2, 12], c_q in [1, 6] and uniform phases.
    """
    rng = np.random.default_rng(seed)
    a = rng.integers(2, 13, size=nbumps)
    c = rng.integers(1, 7, size=nbumps)
    phi = rng.uniform(0.0, 2.0 * np.pi, size=nbumps)
    psi = rng.uniform(0.0, 2.0 * np.pi, size=nbumps)
    u = 2.0 * np.pi * np.arange(nu) / nu
    v = 2.0 * np.pi * np.arange(nv) / nv
    U, Vv = np.meshgrid(u, v, indexing="ij")
    beta = np.zeros_like(U)
    for q in range(nbumps):
        beta += np.sin(a[q] * U + phi[q]) * np.sin(c[q] * Vv + psi[q])
    rr = r0 + amp * beta / np.max(np.abs(beta))
    x = (R + rr * np.cos(Vv)) * np.cos(U)
    y = (R + rr * np.cos(Vv)) * np.sin(U)
    z = rr * np.sin(Vv)
    V = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    return V, _torus_faces(nu, nv)


def _icosahedron():
    t = (1.0 + np.sqrt(5.0)) / 2.0
    V = np.array([
        [-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0],
        [0, -1, t], [0, 1, t], [0, -1, -t], [0, 1, -t],
        [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1],
    ], dtype=np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    F = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1],
    ], dtype=np.int64)
    return V, F


def icosphere(level: int):
    """Unit icosphere by ``level`` rounds of midpoint subdivision.

    n = 10 * 4**level + 2 vertices, 20 * 4**level faces.  New midpoints are
    projected to the unit sphere after every round.
    """
    V, F = _icosahedron()
    for _ in range(level):
        nV = V.shape[0]
        e = np.concatenate([F[:, [0, 1]], F[:, [1, 2]], F[:, [2, 0]]], axis=0)
        e_sorted = np.sort(e, axis=1)
        uniq, inv = np.unique(e_sorted, axis=0, return_inverse=True)
        inv = inv.ravel()
        mid = 0.5 * (V[uniq[:, 0]] + V[uniq[:, 1]])
        mid /= np.linalg.norm(mid, axis=1, keepdims=True)
        V = np.concatenate([V, mid], axis=0)
        m = nV + inv
        nf = F.shape[0]
        m01, m12, m20 = m[:nf], m[nf:2 * nf], m[2 * nf:]
        a, b, c = F[:, 0], F[:, 1], F[:, 2]
        F = np.concatenate([
            np.stack([a, m01, m20], 1),
            np.stack([b, m12, m01], 1),
            np.stack([c, m20, m12], 1),
            np.stack([m01, m12, m20], 1),
        ], axis=0)
    return V, F


def real_sph_harm(ell: int, m: int, polar: np.ndarray, azim: np.ndarray) -> np.ndarray:
    """Real spherical harmonic of degree ell and order m.

    m > 0 uses sqrt(2) * Re(Y_ell^m), m < 0 uses sqrt(2) * Im(Y_ell^|m|),
    m = 0 is Y_ell^0 (complex Y from scipy.special.sph_harm_y).
    """
    from scipy.special import sph_harm_y

    Y = sph_harm_y(ell, abs(m), polar, azim)
    if m > 0:
        return np.sqrt(2.0) * Y.real
    if m < 0:
        return np.sqrt(2.0) * Y.imag
    return Y.real


def _radial_deform(V: np.ndarray, seed: int, amp: float, nterms: int, max_degree: int):
    rng = np.random.default_rng(seed)
    ells = rng.integers(1, max_degree + 1, size=nterms)
    ms = np.array([rng.integers(-l, l + 1) for l in ells])
    coef = rng.normal(0.0, 1.0, size=nterms)
    polar = np.arccos(np.clip(V[:, 2], -1.0, 1.0))
    azim = np.arctan2(V[:, 1], V[:, 0])
    s = np.zeros(V.shape[0])
    for q in range(nterms):
        s += coef[q] * real_sph_harm(int(ells[q]), int(ms[q]), polar, azim)
    radius = 1.0 + amp * s / np.max(np.abs(s))
    return V * radius[:, None]


def deformed_icosphere(level: int, seed: int, amp: float = 0.05, nterms: int = 8,
                       max_degree: int = 6):
    """Icosphere with radius 1 + amp * s(x) / max|s|, s a seeded sum of
    ``nterms`` real spherical harmonics of degree 1..max_degree with N(0,1)
    coefficients."""
    V, F = icosphere(level)
    return _radial_deform(V, seed, amp, nterms, max_degree), F


def geodesic_sphere(freq: int):
    """Class-I geodesic sphere: each icosahedron face split into freq**2
    triangles, vertices projected to the unit sphere.  n = 10 * freq**2 + 2.
    Reaches vertex counts that repeated midpoint subdivision cannot."""
    V0, F0 = _icosahedron()
    key = {}
    verts = []

    def vid(p):
        # Points on shared edges and corners are found again from the
        # neighbouring face; round to merge them.
        k = tuple(np.round(p / np.linalg.norm(p), 12))
        if k not in key:
            key[k] = len(verts)
            verts.append(p / np.linalg.norm(p))
        return key[k]

    faces = []
    for f in F0:
        A, B, C = V0[f[0]], V0[f[1]], V0[f[2]]
        idx = {}
        for i in range(freq + 1):
            for j in range(freq + 1 - i):
                k = freq - i - j
                p = (i * A + j * B + k * C) / freq
                idx[(i, j)] = vid(p)
        for i in range(freq):
            for j in range(freq - i):
                faces.append([idx[(i, j)], idx[(i + 1, j)], idx[(i, j + 1)]])
                if i + j < freq - 1:
                    faces.append([idx[(i + 1, j)], idx[(i + 1, j + 1)], idx[(i, j + 1)]])
    V = np.array(verts)
    F = np.array(faces, dtype=np.int64)
    # orient every face outward
    cen = V[F].mean(axis=1)
    nrm = np.cross(V[F[:, 1]] - V[F[:, 0]], V[F[:, 2]] - V[F[:, 0]])
    flip = np.einsum("ij,ij->i", nrm, cen) < 0
    F[flip] = F[flip][:, [0, 2, 1]]
    return V, F


def flat_grid(nx: int, ny: int, h: float = 1.0, seed: int | None = None, jitter: float = 0.0):
    """Open planar grid in the z = 0 plane, quads split along one diagonal.
    Used only by tests (linear precision of the cotangent Laplacian)."""
    i, j = np.meshgrid(np.arange(nx), np.arange(ny), indexing="ij")
    V = np.stack([h * i.ravel(), h * j.ravel(), np.zeros(nx * ny)], axis=1).astype(np.float64)
    if jitter > 0.0:
        rng = np.random.default_rng(seed)
        interior = (i.ravel() > 0) & (i.ravel() < nx - 1) & (j.ravel() > 0) & (j.ravel() < ny - 1)
        V[interior, :2] += rng.normal(0.0, jitter, size=(interior.sum(), 2))
    ii, jj = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), indexing="ij")
    ii = ii.ravel()
    jj = jj.ravel()
    a = ny * ii + jj
    b = ny * (ii + 1) + jj
    c = ny * (ii + 1) + jj + 1
    d = ny * ii + jj + 1
    F = np.concatenate([np.stack([a, b, c], 1), np.stack([a, c, d], 1)], 0).astype(np.int64)
    return V, F


def equilateral_patch(rings: int = 3):
    """Planar patch of equilateral triangles (unit edges) on a hexagonal
    lattice, all vertices within ``rings`` steps of the origin."""
    pts = {}
    e1 = np.array([1.0, 0.0])
    e2 = np.array([0.5, np.sqrt(3.0) / 2.0])
    for a in range(-rings, rings + 1):
        for b in range(-rings, rings + 1):
            if abs(a) <= rings and abs(b) <= rings and abs(a + b) <= rings:
                pts[(a, b)] = len(pts)
    V = np.zeros((len(pts), 3))
    for (a, b), k in pts.items():
        V[k, :2] = a * e1 + b * e2
    F = []
    for (a, b), k in pts.items():
        if (a + 1, b) in pts and (a, b + 1) in pts:
            F.append([k, pts[(a + 1, b)], pts[(a, b + 1)]])
        if (a + 1, b) in pts and (a + 1, b - 1) in pts:
            F.append([k, pts[(a + 1, b - 1)], pts[(a + 1, b)]])
    return V, np.array(F, dtype=np.int64)
