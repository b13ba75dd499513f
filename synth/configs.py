"""Named synthetic workloads and an on-disk cache of their inputs.

Each builder returns a dict with the float64 operator (``P64`` CSR), the
float32-rounded arrays handed to the embedding path (``rowptr`` int32,
``col`` int32, ``val`` float32/float64, ``W`` float32/float64), landmark
vertex ids, the mesh and the parameters.  The precision of ``val``/``W``
is float64 for the FP64 workload and float32 otherwise; the reference
eigenpairs are always taken on exactly these rounded values, upcast.

Workloads (mesh recipe, landmark count, sparsity):
  torus64x32   n=2,048 torus (R=1, r=0.4) with N(0, 0.01^2) vertex jitter,
               l=64 geodesic farthest-point landmarks, p_row=10 (p=310), FP64
  sphere7      icosphere level 7 (n=163,842) with radius 1 + 0.05 s/max|s|,
               s a sum of 8 seeded real spherical harmonics of degree <= 6,
               l=2,000, p_row=10 (p=809), FP32
  bumpy_torus  nu x nv torus with sinusoidal tube-radius bumps (amp 0.05),
               l = n/50 (or given), p_row=10, FP32
  small meshes for tests (any of the above at reduced sizes)
"""
from __future__ import annotations

import hashlib
import json
import os
import time

import numpy as np
import scipy.sparse as sp

from . import meshes
from . import operator as op

__all__ = ["build_problem", "load", "cache_dir", "torus64x32", "sphere7", "PRESETS"]


def cache_dir() -> str:
    d = os.environ.get("SBMDS_CACHE")
    if not d:
        d = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "_cache")
    os.makedirs(d, exist_ok=True)
    return d


def build_problem(V, F, l: int, p_row: float | None, seed: int, dtype=np.float32,
                  landmarks=None, graph_operator: bool = False, log=None):
    """Full input chain for one mesh.  ``p_row=None`` keeps P dense."""
    t0 = time.time()
    n = V.shape[0]
    M = op.biharmonic(V, F, graph=graph_operator)
    G = op.edge_graph(V, F)
    if landmarks is None:
        landmarks = op.farthest_point_landmarks(G, l, seed=seed)
    landmarks = np.asarray(landmarks, dtype=np.int64)
    if log:
        log(f"  landmarks done ({time.time() - t0:.1f}s)")
    W64 = op.landmark_sq_distances(G, landmarks)
    if log:
        log(f"  W done ({time.time() - t0:.1f}s)")
    p = None if p_row is None else op.p_from_prow(n, l, p_row)
    if l == n:
        P64 = sp.csr_matrix((np.ones(n), (landmarks, np.arange(n))), shape=(n, n))
        P64.sort_indices()
    else:
        P64, _ = op.interpolation_operator(M, landmarks, p)
    if log:
        log(f"  P done ({time.time() - t0:.1f}s)")
    val = P64.data.astype(dtype)
    W = W64.astype(dtype)
    return {
        "n": n, "l": l, "p": p if p is not None else n - l, "p_row": p_row, "seed": seed,
        "V": V, "F": F, "landmarks": landmarks,
        "rowptr": P64.indptr.astype(np.int32), "col": P64.indices.astype(np.int32),
        "val": val, "W": W, "P64": P64, "W64": W64,
    }


def operator_rounded(prob) -> sp.csr_matrix:
    """The CSR P exactly as handed to the path (rounded values), in float64."""
    return sp.csr_matrix((prob["val"].astype(np.float64), prob["col"], prob["rowptr"]),
                         shape=(prob["n"], prob["l"]))


def _key(name: str, params: dict) -> str:
    h = hashlib.sha1(json.dumps(params, sort_keys=True).encode()).hexdigest()[:12]
    return f"{name}_{h}"


_ARRAYS = ["V", "F", "landmarks", "rowptr", "col", "val", "W"]


def _save(path, prob):
    meta = {k: prob[k] for k in ("n", "l", "p", "p_row", "seed")}
    arrays = {k: prob[k] for k in _ARRAYS}
    W = arrays.pop("W")
    if np.array_equal(W, W.T):
        # W is symmetrised before rounding, so its upper triangle holds it
        # exactly (half the bytes of the largest inputs)
        arrays["W_upper"] = W[np.triu_indices(W.shape[0])]
    else:
        arrays["W"] = W
    np.savez(path, meta=json.dumps(meta), **arrays)


def _restore(path):
    z = np.load(path, allow_pickle=False)
    meta = json.loads(str(z["meta"]))
    prob = dict(meta)
    for k in _ARRAYS:
        if k == "W" and "W_upper" in z.files:
            l = int(meta["l"])
            iu = np.triu_indices(l)
            W = np.empty((l, l), dtype=z["W_upper"].dtype)
            W[iu] = z["W_upper"]
            W.T[iu] = z["W_upper"]
            prob[k] = W
        else:
            prob[k] = z[k]
    return prob


def _cached(name, params, make, use_cache=True, log=None, generate=True):
    path = os.path.join(cache_dir(), _key(name, params) + ".npz")
    if use_cache and os.path.exists(path):
        return _restore(path)
    if not generate:
        return None
    if log:
        log(f"generating {name} {params}")
    prob = make()
    if use_cache:
        tmp = path + ".tmp.npz"
        _save(tmp, prob)
        os.replace(tmp, path)
    # drop float64 extras so cached and fresh results look the same
    return {k: prob[k] for k in list(_ARRAYS) + ["n", "l", "p", "p_row", "seed"]}


def torus64x32(p_row=10, l=64, seed=1001, jitter=0.01, fp64=True, use_cache=True, log=None):
    params = dict(p_row=p_row, l=l, seed=seed, jitter=jitter, fp64=fp64, v=1)

    def make():
        V, F = meshes.torus_grid(64, 32, 1.0, 0.4, jitter=jitter, seed=seed)
        return build_problem(V, F, l, p_row, seed, np.float64 if fp64 else np.float32, log=log)

    return _cached("torus64x32", params, make, use_cache, log)


def sphere7(p_row=10, l=2000, seed=2002, level=7, use_cache=True, log=None):
    params = dict(p_row=p_row, l=l, seed=seed, level=level, v=1)

    def make():
        V, F = meshes.deformed_icosphere(level, seed)
        return build_problem(V, F, l, p_row, seed, np.float32, log=log)

    return _cached(f"sphere{level}", params, make, use_cache, log)


def bumpy_torus(nu, nv, l=None, p_row=10, seed=3003, use_cache=True, log=None, generate=True):
    """Bumpy torus of nu x nv vertices.  With ``generate=False`` only a cached
    input is returned (None when there is none): the 1024 x 512 torus with
    10,000 landmarks takes about an hour of host time to generate."""
    n = nu * nv
    l = l if l is not None else max(2, round(n / 50))
    params = dict(nu=nu, nv=nv, l=l, p_row=p_row, seed=seed, v=1)

    def make():
        V, F = meshes.bumpy_torus(nu, nv, seed)
        return build_problem(V, F, l, p_row, seed, np.float32, log=log)

    return _cached(f"bumpy_torus{nu}x{nv}", params, make, use_cache, log, generate)


def batch_meshes(count=16, nmin=2000, nmax=20000, seed0=4004, p_row=10):
    """The meshes of the batched workload's recipe, without their inputs:
    n_i ~ U[nmin, nmax] from default_rng(seed0); even i is a bumpy torus
    with n_v = round(sqrt(n_i / 2)), n_u = round(n_i / n_v); odd i is a
    class-I geodesic sphere of frequency round(sqrt((n_i - 2) / 10)) with the
    radial spherical-harmonic deformation of sphere7; l_i = round(n_i / 50),
    seed seed0 + i for the mesh and its landmarks (the first landmark is
    default_rng(seed).integers(n), as in the input chain).  Returns dicts
    with V, F, n, l, p, seed, first, kind and the mesh's parameters."""
    rng = np.random.default_rng(seed0)
    sizes = rng.integers(nmin, nmax + 1, size=count)
    out = []
    for i, ni in enumerate(sizes):
        seed = seed0 + i
        if i % 2 == 0:
            nv = max(3, int(round(np.sqrt(ni / 2))))
            nu = max(3, int(round(ni / nv)))
            V, F = meshes.bumpy_torus(nu, nv, seed)
            d = {"kind": "torus", "nu": nu, "nv": nv}
        else:
            freq = max(1, int(round(np.sqrt((ni - 2) / 10))))
            V, F = meshes.geodesic_sphere(freq)
            V = meshes._radial_deform(V, seed, 0.05, 8, 6)
            d = {"kind": "geosphere", "freq": freq}
        n = V.shape[0]
        l = max(2, int(round(n / 50)))
        d.update(V=V, F=F, n=n, l=l, p=op.p_from_prow(n, l, p_row), p_row=p_row, seed=seed,
                 first=int(np.random.default_rng(seed).integers(n)))
        out.append(d)
    return out


def mesh_batch(count=16, nmin=2000, nmax=20000, seed0=4004, p_row=10, use_cache=True, log=None):
    """The batched workload's recipe (batch_meshes) at reduced scale with
    every mesh's input chain run on the host (cached)."""
    out = []
    for m in batch_meshes(count, nmin, nmax, seed0, p_row):
        seed, l = m["seed"], m["l"]
        if m["kind"] == "torus":
            prob = bumpy_torus(m["nu"], m["nv"], l=l, p_row=p_row, seed=seed, use_cache=use_cache, log=log)
        else:
            params = dict(freq=m["freq"], l=l, p_row=p_row, seed=seed, v=1)

            def make(m=m):
                return build_problem(m["V"], m["F"], m["l"], p_row, m["seed"], np.float32, log=log)

            prob = _cached(f"geosphere{m['freq']}", params, make, use_cache, log)
        out.append(prob)
    return out


def sphere_family(count=12, level=5, seed0=7001, p_row=10, use_cache=True, log=None):
    """Training meshes for the learned start on the sphere7 workload: icospheres
    of the given level with sphere7's radial deformation (seeds seed0 ..
    seed0 + count - 1, all different from sphere7's), l = round(n / 50)."""
    out = []
    for i in range(count):
        seed = seed0 + i
        V0, F = meshes.icosphere(level)
        l = max(2, int(round(V0.shape[0] / 50)))
        params = dict(level=level, l=l, p_row=p_row, seed=seed, v=1)

        def make(seed=seed, l=l):
            V, F2 = meshes.deformed_icosphere(level, seed)
            return build_problem(V, F2, l, p_row, seed, np.float32, log=log)

        out.append(_cached(f"sphere{level}", params, make, use_cache, log))
    return out


TORUS_FAMILY = [(56, 28, 4101), (64, 32, 4102), (72, 36, 4103), (60, 30, 4104), (68, 34, 4105), (80, 40, 4106),
                (64, 32, 4107), (72, 36, 4108), (56, 28, 4109), (76, 38, 4110), (64, 32, 4111), (84, 42, 4112)]


TORUS_FAMILY_192 = [(192, 96, 4200 + i) for i in range(1, 13)]


def torus_family(size="small", use_cache=True, log=None):
    """Training meshes for the learned start on bumpy tori, l = n/50,
    p_row = 10: "small" is 12 tori from 56 x 28 to 84 x 42 vertices (seeds
    4101-4112); "192" is 12 tori of 192 x 96 vertices (seeds 4201-4212)."""
    fam = TORUS_FAMILY if size == "small" else TORUS_FAMILY_192
    return [bumpy_torus(nu, nv, seed=seed, use_cache=use_cache, log=log) for nu, nv, seed in fam]


def input_digest(prob) -> str:
    """sha1 over the arrays handed to the path (rowptr, col, val, W), to tie
    stored expected values to the exact input they were computed from."""
    h = hashlib.sha1()
    for k in ("rowptr", "col", "val", "W"):
        a = np.ascontiguousarray(prob[k])
        h.update(str(a.dtype).encode())
        h.update(str(a.shape).encode())
        h.update(a.tobytes())
    return h.hexdigest()


def load(name: str, **kw):
    return PRESETS[name](**kw)


PRESETS = {
    "torus64x32": torus64x32,
    "sphere7": sphere7,
}
