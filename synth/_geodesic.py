"""ctypes loader for the generator's shortest-path helpers (synth/_native)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np
import scipy.sparse as sp

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "_native", "geodesic.c")
_LIB = os.path.join(_HERE, "_native", "libsbgen.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile the helper with gcc (OpenMP).  Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        lib = ctypes.CDLL(build())
        p = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.sbgen_fps.argtypes = [i64, p, p, p, i64, i64, p, p]
        lib.sbgen_fps.restype = ctypes.c_int
        lib.sbgen_sssp_to.argtypes = [i64, p, p, p, i64, p, i64, p, p, ctypes.c_int]
        lib.sbgen_sssp_to.restype = ctypes.c_int
        _lib = lib
    return _lib


def _graph_arrays(G: sp.csr_matrix):
    G = sp.csr_matrix(G)
    indptr = np.ascontiguousarray(G.indptr, dtype=np.int64)
    indices = np.ascontiguousarray(G.indices, dtype=np.int32)
    w = np.ascontiguousarray(G.data, dtype=np.float64)
    if np.any(w <= 0):
        raise ValueError("edge weights must be positive")
    return indptr, indices, w


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def fps(G: sp.csr_matrix, l: int, first: int) -> np.ndarray:
    lib = _load()
    indptr, indices, w = _graph_arrays(G)
    n = G.shape[0]
    out = np.empty(l, dtype=np.int64)
    rc = lib.sbgen_fps(n, _ptr(indptr), _ptr(indices), _ptr(w), l, first, _ptr(out), None)
    if rc:
        raise RuntimeError(f"sbgen_fps failed ({rc})")
    return out


def sssp_to(G: sp.csr_matrix, sources: np.ndarray, targets: np.ndarray, threads: int) -> np.ndarray:
    lib = _load()
    indptr, indices, w = _graph_arrays(G)
    n = G.shape[0]
    src = np.ascontiguousarray(sources, dtype=np.int64)
    tgt = np.ascontiguousarray(targets, dtype=np.int64)
    out = np.empty((len(src), len(tgt)), dtype=np.float64)
    rc = lib.sbgen_sssp_to(n, _ptr(indptr), _ptr(indices), _ptr(w), len(src), _ptr(src),
                           len(tgt), _ptr(tgt), _ptr(out), int(threads))
    if rc:
        raise RuntimeError(f"sbgen_sssp_to failed ({rc})")
    return out
