"""Python binding of the sBMDS embedding library (libsbmds.so, include/sbmds.h).

Argument marshalling only: every step of the solve runs in the library's HIP
kernels.  Inputs may be NumPy arrays (host memory) or torch tensors on a
ROCm device (device memory); torch supplies device memory and the stream.

    from paper_1705_10887_amd import embed
    Z, eig, report = embed(rowptr, col, val, W, k=3, block=16)

The library is loaded from this directory; if it has not been built the
import of the binding functions fails loudly (there is no fallback path).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "FP64", "FP32", "BF16_FP32",
    "START_RANDOM", "START_LMDS", "START_LEARNED", "START_USER",
    "FLAG_KERNEL_TIMING", "FLAG_NO_GRAPH", "FLAG_NO_CERTIFY", "FLAG_PACK_W", "FLAG_FULL_W", "FLAG_PUSH_T",
    "INTERP_GRAPH", "INTERP_DENSE", "INTERP_BLOCKED",
    "SbmdsError", "Problem", "Context", "embed", "approx_rows", "lib", "lib_path", "version",
]

FP64, FP32, BF16_FP32 = 0, 1, 2
START_RANDOM, START_LMDS, START_LEARNED, START_USER = 0, 1, 2, 3
MEM_HOST, MEM_DEVICE = 0, 1
FLAG_KERNEL_TIMING, FLAG_NO_GRAPH, FLAG_NO_CERTIFY = 0x1, 0x2, 0x4
FLAG_PACK_W, FLAG_FULL_W, FLAG_PUSH_T = 0x8, 0x10, 0x20
INTERP_GRAPH, INTERP_DENSE, INTERP_BLOCKED = 0x1, 0x2, 0x4  # sbmds_interpolation flags
MAX_BLOCK = 64

_STATUS = {0: "OK", 1: "ENOCONV", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ENODEV", -5: "EBREAKDOWN"}

_HERE = os.path.dirname(os.path.abspath(__file__))
lib_path = os.path.join(_HERE, "libsbmds.so")


class SbmdsError(RuntimeError):
    def __init__(self, code, msg):
        self.code = code
        super().__init__(f"sbmds {_STATUS.get(code, code)}: {msg}")


class _Problem(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64), ("l", ctypes.c_int64), ("nnz", ctypes.c_int64),
        ("P_rowptr", ctypes.c_void_p), ("P_col", ctypes.c_void_p), ("P_val", ctypes.c_void_p),
        ("W", ctypes.c_void_p), ("xyz", ctypes.c_void_p), ("landmark_vertex", ctypes.c_void_p),
        ("X0", ctypes.c_void_p), ("mem", ctypes.c_int),
    ]


class _Options(ctypes.Structure):
    _fields_ = [
        ("k", ctypes.c_int), ("block", ctypes.c_int), ("prec", ctypes.c_int), ("start", ctypes.c_int),
        ("tol", ctypes.c_double), ("max_iter", ctypes.c_int), ("seed", ctypes.c_uint64),
        ("stream", ctypes.c_void_p), ("mlp_weights", ctypes.c_char_p), ("tune_cache", ctypes.c_char_p),
        ("mem_cap", ctypes.c_size_t), ("flags", ctypes.c_uint),
    ]


class _Report(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("iters_bf16", ctypes.c_int), ("iters_fp32", ctypes.c_int),
        ("iters_fp64", ctypes.c_int), ("nonpositive", ctypes.c_int), ("certified", ctypes.c_int),
        ("jacobi_sweeps", ctypes.c_int), ("start_iters", ctypes.c_int),
        ("ms_start", ctypes.c_double), ("ms_iter", ctypes.c_double), ("ms_total", ctypes.c_double),
        ("eig", ctypes.c_double * MAX_BLOCK), ("err_bound", ctypes.c_double * MAX_BLOCK),
        ("resid", ctypes.c_double * MAX_BLOCK),
    ]


class _SolverReport(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int), ("steps", ctypes.c_int), ("basis", ctypes.c_int), ("nonpositive", ctypes.c_int),
        ("ms_total", ctypes.c_double),
        ("eig", ctypes.c_double * MAX_BLOCK), ("err_bound", ctypes.c_double * MAX_BLOCK),
        ("resid", ctypes.c_double * MAX_BLOCK),
    ]


class _KStat(ctypes.Structure):
    _fields_ = [
        ("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("ms_total", ctypes.c_double),
        ("bytes_total", ctypes.c_double), ("flops_total", ctypes.c_double),
    ]


_lib = None

EXPORTS = [
    "sbmds_default_options", "sbmds_create", "sbmds_embed", "sbmds_get_block",
    "sbmds_kernel_stats", "sbmds_reset_kernel_stats", "sbmds_destroy",
    "sbmds_last_error", "sbmds_version", "sbmds_approx_rows", "sbmds_stress",
    "sbmds_embed_lanczos", "sbmds_embed_bmds", "sbmds_landmarks_geodesic", "sbmds_interpolation",
    # learned warm start (include/sbmds_mlp.h)
    "sbmds_mlp_create", "sbmds_mlp_load", "sbmds_mlp_save", "sbmds_mlp_num_params", "sbmds_mlp_get_params",
    "sbmds_mlp_set_params", "sbmds_mlp_set_norm", "sbmds_mlp_features", "sbmds_mlp_forward",
    "sbmds_mlp_loss_grad", "sbmds_mlp_adam_step", "sbmds_mlp_destroy",
    "sbmds_mlp_forward_noalloc",
]


def lib():
    """Load libsbmds.so (once).  Raises ImportError if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(lib_path):
        raise ImportError(f"{lib_path} is missing; build it with `python -m paper_1705_10887_amd._build` "
                          "(there is no CPU fallback)")
    L = ctypes.CDLL(lib_path)
    L.sbmds_default_options.argtypes = [ctypes.POINTER(_Options)]
    L.sbmds_default_options.restype = None
    L.sbmds_create.argtypes = [ctypes.POINTER(_Problem), ctypes.c_int, ctypes.POINTER(_Options),
                               ctypes.POINTER(ctypes.c_void_p)]
    L.sbmds_create.restype = ctypes.c_int
    L.sbmds_embed.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                              ctypes.POINTER(_Report)]
    L.sbmds_embed.restype = ctypes.c_int
    L.sbmds_get_block.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p, ctypes.c_int]
    L.sbmds_get_block.restype = ctypes.c_int
    L.sbmds_kernel_stats.argtypes = [ctypes.c_void_p, ctypes.POINTER(_KStat), ctypes.c_int]
    L.sbmds_kernel_stats.restype = ctypes.c_int
    L.sbmds_reset_kernel_stats.argtypes = [ctypes.c_void_p]
    L.sbmds_reset_kernel_stats.restype = None
    L.sbmds_destroy.argtypes = [ctypes.c_void_p]
    L.sbmds_destroy.restype = None
    L.sbmds_last_error.argtypes = []
    L.sbmds_last_error.restype = ctypes.c_char_p
    L.sbmds_version.argtypes = []
    L.sbmds_version.restype = ctypes.c_int
    vp, i64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
    for name, args, res in [
        ("sbmds_mlp_create", [ci, ctypes.c_uint64, vp, ctypes.POINTER(vp)], ci),
        ("sbmds_mlp_load", [ctypes.c_char_p, vp, ctypes.POINTER(vp)], ci),
        ("sbmds_mlp_save", [vp, ctypes.c_char_p], ci),
        ("sbmds_mlp_num_params", [vp], i64),
        ("sbmds_mlp_get_params", [vp, vp], ci),
        ("sbmds_mlp_set_params", [vp, vp], ci),
        ("sbmds_mlp_set_norm", [vp, vp, vp], ci),
        ("sbmds_mlp_features", [vp, i64, vp, vp, i64, ci, vp, ci, vp], ci),
        ("sbmds_mlp_forward", [vp, vp, i64, vp, ci], ci),
        ("sbmds_mlp_loss_grad", [vp, vp, vp, vp, ci, vp, vp, ci], ci),
        ("sbmds_mlp_adam_step", [vp, ctypes.c_float], ci),
        ("sbmds_mlp_destroy", [vp], None),
        ("sbmds_mlp_forward_noalloc", [vp, vp, i64, vp], ci),
        ("sbmds_approx_rows", [ctypes.POINTER(_Problem), ci, vp, vp, i64, vp, vp, vp, ci, vp], ci),
        ("sbmds_stress", [vp, i64, ci, vp, ci, ci, vp, vp], ci),
        ("sbmds_embed_lanczos", [vp, ci, ci, vp, vp, ci, ctypes.POINTER(_SolverReport)], ci),
        ("sbmds_embed_bmds", [vp, vp, vp, ci, ctypes.POINTER(_SolverReport)], ci),
        ("sbmds_landmarks_geodesic", [vp, vp, vp, i64, i64, ctypes.c_int32, vp, vp, ci, ci, vp], ci),
        ("sbmds_interpolation", [vp, i64, vp, i64, vp, i64, i64, ci, vp, vp, vp, i64, vp, ci, vp], ci),
    ]:
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def version():
    v = lib().sbmds_version()
    return (v >> 16, v & 0xFFFF)


def _check(rc):
    if rc < 0:
        raise SbmdsError(rc, lib().sbmds_last_error().decode())
    return rc


def _is_torch(x):
    return type(x).__module__.startswith("torch")


def _ptr_any(a, dtype):
    """(pointer, mem) of a NumPy array (converted to a contiguous `dtype`
    copy, kept alive on the function) or a contiguous CUDA tensor."""
    if _is_torch(a) and a.is_cuda:
        return a.data_ptr(), MEM_DEVICE
    arr = np.ascontiguousarray(a, dtype=dtype)
    _ptr_any.keep.append(arr)
    del _ptr_any.keep[:-8]
    return arr.ctypes.data, MEM_HOST


_ptr_any.keep = []


@dataclass
class Problem:
    """One mesh's operator: CSR of P (n x l) and W (l x l).

    Arrays are NumPy (host) or torch tensors on the GPU (device); the value
    dtype must be float64 for FP64 and float32 otherwise.
    """
    rowptr: object
    col: object
    val: object
    W: object
    n: int
    l: int
    X0: object = None
    xyz: object = None
    landmark_vertex: object = None
    _keep: list = field(default_factory=list, repr=False)

    @classmethod
    def from_arrays(cls, rowptr, col, val, W, X0=None, xyz=None, landmark_vertex=None):
        n = int(rowptr.shape[0]) - 1
        l = int(W.shape[0])
        return cls(rowptr, col, val, W, n, l, X0, xyz, landmark_vertex)

    def _struct(self, fdtype):
        dev = _is_torch(self.W) and self.W.is_cuda
        keep = []

        def ptr(a, dtype):
            if a is None:
                return None
            if dev:
                import torch
                tdt = {np.int32: torch.int32, np.float32: torch.float32, np.float64: torch.float64}[dtype]
                if a.dtype != tdt or not a.is_contiguous():
                    raise TypeError(f"expected contiguous {tdt} tensor, got {a.dtype}")
                keep.append(a)
                return a.data_ptr()
            arr = np.ascontiguousarray(a, dtype=dtype)
            keep.append(arr)
            return arr.ctypes.data

        s = _Problem()
        s.n = self.n
        s.l = self.l
        s.nnz = int(self.col.shape[0])
        s.P_rowptr = ptr(self.rowptr, np.int32)
        s.P_col = ptr(self.col, np.int32)
        s.P_val = ptr(self.val, fdtype)
        s.W = ptr(self.W, fdtype)
        s.X0 = ptr(self.X0, fdtype)
        s.xyz = ptr(self.xyz, np.float32)
        s.landmark_vertex = ptr(self.landmark_vertex, np.int32)
        s.mem = MEM_DEVICE if dev else MEM_HOST
        self._keep = keep
        return s


class Context:
    """A created solver context (sbmds_create) over one or more problems."""

    def __init__(self, problems, k=3, block=16, prec=FP32, start=START_RANDOM, tol=1e-6, max_iter=500,
                 seed=12345, stream=None, mlp_weights=None, tune_cache=None, mem_cap=0, flags=0):
        L = lib()
        if isinstance(problems, Problem):
            problems = [problems]
        self.problems = list(problems)
        self.prec = prec
        self.k = k
        self.block = block
        fdtype = np.float64 if prec == FP64 else np.float32
        arr = (_Problem * len(self.problems))()
        for i, p in enumerate(self.problems):
            arr[i] = p._struct(fdtype)
        o = _Options()
        L.sbmds_default_options(ctypes.byref(o))
        o.k, o.block, o.prec, o.start = k, block, prec, start
        o.tol, o.max_iter, o.seed = tol, max_iter, seed
        if stream is None and any(_is_torch(p.W) and p.W.is_cuda for p in self.problems):
            import torch
            stream = torch.cuda.current_stream().cuda_stream
        o.stream = stream
        self._mlp = mlp_weights.encode() if isinstance(mlp_weights, str) else mlp_weights
        self._tune = tune_cache.encode() if isinstance(tune_cache, str) else tune_cache
        o.mlp_weights = self._mlp
        o.tune_cache = self._tune
        o.mem_cap = mem_cap
        o.flags = flags
        self._opt = o
        h = ctypes.c_void_p()
        _check(L.sbmds_create(arr, len(self.problems), ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        for p in self.problems:  # inputs may be released after create
            p._keep = []

    def embed(self, Z_out=None):
        """Run the solve.  Returns (Z, eigvals [nprob, k], reports).

        Z is written into ``Z_out`` if given (a device tensor or a host
        array of shape [sum n, k]); otherwise a host NumPy array is returned.
        """
        L = lib()
        nprob = len(self.problems)
        eig = np.zeros((nprob, self.k), dtype=np.float64)
        reps = (_Report * nprob)()
        ntot = sum(p.n for p in self.problems)
        zdt = np.float64 if self.prec == FP64 else np.float32
        if Z_out is None:
            Z = np.zeros((ntot, self.k), dtype=zdt)
            zptr, zmem = Z.ctypes.data, MEM_HOST
        elif _is_torch(Z_out) and Z_out.is_cuda:
            Z = Z_out
            zptr, zmem = Z_out.data_ptr(), MEM_DEVICE
        else:
            Z = Z_out
            zptr, zmem = Z_out.ctypes.data, MEM_HOST
        rc = _check(L.sbmds_embed(self._h, eig.ctypes.data, zptr, zmem, reps))
        reports = [_report_dict(r, self.k, self.block) for r in reps]
        return Z, eig, reports, rc

    def _z_target(self, Z_out):
        ntot = sum(p.n for p in self.problems)
        zdt = np.float64 if self.prec == FP64 else np.float32
        if Z_out is None:
            Z = np.zeros((ntot, self.k), dtype=zdt)
            return Z, Z.ctypes.data, MEM_HOST
        if _is_torch(Z_out) and Z_out.is_cuda:
            return Z_out, Z_out.data_ptr(), MEM_DEVICE
        return Z_out, Z_out.ctypes.data, MEM_HOST

    def _compare(self, fn, *args, Z_out=None):
        nprob = len(self.problems)
        eig = np.zeros((nprob, self.k), dtype=np.float64)
        reps = (_SolverReport * nprob)()
        Z, zptr, zmem = self._z_target(Z_out)
        rc = _check(fn(self._h, *args, eig.ctypes.data, zptr, zmem, reps))
        reports = [dict(status=r.status, steps=r.steps, basis=r.basis, nonpositive=r.nonpositive,
                        ms_total=r.ms_total, eig=list(r.eig[:self.k]), err_bound=list(r.err_bound[:self.k]),
                        resid=list(r.resid[:self.k])) for r in reps]
        return Z, eig, reports, rc

    def embed_lanczos(self, block=1, max_steps=300, Z_out=None):
        """The paper's sBMDS route (sbmds_embed_lanczos): (block) Lanczos on
        the implicit operator, on the context's problems.  Returns
        (Z, eigvals [nprob, k], reports, status)."""
        return self._compare(lib().sbmds_embed_lanczos, block, max_steps, Z_out=Z_out)

    def embed_bmds(self, Z_out=None):
        """BMDS (sbmds_embed_bmds): QR of the dense J P, eigendecomposition of
        -1/2 R W R^T.  Returns (Z, eigvals [nprob, k], reports, status)."""
        return self._compare(lib().sbmds_embed_bmds, Z_out=Z_out)

    def get_block(self, prob=0):
        """Current orthonormal basis X (n x block) of problem `prob` (host array)."""
        p = self.problems[prob]
        X = np.zeros((p.n, self.block), dtype=np.float64 if self.prec == FP64 else np.float32)
        _check(lib().sbmds_get_block(self._h, prob, X.ctypes.data, MEM_HOST))
        return X

    def kernel_stats(self):
        L = lib()
        n = _check(L.sbmds_kernel_stats(self._h, None, 0))
        arr = (_KStat * max(n, 1))()
        L.sbmds_kernel_stats(self._h, arr, n)
        return [dict(name=s.name.decode(), launches=s.launches, ms_total=s.ms_total,
                     bytes_total=s.bytes_total, flops_total=s.flops_total) for s in arr[:n]]

    def reset_kernel_stats(self):
        lib().sbmds_reset_kernel_stats(self._h)

    def close(self):
        if getattr(self, "_h", None):
            lib().sbmds_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def _report_dict(r, k, block):
    return dict(status=r.status, iters_bf16=r.iters_bf16, iters_fp32=r.iters_fp32, iters_fp64=r.iters_fp64,
                nonpositive=r.nonpositive, certified=bool(r.certified), jacobi_sweeps=r.jacobi_sweeps, start_iters=r.start_iters,
                ms_start=r.ms_start,
                ms_iter=r.ms_iter, ms_total=r.ms_total, eig=list(r.eig[:block]),
                err_bound=list(r.err_bound[:block]), resid=list(r.resid[:block]))


def embed(rowptr, col, val, W, k=3, block=16, prec=FP32, **kw):
    """One-shot: create a context for one problem, solve, destroy.

    Returns (Z [n, k], eigenvalues [k], report dict).
    """
    p = Problem.from_arrays(rowptr, col, val, W, X0=kw.pop("X0", None))
    with Context([p], k=k, block=block, prec=prec, **kw) as ctx:
        Z, eig, reps, _ = ctx.embed()
    return Z, eig[0], reps[0]


def approx_rows(rowptr, col, val, L, rows, K_rows=None, want_rows=False):
    """Rows `rows` of K~ = P L P^T and, with the exact rows K_rows, the
    relative error eps = sum ||K~_s - K_s||^2 / sum ||K_s||^2 on them
    (sbmds_approx_rows).  Arrays are NumPy (host) or torch CUDA tensors
    (device), all in one place; float64 values select the float64 path.
    Returns (eps or None, (num, den) or None, K~ rows or None)."""
    fp64 = (str(getattr(val, "dtype", "")) in ("float64", "torch.float64"))
    fdt = np.float64 if fp64 else np.float32
    n = int(rowptr.shape[0]) - 1
    L_ = L
    l = int(L_.shape[0])
    p = Problem.from_arrays(rowptr, col, val, L_)
    s = p._struct(fdt)
    pr, mem = _ptr_any(rows, np.int32)
    pK, _ = _ptr_any(K_rows, fdt) if K_rows is not None else (None, mem)
    S = int(rows.shape[0])
    err = (ctypes.c_double * 2)()
    out = None
    pout, out_mem = None, mem
    if want_rows:
        if mem == MEM_DEVICE:
            import torch
            out = torch.empty((S, n), dtype=torch.float64, device=rows.device)
        else:
            out = np.empty((S, n), dtype=np.float64)
        pout, _ = _ptr_any(out, np.float64)
    stream = None
    if mem == MEM_DEVICE:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    _check(lib().sbmds_approx_rows(ctypes.byref(s), 1 if fp64 else 0, s.W, pr, S, pK,
                                   err if K_rows is not None else None, pout, out_mem, stream))
    if K_rows is None:
        return None, None, out
    return (err[0] / err[1] if err[1] > 0 else float("nan")), (err[0], err[1]), out


def interpolation(V, F, landmarks, p=None, graph=False, route=None):
    """P of Eq. (PDefinition) built on the device (sbmds_interpolation) from
    the mesh (V [n, 3], F [nf, 3]) and its landmarks, thresholded to p
    entries per column (None: unthresholded).  ``route`` is "dense",
    "blocked" or None (the library's choice by size).  Host NumPy inputs and
    outputs: returns (rowptr, col, val) of the n x l CSR."""
    V = np.ascontiguousarray(V, dtype=np.float64)
    F = np.ascontiguousarray(F, dtype=np.int32)
    lm = np.ascontiguousarray(landmarks, dtype=np.int32)
    n, l = V.shape[0], lm.shape[0]
    m = n - l
    pk = 0 if p is None else int(p)
    flags = INTERP_GRAPH if graph else 0
    if route is not None:
        if route not in ("dense", "blocked"):
            raise ValueError(f"route must be 'dense', 'blocked' or None, not {route!r}")
        flags |= INTERP_DENSE if route == "dense" else INTERP_BLOCKED
    cap = l + l * (m if pk <= 0 or pk >= m else pk)
    rowptr = np.empty(n + 1, dtype=np.int32)
    col = np.empty(max(cap, 1), dtype=np.int32)
    val = np.empty(max(cap, 1), dtype=np.float64)
    nnz = ctypes.c_int64(0)
    _check(lib().sbmds_interpolation(V.ctypes.data, n, F.ctypes.data, F.shape[0], lm.ctypes.data, l, pk, flags,
                                     rowptr.ctypes.data, col.ctypes.data, val.ctypes.data, cap, ctypes.byref(nnz),
                                     MEM_HOST, None))
    return rowptr, col[:nnz.value].copy(), val[:nnz.value].copy()


def landmarks_geodesic(rowptr, col, w, l, first, want_W=True, batch=64):
    """Farthest-point landmarks and W = D_ll o D_ll on the device
    (sbmds_landmarks_geodesic) for the weighted graph CSR (rowptr, col, w),
    NumPy (host) or torch CUDA tensors.  Returns (landmarks [l] int32,
    W [l, l] float64 or None) in the same place as the inputs."""
    n = int(rowptr.shape[0]) - 1
    prp, mem = _ptr_any(rowptr, np.int32)
    pci, _ = _ptr_any(col, np.int32)
    pw, _ = _ptr_any(w, np.float64)
    stream = None
    if mem == MEM_DEVICE:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
        lm = torch.empty(l, dtype=torch.int32, device=rowptr.device)
        W = torch.empty((l, l), dtype=torch.float64, device=rowptr.device) if want_W else None
        plm, pW = lm.data_ptr(), (W.data_ptr() if want_W else None)
    else:
        lm = np.empty(l, dtype=np.int32)
        W = np.empty((l, l), dtype=np.float64) if want_W else None
        plm, pW = lm.ctypes.data, (W.ctypes.data if want_W else None)
    _check(lib().sbmds_landmarks_geodesic(prp, pci, pw, n, l, int(first), plm, pW, mem, batch, stream))
    return lm, W


def stress(Z, K):
    """Stress ||Z Z^T + 1/2 J E J||_F of the embedding Z (n x m) against the
    dense symmetric distances K (n x n), E = K o K (sbmds_stress), and the
    scale ||1/2 J E J||_F.  NumPy (host) or torch CUDA tensors, both float64
    or both float32.  Returns (stress, scale)."""
    fp64 = str(getattr(Z, "dtype", "")) in ("float64", "torch.float64")
    fdt = np.float64 if fp64 else np.float32
    n, m = int(Z.shape[0]), int(Z.shape[1])
    if tuple(K.shape) != (n, n):
        raise ValueError(f"K must be {n} x {n}")
    pZ, mem = _ptr_any(Z, fdt)
    pK, memK = _ptr_any(K, fdt)
    if memK != mem:
        raise ValueError("Z and K must be in the same memory")
    stream = None
    if mem == MEM_DEVICE:
        import torch
        stream = torch.cuda.current_stream().cuda_stream
    out = (ctypes.c_double * 2)()
    _check(lib().sbmds_stress(pZ, n, m, pK, 1 if fp64 else 0, mem, out, stream))
    return out[0], out[1]
