"""Learned warm start: binding of include/sbmds_mlp.h and the training driver.

The network (19 landmark features -> 128 -> 128 -> k, GELU, float32) is
trained on the GPU by the library's own forward, backward and Adam kernels,
on targets the solver itself produces: the landmark rows of converged
embeddings.  A trained network is saved to a weights file that a solver
context loads with ``start=START_LEARNED, mlp_weights=path``.

Arrays are NumPy (host) or CUDA torch tensors (device); every call marshals
pointers only.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import MEM_DEVICE, MEM_HOST, SbmdsError, _check, _is_torch, lib

N_FEAT = 19
HIDDEN = 128


def _ptr(a, dtype):
    """(pointer, mem) of a contiguous array of the given dtype."""
    if _is_torch(a):
        import torch
        want = {np.float32: torch.float32, np.float64: torch.float64, np.int32: torch.int32,
                np.int64: torch.int64}[dtype]
        if a.dtype != want or not a.is_contiguous():
            raise TypeError(f"expected a contiguous {want} tensor")
        return a.data_ptr(), (MEM_DEVICE if a.is_cuda else MEM_HOST)
    if not isinstance(a, np.ndarray) or a.dtype != dtype or not a.flags["C_CONTIGUOUS"]:
        raise TypeError(f"expected a C-contiguous {np.dtype(dtype).name} array")
    return a.ctypes.data, MEM_HOST


def features(xyz, landmarks, W, stream=None):
    """[l, 19] float32 features of one mesh (host arrays in, host array out;
    CUDA tensors in, CUDA tensor out)."""
    l = int(landmarks.shape[0])
    n = int(xyz.shape[0])
    wd = np.float64 if (W.dtype == np.float64 or str(W.dtype) == "torch.float64") else np.float32
    px, mx = _ptr(xyz, np.float32)
    pl, ml = _ptr(landmarks, np.int32)
    pw, mw = _ptr(W, wd)
    if len({mx, ml, mw}) != 1:
        raise ValueError("xyz, landmarks and W must all be on the host or all on the device")
    if mx == MEM_DEVICE:
        import torch
        F = torch.empty((l, N_FEAT), dtype=torch.float32, device=xyz.device)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
    else:
        F = np.empty((l, N_FEAT), dtype=np.float32)
    pf, _ = _ptr(F, np.float32)
    _check(lib().sbmds_mlp_features(px, n, pl, pw, l, 1 if wd == np.float64 else 0, pf, mx, stream))
    return F


class Net:
    """A network handle (sbmds_mlp)."""

    def __init__(self, k=3, seed=0, stream=None, _handle=None):
        L = lib()
        if _handle is None:
            h = ctypes.c_void_p()
            _check(L.sbmds_mlp_create(k, seed, stream, ctypes.byref(h)))
            _handle = h
        self._h = _handle
        self.k = k
        self.n_params = int(L.sbmds_mlp_num_params(self._h))

    @classmethod
    def load(cls, path, stream=None):
        h = ctypes.c_void_p()
        _check(lib().sbmds_mlp_load(path.encode(), stream, ctypes.byref(h)))
        net = cls.__new__(cls)
        net._h = h
        net.n_params = int(lib().sbmds_mlp_num_params(h))
        # n_params = 19*128 + 128 + 128*128 + 128 + 129*k
        net.k = (net.n_params - (N_FEAT * HIDDEN + HIDDEN + HIDDEN * HIDDEN + HIDDEN)) // (HIDDEN + 1)
        return net

    def save(self, path):
        _check(lib().sbmds_mlp_save(self._h, path.encode()))

    def get_params(self):
        th = np.empty(self.n_params, dtype=np.float32)
        _check(lib().sbmds_mlp_get_params(self._h, th.ctypes.data))
        return th

    def set_params(self, theta):
        th = np.ascontiguousarray(theta, dtype=np.float32)
        if th.size != self.n_params:
            raise ValueError(f"expected {self.n_params} parameters")
        _check(lib().sbmds_mlp_set_params(self._h, th.ctypes.data))

    def set_norm(self, mean, std):
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(std, dtype=np.float32)
        _check(lib().sbmds_mlp_set_norm(self._h, m.ctypes.data, s.ctypes.data))

    def forward(self, feat):
        rows = int(feat.shape[0])
        pf, mem = _ptr(feat, np.float32)
        if mem == MEM_DEVICE:
            import torch
            Y = torch.empty((rows, self.k), dtype=torch.float32, device=feat.device)
        else:
            Y = np.empty((rows, self.k), dtype=np.float32)
        py, _ = _ptr(Y, np.float32)
        _check(lib().sbmds_mlp_forward(self._h, pf, rows, py, mem))
        return Y

    def loss_grad(self, feat, T, seg, want_grad=True):
        """Loss over meshes seg[m]..seg[m+1]-1 and (optionally) the gradient
        as a host array; the gradient also stays on the device for adam_step."""
        pf, mf = _ptr(feat, np.float32)
        pt, mt = _ptr(T, np.float32)
        ps, ms = _ptr(seg, np.int64)
        if len({mf, mt, ms}) != 1:
            raise ValueError("feat, T and seg must all be on the host or all on the device")
        loss = ctypes.c_double()
        g = np.empty(self.n_params, dtype=np.float32) if want_grad else None
        _check(lib().sbmds_mlp_loss_grad(self._h, pf, pt, ps, int(seg.shape[0]) - 1, ctypes.byref(loss),
                                         g.ctypes.data if want_grad else None, mf))
        return loss.value, g

    def adam_step(self, lr):
        _check(lib().sbmds_mlp_adam_step(self._h, ctypes.c_float(lr)))

    def close(self):
        if getattr(self, "_h", None):
            lib().sbmds_mlp_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def landmark_targets(Z, landmarks):
    """The landmark rows of a converged embedding: the training target."""
    return np.ascontiguousarray(np.asarray(Z)[np.asarray(landmarks)], dtype=np.float32)


def solve_targets(meshes, k=3, block=16):
    """Converged embeddings of training meshes from the solver itself (FP32,
    random start), one context per mesh; returns the landmark rows of each."""
    from . import FP32, Context, Problem
    out = []
    for m in meshes:
        p = Problem.from_arrays(m["rowptr"], m["col"], m["val"], m["W"])
        with Context([p], k=k, block=block, prec=FP32) as ctx:
            Z, _, reps, rc = ctx.embed()
        if rc != 0:
            raise SbmdsError(rc, "a training mesh did not converge")
        out.append(landmark_targets(Z, m["landmarks"]))
    return out


def train(feats, targets, k=3, steps=600, lr=3e-3, seed=0, log=None, log_every=100):
    """Full-batch Adam on the concatenation of the meshes (device resident).

    feats / targets: per mesh [l_m, 19] and [l_m, k] float32 arrays.
    Returns (net, losses).  The standardisation is the mean and standard
    deviation of the training features."""
    import torch
    F = np.concatenate(feats).astype(np.float32)
    T = np.concatenate(targets).astype(np.float32)
    seg = np.concatenate([[0], np.cumsum([f.shape[0] for f in feats])]).astype(np.int64)
    mean = F.mean(axis=0)
    std = np.maximum(F.std(axis=0), 1e-3)
    net = Net(k=k, seed=seed, stream=torch.cuda.current_stream().cuda_stream)
    net.set_norm(mean, std)
    Fd = torch.from_numpy(F).cuda()
    Td = torch.from_numpy(T).cuda()
    Sd = torch.from_numpy(seg).cuda()
    losses = []
    for step in range(steps):
        loss, _ = net.loss_grad(Fd, Td, Sd, want_grad=False)
        net.adam_step(lr)
        losses.append(loss)
        if log and (step % log_every == 0 or step == steps - 1):
            log(f"step {step} loss {loss:.4e}")
    return net, losses
