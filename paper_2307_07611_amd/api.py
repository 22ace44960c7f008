"""PyTorch-facing wrappers of libtrinv (argument marshalling only).

PyTorch supplies device memory (outputs and workspaces) and the current HIP
stream; every step of the computation runs in the library's HIP kernels.
"""

from __future__ import annotations

import ctypes

import torch

from . import _lib

_DT = {torch.float64: "f64", torch.float32: "f32"}


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_dev(*ts):
    for t in ts:
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError("expected CUDA (HIP) tensors")


def _mode_for(t: torch.Tensor, mode):
    if mode is None:
        if t.dtype not in _DT:
            raise ValueError(f"unsupported dtype {t.dtype}")
        mode = _DT[t.dtype]
    m = _lib.MODES[mode]
    want = torch.float32 if m == _lib.F32 else torch.float64
    if t.dtype != want:
        raise ValueError(f"mode {mode} needs {want} inputs, got {t.dtype}")
    return m


def _opts(leaf=0, unit_diag=False, upper=False, max_iter=4, tol=1e-12, blocking=True, check=False, beta=0,
          resid="auto"):
    o = _lib.Opts()
    _lib.load().trinv_default_opts(ctypes.byref(o))
    o.leaf, o.unit_diag, o.upper = int(leaf), int(unit_diag), int(upper)
    o.max_iter, o.tol, o.blocking, o.check = int(max_iter), float(tol), int(blocking), int(check)
    o.beta = int(beta)
    o.resid = _lib.RESID[resid] if isinstance(resid, str) else int(resid)
    return o


def _workspace(nbytes: int, device):
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


def _info_dict(info: _lib.Info) -> dict:
    return {"rel_residual": info.rel_residual, "resid_error_est": info.resid_error_est,
            "resid_error_bound": info.resid_error_bound, "iterations": info.iterations,
            "first_bad_index": info.first_bad_index}


def tril_inverse(L: torch.Tensor, mode=None, *, leaf=0, unit_diag=False, upper=False, max_iter=4, tol=1e-12,
                 blocking=True, check=False, beta=0, resid="auto", out=None, workspace=None, return_info=False):
    """X = L^-1 for one triangular matrix (lower; ``upper=True`` for upper).
    ``beta`` > 2: top level of algorithm COMBRIT on a beta x beta block grid.
    ``resid`` (refine modes): "auto", "split" or "fp64" residual product."""
    _check_dev(L)
    if L.dim() != 2 or L.shape[0] != L.shape[1] or L.stride(1) != 1:
        raise ValueError("L must be a square matrix with unit column stride")
    m = _mode_for(L, mode)
    n = L.shape[0]
    X = out if out is not None else torch.empty((n, n), dtype=L.dtype, device=L.device)
    lib = _lib.load()
    o = _opts(leaf, unit_diag, upper, max_iter, tol, blocking, check, beta, resid)
    nbytes = lib.trinv_workspace_bytes(m, n, ctypes.byref(o))
    ws = workspace if workspace is not None else _workspace(nbytes, L.device)
    info = _lib.Info()
    st = lib.trinv_tril_inverse(m, n, L.data_ptr(), L.stride(0), X.data_ptr(), X.stride(0), ctypes.byref(o),
                                ws.data_ptr(), ws.numel(), _stream(), ctypes.byref(info))
    if st != _lib.OK:
        raise _lib.TrinvError(st, "trinv_tril_inverse", _info_dict(info))
    return (X, _info_dict(info)) if return_info else X


def workspace_bytes(n: int, mode="f64", **kw) -> int:
    return int(_lib.load().trinv_workspace_bytes(_lib.MODES[mode], n, ctypes.byref(_opts(**kw))))


def residual(L: torch.Tensor, X: torch.Tensor) -> dict:
    """FP64 ||LX - I||_F, ||L||_F, ||X||_F computed on the GPU (FP64 MFMA)."""
    _check_dev(L, X)
    m = _mode_for(L, None)
    n = L.shape[0]
    lib = _lib.load()
    ws = _workspace(lib.trinv_residual_workspace_bytes(m, n), L.device)
    out = (ctypes.c_double * 3)()
    st = lib.trinv_residual(m, n, L.data_ptr(), L.stride(0), X.data_ptr(), X.stride(0), ws.data_ptr(), ws.numel(),
                            _stream(), out)
    if st != _lib.OK:
        raise _lib.TrinvError(st, "trinv_residual")
    r = {"lx": out[0], "norm_l": out[1], "norm_x": out[2]}
    r["rel"] = r["lx"] / (r["norm_l"] * r["norm_x"]) if r["norm_l"] * r["norm_x"] else 0.0
    return r


def refine_residual(L: torch.Tensor, X: torch.Tensor, mode="bf16_refine", nsplit=3, R=None) -> dict:
    """R = I - L X by the refinement's split residual product
    (trinv_refine_residual): returns R (FP32, lower triangle; zeros above
    it), its norms, the estimated error of the relative residual and its
    worst-case bound."""
    _check_dev(L, X)
    n = L.shape[0]
    m = _lib.MODES[mode]
    if R is None:
        R = torch.zeros((n, n), dtype=torch.float32, device=L.device)
    lib = _lib.load()
    ws = _workspace(lib.trinv_refine_residual_workspace_bytes(m, n), L.device)
    out = (ctypes.c_double * 5)()
    st = lib.trinv_refine_residual(m, n, L.data_ptr(), L.stride(0), X.data_ptr(), X.stride(0), int(nsplit),
                                   R.data_ptr(), R.stride(0), ws.data_ptr(), ws.numel(), _stream(), out)
    if st != _lib.OK:
        raise _lib.TrinvError(st, "trinv_refine_residual")
    r = {"R": R, "r": out[0], "norm_l": out[1], "norm_x": out[2], "est": out[3], "bound": out[4]}
    r["rel"] = r["r"] / (r["norm_l"] * r["norm_x"]) if r["norm_l"] * r["norm_x"] else 0.0
    return r


def tril_inverse_backward(X: torch.Tensor, G: torch.Tensor) -> torch.Tensor:
    """-tril(X^T G X^T) for a matrix or a batch (leading dimension) of matrices."""
    _check_dev(X, G)
    squeeze = X.dim() == 2
    Xb = X.unsqueeze(0) if squeeze else X
    Gb = (G.unsqueeze(0) if squeeze else G).contiguous()
    Xb = Xb.contiguous()
    batch, n = Xb.shape[0], Xb.shape[-1]
    m = _mode_for(Xb, None)
    grad = torch.empty_like(Xb)
    lib = _lib.load()
    ws = _workspace(lib.trinv_backward_workspace_bytes(m, batch, n), X.device)
    st = lib.trinv_tril_inverse_backward(m, batch, n, Xb.data_ptr(), Gb.data_ptr(), grad.data_ptr(), n * n,
                                         ws.data_ptr(), ws.numel(), _stream())
    if st != _lib.OK:
        raise _lib.TrinvError(st, "trinv_tril_inverse_backward")
    return grad[0] if squeeze else grad


def factored_inverse(L: torch.Tensor, U: torch.Tensor, *, l_unit=False, u_unit=False, want_ainv=True, leaf=0,
                     blocking=True):
    """(Linv, Uinv, Ainv) with A = L U; Ainv = Uinv Linv (None if not wanted).
    L and U may be row-strided views (unit column stride); the outputs are
    new contiguous matrices."""
    _check_dev(L, U)
    for t in (L, U):
        if t.dim() != 2 or t.shape[0] != t.shape[1] or t.stride(1) != 1:
            raise ValueError("factored_inverse: L and U must be square matrices with unit column stride")
    m = _mode_for(L, None)
    n = L.shape[0]
    Linv = torch.empty((n, n), dtype=L.dtype, device=L.device)
    Uinv = torch.empty_like(Linv)
    Ainv = torch.empty_like(Linv) if want_ainv else None
    lib = _lib.load()
    o = _opts(leaf=leaf, blocking=blocking)
    ws = _workspace(lib.trinv_factored_workspace_bytes(m, n, ctypes.byref(o)), L.device)
    info = _lib.Info()
    st = lib.trinv_factored_inverse(m, n, L.data_ptr(), max(L.stride(0), 1), int(l_unit), U.data_ptr(),
                                    max(U.stride(0), 1), int(u_unit), Linv.data_ptr(), n, Uinv.data_ptr(), n,
                                    Ainv.data_ptr() if Ainv is not None else None, n,
                                    ctypes.byref(o), ws.data_ptr(), ws.numel(), _stream(), ctypes.byref(info))
    if st != _lib.OK:
        raise _lib.TrinvError(st, "trinv_factored_inverse", _info_dict(info))
    return Linv, Uinv, Ainv


def tril_inverse_batched(L_packed: torch.Tensor, sizes, offsets=None, mode=None, *, blocking=True, leaf=0,
                         upper=False, out=None, workspace=None, n_dev=None, off_dev=None, status=None):
    """Inverse of every matrix of a packed batch (dense n_i x n_i blocks at
    element offsets ``offsets``); returns (X_packed, status per matrix).
    Uneven orders run in one persistent launch (after a one-block plan
    kernel); uniform ones as batched level products. ``upper``: the matrices
    are upper triangular (inverted through their transposes)."""
    _check_dev(L_packed)
    import numpy as np

    sizes_np = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32))
    if offsets is None:
        offsets = np.zeros(len(sizes_np), dtype=np.int64)
        if len(sizes_np) > 1:
            offsets[1:] = np.cumsum(sizes_np[:-1].astype(np.int64) ** 2)
    off_np = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    m = _mode_for(L_packed, mode)
    batch = len(sizes_np)
    dev = L_packed.device
    if n_dev is None:
        n_dev = torch.from_numpy(sizes_np).to(dev)
    if off_dev is None:
        off_dev = torch.from_numpy(off_np).to(dev)
    X = out if out is not None else torch.empty_like(L_packed)
    if status is None:
        status = torch.empty(batch, dtype=torch.int32, device=dev)
    lib = _lib.load()
    o = _opts(leaf=leaf, blocking=blocking, upper=upper)
    nbytes = lib.trinv_batched_workspace_bytes(m, batch, sizes_np.ctypes.data, ctypes.byref(o))
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    st = lib.trinv_tril_inverse_batched(m, batch, sizes_np.ctypes.data, n_dev.data_ptr(), off_np.ctypes.data,
                                        off_dev.data_ptr(), L_packed.data_ptr(), X.data_ptr(), status.data_ptr(),
                                        ctypes.byref(o), ws.data_ptr(), ws.numel(), _stream())
    if st not in (_lib.OK, _lib.ERR_SINGULAR, _lib.ERR_NONFINITE):  # those two: per matrix, in ``status``
        raise _lib.TrinvError(st, "trinv_tril_inverse_batched")
    return X, status


def batched_autotune(L_packed: torch.Tensor, sizes, offsets=None, mode=None, *, leaf=0, out=None, workspace=None,
                     n_dev=None, off_dev=None, status=None) -> dict:
    """Times the persistent batched launch's configurations on this batch and
    keeps the fastest for batches with the same orders (trinv_batched_autotune);
    returns it as a dict (leaf, wgs_per_cu, ms). X (``out``) and
    ``status`` hold the result of the chosen configuration."""
    _check_dev(L_packed)
    import numpy as np

    sizes_np = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32))
    if offsets is None:
        offsets = np.zeros(len(sizes_np), dtype=np.int64)
        if len(sizes_np) > 1:
            offsets[1:] = np.cumsum(sizes_np[:-1].astype(np.int64) ** 2)
    off_np = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    m = _mode_for(L_packed, mode)
    batch = len(sizes_np)
    dev = L_packed.device
    if n_dev is None:
        n_dev = torch.from_numpy(sizes_np).to(dev)
    if off_dev is None:
        off_dev = torch.from_numpy(off_np).to(dev)
    X = out if out is not None else torch.empty_like(L_packed)
    if status is None:
        status = torch.empty(batch, dtype=torch.int32, device=dev)
    lib = _lib.load()
    o = _opts(leaf=leaf, blocking=False)
    nbytes = lib.trinv_batched_workspace_bytes(m, batch, sizes_np.ctypes.data, ctypes.byref(o))
    ws = workspace if workspace is not None else _workspace(nbytes, dev)
    cfg = _lib.BatchedConfig()
    st = lib.trinv_batched_autotune(m, batch, sizes_np.ctypes.data, n_dev.data_ptr(), off_np.ctypes.data,
                                    off_dev.data_ptr(), L_packed.data_ptr(), X.data_ptr(), status.data_ptr(),
                                    ctypes.byref(o), ws.data_ptr(), ws.numel(), _stream(), ctypes.byref(cfg))
    if st != _lib.OK:
        raise _lib.TrinvError(st, "trinv_batched_autotune")
    return {"leaf": cfg.leaf, "wgs_per_cu": cfg.wgs_per_cu, "tile": cfg.tile, "ms": cfg.ms}


def batched_set_config(sizes, mode, leaf, wgs_per_cu=0, tile=0):
    """Pin the persistent batched launch's configuration for batches with these
    orders (trinv_batched_set_config)."""
    import numpy as np

    sizes_np = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32))
    cfg = _lib.BatchedConfig(leaf, wgs_per_cu, -1.0, tile)
    st = _lib.load().trinv_batched_set_config(_lib.MODES[mode], len(sizes_np), sizes_np.ctypes.data,
                                              ctypes.byref(cfg))
    if st != _lib.OK:
        raise _lib.TrinvError(st, "trinv_batched_set_config")


def batched_get_config(sizes, mode) -> dict:
    """The persistent batched launch's configuration for batches with these
    orders: set, tuned in this process or loaded from the TRINV_TUNE_CACHE
    file, else the defaults (trinv_batched_get_config)."""
    import numpy as np

    sizes_np = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32))
    cfg = _lib.BatchedConfig()
    st = _lib.load().trinv_batched_get_config(_lib.MODES[mode], len(sizes_np), sizes_np.ctypes.data,
                                              ctypes.byref(cfg))
    if st != _lib.OK:
        raise _lib.TrinvError(st, "trinv_batched_get_config")
    return {"leaf": cfg.leaf, "wgs_per_cu": cfg.wgs_per_cu, "tile": cfg.tile}


def skul(A: torch.Tensor, *, want_ainv=True, leaf=0, blocking=True):
    """Algorithm SKUL: (L, U, S, K, Ainv) with A = L U (Crout, U unit upper, no
    pivoting), S = U^-1, K = L^-1 and Ainv = S K (None if not wanted)."""
    _check_dev(A)
    A = A.contiguous()
    m = _mode_for(A, None)
    n = A.shape[0]
    L, U, S, K = (torch.empty_like(A) for _ in range(4))
    Ainv = torch.empty_like(A) if want_ainv else None
    lib = _lib.load()
    o = _opts(leaf=leaf, blocking=blocking)
    ws = _workspace(lib.trinv_skul_workspace_bytes(m, n, ctypes.byref(o)), A.device)
    info = _lib.Info()
    st = lib.trinv_skul(m, n, A.data_ptr(), L.data_ptr(), U.data_ptr(), S.data_ptr(), K.data_ptr(),
                        Ainv.data_ptr() if want_ainv else None, ctypes.byref(o), ws.data_ptr(), ws.numel(), _stream(),
                        ctypes.byref(info))
    if st != _lib.OK:
        raise _lib.TrinvError(st, "trinv_skul", _info_dict(info))
    return L, U, S, K, Ainv


def sqr(A: torch.Tensor, *, want_ainv=True, leaf=0, blocking=True):
    """Algorithm SQR: (Q, R, S, Ainv) with A = Q R (modified Gram-Schmidt,
    R(j, j) > 0), S = R^-1 and Ainv = S Q^T (None if not wanted)."""
    _check_dev(A)
    A = A.contiguous()
    m = _mode_for(A, None)
    n = A.shape[0]
    Q, R, S = (torch.empty_like(A) for _ in range(3))
    Ainv = torch.empty_like(A) if want_ainv else None
    lib = _lib.load()
    o = _opts(leaf=leaf, blocking=blocking)
    ws = _workspace(lib.trinv_sqr_workspace_bytes(m, n, ctypes.byref(o)), A.device)
    info = _lib.Info()
    st = lib.trinv_sqr(m, n, A.data_ptr(), Q.data_ptr(), R.data_ptr(), S.data_ptr(),
                       Ainv.data_ptr() if want_ainv else None, ctypes.byref(o), ws.data_ptr(), ws.numel(), _stream(),
                       ctypes.byref(info))
    if st != _lib.OK:
        raise _lib.TrinvError(st, "trinv_sqr", _info_dict(info))
    return Q, R, S, Ainv


def brsi(A: torch.Tensor, *, blocking=True):
    """General inverse by BRSI with gamma = 2 (no pivoting)."""
    _check_dev(A)
    if A.dim() != 2 or A.shape[0] != A.shape[1] or A.stride(1) != 1:
        raise ValueError("brsi: A must be a square matrix with unit column stride")
    m = _mode_for(A, None)
    n = A.shape[0]
    X = torch.empty((n, n), dtype=A.dtype, device=A.device)
    lib = _lib.load()
    o = _opts(blocking=blocking)
    ws = _workspace(lib.trinv_brsi_workspace_bytes(m, n, ctypes.byref(o)), A.device)
    info = _lib.Info()
    st = lib.trinv_brsi(m, n, A.data_ptr(), max(A.stride(0), 1), X.data_ptr(), n, ctypes.byref(o), ws.data_ptr(),
                        ws.numel(), _stream(), ctypes.byref(info))
    if st != _lib.OK:
        raise _lib.TrinvError(st, "trinv_brsi", _info_dict(info))
    return X


class BatchedGraph:
    """A fixed batch layout with static device buffers whose inversion is
    captured once in a graph (``torch.cuda.CUDAGraph``) and replayed.

    Write the inputs into ``self.L`` (packed, dense n_i x n_i blocks at
    ``self.offsets``), call ``replay()``; the inverses land in ``self.X`` and
    the per-matrix status in ``self.status``."""

    def __init__(self, sizes, offsets=None, dtype=torch.float32, device="cuda", leaf=0):
        import numpy as np

        self.sizes = np.ascontiguousarray(np.asarray(sizes, dtype=np.int32))
        if offsets is None:
            offsets = np.zeros(len(self.sizes), dtype=np.int64)
            if len(self.sizes) > 1:
                offsets[1:] = np.cumsum(self.sizes[:-1].astype(np.int64) ** 2)
        self.offsets = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
        total = int(np.max(self.offsets + self.sizes.astype(np.int64) ** 2)) if len(self.sizes) else 0
        self.mode_name = "f32" if dtype == torch.float32 else "f64"
        self.mode = _lib.MODES[self.mode_name]
        self.leaf = leaf
        self.L = torch.zeros(total, dtype=dtype, device=device)
        self.X = torch.empty_like(self.L)
        self.status = torch.empty(len(self.sizes), dtype=torch.int32, device=device)
        self.n_dev = torch.from_numpy(self.sizes).to(device)
        self.off_dev = torch.from_numpy(self.offsets).to(device)
        lib = _lib.load()
        o = _opts(leaf=leaf, blocking=False)
        nbytes = lib.trinv_batched_workspace_bytes(self.mode, len(self.sizes), self.sizes.ctypes.data,
                                                   ctypes.byref(o))
        self.ws = _workspace(nbytes, self.L.device)
        self.graph = None
        self.config = None

    def _call(self):
        tril_inverse_batched(self.L, self.sizes, self.offsets, self.mode_name, blocking=False, leaf=self.leaf,
                             out=self.X, workspace=self.ws, n_dev=self.n_dev, off_dev=self.off_dev,
                             status=self.status)

    def run_eager(self):
        self._call()

    def tune(self):
        """Run the autotuner on this batch layout (the current contents of
        ``self.L``); the chosen configuration is used by every later launch,
        captured ones included."""
        self.config = batched_autotune(self.L, self.sizes, self.offsets, self.mode_name, leaf=self.leaf, out=self.X,
                                       workspace=self.ws, n_dev=self.n_dev, off_dev=self.off_dev, status=self.status)
        return self.config

    def capture(self, tune=True):
        if tune:
            self.tune()  # outside the graph: it times launches and synchronises
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self._call()  # warm-up outside the graph (kernel loading, occupancy query)
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        self.graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(self.graph):
            self._call()
        return self

    def replay(self):
        if self.graph is None:
            self.capture()
        self.graph.replay()


class TrilInverse(torch.autograd.Function):
    """X = L^-1 with the hand-written adjoint gradL = -tril(X^T G X^T).

    The forward's X is saved and reused by the backward (no recomputation)."""

    @staticmethod
    def forward(ctx, L, mode=None):
        if L.dim() == 2:
            X = tril_inverse(L, mode)
        else:
            X = batched_uniform_inverse(L, mode)
        ctx.save_for_backward(X)
        return X

    @staticmethod
    def backward(ctx, G):
        (X,) = ctx.saved_tensors
        return tril_inverse_backward(X, G), None


def batched_uniform_inverse(L: torch.Tensor, mode=None) -> torch.Tensor:
    """Inverse of a (batch, n, n) stack of lower-triangular matrices. Raises
    TrinvError (ERR_SINGULAR / ERR_NONFINITE) naming the offending matrices
    if any of them has an exact zero diagonal entry or a non-finite inverse."""
    _check_dev(L)
    L = L.contiguous()
    batch, n = L.shape[0], L.shape[-1]
    sizes = [n] * batch
    X, status = tril_inverse_batched(L.view(-1), sizes, mode=mode)
    st = status.cpu()
    if bool((st != 0).any()):
        bad = torch.nonzero(st != 0).flatten().tolist()
        code = _lib.ERR_SINGULAR if bool((st[bad] > 0).any()) else _lib.ERR_NONFINITE
        raise _lib.TrinvError(code, "batched_uniform_inverse",
                              {"matrices": bad, "status": [int(st[i]) for i in bad]})
    return X.view(batch, n, n)


def profile_enable(on: bool = True) -> None:
    """Start (dropping any previous one) or stop recording launch profiles."""
    _lib.load().trinv_profile_enable(int(on))


def profile_select(classes=None) -> None:
    """Record only the named kernel classes (an iterable of names; None: all)."""
    arg = None if not classes else ",".join(classes).encode()
    _lib.load().trinv_profile_select(arg)


def profile_read() -> dict:
    """Per kernel class: launches, total_ms, flops, bytes (waits for the GPU)."""
    lib = _lib.load()
    buf = (_lib.ProfileEntry * 64)()
    n = lib.trinv_profile_read(buf, 64)
    if n < 0:
        raise _lib.TrinvError(-n, "trinv_profile_read")
    return {buf[i].name.decode(): {"launches": buf[i].launches, "total_ms": buf[i].total_ms,
                                   "flops": buf[i].flops, "bytes": buf[i].bytes} for i in range(min(n, 64))}
