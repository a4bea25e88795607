"""ctypes binding of liblsq (include/lsq.h).

Argument marshalling only: every step of the method runs in the library's
HIP kernels. PyTorch provides the device memory (tensors) and the stream.
"""
from __future__ import annotations

import ctypes as C
import os
import warnings
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblsq.so")

LSQ_OK, LSQ_ENOCONV = 0, 1
LSQ_EINVAL, LSQ_ESINGULAR, LSQ_ENONFINITE, LSQ_ENOMEM, LSQ_EHIP, LSQ_EBREAKDOWN, LSQ_ESTATE = range(-1, -8, -1)
LSQ_DENSE, LSQ_CSR = 0, 1
LSQ_F64, LSQ_F32 = 0, 1
LSQ_MODE_FP64, LSQ_MODE_FP32_REFINE = 0, 1

EXPORTS = ("lsq_default_options", "lsq_setup", "lsq_solve", "lsq_solve_many", "lsq_backward", "lsq_get_setup",
           "lsq_get_M_nnz", "lsq_get_M", "lsq_apply_P", "lsq_apply_K", "lsq_get_info", "lsq_get_kernel_stats", "lsq_destroy",
           "lsq_strerror", "lsq_last_error")


class LsqError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__("%s (%d): %s" % (_lib_strerror(code), code, msg))
        self.code = code


class Matrix(C.Structure):
    _fields_ = [("format", C.c_int32), ("dtype", C.c_int32), ("m", C.c_int64), ("n", C.c_int64),
                ("ld", C.c_int64), ("nnz", C.c_int64), ("values", C.c_void_p), ("row_ptr", C.c_void_p),
                ("col_idx", C.c_void_p)]


class Options(C.Structure):
    _fields_ = [("mode", C.c_int32), ("tol", C.c_double), ("max_iter", C.c_int64), ("fixed_iters", C.c_int64),
                ("max_replace", C.c_int32), ("inner_tol", C.c_double), ("max_inner", C.c_int64),
                ("max_outer", C.c_int32), ("tie_eps", C.c_double), ("atap_algo", C.c_int32),
                ("profile", C.c_int32), ("near_levels", C.c_int32), ("chain_levels", C.c_int32)]


class KernelStats(C.Structure):
    _fields_ = [("launches", C.c_int64 * 5), ("ms", C.c_double * 5), ("bytes", C.c_double * 5)]

    CLASSES = ("trsv", "sgs_rhs", "atap", "vec", "gram")  # "gram": bytes holds flops

    def as_dict(self) -> dict:
        return {name: dict(launches=int(self.launches[i]), ms=float(self.ms[i]), bytes=float(self.bytes[i]))
                for i, name in enumerate(self.CLASSES)}


class Info(C.Structure):
    _fields_ = [("s", C.c_int64), ("s_distinct", C.c_int64), ("nnz_M", C.c_int64), ("levels_fwd", C.c_int64),
                ("levels_bwd", C.c_int64), ("ties", C.c_int64), ("diag_fixes", C.c_int64), ("iters", C.c_int64),
                ("outer_iters", C.c_int64), ("replacements", C.c_int64), ("W", C.c_double),
                ("relres", C.c_double), ("relres_true", C.c_double), ("setup_ms", C.c_double),
                ("solve_ms", C.c_double), ("converged", C.c_int32), ("status", C.c_int32),
                ("trsv_mode", C.c_int32), ("atap_algo", C.c_int32),
                ("chain_levels", C.c_int32), ("chain_max", C.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def lib():
    """Load liblsq.so. Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblsq.so is not built (run __graft_entry__.build()): %s" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        P, I64, D = C.c_void_p, C.c_int64, C.c_double
        L.lsq_default_options.argtypes = [C.POINTER(Options)]
        L.lsq_default_options.restype = None
        L.lsq_setup.argtypes = [C.POINTER(Matrix), P, D, C.c_int32, C.c_uint64, C.POINTER(Options), P,
                                C.POINTER(P)]
        L.lsq_setup.restype = C.c_int
        L.lsq_solve.argtypes = [P, P, C.POINTER(Info)]
        L.lsq_solve.restype = C.c_int
        L.lsq_solve_many.argtypes = [P, C.c_int32, P, I64, P, I64, P]
        L.lsq_solve_many.restype = C.c_int
        L.lsq_backward.argtypes = [P, P, P, P, P, P, C.POINTER(Info)]
        L.lsq_backward.restype = C.c_int
        L.lsq_get_setup.argtypes = [P, P, P, P, P]
        L.lsq_get_setup.restype = C.c_int
        L.lsq_get_M_nnz.argtypes = [P]
        L.lsq_get_M_nnz.restype = I64
        L.lsq_get_M.argtypes = [P, P, P, P]
        L.lsq_get_M.restype = C.c_int
        L.lsq_apply_P.argtypes = [P, P, P]
        L.lsq_apply_P.restype = C.c_int
        L.lsq_apply_K.argtypes = [P, P, P]
        L.lsq_apply_K.restype = C.c_int
        L.lsq_get_kernel_stats.argtypes = [P, C.POINTER(KernelStats), C.c_int32]
        L.lsq_get_kernel_stats.restype = C.c_int
        L.lsq_get_info.argtypes = [P, C.POINTER(Info)]
        L.lsq_get_info.restype = C.c_int
        L.lsq_destroy.argtypes = [P]
        L.lsq_destroy.restype = None
        L.lsq_strerror.argtypes = [C.c_int]
        L.lsq_strerror.restype = C.c_char_p
        L.lsq_last_error.argtypes = [P]
        L.lsq_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def _lib_strerror(code: int) -> str:
    try:
        return lib().lsq_strerror(code).decode()
    except Exception:  # pragma: no cover - only when the library is missing
        return "error"


def default_options() -> Options:
    o = Options()
    lib().lsq_default_options(C.byref(o))
    return o


def _ptr(t) -> int:
    return 0 if t is None else int(t.data_ptr())


def _stream() -> int:
    import torch
    return int(torch.cuda.current_stream().cuda_stream)


class Solver:
    """One set-up context: Algorithm 2 steps 1-3 run in the constructor.

    Dense A: a 2-D CUDA tensor (float64 or float32, row-major, unit column
    stride). CSR A: ``values`` (float64/float32), ``row_ptr`` (int64),
    ``col_idx`` (int32) CUDA tensors and ``shape=(m, n)``. ``b`` is a float64
    CUDA tensor. The tensors must stay alive and unchanged while the solver
    lives (the library borrows them).
    """

    def __init__(self, A=None, b=None, *, values=None, row_ptr=None, col_idx=None, shape=None, C_: float = 4.0,
                 sweeps: int = 1, seed: int = 0, mode: str = "fp64", tol: float = 1e-10, max_iter: int = 0,
                 fixed_iters: int = -1, max_replace: int = 3, inner_tol: float = 1e-5, max_inner: int = 0,
                 max_outer: int = 30, tie_eps: float = 2.0 ** -44, atap_algo: int = 0, profile: bool = False,
                 near_levels: int = 0, chain_levels: int = 0):
        import torch
        if b is None or not b.is_cuda or b.dtype != torch.float64 or not b.is_contiguous():
            raise ValueError("b must be a contiguous float64 CUDA tensor")
        mat = Matrix()
        if A is not None:
            if A.dim() != 2 or not A.is_cuda or A.stride(1) != 1 or A.dtype not in (torch.float64, torch.float32):
                raise ValueError("dense A must be a 2-D float64/float32 CUDA tensor with unit column stride")
            mat.format = LSQ_DENSE
            mat.dtype = LSQ_F64 if A.dtype == torch.float64 else LSQ_F32
            mat.m, mat.n = A.shape
            mat.ld = A.stride(0)
            mat.nnz = A.shape[0] * A.shape[1]
            mat.values = _ptr(A)
            self._keep = (A, b)
            self.fmt = "dense"
        else:
            if values is None or row_ptr is None or col_idx is None or shape is None:
                raise ValueError("CSR A needs values, row_ptr, col_idx and shape")
            if row_ptr.dtype != torch.int64 or col_idx.dtype != torch.int32:
                raise ValueError("row_ptr must be int64 and col_idx int32")
            if values.dtype not in (torch.float64, torch.float32):
                raise ValueError("values must be float64 or float32")
            for t in (values, row_ptr, col_idx):
                if not t.is_cuda or not t.is_contiguous():
                    raise ValueError("CSR arrays must be contiguous CUDA tensors")
            mat.format = LSQ_CSR
            mat.dtype = LSQ_F64 if values.dtype == torch.float64 else LSQ_F32
            mat.m, mat.n = shape
            mat.ld = shape[1]
            mat.nnz = values.shape[0]
            mat.values = _ptr(values)
            mat.row_ptr = _ptr(row_ptr)
            mat.col_idx = _ptr(col_idx)
            self._keep = (values, row_ptr, col_idx, b)
            self.fmt = "csr"
        if b.shape[0] != mat.m:
            raise ValueError("b has %d entries, A has %d rows" % (b.shape[0], mat.m))
        opt = default_options()
        opt.mode = {"fp64": LSQ_MODE_FP64, "fp32_refine": LSQ_MODE_FP32_REFINE}[mode]
        opt.tol = tol
        opt.max_iter = max_iter
        opt.fixed_iters = fixed_iters
        opt.max_replace = max_replace
        opt.inner_tol = inner_tol
        opt.max_inner = max_inner
        opt.max_outer = max_outer
        opt.tie_eps = tie_eps
        opt.atap_algo = atap_algo
        opt.profile = 1 if profile else 0
        opt.near_levels = near_levels
        opt.chain_levels = chain_levels
        self.m, self.n = int(mat.m), int(mat.n)
        self.mode = mode
        self.dtype = A.dtype if A is not None else values.dtype
        self._ctx = C.c_void_p(0)
        rc = lib().lsq_setup(C.byref(mat), _ptr(b), float(C_), int(sweeps), int(seed) & (2 ** 64 - 1),
                             C.byref(opt), _stream(), C.byref(self._ctx))
        if rc != LSQ_OK:
            raise LsqError(rc, "lsq_setup failed")

    # -- lifecycle
    def close(self):
        if getattr(self, "_ctx", None) and self._ctx.value:
            lib().lsq_destroy(self._ctx)
            self._ctx = C.c_void_p(0)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if rc < 0:
            raise LsqError(rc, "%s: %s" % (what, lib().lsq_last_error(self._ctx).decode()))
        if rc == LSQ_ENOCONV:
            warnings.warn("%s: tolerance not reached" % what, RuntimeWarning, stacklevel=3)

    # -- the method
    def solve(self, out=None):
        import torch
        x = out if out is not None else torch.empty(self.n, dtype=torch.float64, device="cuda")
        info = Info()
        rc = lib().lsq_solve(self._ctx, _ptr(x), C.byref(info))
        self._check(rc, "lsq_solve")
        return x, info.as_dict()

    def solve_many(self, B):
        """Columns of B (m x k, float64 on the device) solved on this setup;
        returns X (n x k) and one info dict per column."""
        import torch
        if B.dim() != 2 or B.shape[0] != self.m or B.dtype != torch.float64 or not B.is_cuda:
            raise ValueError("B must be a float64 device tensor of shape (%d, k)" % self.m)
        k = int(B.shape[1])
        Bc = B.t().contiguous()  # column j at Bc[j], stride m
        X = torch.empty(k, self.n, dtype=torch.float64, device="cuda")  # row j = column j of the result
        infos = (Info * max(k, 1))()
        rc = lib().lsq_solve_many(self._ctx, k, _ptr(Bc), self.m, _ptr(X), self.n, infos)
        self._check(rc, "lsq_solve_many")
        return X.t(), [infos[j].as_dict() for j in range(k)]

    def backward(self, x, grad_x, want_grad_A: bool = True, want_grad_b: bool = True):
        import torch
        lam = torch.empty(self.n, dtype=torch.float64, device="cuda")
        gb = torch.empty(self.m, dtype=torch.float64, device="cuda") if want_grad_b else None
        gA = None
        if want_grad_A:
            src = self._keep[0]
            gA = torch.empty_like(src)
        info = Info()
        rc = lib().lsq_backward(self._ctx, _ptr(x), _ptr(grad_x.contiguous()), _ptr(lam), _ptr(gb), _ptr(gA),
                                C.byref(info))
        self._check(rc, "lsq_backward")
        return lam, gb, gA, info.as_dict()

    # -- inspection
    def kernel_stats(self, reset: bool = False) -> dict:
        st = KernelStats()
        self._check(lib().lsq_get_kernel_stats(self._ctx, C.byref(st), 1 if reset else 0), "lsq_get_kernel_stats")
        return st.as_dict()

    def info(self) -> dict:
        inf = Info()
        lib().lsq_get_info(self._ctx, C.byref(inf))
        return inf.as_dict()

    def setup_arrays(self, want_w: bool = True):
        inf = self.info()
        s = inf["s"]
        D = np.zeros(self.n)
        w = np.zeros(self.m) if want_w else None
        idx = np.zeros(s, dtype=np.int64)
        gap = np.zeros(s)
        rc = lib().lsq_get_setup(self._ctx, D.ctypes.data, 0 if w is None else w.ctypes.data, idx.ctypes.data,
                                 gap.ctypes.data)
        self._check(rc, "lsq_get_setup")
        return D, w, idx, gap

    def M_csr(self):
        nnz = lib().lsq_get_M_nnz(self._ctx)
        rp = np.zeros(self.n + 1, dtype=np.int64)
        ci = np.zeros(nnz, dtype=np.int32)
        v = np.zeros(nnz)
        rc = lib().lsq_get_M(self._ctx, rp.ctypes.data, ci.ctypes.data, v.ctypes.data)
        self._check(rc, "lsq_get_M")
        return rp, ci, v

    def M_dense(self):
        rp, ci, v = self.M_csr()
        out = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(rp))
        out[rows, ci] = v
        return out

    def apply_P(self, r):
        import torch
        z = torch.empty_like(r)
        self._check(lib().lsq_apply_P(self._ctx, _ptr(r.contiguous()), _ptr(z)), "lsq_apply_P")
        return z

    def apply_K(self, p):
        import torch
        q = torch.empty_like(p)
        self._check(lib().lsq_apply_K(self._ctx, _ptr(p.contiguous()), _ptr(q)), "lsq_apply_K")
        return q


def _autograd_function():
    import torch

    class LsqSolve(torch.autograd.Function):
        """x = argmin ||A x - b|| by Algorithm 2; backward by the adjoint solve
        A^T A lambda = dL/dx with the same preconditioner:
        dL/db = A lambda, dL/dA = (b - A x) lambda^T - (A lambda) x^T on A's pattern.

        Dense: apply(A, b, opts). CSR: apply(values, b, opts) with
        opts["row_ptr"], opts["col_idx"], opts["shape"]; the gradient of a CSR
        matrix is returned on ``values``.
        """

        @staticmethod
        def forward(ctx, A_or_values, b, opts):
            kw = dict(opts)
            csr = "row_ptr" in kw
            if csr:
                solver = Solver(values=A_or_values.detach(), b=b.detach(), **kw)
            else:
                solver = Solver(A_or_values.detach(), b.detach(), **kw)
            x, info = solver.solve()
            ctx.solver = solver
            ctx.save_for_backward(x)
            ctx.info = info
            return x

        @staticmethod
        def backward(ctx, gx):
            (x,) = ctx.saved_tensors
            need_A, need_b = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
            _, gb, gA, _ = ctx.solver.backward(x, gx.to(torch.float64), want_grad_A=need_A, want_grad_b=need_b)
            return gA, gb, None

    return LsqSolve


_LsqSolve = None


def LsqSolve():
    global _LsqSolve
    if _LsqSolve is None:
        _LsqSolve = _autograd_function()
    return _LsqSolve


def solve(A=None, b=None, *, values=None, row_ptr=None, col_idx=None, shape=None, **kw):
    """Differentiable least-squares solve (returns x, float64)."""
    F = LsqSolve()
    if A is not None:
        return F.apply(A, b, kw)
    opts = dict(kw, row_ptr=row_ptr, col_idx=col_idx, shape=tuple(shape))
    return F.apply(values, b, opts)
