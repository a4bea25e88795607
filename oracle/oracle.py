"""ctypes wrapper around the C oracle ``liblsq_oracle.so`` (test infrastructure only).

Arrays are passed as numpy buffers; matrices come from ``workloads.Problem``.
The shared library is compiled by :func:`build` (gcc, strict IEEE float64: no
fast-math, no FMA contraction).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lsq_oracle.c")
_LIB = os.path.join(_HERE, "liblsq_oracle.so")

_lib = None


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into oracle/liblsq_oracle.so."""
    global _lib
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
               "-Wall", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
        _lib = None
    return _LIB


class _Matrix(C.Structure):
    _fields_ = [("fmt", C.c_int32), ("dtype", C.c_int32), ("m", C.c_int64), ("n", C.c_int64),
                ("ld", C.c_int64), ("nnz", C.c_int64), ("values", C.c_void_p),
                ("row_ptr", C.c_void_p), ("col_idx", C.c_void_p)]


class Info(C.Structure):
    _fields_ = [("s", C.c_int64), ("iters", C.c_int64), ("replacements", C.c_int64),
                ("ties", C.c_int64), ("diag_fixes", C.c_int64), ("nnz_M", C.c_int64),
                ("W", C.c_double), ("relres", C.c_double), ("relres_true", C.c_double),
                ("status", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_P = C.c_void_p
_I64 = C.c_int64
_D = C.c_double


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = C.CDLL(_LIB)
        L.orc_philox4x64_10.argtypes = [_P, _P, _P]
        L.orc_uniform.argtypes = [C.c_uint64, _I64]
        L.orc_uniform.restype = _D
        L.orc_sample_size.argtypes = [_D, _I64]
        L.orc_sample_size.restype = _I64
        L.orc_column_norms.argtypes = [C.POINTER(_Matrix), _P]
        L.orc_column_norms.restype = C.c_int
        L.orc_row_weights.argtypes = [C.POINTER(_Matrix), _P, _P]
        L.orc_cdf.argtypes = [_I64, _P, _P]
        L.orc_cdf.restype = _D
        L.orc_draw.argtypes = [_I64, _P, _P, _D, _P]
        L.orc_draw.restype = _I64
        L.orc_setup.argtypes = [C.POINTER(_Matrix), _D, C.c_int32, C.c_uint64, _D, _P, _I64,
                                C.POINTER(C.c_int32)]
        L.orc_setup.restype = _P
        L.orc_free.argtypes = [_P]
        L.orc_n.argtypes = [_P]
        L.orc_n.restype = _I64
        L.orc_s.argtypes = [_P]
        L.orc_s.restype = _I64
        for f in ("orc_get_D", "orc_get_w", "orc_get_M_dense"):
            getattr(L, f).argtypes = [_P, _P]
        L.orc_get_samples.argtypes = [_P, _P, _P]
        L.orc_get_info.argtypes = [_P, C.POINTER(Info)]
        L.orc_M_nnz.argtypes = [_P]
        L.orc_M_nnz.restype = _I64
        L.orc_get_M_csr.argtypes = [_P, _P, _P, _P]
        L.orc_M_entry.argtypes = [_P, _I64, _I64]
        L.orc_M_entry.restype = _D
        L.orc_apply_P.argtypes = [_P, _P, _P]
        L.orc_apply_K.argtypes = [_P, _P, _P]
        L.orc_solve.argtypes = [_P, _P, _D, _I64, _I64, C.c_int32, _P, C.POINTER(Info)]
        L.orc_solve.restype = C.c_int
        L.orc_backward.argtypes = [_P, _P, _P, _P, _D, _I64, _I64, C.c_int32, _P, _P, _P,
                                   C.POINTER(Info)]
        L.orc_backward.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class _MatrixHolder:
    """Keeps the numpy buffers of a matrix alive while the C side uses them."""

    def __init__(self, problem):
        p = problem
        if p.fmt == "dense":
            A = np.ascontiguousarray(p.A)
            if A.dtype not in (np.float64, np.float32):
                A = A.astype(np.float64)
            self.keep = (A,)
            self.s = _Matrix(0, 0 if A.dtype == np.float64 else 1, p.m, p.n, A.shape[1], p.m * p.n,
                             A.ctypes.data, None, None)
        else:
            v = np.ascontiguousarray(p.values)
            if v.dtype not in (np.float64, np.float32):
                v = v.astype(np.float64)
            rp = np.ascontiguousarray(p.row_ptr, dtype=np.int64)
            ci = np.ascontiguousarray(p.col_idx, dtype=np.int32)
            self.keep = (v, rp, ci)
            self.s = _Matrix(1, 0 if v.dtype == np.float64 else 1, p.m, p.n, p.n, v.shape[0],
                             v.ctypes.data, rp.ctypes.data, ci.ctypes.data)


# ---- building blocks -----------------------------------------------------


def philox4x64_10(ctr, key) -> np.ndarray:
    c = np.asarray(ctr, dtype=np.uint64).copy()
    k = np.asarray(key, dtype=np.uint64).copy()
    out = np.zeros(4, dtype=np.uint64)
    lib().orc_philox4x64_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def uniform(seed: int, t: int) -> float:
    return lib().orc_uniform(seed, t)


def sample_size(C_: float, n: int) -> int:
    return lib().orc_sample_size(C_, n)


def column_norms(problem) -> tuple:
    h = _MatrixHolder(problem)
    D = np.zeros(problem.n)
    rc = lib().orc_column_norms(C.byref(h.s), _ptr(D))
    return D, rc


def row_weights(problem, invD) -> np.ndarray:
    h = _MatrixHolder(problem)
    invD = _f64(invD)
    w = np.zeros(problem.m)
    lib().orc_row_weights(C.byref(h.s), _ptr(invD), _ptr(w))
    return w


def cdf(w) -> tuple:
    w = _f64(w)
    out = np.zeros_like(w)
    W = lib().orc_cdf(w.shape[0], _ptr(w), _ptr(out))
    return out, W


def draw(w, cdf_, tau) -> tuple:
    w = _f64(w)
    c = _f64(cdf_)
    g = np.zeros(1)
    i = lib().orc_draw(w.shape[0], _ptr(w), _ptr(c), float(tau), _ptr(g))
    return int(i), float(g[0])


# ---- the method ----------------------------------------------------------


class Oracle:
    """Algorithm 2 on the CPU in float64. Holds the setup (D, draws, M)."""

    TIE_EPS = 2.0 ** -44

    def __init__(self, problem, C_: float = 4.0, sweeps: int = 1, seed: int = 0,
                 tie_eps: float = TIE_EPS, samples: Optional[np.ndarray] = None):
        self.problem = problem
        self._h = _MatrixHolder(problem)
        st = C.c_int32(0)
        idx = None
        if samples is not None:
            idx = np.ascontiguousarray(samples, dtype=np.int64)
        self._idx_keep = idx
        self._st = lib().orc_setup(C.byref(self._h.s), float(C_), int(sweeps), int(seed) & (2**64 - 1),
                                   float(tie_eps), _ptr(idx), 0 if idx is None else idx.shape[0],
                                   C.byref(st))
        self.status = st.value
        if not self._st:
            raise ValueError("oracle setup failed with status %d" % st.value)
        self.m, self.n = problem.m, problem.n
        self.s = lib().orc_s(self._st)

    def __del__(self):
        if getattr(self, "_st", None):
            lib().orc_free(self._st)
            self._st = None

    # accessors
    @property
    def D(self):
        out = np.zeros(self.n)
        lib().orc_get_D(self._st, _ptr(out))
        return out

    @property
    def w(self):
        out = np.zeros(self.m)
        lib().orc_get_w(self._st, _ptr(out))
        return out

    def samples(self):
        idx = np.zeros(self.s, dtype=np.int64)
        gap = np.zeros(self.s)
        lib().orc_get_samples(self._st, _ptr(idx), _ptr(gap))
        return idx, gap

    def info(self) -> dict:
        inf = Info()
        lib().orc_get_info(self._st, C.byref(inf))
        return inf.as_dict()

    def M_dense(self):
        out = np.zeros((self.n, self.n))
        lib().orc_get_M_dense(self._st, _ptr(out))
        return out

    def M_csr(self):
        nnz = lib().orc_M_nnz(self._st)
        rp = np.zeros(self.n + 1, dtype=np.int64)
        ci = np.zeros(nnz, dtype=np.int32)
        v = np.zeros(nnz)
        lib().orc_get_M_csr(self._st, _ptr(rp), _ptr(ci), _ptr(v))
        return rp, ci, v

    def M_entry(self, j: int, l: int) -> float:
        return lib().orc_M_entry(self._st, j, l)

    def apply_P(self, r):
        r = _f64(r)
        z = np.zeros(self.n)
        lib().orc_apply_P(self._st, _ptr(r), _ptr(z))
        return z

    def apply_K(self, p):
        p = _f64(p)
        q = np.zeros(self.n)
        lib().orc_apply_K(self._st, _ptr(p), _ptr(q))
        return q

    def solve(self, b=None, tol: float = 1e-10, max_iter: int = 0, fixed_iters: int = -1,
              max_replace: int = 3):
        b = _f64(self.problem.b if b is None else b)
        x = np.zeros(self.n)
        inf = Info()
        lib().orc_solve(self._st, _ptr(b), tol, max_iter, fixed_iters, max_replace, _ptr(x), C.byref(inf))
        return x, inf.as_dict()

    def backward(self, x, gx, b=None, tol: float = 1e-10, max_iter: int = 0, fixed_iters: int = -1,
                 max_replace: int = 3, want_grad_A: bool = True):
        b = _f64(self.problem.b if b is None else b)
        x = _f64(x)
        gx = _f64(gx)
        lam = np.zeros(self.n)
        gb = np.zeros(self.m)
        p = self.problem
        gA = None
        if want_grad_A:
            gA = np.zeros(p.values.shape[0]) if p.fmt == "csr" else np.zeros((p.m, p.n))
        inf = Info()
        lib().orc_backward(self._st, _ptr(b), _ptr(x), _ptr(gx), tol, max_iter, fixed_iters, max_replace,
                           _ptr(lam), _ptr(gb), _ptr(gA), C.byref(inf))
        return lam, gb, gA, inf.as_dict()
