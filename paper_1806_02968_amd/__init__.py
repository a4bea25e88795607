"""Row-sampling preconditioned least squares (Chen & Wu, arXiv:1806.02968) on MI355X.

The solver lives in the HIP library ``liblsq.so`` (C ABI in include/lsq.h);
this package is its Python binding and autograd wrapper.
"""
from .lsq import (  # noqa: F401
    EXPORTS,
    LIB_PATH,
    LsqError,
    LsqSolve,
    Solver,
    default_options,
    lib,
    solve,
)
