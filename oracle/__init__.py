"""CPU float64 oracle for the row-sampling preconditioned least-squares solver.

TEST INFRASTRUCTURE ONLY. The tests, the smoke check and the benchmark's
CPU-baseline leg use it to check and time the GPU library; the GPU library
never imports, links or calls anything here.
"""
from .oracle import (  # noqa: F401
    Oracle,
    build,
    lib,
    philox4x64_10,
    uniform,
    sample_size,
    column_norms,
    row_weights,
    cdf,
    draw,
)
