"""Seeded synthetic inputs shaped like the paper's matrix families.

This package only draws random matrices and right-hand sides. It holds none of
the solver's arithmetic (no norms, no sampling, no Gram products, no solves),
so both the CPU oracle and the HIP path can take their inputs from it.
"""
from .generators import (  # noqa: F401
    Problem,
    gaussian_dense,
    sparse_rowscaled,
    udv_dense,
    er_incidence,
    semi_gaussian_dense,
    powerlaw_laplacian,
    coherent_identity,
    semi_coherent_block,
    make_config,
    CONFIG_NAMES,
)
