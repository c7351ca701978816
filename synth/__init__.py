"""Seeded synthetic CSR inputs shared by the tests, the benchmark and the oracle checks.

This module only builds input matrices (patterns and values). It holds none of the
sparse-product arithmetic: neither the GPU path nor the oracle lives here, and
nothing here imports either of them.
"""
from .csr import (
    CSR,
    uniform_rows,
    erdos_renyi,
    stencil27,
    rmat,
    transpose,
    from_dense,
    to_dense,
    random_tiny,
    batched_set,
    served_jobs,
)

__all__ = [
    "CSR",
    "uniform_rows",
    "erdos_renyi",
    "stencil27",
    "rmat",
    "transpose",
    "from_dense",
    "to_dense",
    "random_tiny",
    "batched_set",
    "served_jobs",
]
