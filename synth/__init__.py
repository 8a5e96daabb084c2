"""Seeded synthetic sparse matrices with the shapes and structure of the paper's workloads.

This module only builds inputs (sparsity patterns and values). It holds none of the
randomized-PCA arithmetic, so both the CPU oracle and the HIP path can consume it.
"""
from .matrices import (  # noqa: F401
    Csr,
    small_decay,
    zipf_rows,
    zipf_lognormal,
    aminer_tfidf,
    zipf_normal,
    planted_blocks,
    ratings_zipf,
    from_dense,
    random_sparse,
    WORKLOADS,
)
