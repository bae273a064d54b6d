"""Seeded synthetic fragment inputs shared by the oracle and the GPU path.

This package draws random numbers and arranges them into the fragment-problem
inputs (three-index DF factors and semi-canonical orbital energies).  It holds
none of the coupled-cluster arithmetic.
"""
from .fragments import (
    Fragment,
    make_fragment,
    batch_shapes,
    CONFIG_SHAPES,
    random_amplitudes,
    System,
    make_system,
    BATCH_ORACLE_SUBSET,
    LARGE_TRIPLES_SHAPE,
    random_orthonormal,
)

__all__ = ["Fragment", "make_fragment", "batch_shapes", "CONFIG_SHAPES", "random_amplitudes", "System", "make_system",
           "BATCH_ORACLE_SUBSET", "LARGE_TRIPLES_SHAPE",
           "random_orthonormal"]
