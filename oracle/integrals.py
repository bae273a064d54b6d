"""Two-electron integrals of the fragment Hamiltonian from DF factors.

Eq. 27a of the paper writes each ERI of the local Hamiltonian as a sum over
auxiliary functions of products of three-index factors.  With real orbitals and
the momentum sum folded into the auxiliary index this is
    (pq|rs) = sum_Q B[Q,p,q] B[Q,r,s]
in chemists' (11|22) notation (Eq. 2).  Occupied orbitals come first.
"""
from __future__ import annotations

import numpy as np


def eri(B1: np.ndarray, B2: np.ndarray) -> np.ndarray:
    """(pq|rs) = sum_Q B1[Q,p,q] B2[Q,r,s] for two (possibly different) blocks."""
    return np.einsum("Qpq,Qrs->pqrs", B1, B2, optimize=True)


def full_eri(B: np.ndarray) -> np.ndarray:
    """The whole (pq|rs) tensor (small cases only)."""
    return eri(B, B)


def slices(nocc: int, n: int):
    return slice(0, nocc), slice(nocc, n)
