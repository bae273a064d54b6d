"""Fragment pair energies and their projection onto localized orbitals, FP64,
plain NumPy (test infrastructure; the library never imports this module).

Sec. II.B of the paper writes the correlation energy of each fragment F as a
projection of an occupied-occupied pair matrix onto the fragment's localized
orbitals (LOs) alpha, with U[i, alpha] the coefficient of LO alpha on occupied
orbital i (real orbitals, so U* = U):

  E_c^(F)     = sum_{alpha in F} sum_{i i'} U[i, alpha] E[i, i'] U[i', alpha]     (Eqs. 8, 12)
  E[i, i']    = sum_{j a b} tau_ij^ab (2 (i'a|jb) - (i'b|ja)),  tau = t2 + t1 t1     (Eqs. 9, 13)
  E_T[i, i']  = -1/3 sum_{j k a b c} (4 w_ijk^abc + w_ijk^bca + w_ijk^cab)
                                    (v_i'jk^abc - v_i'jk^cba)                       (Eq. 16)
  w_ijk = W_ijk / sqrt(-Delta_ijk),  v_i'jk = V_i'jk / sqrt(-Delta_i'jk)            (SI Sec. S1)

with W, V and Delta those of the (T) module (SI Sec. S1).  The sum over all
alpha of the projected energies is the trace of E when the LOs span the
occupied space (Eq. 5), which is the canonical correlation energy (Eq. 7 for
CCSD, Eq. 16 at i = i' summed for (T)).

Parity unpinned: the off-diagonal elements (i != i') of E_T.  Their sum with
the diagonal is pinned (trace, projection identity, block structure of
non-interacting fragments), but no closed form or brute-force route checks
the Delta_i'jk scaling of v for i != i' on its own.
"""
from __future__ import annotations

import numpy as np

from .ccsd import ovov
from .triples import TriplesIntegrals, _perm, w_v


def ccsd_pair_matrix(B: np.ndarray, nocc: int, t1: np.ndarray, t2: np.ndarray) -> np.ndarray:
    """E[i, i'] of Eqs. 9 / 13 (tau = t2 + t1 t1, the sign reading of Eq. 7)."""
    g = ovov(B, nocc)                           # (ia|jb) as [i, a, j, b]
    tau = t2 + np.einsum("ia,jb->ijab", t1, t1)
    L = 2.0 * g - g.transpose(0, 3, 2, 1)       # L[i', a, j, b] = 2 (i'a|jb) - (i'b|ja)
    return np.einsum("ijab,kajb->ik", tau, L, optimize=True)


def triples_pair_matrix(B: np.ndarray, eps_occ: np.ndarray, eps_vir: np.ndarray,
                        t1: np.ndarray, t2: np.ndarray) -> np.ndarray:
    """E_T[i, i'] of Eq. 16 with the intermediates of SI Sec. S1, summed over every
    ordered pair (j, k)."""
    nocc = eps_occ.size
    ints = TriplesIntegrals(B, nocc)
    ev = eps_vir
    E = np.zeros((nocc, nocc))
    for j in range(nocc):
        for k in range(nocc):
            Y = []
            Z = []
            for i in range(nocc):
                W, V = w_v(ints, t1, t2, i, j, k)
                delta = (eps_occ[i] + eps_occ[j] + eps_occ[k]
                         - ev[:, None, None] - ev[None, :, None] - ev[None, None, :])
                s = 1.0 / np.sqrt(-delta)
                w = W * s
                v = V * s
                Y.append(4.0 * w + _perm(w, "bca") + _perm(w, "cab"))
                Z.append(v - _perm(v, "cba"))
            for i in range(nocc):
                for ip in range(nocc):
                    E[i, ip] += -np.sum(Y[i] * Z[ip]) / 3.0
    return E


def project(E: np.ndarray, U: np.ndarray) -> np.ndarray:
    """Projected energy of every LO alpha: sum_{i i'} U[i, alpha] E[i, i'] U[i', alpha]
    (the summand of Eqs. 8 / 12 / 15 for one alpha)."""
    return np.einsum("ia,ij,ja->a", U, E, U)
