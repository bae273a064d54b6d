"""Perturbative triples (T) on one fragment, FP64, plain NumPy.

Follows SI Sec. S1 (intermediates after Nagy and Kallay) and the pair energy of
Eq. 16 taken at i = i' and summed over i, which is the canonical (T) energy of
the fragment (the full-active-space limit stated after Eq. 16):

  W_ijk^abc = P_ijk^abc { sum_d (bd|ai) t_kj^cd - sum_l (ck|jl) t_il^ab }
  V_ijk^abc = W_ijk^abc + (ai|bj) t_k^c + (ai|ck) t_j^b + (bj|ck) t_i^a
  Delta     = e_i + e_j + e_k - e_a - e_b - e_c
  P_ijk^abc { X } = X_ijk^abc + X_ikj^acb + X_jik^bac + X_jki^bca + X_kij^cab + X_kji^cba

"1/2 P {V_aibj t_kc}" is read as its three distinct terms (the six
permutations produce each twice).  With w = W / sqrt(-Delta) and
v = V / sqrt(-Delta) at i = i', Eq. 16 summed over i gives

  E_(T) = 1/3 sum_ijk sum_abc (4 W^abc + W^bca + W^cab)(V^abc - V^cba) / Delta

where W^bca denotes W_ijk with its virtual labels read in the order (b, c, a).

Two loops are provided:
  e_triples_full        every ordered (i, j, k), the expression above;
  e_triples_restricted  i <= j <= k only, with the integrand averaged over the
                        six simultaneous relabellings of (ijk, abc), which is
                        V^abc (4 W^abc + W^bca + W^cab - 2 W^acb - 2 W^bac
                        - 2 W^cba) / (3 Delta), weighted 6 / 3 / 1 for three /
                        two / one distinct occupied labels.
"""
from __future__ import annotations

import numpy as np

from .integrals import eri


def _perm(X: np.ndarray, src: str) -> np.ndarray:
    """Array Y[a,b,c] = X[<src order>], e.g. src='bca' gives Y[a,b,c] = X[b,c,a]."""
    return np.einsum(f"{src}->abc", X)


class TriplesIntegrals:
    """The integral blocks that enter W and V."""

    def __init__(self, B: np.ndarray, nocc: int):
        n = B.shape[1]
        o, v = slice(0, nocc), slice(nocc, n)
        self.vvvo = eri(B[:, v, v], B[:, v, o])   # (bd|ai) [b,d,a,i]
        self.vooo = eri(B[:, v, o], B[:, o, o])   # (ck|jl) [c,k,j,l]
        self.vovo = eri(B[:, v, o], B[:, v, o])   # (ai|bj) [a,i,b,j]


def _x(ints: TriplesIntegrals, t2: np.ndarray, i: int, j: int, k: int) -> np.ndarray:
    """X_ijk[a,b,c] = sum_d (bd|ai) t_kj^cd - sum_l (ck|jl) t_il^ab."""
    part = np.einsum("bda,cd->abc", ints.vvvo[:, :, :, i], t2[k, j], optimize=True)
    hole = np.einsum("cl,lab->abc", ints.vooo[:, k, j, :], t2[i], optimize=True)
    return part - hole


def w_v(ints: TriplesIntegrals, t1: np.ndarray, t2: np.ndarray, i: int, j: int, k: int):
    """W_ijk[a,b,c] and V_ijk[a,b,c]."""
    W = (_x(ints, t2, i, j, k)
         + _perm(_x(ints, t2, i, k, j), "acb")
         + _perm(_x(ints, t2, j, i, k), "bac")
         + _perm(_x(ints, t2, j, k, i), "bca")
         + _perm(_x(ints, t2, k, i, j), "cab")
         + _perm(_x(ints, t2, k, j, i), "cba"))
    g = ints.vovo
    V = (W + np.einsum("ab,c->abc", g[:, i, :, j], t1[k])
         + np.einsum("ac,b->abc", g[:, i, :, k], t1[j])
         + np.einsum("bc,a->abc", g[:, j, :, k], t1[i]))
    return W, V


def _delta(eps_occ, eps_vir, i, j, k):
    ev = eps_vir
    return (eps_occ[i] + eps_occ[j] + eps_occ[k]
            - ev[:, None, None] - ev[None, :, None] - ev[None, None, :])


def e_triples_full(B, eps_occ, eps_vir, t1, t2) -> float:
    nocc = eps_occ.size
    ints = TriplesIntegrals(B, nocc)
    e = 0.0
    for i in range(nocc):
        for j in range(nocc):
            for k in range(nocc):
                W, V = w_v(ints, t1, t2, i, j, k)
                Y = 4.0 * W + _perm(W, "bca") + _perm(W, "cab")
                Z = V - _perm(V, "cba")
                e += float(np.sum(Y * Z / _delta(eps_occ, eps_vir, i, j, k))) / 3.0
    return e


def e_triples_restricted(B, eps_occ, eps_vir, t1, t2) -> float:
    nocc = eps_occ.size
    ints = TriplesIntegrals(B, nocc)
    e = 0.0
    for i in range(nocc):
        for j in range(i, nocc):
            for k in range(j, nocc):
                m = 6.0 if (i < j < k) else (1.0 if i == k else 3.0)
                W, V = w_v(ints, t1, t2, i, j, k)
                Z = (4.0 * W + _perm(W, "bca") + _perm(W, "cab")
                     - 2.0 * _perm(W, "acb") - 2.0 * _perm(W, "bac") - 2.0 * _perm(W, "cba"))
                e += m * float(np.sum(V * Z / _delta(eps_occ, eps_vir, i, j, k))) / 3.0
    return e
