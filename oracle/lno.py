"""Local active spaces of LNO-CC (Sec. II.C-E), FP64, plain NumPy (test
infrastructure; the library never imports this module).

For one fragment F with LO coefficients U_occ [N_occ, n_F] on the canonical
occupied orbitals (and, for LOs that reach into the virtual space, U_vir
[N_vir, n_F]):

  1. Internal / external split (Eqs. 18-19): the left singular vectors of U_occ
     with non-zero singular values span the internal occupied space, the rest
     the external one.  They are the eigenvectors of U_occ U_occ^T with non-zero
     / zero eigenvalues.  Same for U_vir (no internal virtuals without it).
  2. Semi-canonical internal orbitals: the Fock matrix (diagonal eps in the
     canonical basis) is diagonalized inside the internal space, which fixes
     f_{i_F i_F} of Eq. 21.
  3. MP1 amplitudes with one internal occupied index (Eqs. 21-23):
     t[k, a, j, b] = (k a|j b) / (f_k + e_j - e_a - e_b), (k a|j b) = sum_P
     (sum_i W[i, k] L[P, i, a]) L[P, j, b] with W the internal orbitals.
  4. Densities with one internal occupied index (Eq. 20) or, the CBNO variant,
     with internal-only pair indices (Eq. 28).
  5. Diagonalization inside the external spaces (Eqs. 24-25) and selection by
     |lambda| >= eta (Eq. 26); the active space is the internal orbitals plus
     the selected LNOs, semi-canonicalized (occupied and virtual separately).
The local Hamiltonian's DF factors follow from the AO-basis factors (Eq. 27b),
and the MP2 composite correction is Eq. 17.
"""
from __future__ import annotations

import numpy as np

SVD_TOL = 1e-10


def split_space(U: np.ndarray | None, n: int):
    """(internal, external) orthonormal bases of R^n from LO coefficients U [n, m]
    (Eqs. 18-19: the left singular vectors with non-zero / zero singular values)."""
    if U is None or U.shape[1] == 0:
        return np.zeros((n, 0)), np.eye(n)
    w, V = np.linalg.eigh(U @ U.T)
    keep = w > SVD_TOL * max(1.0, w.max())
    return V[:, keep], V[:, ~keep]


def semicanonical(Wsub: np.ndarray, eps: np.ndarray):
    """Rotate the orbitals Wsub [n, m] so that the Fock matrix diag(eps) is diagonal
    inside their span; returns (rotated orbitals, their orbital energies)."""
    if Wsub.shape[1] == 0:
        return Wsub, np.zeros(0)
    e, R = np.linalg.eigh(Wsub.T @ np.diag(eps) @ Wsub)
    return Wsub @ R, e


def mp1_one_internal(Lov: np.ndarray, eps_occ, eps_vir, Wint, f_int) -> np.ndarray:
    """t[k, a, j, b] of Eq. 21 with k internal (orbitals Wint, energies f_int)."""
    Lk = np.einsum("ik,Pia->Pka", Wint, Lov)
    V = np.einsum("Pka,Pjb->kajb", Lk, Lov, optimize=True)
    D = (f_int[:, None, None, None] + eps_occ[None, None, :, None]
         - eps_vir[None, :, None, None] - eps_vir[None, None, None, :])
    return V / D


def lno_densities(t: np.ndarray):
    """Eq. 20 from t[k, a, j, b] (k internal):
    D_ij = 2 sum_{k a b} t_{i a k b} (2 t_{j a k b} - t_{j b k a}) with t_{iakb} = t[k, b, i, a];
    D_ab = sum_{k j c} 2 (t_{kajc} t_{kbjc} + t_{kcja} t_{kcjb}) - (t_{kcja} t_{kbjc} + t_{kajc} t_{kcjb})."""
    tt = t.transpose(0, 3, 2, 1)               # tt[k, b, i, a] = t_{iakb}
    Dij = 2.0 * (2.0 * np.einsum("kbia,kbja->ij", tt, tt, optimize=True)
                 - np.einsum("kbia,kajb->ij", tt, tt, optimize=True))
    Dab = (2.0 * (np.einsum("kajc,kbjc->ab", t, t, optimize=True)
                  + np.einsum("kcja,kcjb->ab", t, t, optimize=True))
           - (np.einsum("kcja,kbjc->ab", t, t, optimize=True)
              + np.einsum("kajc,kcjb->ab", t, t, optimize=True)))
    return Dij, Dab


def cbno_densities(Lov: np.ndarray, eps_occ, eps_vir, Wo, fo, Wv, fv):
    """Eq. 28: D_ij = 2 sum_{a_F b_F} sum_k t_{i a_F k b_F} (2 t_{j a_F k b_F} - t_{j b_F k a_F})
    (internal virtuals Wv, energies fv; the first factor read with internal
    virtuals as the sum says) and D_ab = 2 sum_{i_F j_F} sum_c t_{i_F a j_F c}
    (2 t_{i_F b j_F c} - t_{i_F c j_F b}) (internal occupied Wo, energies fo)."""
    no, nv = eps_occ.size, eps_vir.size
    Dij = np.zeros((no, no))
    Dab = np.zeros((nv, nv))
    if Wv.shape[1] > 0:
        Lv = np.einsum("Pia,aA->PiA", Lov, Wv)
        V = np.einsum("PiA,PkB->iAkB", Lv, Lv, optimize=True)
        D = (eps_occ[:, None, None, None] + eps_occ[None, None, :, None]
             - fv[None, :, None, None] - fv[None, None, None, :])
        t = V / D                                   # t[i, A, k, B]
        Dij = 2.0 * (2.0 * np.einsum("iAkB,jAkB->ij", t, t, optimize=True)
                     - np.einsum("iAkB,jBkA->ij", t, t, optimize=True))
    if Wo.shape[1] > 0:
        Lo = np.einsum("iI,Pia->PIa", Wo, Lov)
        V = np.einsum("PIa,PJc->IaJc", Lo, Lo, optimize=True)
        D = (fo[:, None, None, None] + fo[None, None, :, None]
             - eps_vir[None, :, None, None] - eps_vir[None, None, None, :])
        t = V / D                                   # t[I, a, J, c]
        Dab = 2.0 * (2.0 * np.einsum("IaJc,IbJc->ab", t, t, optimize=True)
                     - np.einsum("IaJc,IcJb->ab", t, t, optimize=True))
    return Dij, Dab


def select(D: np.ndarray, Wext: np.ndarray, eta: float):
    """Eqs. 24-26: diagonalize D inside the external space; keep |lambda| >= eta.
    Returns (selected LNO coefficients [n, m], all eigenvalues, descending |lambda|)."""
    if Wext.shape[1] == 0:
        return Wext, np.zeros(0)
    lam, X = np.linalg.eigh(Wext.T @ D @ Wext)
    order = np.argsort(-np.abs(lam), kind="stable")
    lam, X = lam[order], X[:, order]
    keep = np.abs(lam) >= eta
    return Wext @ X[:, keep], lam


def active_space(Lov, eps_occ, eps_vir, U_occ, U_vir, eta_occ, eta_vir, cbno=False):
    """Active occupied / virtual orbitals (coefficients on the canonical ones,
    semi-canonical) and their orbital energies for one fragment."""
    no, nv = eps_occ.size, eps_vir.size
    Wo, Wo_ext = split_space(U_occ, no)
    Wv, Wv_ext = split_space(U_vir, nv)
    Wo, fo = semicanonical(Wo, eps_occ)
    Wv, fv = semicanonical(Wv, eps_vir)
    if cbno:
        Dij, Dab = cbno_densities(Lov, eps_occ, eps_vir, Wo, fo, Wv, fv)
    else:
        Dij, Dab = lno_densities(mp1_one_internal(Lov, eps_occ, eps_vir, Wo, fo))
    Xo, lam_o = select(Dij, Wo_ext, eta_occ)
    Xv, lam_v = select(Dab, Wv_ext, eta_vir)
    Co, eo = semicanonical(np.hstack([Wo, Xo]), eps_occ)
    Cv, ev = semicanonical(np.hstack([Wv, Xv]), eps_vir)
    return Co, eo, Cv, ev, lam_o, lam_v


def df_transform(Lao: np.ndarray, C: np.ndarray) -> np.ndarray:
    """Eq. 27b: B[P, p, q] = sum_{mu nu} L[P, mu, nu] C[mu, p] C[nu, q]."""
    return np.einsum("Pmn,mp,nq->Ppq", Lao, C, C, optimize=True)


def mp2_composite(e_mp2_full: float, e_mp2_fragments) -> float:
    """Eq. 17: the full-system MP2 energy minus the sum of the fragment MP2 energies."""
    return e_mp2_full - float(np.sum(e_mp2_fragments))
