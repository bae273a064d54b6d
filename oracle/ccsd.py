"""Closed-shell CCSD on one fragment Hamiltonian, FP64, plain NumPy.

What the paper fixes
  * The fragment problem (Sec. II.B, Eqs. 10-11): a Hamiltonian on the active
    space with a semi-canonical Fock operator (diagonal, no occupied-virtual
    block because occupied and virtual orbitals are rotated separately, Sec. II.C
    end) and ERIs from DF factors (Eq. 27a).
  * The amplitudes t_ia, t_iajb = t_ij^ab are obtained "using CCSD with the
    fragment Hamiltonian" (Sec. II.B); the paper prints no CCSD equations.
  * The correlation energy (Eq. 7): sum_ijab tau_ij^ab (2 V_iajb - V_ibja) with
    tau = t2 + t1 t1 (the printed minus sign is read as a typo: the t1 t1 term
    is even in T1 and the determinant-space definition below gives +).
  * MP1 amplitudes (Eq. 21) with i_F running over all occupied orbitals give
    the starting guess; the MP2 energy is Eq. 7 evaluated with them and T1 = 0.

CCSD equations used here (published closed-shell form, written with the
T1-similarity-transformed Hamiltonian H~ = exp(-T1) H exp(T1)).  The residual
vector is the projection of exp(-T) H exp(T)|HF> on the singly and doubly
excited determinants:
    R1[i,a]     = <Phi_{i alpha}^{a alpha}| e^{-T} H e^{T} |HF>
    R2[i,j,a,b] = <Phi_{i alpha, j beta}^{a alpha, b beta}| e^{-T} H e^{T} |HF>
The determinant-space module (``brute``) computes the same quantities from
their definition and the tests compare the two at random amplitudes.

Amplitude step: Jacobi, t <- t + R / D with D_i^a = e_i - e_a and
D_ij^ab = e_i + e_j - e_a - e_b, followed by Pulay DIIS on the concatenated
(t1, t2) vector with error = (new - old); the residual norm used for
convergence is ||new - old||_2 over the full t1[o,v] and t2[o,o,v,v] arrays,
taken before extrapolation.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .integrals import eri


# ---------------------------------------------------------------- helpers
def _blocks(nocc: int, n: int):
    return slice(0, nocc), slice(nocc, n)


def _pswap(X: np.ndarray) -> np.ndarray:
    """(ai) <-> (bj) partner of an [i,j,a,b] array."""
    return X.transpose(1, 0, 3, 2)


def denominators(eps_occ: np.ndarray, eps_vir: np.ndarray):
    """D_i^a = e_i - e_a [o,v] and D_ij^ab = e_i + e_j - e_a - e_b [o,o,v,v]."""
    d1 = eps_occ[:, None] - eps_vir[None, :]
    d2 = (eps_occ[:, None, None, None] + eps_occ[None, :, None, None]
          - eps_vir[None, None, :, None] - eps_vir[None, None, None, :])
    return d1, d2


# ---------------------------------------------------------------- energies
def ovov(B: np.ndarray, nocc: int) -> np.ndarray:
    """(ia|jb) as an [i,a,j,b] array (undressed)."""
    o, v = _blocks(nocc, B.shape[1])
    return eri(B[:, o, v], B[:, o, v])


def energy(B: np.ndarray, nocc: int, t1: np.ndarray, t2: np.ndarray) -> float:
    """Eq. 7: sum_ijab (t_ij^ab + t_i^a t_j^b) (2 (ia|jb) - (ib|ja))."""
    g = ovov(B, nocc)
    tau = t2 + np.einsum("ia,jb->ijab", t1, t1)
    return float(np.einsum("ijab,iajb->", tau, 2.0 * g)
                 - np.einsum("ijab,ibja->", tau, g))


def mp2(B: np.ndarray, eps_occ: np.ndarray, eps_vir: np.ndarray):
    """MP1 amplitudes (Eq. 21, i_F = every occupied) and the MP2 energy."""
    nocc = eps_occ.size
    g = ovov(B, nocc)
    _, d2 = denominators(eps_occ, eps_vir)
    t2 = g.transpose(0, 2, 1, 3) / d2
    return t2, energy(B, nocc, np.zeros((nocc, eps_vir.size)), t2)


# ---------------------------------------------------------------- T1 dressing
def t1_transform(nocc: int, n: int, t1: np.ndarray):
    """Matrices of the exp(-T1) ... exp(T1) similarity transformation.

    exp(-T1) a+_p exp(T1) = sum_x a+_x Lm[x,p] and
    exp(-T1) a_q  exp(T1) = sum_y a_y  Rm[y,q] with
    Lm = 1 - T, Rm = 1 + T^T and T[a,i] = t_i^a.
    """
    T = np.zeros((n, n))
    T[nocc:, :nocc] = t1.T
    return np.eye(n) - T, np.eye(n) + T.T


def dress_B(B: np.ndarray, nocc: int, t1: np.ndarray) -> np.ndarray:
    """B~[Q,x,y] = sum_pq Lm[x,p] B[Q,p,q] Rm[y,q]."""
    Lm, Rm = t1_transform(nocc, B.shape[1], t1)
    return np.einsum("xp,Qpq,yq->Qxy", Lm, B, Rm, optimize=True)


def two_electron_fock(B: np.ndarray, nocc: int) -> np.ndarray:
    """G_pq = sum_k [2 (pq|kk) - (pk|kq)] over the occupied k."""
    o = slice(0, nocc)
    J = np.einsum("Qkk->Q", B[:, o, o])
    return (2.0 * np.einsum("Q,Qpq->pq", J, B)
            - np.einsum("Qpk,Qkq->pq", B[:, :, o], B[:, o, :], optimize=True))


def dressed_fock(B: np.ndarray, Bt: np.ndarray, eps: np.ndarray, nocc: int,
                 t1: np.ndarray) -> np.ndarray:
    """Fock matrix of H~.

    The bare one-electron operator is recovered from the semi-canonical Fock
    diagonal, h = diag(eps) - G(B) (Eq. 11 with every occupied orbital of the
    fragment inside the active space), then transformed and re-dressed:
    F~ = Lm h Rm^T + G(B~).
    """
    Lm, Rm = t1_transform(nocc, B.shape[1], t1)
    h = np.diag(eps) - two_electron_fock(B, nocc)
    return Lm @ h @ Rm.T + two_electron_fock(Bt, nocc)


# ---------------------------------------------------------------- residuals
def ladder(Bvv: np.ndarray, t2: np.ndarray, block: int = 8) -> np.ndarray:
    """Particle-particle ladder sum_cd t_ij^cd (ac|bd)~ as an [i,j,a,b] array.

    (ac|bd)~ = sum_Q B~[Q,a,c] B~[Q,b,d] is formed for a few values of a at a
    time, so that no v^4 array is held; the sum itself is the plain one.
    """
    nocc, nvir = t2.shape[0], t2.shape[2]
    R = np.zeros((nocc, nocc, nvir, nvir))
    for a0 in range(0, nvir, block):
        a1 = min(nvir, a0 + block)
        g = eri(Bvv[:, a0:a1, :], Bvv)                     # (ac|bd)~ [a,c,b,d]
        R[:, :, a0:a1, :] = np.einsum("ijcd,acbd->ijab", t2, g, optimize=True)
    return R


def residuals(B: np.ndarray, eps_occ: np.ndarray, eps_vir: np.ndarray,
              t1: np.ndarray, t2: np.ndarray):
    """CCSD residuals R1[i,a], R2[i,j,a,b] (see module docstring)."""
    nocc, nvir = t1.shape
    n = nocc + nvir
    o, v = _blocks(nocc, n)
    eps = np.concatenate([eps_occ, eps_vir])
    Bt = dress_B(B, nocc, t1)
    F = dressed_fock(B, Bt, eps, nocc, t1)
    Boo, Bov, Bvo, Bvv = Bt[:, o, o], Bt[:, o, v], Bt[:, v, o], Bt[:, v, v]

    g_vovo = eri(Bvo, Bvo)      # (ai|bj)~
    g_oooo = eri(Boo, Boo)      # (ki|lj)~
    g_ovov = eri(Bov, Bov)      # (kc|ld)   (the ov block is not dressed)
    g_oovv = eri(Boo, Bvv)      # (ki|ac)~
    g_voov = eri(Bvo, Bov)      # (ai|kc)~
    g_vvov = eri(Bvv, Bov)      # (ad|kc)~
    g_ooov = eri(Boo, Bov)      # (ki|lc)~

    u = 2.0 * t2 - t2.transpose(1, 0, 2, 3)          # u_ij^ab = 2 t_ij^ab - t_ji^ab
    L_ovov = 2.0 * g_ovov - g_ovov.transpose(0, 3, 2, 1)   # L_ldkc = 2(ld|kc) - (lc|kd)

    # singles
    R1 = np.einsum("kicd,adkc->ia", u, g_vvov, optimize=True)
    R1 -= np.einsum("klac,kilc->ia", u, g_ooov, optimize=True)
    R1 += np.einsum("ikac,kc->ia", u, F[o, v])
    R1 += F[v, o].T

    # doubles: bare coupling and particle-particle ladder
    R2 = g_vovo.transpose(1, 3, 0, 2).copy()
    R2 += ladder(Bvv, t2)
    # hole-hole ladder
    Wkl = g_oooo.transpose(0, 2, 1, 3) + np.einsum("ijcd,kcld->klij", t2, g_ovov,
                                                   optimize=True)
    R2 += np.einsum("klab,klij->ijab", t2, Wkl, optimize=True)
    # exchange-type rings
    Cint = g_oovv - 0.5 * np.einsum("liad,kdlc->kiac", t2, g_ovov, optimize=True)
    X = np.einsum("kjbc,kiac->ijab", t2, Cint, optimize=True)
    Y = np.einsum("kibc,kjac->ijab", t2, Cint, optimize=True)
    R2 += -0.5 * (X + _pswap(X)) - (Y + _pswap(Y))
    # coulomb-type rings
    Dint = (2.0 * g_voov - g_oovv.transpose(2, 1, 0, 3)
            + 0.5 * np.einsum("ilad,ldkc->aikc", u, L_ovov, optimize=True))
    Z = np.einsum("jkbc,aikc->ijab", u, Dint, optimize=True)
    R2 += 0.5 * (Z + _pswap(Z))
    # dressed Fock terms
    Fvv = F[v, v] - np.einsum("klbd,ldkc->bc", u, g_ovov, optimize=True)
    Foo = F[o, o] + np.einsum("ljcd,kdlc->kj", u, g_ovov, optimize=True)
    E = (np.einsum("ijac,bc->ijab", t2, Fvv, optimize=True)
         - np.einsum("ikab,kj->ijab", t2, Foo, optimize=True))
    R2 += E + _pswap(E)
    return R1, R2


# ---------------------------------------------------------------- DIIS
class DIIS:
    """Pulay extrapolation on the concatenated amplitude vector."""

    def __init__(self, space: int = 8):
        self.space = space
        self.vecs: list[np.ndarray] = []
        self.errs: list[np.ndarray] = []

    def reset(self):
        self.vecs.clear()
        self.errs.clear()

    def update(self, x: np.ndarray, e: np.ndarray) -> np.ndarray:
        self.vecs.append(x.copy())
        self.errs.append(e.copy())
        if len(self.vecs) > self.space:
            self.vecs.pop(0)
            self.errs.pop(0)
        m = len(self.vecs)
        if m < 2:
            return x
        A = np.zeros((m + 1, m + 1))
        for i in range(m):
            for j in range(i + 1):
                A[i, j] = A[j, i] = float(np.dot(self.errs[i], self.errs[j]))
        A[m, :m] = A[:m, m] = -1.0
        rhs = np.zeros(m + 1)
        rhs[m] = -1.0
        c = np.linalg.solve(A, rhs)[:m]
        return sum(ci * xi for ci, xi in zip(c, self.vecs))


# ---------------------------------------------------------------- driver
@dataclasses.dataclass
class CCSDResult:
    e_mp2: float
    e_ccsd: float
    t1: np.ndarray
    t2: np.ndarray
    n_iter: int
    residual: float
    converged: bool
    history: list


def ccsd(B: np.ndarray, eps_occ: np.ndarray, eps_vir: np.ndarray, *,
         conv_tol: float = 1e-8, max_iter: int = 100, diis_space: int = 8,
         diis_start: int = 2, t1: np.ndarray | None = None,
         t2: np.ndarray | None = None) -> CCSDResult:
    """Iterate the CCSD equations from the MP2 guess (or given amplitudes)."""
    nocc, nvir = eps_occ.size, eps_vir.size
    t2_mp2, e_mp2 = mp2(B, eps_occ, eps_vir)
    if t2 is None:
        t1 = np.zeros((nocc, nvir))
        t2 = t2_mp2
    elif t1 is None:
        t1 = np.zeros((nocc, nvir))
    t1 = np.array(t1, dtype=np.float64)
    t2 = np.array(t2, dtype=np.float64)
    d1, d2 = denominators(eps_occ, eps_vir)
    diis = DIIS(diis_space)
    n1 = t1.size
    history = []
    r = np.inf
    it = 0
    converged = False
    for it in range(1, max_iter + 1):
        R1, R2 = residuals(B, eps_occ, eps_vir, t1, t2)
        t1n = t1 + R1 / d1
        t2n = t2 + R2 / d2
        dx = np.concatenate([(t1n - t1).ravel(), (t2n - t2).ravel()])
        r = float(np.linalg.norm(dx))
        xn = np.concatenate([t1n.ravel(), t2n.ravel()])
        if r <= conv_tol:
            t1, t2 = t1n, t2n
            history.append((it, energy(B, nocc, t1, t2), r))
            converged = True
            break
        if it >= diis_start:
            xn = diis.update(xn, dx)
        t1 = xn[:n1].reshape(nocc, nvir)
        t2 = xn[n1:].reshape(nocc, nocc, nvir, nvir)
        history.append((it, energy(B, nocc, t1, t2), r))
    return CCSDResult(e_mp2, energy(B, nocc, t1, t2), t1, t2, it, r, converged,
                      history)
