"""Determinant-space definitions used to pin the CCSD and (T) oracles.

Everything here is written from the definitions of second quantization, for
tiny active spaces only.  The Hamiltonian is Eq. 2 restricted to the fragment
(Eq. 10): H = sum_pq h_pq E_pq + 1/2 sum_pqrs (pq|rs) (E_pq E_rs - delta_qr E_ps)
with E_pq = sum_sigma a+_{p sigma} a_{q sigma}.  The one-electron part is
recovered from the semi-canonical Fock diagonal: h = diag(eps) - G with
G_pq = sum_k [2 (pq|kk) - (pk|kq)] (k occupied), i.e. f = h + G (Eq. 11).

Spin orbitals are numbered p (alpha) and p + n (beta); a determinant is a bit
string and a_s carries the Jordan-Wigner sign (-1)^(occupied orbitals below s).
The space is the N = 2 nocc, S_z = 0 sector, which every operator used here
(spin-free excitations) leaves invariant.

  cc_residuals   <mu| e^{-T} H e^{T} |HF>, mu = single (alpha) and double
                 (alpha-beta) excitations, plus E_corr = <HF|H e^T|HF> - E_HF,
                 at any closed-shell T1 = sum t_i^a E_ai,
                 T2 = 1/2 sum t_ij^ab E_ai E_bj.
  fci_energy     lowest eigenvalue of H in the sector (exact for 2 electrons).
  triples_energy the (T) correction as a sum over triply excited determinants
                 mu3 of c (c + d) / D with c = <mu3|H T2|HF>,
                 d = <mu3|H T1|HF> and D the orbital-energy difference (the
                 fourth-order triples term plus the fifth-order singles-triples
                 term of Raghavachari et al., Chem. Phys. Lett. 157, 479).
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp


def _parity_below(det: int, s: int) -> int:
    return -1 if bin(det & ((1 << s) - 1)).count("1") & 1 else 1


class Sector:
    """Determinants with nocc alpha and nocc beta electrons in n orbitals."""

    def __init__(self, n: int, nocc: int):
        self.n, self.nocc = n, nocc
        strings = [sum(1 << p for p in occ)
                   for occ in itertools.combinations(range(n), nocc)]
        self.dets = [a | (b << n) for a in strings for b in strings]
        self.index = {d: k for k, d in enumerate(self.dets)}
        self.dim = len(self.dets)
        self.hf = sum(1 << p for p in range(nocc)) | (sum(1 << p for p in range(nocc)) << n)
        self._E = {}

    def e_spin(self, p: int, q: int, sigma: int) -> sp.csr_matrix:
        """Matrix of a+_{p sigma} a_{q sigma} on the sector."""
        key = (p, q, sigma)
        if key in self._E:
            return self._E[key]
        ps, qs = p + sigma * self.n, q + sigma * self.n
        rows, cols, vals = [], [], []
        for col, d in enumerate(self.dets):
            if not (d >> qs) & 1:
                continue
            s1 = _parity_below(d, qs)
            d1 = d ^ (1 << qs)
            if (d1 >> ps) & 1:
                continue
            s2 = _parity_below(d1, ps)
            rows.append(self.index[d1 | (1 << ps)])
            cols.append(col)
            vals.append(float(s1 * s2))
        M = sp.csr_matrix((vals, (rows, cols)), shape=(self.dim, self.dim))
        self._E[key] = M
        return M

    def e(self, p: int, q: int) -> sp.csr_matrix:
        return self.e_spin(p, q, 0) + self.e_spin(p, q, 1)

    def unit(self, det: int) -> np.ndarray:
        x = np.zeros(self.dim)
        x[self.index[det]] = 1.0
        return x

    def hf_vector(self) -> np.ndarray:
        return self.unit(self.hf)

    def excitation_level(self) -> np.ndarray:
        hf = self.hf
        return np.array([bin(d & ~hf).count("1") for d in self.dets])


def one_electron(B: np.ndarray, eps: np.ndarray, nocc: int) -> np.ndarray:
    g = np.einsum("Qpq,Qrs->pqrs", B, B)
    o = range(nocc)
    G = sum(2.0 * g[:, :, k, k] - g[:, k, k, :] for k in o)
    return np.diag(eps) - G, g


def apply_h(sec: Sector, h: np.ndarray, g: np.ndarray, psi: np.ndarray) -> np.ndarray:
    n = sec.n
    phi = np.array([[sec.e(r, s) @ psi for s in range(n)] for r in range(n)])
    out = np.einsum("pq,pqx->x", h, phi)
    chi = np.einsum("pqrs,rsx->pqx", g, phi)
    for p in range(n):
        for q in range(n):
            out += 0.5 * (sec.e(p, q) @ chi[p, q])
    k = np.einsum("pqqs->ps", g)
    out -= 0.5 * np.einsum("ps,psx->x", k, phi)
    return out


def apply_t(sec: Sector, t1: np.ndarray, t2: np.ndarray, psi: np.ndarray) -> np.ndarray:
    nocc, nvir = t1.shape
    out = np.zeros_like(psi)
    for i in range(nocc):
        for a in range(nvir):
            out += t1[i, a] * (sec.e(nocc + a, i) @ psi)
    phi = np.array([[sec.e(nocc + b, j) @ psi for j in range(nocc)] for b in range(nvir)])
    kappa = np.einsum("ijab,bjx->aix", t2, phi)
    for i in range(nocc):
        for a in range(nvir):
            out += 0.5 * (sec.e(nocc + a, i) @ kappa[a, i])
    return out


def apply_exp_t(sec, t1, t2, psi, sign=1.0):
    out = psi.copy()
    term = psi.copy()
    for k in range(1, 4 * sec.nocc + 3):
        term = sign * apply_t(sec, t1, t2, term) / k
        if not np.any(term):
            break
        out += term
    return out


def cc_residuals(B, eps_occ, eps_vir, t1, t2):
    """Projections of e^{-T} H e^{T}|HF> and the correlation energy."""
    nocc, nvir = t1.shape
    n = nocc + nvir
    eps = np.concatenate([eps_occ, eps_vir])
    h, g = one_electron(B, eps, nocc)
    sec = Sector(n, nocc)
    hf = sec.hf_vector()
    psi = apply_exp_t(sec, t1, t2, hf)
    hpsi = apply_h(sec, h, g, psi)
    hbar = apply_exp_t(sec, t1, t2, hpsi, sign=-1.0)
    e_hf = float(hf @ apply_h(sec, h, g, hf))
    e_corr = float(hf @ hpsi) - e_hf
    R1 = np.zeros((nocc, nvir))
    R2 = np.zeros((nocc, nocc, nvir, nvir))
    for i in range(nocc):
        for a in range(nvir):
            mu = sec.e_spin(nocc + a, i, 0) @ hf
            R1[i, a] = mu @ hbar
            for j in range(nocc):
                for b in range(nvir):
                    mu2 = sec.e_spin(nocc + a, i, 0) @ (sec.e_spin(nocc + b, j, 1) @ hf)
                    R2[i, j, a, b] = mu2 @ hbar
    return R1, R2, e_corr


def fci_energy(B, eps_occ, eps_vir):
    """Lowest eigenvalue of H in the sector and E_HF, as (E_FCI, E_HF)."""
    nocc = eps_occ.size
    n = nocc + eps_vir.size
    eps = np.concatenate([eps_occ, eps_vir])
    h, g = one_electron(B, eps, nocc)
    sec = Sector(n, nocc)
    H = np.array([apply_h(sec, h, g, sec.unit(d)) for d in sec.dets]).T
    w = np.linalg.eigvalsh(0.5 * (H + H.T))
    hf = sec.hf_vector()
    return float(w[0]), float(hf @ H @ hf)


def triples_energy(B, eps_occ, eps_vir, t1, t2):
    """(T) as a sum over triply excited determinants (see module docstring)."""
    nocc, nvir = t1.shape
    n = nocc + nvir
    eps = np.concatenate([eps_occ, eps_vir])
    h, g = one_electron(B, eps, nocc)
    sec = Sector(n, nocc)
    hf = sec.hf_vector()
    zero1 = np.zeros_like(t1)
    zero2 = np.zeros_like(t2)
    c = apply_h(sec, h, g, apply_t(sec, zero1, t2, hf))
    d = apply_h(sec, h, g, apply_t(sec, t1, zero2, hf))
    level = sec.excitation_level()
    e = 0.0
    for k, det in enumerate(sec.dets):
        if level[k] != 3:
            continue
        holes = [s for s in range(2 * n) if (sec.hf >> s) & 1 and not (det >> s) & 1]
        parts = [s for s in range(2 * n) if (det >> s) & 1 and not (sec.hf >> s) & 1]
        D = sum(eps[s % n] for s in holes) - sum(eps[s % n] for s in parts)
        e += c[k] * (c[k] + d[k]) / D
    return float(e)
