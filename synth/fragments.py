"""Seeded synthetic fragments with the structure of an LNO active-space problem.

A fragment problem (paper, Sec. II.B, Eqs. 10-11 and 27) is the semi-canonical
Fock diagonal (occupied energies, then virtual energies) and real
density-fitting factors B[Q, p, q] with (pq|rs) = sum_Q B[Q,p,q] B[Q,r,s].
Orbitals are ordered occupied first.

Recipe (fixed reading; the paper gives no fragment-level data):
  rng = numpy.random.default_rng(seed)            # PCG64
  Z   = rng.standard_normal((naux, n, n))
  B   = 0.1 * exp(-|p-q|/8) * exp(-3 Q / naux) * Z
  B   = (B + B^T_pq) / 2                         # symmetric in p, q
  eps_occ = sort(rng.uniform(-1.2, -0.4, nocc))
  eps_vir = sort(rng.uniform( 0.3,  4.0, nvir))
Draws happen in exactly this order.  The decay in |p-q| mimics locality of the
orbital products and the decay in Q mimics a Cholesky/DF spectrum.
"""
from __future__ import annotations

import dataclasses
import hashlib

import numpy as np

# (nocc, nvir, naux, seed) of the named single-fragment workloads.
CONFIG_SHAPES = {
    "single_small": (4, 20, 72, 0),
    "single_realistic": (16, 160, 528, 1),
    "large": (32, 400, 1300, 4),
}


@dataclasses.dataclass
class Fragment:
    nocc: int
    nvir: int
    naux: int
    B: np.ndarray        # float64 [naux, n, n], occupied first, symmetric in (p, q)
    eps_occ: np.ndarray  # float64 [nocc], ascending
    eps_vir: np.ndarray  # float64 [nvir], ascending
    seed: int | None = None

    @property
    def n(self) -> int:
        return self.nocc + self.nvir

    def sha256(self) -> str:
        h = hashlib.sha256()
        for a in (self.B, self.eps_occ, self.eps_vir):
            h.update(np.ascontiguousarray(a, dtype=np.float64).tobytes())
        return h.hexdigest()


def make_fragment(nocc: int, nvir: int, naux: int, seed: int) -> Fragment:
    """Draw one fragment with the recipe in the module docstring."""
    if nocc <= 0 or nvir <= 0 or naux <= 0:
        raise ValueError("nocc, nvir and naux must be positive")
    n = nocc + nvir
    rng = np.random.default_rng(seed)
    B = rng.standard_normal((naux, n, n))
    p = np.arange(n)
    B *= 0.1 * np.exp(-np.abs(p[:, None] - p[None, :]) / 8.0)[None, :, :]
    B *= np.exp(-3.0 * np.arange(naux) / naux)[:, None, None]
    B = 0.5 * (B + B.transpose(0, 2, 1))
    eps_occ = np.sort(rng.uniform(-1.2, -0.4, nocc))
    eps_vir = np.sort(rng.uniform(0.3, 4.0, nvir))
    return Fragment(nocc, nvir, naux, np.ascontiguousarray(B), eps_occ, eps_vir, seed)


def batch_shapes(nfrag: int = 64, seed: int = 3):
    """Uneven fragment shapes of the batched workload.

    nocc ~ U{6..24}, nvir ~ U{60..220}, naux = 3 (nocc + nvir); fragment f is
    drawn with seed 1000 * seed + f.  Returns a list of (nocc, nvir, naux, seed).
    """
    rng = np.random.default_rng(seed)
    o = rng.integers(6, 25, size=nfrag)
    v = rng.integers(60, 221, size=nfrag)
    return [(int(o[f]), int(v[f]), int(3 * (o[f] + v[f])), 1000 * seed + f)
            for f in range(nfrag)]


def random_amplitudes(nocc: int, nvir: int, seed: int, scale1: float = 5e-3,
                      scale2: float = 1e-2):
    """Seeded amplitudes (t1[o,v], t2[o,o,v,v]) with t2[i,j,a,b] = t2[j,i,b,a].

    rng = default_rng(seed); t1 = scale1 N(0,1) drawn first, then
    Z = scale2 N(0,1) of shape (o,o,v,v) and t2 = (Z + Z^T_(ij)(ab)) / 2.
    """
    rng = np.random.default_rng(seed)
    t1 = scale1 * rng.standard_normal((nocc, nvir))
    z = scale2 * rng.standard_normal((nocc, nocc, nvir, nvir))
    t2 = 0.5 * (z + z.transpose(1, 0, 3, 2))
    return t1, np.ascontiguousarray(t2)


# Fragments of the batched workload (indices into batch_shapes()) that carry
# full oracle CCSD and (T) values: they span nocc 6..24 and nvir 60..214,
# including the largest fragment of the batch.
BATCH_ORACLE_SUBSET = (20, 48, 31, 51, 53, 4, 49, 26)

# (T) at the virtual and auxiliary size of the large workload with few
# occupied orbitals, on seeded amplitudes: (nocc, nvir, naux, fragment seed,
# amplitude seed).
LARGE_TRIPLES_SHAPE = (6, 400, 1300, 4, 44)



@dataclasses.dataclass
class System:
    """A whole (Gamma-point supercell) system upstream of the fragment problems:
    canonical orbital energies, AO-basis DF factors, canonical MO coefficients
    and the LO coefficients of its fragments."""
    nocc: int
    nvir: int
    naux: int
    Lao: np.ndarray      # [naux, n, n] AO-basis DF factors, symmetric in (mu, nu)
    C: np.ndarray        # [n, n] canonical MO coefficients (orthogonal), occupied first
    eps_occ: np.ndarray  # [nocc] ascending
    eps_vir: np.ndarray  # [nvir] ascending
    U_occ: np.ndarray    # [nocc, nlo] LO coefficients on the occupied orbitals
    U_vir: np.ndarray    # [nvir, nlo] LO coefficients on the virtual orbitals (zero for
                         # LOs inside the occupied space)
    fragments: list      # list of lists of LO indices

    @property
    def n(self) -> int:
        return self.nocc + self.nvir

    @property
    def B(self) -> np.ndarray:
        """DF factors in the canonical MO basis."""
        return np.einsum("Pmn,mp,nq->Ppq", self.Lao, self.C, self.C, optimize=True)


def make_system(nocc: int, nvir: int, naux: int, seed: int, nlo_vir: int = 0,
                nfrag: int = 2) -> System:
    """Seeded synthetic system.  rng = default_rng(seed); draws in this order:
    Z ~ N(0,1) (naux, n, n) for L = 0.1 e^{-|mu-nu|/8} e^{-3P/naux} Z symmetrized in
    (mu, nu); M ~ N(0,1) (n, n), C = Q of its QR factorization (columns occupied
    first); eps_occ ~ U[-1.2,-0.4], eps_vir ~ U[0.3,4.0] sorted; R ~ N(0,1)
    (nlo, nlo), O = Q of its QR (nlo = nocc + nlo_vir); S ~ N(0,1) (nvir, nlo_vir),
    Vs = Q of its QR.  LOs: U_occ = O[:nocc], U_vir = Vs O[nocc:] (rows of U_occ are
    orthonormal, so the LOs span the occupied space, Eq. 5; nlo_vir > 0 gives LOs
    that also reach into nlo_vir virtual directions).  Fragments: the LOs dealt
    round-robin into nfrag groups."""
    n = nocc + nvir
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((naux, n, n))
    p = np.arange(n)
    L = Z * (0.1 * np.exp(-np.abs(p[:, None] - p[None, :]) / 8.0))[None]
    L *= np.exp(-3.0 * np.arange(naux) / naux)[:, None, None]
    L = 0.5 * (L + L.transpose(0, 2, 1))
    C, _ = np.linalg.qr(rng.standard_normal((n, n)))
    eps_occ = np.sort(rng.uniform(-1.2, -0.4, nocc))
    eps_vir = np.sort(rng.uniform(0.3, 4.0, nvir))
    nlo = nocc + nlo_vir
    O, _ = np.linalg.qr(rng.standard_normal((nlo, nlo)))
    U_occ = np.ascontiguousarray(O[:nocc])
    if nlo_vir > 0:
        Vs, _ = np.linalg.qr(rng.standard_normal((nvir, nlo_vir)))
        U_vir = Vs @ O[nocc:]
    else:
        U_vir = np.zeros((nvir, nlo))
    frags = [list(range(f, nlo, nfrag)) for f in range(nfrag)]
    return System(nocc, nvir, naux, np.ascontiguousarray(L), C, eps_occ, eps_vir, U_occ,
                  np.ascontiguousarray(U_vir), frags)


def random_orthonormal(n: int, k: int, seed: int) -> np.ndarray:
    """[n, k] matrix with orthonormal columns: Q of the QR factorization of an
    N(0,1) draw (default_rng(seed))."""
    Q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((n, k)))
    return np.ascontiguousarray(Q)
