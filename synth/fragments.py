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

