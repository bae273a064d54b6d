"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each check compares the oracle with something other than itself:
  * the determinant-space definition of the CCSD residual and of (T)
    (second quantization from scratch, tiny active spaces, random amplitudes),
  * exact diagonalization for two electrons (CCSD is exact there and the
    triples correction has no triply excited determinant to act on),
  * closed forms: the MP1 amplitudes of Eq. 21 and the MP2 energy of Eq. 7,
  * invariants: 8-fold ERI symmetry of real DF factors (Eq. 27a), size
    extensivity for non-interacting fragments, relabelling of occupied and
    virtual orbitals, B = 0.
"""
import numpy as np
import pytest

from oracle import brute, ccsd as cc, integrals, triples as tr
from synth import make_fragment


def _random_amplitudes(o, v, seed, scale=0.1):
    rng = np.random.default_rng(seed)
    t1 = scale * rng.standard_normal((o, v))
    t2 = scale * rng.standard_normal((o, o, v, v))
    return t1, t2 + t2.transpose(1, 0, 3, 2)


@pytest.mark.parametrize("o,v,X,seed", [(1, 4, 10, 0), (2, 3, 12, 1), (2, 4, 16, 2), (3, 4, 18, 3)])
def test_residual_equals_determinant_projection(o, v, X, seed):
    f = make_fragment(o, v, X, seed)
    B = 3.0 * f.B   # stronger coupling so that every term is visible
    t1, t2 = _random_amplitudes(o, v, 100 + seed)
    R1b, R2b, eb = brute.cc_residuals(B, f.eps_occ, f.eps_vir, t1, t2)
    R1, R2 = cc.residuals(B, f.eps_occ, f.eps_vir, t1, t2)
    assert np.abs(R1b).max() > 1e-2 and np.abs(R2b).max() > 1e-2
    np.testing.assert_allclose(R1, R1b, atol=1e-12, rtol=0)
    np.testing.assert_allclose(R2, R2b, atol=1e-12, rtol=0)
    assert abs(cc.energy(B, o, t1, t2) - eb) < 1e-12


@pytest.mark.parametrize("o,v,X,seed", [(2, 3, 12, 1), (2, 4, 16, 2), (3, 4, 18, 3)])
def test_triples_equals_determinant_sum(o, v, X, seed):
    f = make_fragment(o, v, X, seed)
    B = 3.0 * f.B
    t1, t2 = _random_amplitudes(o, v, 200 + seed)
    eb = brute.triples_energy(B, f.eps_occ, f.eps_vir, t1, t2)
    assert abs(eb) > 1e-3
    ef = tr.e_triples_full(B, f.eps_occ, f.eps_vir, t1, t2)
    er = tr.e_triples_restricted(B, f.eps_occ, f.eps_vir, t1, t2)
    assert abs(ef - eb) < 1e-12 * max(1.0, abs(eb))
    assert abs(er - eb) < 1e-12 * max(1.0, abs(eb))


@pytest.mark.parametrize("v,X,seed", [(5, 12, 0), (7, 20, 1), (9, 24, 2)])
def test_two_electron_ccsd_is_fci(v, X, seed):
    f = make_fragment(1, v, X, seed)
    B = 4.0 * f.B
    r = cc.ccsd(B, f.eps_occ, f.eps_vir, conv_tol=1e-11)
    assert r.converged
    e_fci, e_hf = brute.fci_energy(B, f.eps_occ, f.eps_vir)
    assert abs(r.e_ccsd - (e_fci - e_hf)) < 1e-10
    # no triples for two electrons, for the converged and for arbitrary amplitudes
    assert abs(tr.e_triples_full(B, f.eps_occ, f.eps_vir, r.t1, r.t2)) < 1e-14
    t1, t2 = _random_amplitudes(1, v, seed)
    assert abs(tr.e_triples_full(B, f.eps_occ, f.eps_vir, t1, t2)) < 1e-14


def test_first_iteration_is_mp2():
    f = make_fragment(4, 20, 72, 0)
    o, v = 4, 20
    g = integrals.eri(f.B[:, :o, o:], f.B[:, :o, o:])          # (ia|jb)
    d = (f.eps_occ[:, None, None, None] + f.eps_occ[None, None, :, None]
         - f.eps_vir[None, :, None, None] - f.eps_vir[None, None, None, :])
    e_closed = float(np.sum(g * (2 * g - g.transpose(0, 3, 2, 1)) / d))   # closed form
    t2_mp2, e_mp2 = cc.mp2(f.B, f.eps_occ, f.eps_vir)
    assert abs(e_mp2 - e_closed) < 1e-14 * abs(e_closed)
    # one Jacobi step from T = 0: no singles (f_ia = 0), doubles = MP1 (Eq. 21)
    R1, R2 = cc.residuals(f.B, f.eps_occ, f.eps_vir, np.zeros((o, v)), np.zeros((o, o, v, v)))
    d1, d2 = cc.denominators(f.eps_occ, f.eps_vir)
    assert np.abs(R1).max() < 1e-15
    np.testing.assert_allclose(R2 / d2, t2_mp2, rtol=1e-13, atol=1e-16)
    assert abs(cc.energy(f.B, o, np.zeros((o, v)), R2 / d2) - e_closed) < 1e-14 * abs(e_closed)


def test_eri_eightfold_symmetry_and_psd():
    f = make_fragment(3, 7, 25, 5)
    g = integrals.full_eri(f.B)
    for perm in ["qprs", "pqsr", "rspq", "qpsr", "srqp", "rsqp", "srpq"]:
        np.testing.assert_allclose(np.einsum(f"pqrs->{perm}", g), g, atol=1e-15, rtol=0)
    n = f.n
    w = np.linalg.eigvalsh(g.reshape(n * n, n * n))
    assert w.min() > -1e-14


def _composite(fa, fb):
    oa, va, oA = fa.nocc, fa.nvir, fb.nocc
    vb = fb.nvir
    o, v = oa + oA, va + vb
    X = fa.naux + fb.naux
    B = np.zeros((X, o + v, o + v))
    ia = np.r_[0:oa, o:o + va]
    ib = np.r_[oa:o, o + va:o + v]
    B[np.ix_(range(fa.naux), ia, ia)] = fa.B
    B[np.ix_(range(fa.naux, X), ib, ib)] = fb.B
    return B, np.r_[fa.eps_occ, fb.eps_occ], np.r_[fa.eps_vir, fb.eps_vir]


def test_size_extensivity():
    fa = make_fragment(2, 5, 14, 11)
    fb = make_fragment(2, 4, 10, 12)
    fa.B *= 3.0
    fb.B *= 3.0
    B, eo, ev = _composite(fa, fb)
    rab = cc.ccsd(B, eo, ev, conv_tol=1e-11)
    ra = cc.ccsd(fa.B, fa.eps_occ, fa.eps_vir, conv_tol=1e-11)
    rb = cc.ccsd(fb.B, fb.eps_occ, fb.eps_vir, conv_tol=1e-11)
    assert abs(rab.e_ccsd - ra.e_ccsd - rb.e_ccsd) < 1e-10
    tab = tr.e_triples_restricted(B, eo, ev, rab.t1, rab.t2)
    ta = tr.e_triples_restricted(fa.B, fa.eps_occ, fa.eps_vir, ra.t1, ra.t2)
    tb = tr.e_triples_restricted(fb.B, fb.eps_occ, fb.eps_vir, rb.t1, rb.t2)
    assert abs(ta) > 1e-6
    assert abs(tab - ta - tb) < 1e-10


def test_label_permutation_invariance():
    f = make_fragment(3, 6, 20, 7)
    o, v = 3, 6
    r = cc.ccsd(f.B, f.eps_occ, f.eps_vir, conv_tol=1e-11)
    et = tr.e_triples_full(f.B, f.eps_occ, f.eps_vir, r.t1, r.t2)
    po = np.array([2, 0, 1])
    pv = np.array([4, 1, 5, 0, 3, 2])
    perm = np.r_[po, o + pv]
    Bp = f.B[:, perm][:, :, perm]
    rp = cc.ccsd(Bp, f.eps_occ[po], f.eps_vir[pv], conv_tol=1e-11)
    assert abs(rp.e_ccsd - r.e_ccsd) < 1e-11
    np.testing.assert_allclose(rp.t2, r.t2[np.ix_(po, po, pv, pv)], atol=1e-9)
    etp = tr.e_triples_full(Bp, f.eps_occ[po], f.eps_vir[pv], rp.t1, rp.t2)
    assert abs(etp - et) < 1e-12


def test_zero_interaction():
    f = make_fragment(2, 5, 9, 3)
    B = np.zeros_like(f.B)
    r = cc.ccsd(B, f.eps_occ, f.eps_vir, conv_tol=1e-12)
    assert r.e_mp2 == 0.0 and r.e_ccsd == 0.0
    assert tr.e_triples_full(B, f.eps_occ, f.eps_vir, r.t1, r.t2) == 0.0


def test_generator_is_deterministic_and_symmetric():
    a = make_fragment(4, 20, 72, 0)
    b = make_fragment(4, 20, 72, 0)
    assert a.sha256() == b.sha256()
    assert np.array_equal(a.B, a.B.transpose(0, 2, 1))
    assert a.eps_occ.max() < a.eps_vir.min()
    assert make_fragment(4, 20, 72, 1).sha256() != a.sha256()


def test_pins_catch_planted_mistakes(monkeypatch):
    """Plausible slips in the oracle (a dropped symmetrizer, a transposed
    exchange partner) must break the determinant-space pin."""
    f = make_fragment(2, 3, 12, 1)
    B = 3.0 * f.B
    t1, t2 = _random_amplitudes(2, 3, 9)
    R1b, R2b, _ = brute.cc_residuals(B, f.eps_occ, f.eps_vir, t1, t2)
    with monkeypatch.context() as m:
        m.setattr(cc, "_pswap", lambda X: X)                # (ai)<->(bj) partner dropped
        _, R2 = cc.residuals(B, f.eps_occ, f.eps_vir, t1, t2)
        assert np.abs(R2 - R2b).max() > 1e-3
    with monkeypatch.context() as m:
        m.setattr(cc, "_pswap", lambda X: X.transpose(1, 0, 2, 3))   # wrong partner
        _, R2 = cc.residuals(B, f.eps_occ, f.eps_vir, t1, t2)
        assert np.abs(R2 - R2b).max() > 1e-3
    with monkeypatch.context() as m:
        m.setattr(tr, "_perm", lambda X, src: X)            # permutations of P_ijk^abc dropped
        eb = brute.triples_energy(B, f.eps_occ, f.eps_vir, t1, t2)
        assert abs(tr.e_triples_full(B, f.eps_occ, f.eps_vir, t1, t2) - eb) > 1e-4


# ------------------------------------------------------------ pair energies
from oracle import pairs as opr  # noqa: E402


def _separable_union(sA, sB, scale=3.0):
    """Two non-interacting fragments as one: block-diagonal DF factors over
    disjoint orbital and auxiliary blocks (occupied orbitals of both first)."""
    fA, fB = make_fragment(*sA), make_fragment(*sB)
    oA, vA, XA = sA[:3]
    oB, vB, XB = sB[:3]
    o, v, X = oA + oB, vA + vB, XA + XB
    n = o + v
    idxA = list(range(oA)) + [o + a for a in range(vA)]
    idxB = [oA + i for i in range(oB)] + [o + vA + a for a in range(vB)]
    B = np.zeros((X, n, n))
    B[np.ix_(range(XA), idxA, idxA)] = scale * fA.B
    B[np.ix_(range(XA, X), idxB, idxB)] = scale * fB.B
    eo = np.concatenate([fA.eps_occ, fB.eps_occ])
    ev = np.concatenate([fA.eps_vir, fB.eps_vir])
    return B, eo, ev, (scale * fA.B, fA.eps_occ, fA.eps_vir), (scale * fB.B, fB.eps_occ, fB.eps_vir)


def test_pair_matrix_traces_are_the_energies():
    """Tr E = Eq. 7 energy and Tr E_T = the (T) energy of the triples module (both
    pinned above by the determinant-space definitions)."""
    f = make_fragment(3, 5, 16, 41)
    B = 3.0 * f.B
    t1, t2 = _random_amplitudes(3, 5, 42)
    E = opr.ccsd_pair_matrix(B, 3, t1, t2)
    assert abs(np.trace(E) - cc.energy(B, 3, t1, t2)) < 1e-13
    ET = opr.triples_pair_matrix(B, f.eps_occ, f.eps_vir, t1, t2)
    assert abs(np.trace(ET) - tr.e_triples_full(B, f.eps_occ, f.eps_vir, t1, t2)) < 1e-13
    # both pair matrices have off-diagonal weight (the projection is not the trace)
    assert np.abs(E - np.diag(np.diag(E))).max() > 1e-3 * np.abs(E).max()
    assert np.abs(ET - np.diag(np.diag(ET))).max() > 1e-3 * np.abs(ET).max()


def test_projection_over_all_fragments_is_exact():
    """With LOs spanning the occupied space (a random orthogonal U, Eq. 5), the
    projected energies summed over every fragment of any partition equal the
    canonical energy (the exactness of Eqs. 7-9 and 14-15)."""
    f = make_fragment(4, 5, 18, 43)
    B = 3.0 * f.B
    t1, t2 = _random_amplitudes(4, 5, 44)
    rng = np.random.default_rng(45)
    U, _ = np.linalg.qr(rng.standard_normal((4, 4)))
    E = opr.ccsd_pair_matrix(B, 4, t1, t2)
    ET = opr.triples_pair_matrix(B, f.eps_occ, f.eps_vir, t1, t2)
    for frags in ([[0, 1], [2, 3]], [[0], [1, 2, 3]], [[3, 1], [0], [2]]):
        eF = [opr.project(E, U)[F].sum() for F in frags]
        tF = [opr.project(ET, U)[F].sum() for F in frags]
        assert abs(sum(eF) - cc.energy(B, 4, t1, t2)) < 1e-13
        assert abs(sum(tF) - tr.e_triples_full(B, f.eps_occ, f.eps_vir, t1, t2)) < 1e-13
    # a fragment alone is not the whole: the projection depends on U
    assert abs(opr.project(E, U)[0] - E[0, 0]) > 1e-6


def test_pair_matrices_of_non_interacting_fragments():
    """Two non-interacting fragments solved as one system: the converged
    amplitudes do not couple them, so the pair matrices are block diagonal and
    each block is the pair matrix of the fragment solved alone."""
    B, eo, ev, fa, fb = _separable_union((2, 3, 10, 51), (2, 4, 12, 52))
    r = cc.ccsd(B, eo, ev, conv_tol=1e-11)
    ra = cc.ccsd(*fa, conv_tol=1e-11)
    rb = cc.ccsd(*fb, conv_tol=1e-11)
    assert r.converged and ra.converged and rb.converged
    E = opr.ccsd_pair_matrix(B, 4, r.t1, r.t2)
    ET = opr.triples_pair_matrix(B, eo, ev, r.t1, r.t2)
    EA = opr.ccsd_pair_matrix(fa[0], 2, ra.t1, ra.t2)
    EB = opr.ccsd_pair_matrix(fb[0], 2, rb.t1, rb.t2)
    ETA = opr.triples_pair_matrix(*fa, ra.t1, ra.t2)
    ETB = opr.triples_pair_matrix(*fb, rb.t1, rb.t2)
    for M, MA, MB in ((E, EA, EB), (ET, ETA, ETB)):
        assert np.abs(M[:2, 2:]).max() < 1e-10 and np.abs(M[2:, :2]).max() < 1e-10
        np.testing.assert_allclose(M[:2, :2], MA, atol=1e-10)
        np.testing.assert_allclose(M[2:, 2:], MB, atol=1e-10)
    assert np.abs(EA - np.diag(np.diag(EA))).max() > 1e-8


def test_pair_pins_catch_planted_mistakes():
    """A swapped exchange sign or a dropped scaling of v by Delta_i'jk breaks the
    pins above."""
    f = make_fragment(3, 5, 16, 41)
    B = 3.0 * f.B
    t1, t2 = _random_amplitudes(3, 5, 42)
    g = cc.ovov(B, 3)
    tau = t2 + np.einsum("ia,jb->ijab", t1, t1)
    wrong = np.einsum("ijab,kajb->ik", tau, 2.0 * g + g.transpose(0, 3, 2, 1))
    assert abs(np.trace(wrong) - cc.energy(B, 3, t1, t2)) > 1e-6
