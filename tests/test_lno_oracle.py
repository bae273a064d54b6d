"""Pins of the local-active-space oracle (oracle/lno.py, Sec. II.C-E) against
what the mathematics fixes:
  * with every LO in one fragment the densities of Eq. 20 are the MP2 densities
    of the whole system: the occupied and virtual traces agree (the correlation
    hole holds as many electrons as the particle density), and the CBNO
    contraction pattern of Eq. 28 gives the same matrices;
  * with a canonical orbital as the only internal one, the amplitudes of Eq. 21
    are the canonical MP1 amplitudes of that orbital;
  * with every LNO kept (eta = 0) the active space is the whole orbital space:
    the projected fragment energies add up to the canonical CCSD, (T) and MP2
    energies of the system, and the composite correction of Eq. 17 vanishes;
  * thresholds: a larger eta never keeps more LNOs, and eta above every |lambda|
    leaves the internal orbitals only.
"""
import numpy as np
import pytest

from oracle import ccsd as cc, lno, pairs as opr, triples as tr
from synth import make_system


def _lov(s):
    return s.B[:, :s.nocc, s.nocc:]


def test_all_internal_densities_conserve_electrons_and_agree():
    s = make_system(3, 5, 18, 11, nlo_vir=5)
    Lov = _lov(s)
    Wo, Wo_ext = lno.split_space(s.U_occ, 3)
    Wv, Wv_ext = lno.split_space(s.U_vir, 5)
    assert Wo.shape[1] == 3 and Wv.shape[1] == 5 and Wo_ext.shape[1] == 0
    Wo, fo = lno.semicanonical(Wo, s.eps_occ)
    Wv, fv = lno.semicanonical(Wv, s.eps_vir)
    np.testing.assert_allclose(fo, s.eps_occ, atol=1e-13)
    Dij, Dab = lno.lno_densities(lno.mp1_one_internal(Lov, s.eps_occ, s.eps_vir, Wo, fo))
    Cij, Cab = lno.cbno_densities(Lov, s.eps_occ, s.eps_vir, Wo, fo, Wv, fv)
    assert abs(np.trace(Dij) - np.trace(Dab)) < 1e-13 * max(1.0, np.trace(Dab))
    assert np.trace(Dab) > 1e-4
    np.testing.assert_allclose(Cij, Dij, atol=1e-14)
    np.testing.assert_allclose(Cab, Dab, atol=1e-14)
    np.testing.assert_allclose(Dij, Dij.T, atol=1e-15)
    assert np.linalg.eigvalsh(Dab).min() > -1e-14        # a density: positive semidefinite


def test_one_canonical_internal_orbital_gives_mp1():
    s = make_system(4, 6, 20, 12)
    B = s.B
    t2, _ = cc.mp2(B, s.eps_occ, s.eps_vir)
    for k in range(4):
        W = np.zeros((4, 1))
        W[k, 0] = 1.0
        t = lno.mp1_one_internal(_lov(s), s.eps_occ, s.eps_vir, W, s.eps_occ[[k]])
        np.testing.assert_allclose(t[0], t2[k].transpose(1, 0, 2), atol=1e-15)   # t[k,a,j,b] = t_kj^ab


def _fragment_energies(s, eta, cbno=False):
    Lov = _lov(s)
    e_cc = e_t = e_mp2 = 0.0
    sizes = []
    for F in s.fragments:
        Uv = s.U_vir[:, F] if np.abs(s.U_vir).max() > 0 else None
        Co, eo, Cv, ev, lo, lv = lno.active_space(Lov, s.eps_occ, s.eps_vir, s.U_occ[:, F], Uv,
                                                  eta, eta, cbno=cbno)
        no, nv = Co.shape[1], Cv.shape[1]
        sizes.append((no, nv))
        Cact = np.zeros((s.n, no + nv))
        Cact[:s.nocc, :no] = Co
        Cact[s.nocc:, no:] = Cv
        BF = lno.df_transform(s.Lao, s.C @ Cact)
        UF = Co.T @ s.U_occ[:, F]          # the fragment's LOs on its active occupied orbitals
        r = cc.ccsd(BF, eo, ev, conv_tol=1e-11)
        assert r.converged
        e_cc += opr.project(opr.ccsd_pair_matrix(BF, no, r.t1, r.t2), UF).sum()
        e_t += opr.project(opr.triples_pair_matrix(BF, eo, ev, r.t1, r.t2), UF).sum()
        t2m, _ = cc.mp2(BF, eo, ev)
        e_mp2 += opr.project(opr.ccsd_pair_matrix(BF, no, np.zeros((no, nv)), t2m), UF).sum()
    return e_cc, e_t, e_mp2, sizes


@pytest.mark.parametrize("nlo_vir,cbno", [(0, False), (2, False), (2, True)])
def test_all_lnos_recover_the_canonical_energies(nlo_vir, cbno):
    s = make_system(3, 6, 20, 13, nlo_vir=nlo_vir, nfrag=2)
    B = 3.0 * s.B
    s.Lao = 3.0 * s.Lao
    ref = cc.ccsd(B, s.eps_occ, s.eps_vir, conv_tol=1e-11)
    ref_t = tr.e_triples_full(B, s.eps_occ, s.eps_vir, ref.t1, ref.t2)
    e_cc, e_t, e_mp2, sizes = _fragment_energies(s, 0.0, cbno)
    assert all(sz == (3, 6) for sz in sizes)
    assert abs(e_cc - ref.e_ccsd) < 1e-9
    assert abs(e_t - ref_t) < 1e-10
    assert abs(lno.mp2_composite(ref.e_mp2, [e_mp2])) < 1e-11


def test_thresholds_select_fewer_lnos():
    s = make_system(4, 10, 30, 14, nfrag=4)
    Lov = _lov(s)
    counts = []
    for eta in (0.0, 1e-6, 1e-4, 1e-2, 1e3):
        Co, eo, Cv, ev, lo, lv = lno.active_space(Lov, s.eps_occ, s.eps_vir,
                                                  s.U_occ[:, [0]], None, eta, eta)
        counts.append((Co.shape[1], Cv.shape[1]))
        np.testing.assert_allclose(Co.T @ Co, np.eye(Co.shape[1]), atol=1e-12)
        np.testing.assert_allclose(Co.T @ np.diag(s.eps_occ) @ Co, np.diag(eo), atol=1e-12)
    assert counts[0] == (4, 10) and counts[-1] == (1, 0)
    assert all(a[0] >= b[0] and a[1] >= b[1] for a, b in zip(counts, counts[1:]))
