"""GPU: local active spaces (Sec. II.C-E), the local Hamiltonian's DF factors
(Eq. 27b), MP2 and the composite correction (Eq. 17) through the C ABI, against
the oracle (oracle/lno.py, oracle/ccsd.py, oracle/pairs.py).

Orbitals are defined up to sign (and rotations inside degenerate eigenspaces),
so the comparisons use what is unique: the active sizes, orbital energies,
external eigenvalues, the projectors onto the active spaces and the Gram
matrix of the projected LOs.  Thresholds are placed inside a gap of the
oracle's eigenvalues (ratio >= 1.01), where both sides select the same LNOs.
Tolerances: eigenvalues and orbital energies 1e-10 (Jacobi and the FP64
products agree to rounding; the tolerance leaves room for the eigenvector
error ~1e-16 |D| / gap), projectors 1e-8, DF factors 1e-12 of the largest,
MP2 energies 1e-12 relative, chained fragment energies 1e-8 Eh (CCSD
converged to 1e-10 on both sides)."""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2407_11258_amd import lnocc as L  # noqa: E402
from oracle import ccsd as occ, lno, pairs as opr, triples as otr  # noqa: E402
from synth import make_fragment, make_system, random_orthonormal  # noqa: E402

DEV = "cuda:0"


def say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


def host(x):
    return x.detach().cpu().numpy()


def _gap_eta(lam, frac):
    """A threshold between two consecutive |lambda| (descending): the cut with
    the largest ratio among those that keep 30-80 % of them (ratio >= 1.01, so
    the margin on either side is far above the eigenvalue error); 0 when none."""
    a = np.sort(np.abs(lam))[::-1]
    if a.size < 2:
        return 0.0
    ks = range(max(1, int(0.3 * a.size)), min(a.size, int(0.8 * a.size) + 1))
    k = max(ks, key=lambda k: a[k - 1] / a[k], default=None)
    if k is None or a[k - 1] / a[k] < 1.01:
        return 0.0
    return float(np.sqrt(a[k - 1] * a[k]))


class Sys:
    def __init__(self, s):
        self.s = s
        self.Lao, self.C = dev(s.Lao), dev(s.C)
        self.eo, self.ev = dev(s.eps_occ), dev(s.eps_vir)
        self.has_vir = np.abs(s.U_vir).max() > 0

    def U(self, F):
        Uo = dev(self.s.U_occ[:, F])
        Uv = dev(self.s.U_vir[:, F]) if self.has_vir else None
        return Uo, Uv

    def oracle_space(self, F, eta_o, eta_v, cbno):
        Uv = self.s.U_vir[:, F] if self.has_vir else None
        return lno.active_space(self.s.B[:, :self.s.nocc, self.s.nocc:], self.s.eps_occ,
                                self.s.eps_vir, self.s.U_occ[:, F], Uv, eta_o, eta_v, cbno=cbno)

    def etas(self, F, cbno):
        *_, lam_o, lam_v = self.oracle_space(F, 0.0, 0.0, cbno)
        return _gap_eta(lam_o, 0.5), _gap_eta(lam_v, 0.5)


SPACE_CASES = [(6, 41, 120, 21, 0, 3, False), (6, 41, 120, 22, 3, 2, False),
               (6, 41, 120, 22, 3, 2, True), (10, 89, 260, 23, 0, 4, False),
               (10, 89, 260, 24, 4, 3, True), (3, 8, 24, 25, 2, 1, False)]


@pytest.mark.parametrize("o,v,X,seed,nlo_vir,nfrag,cbno", SPACE_CASES)
def test_active_space_matches_oracle(o, v, X, seed, nlo_vir, nfrag, cbno):
    s = make_system(o, v, X, seed, nlo_vir=nlo_vir, nfrag=nfrag)
    S = Sys(s)
    for F in s.fragments[:2]:
        eta_o, eta_v = S.etas(F, cbno)
        say(f"active space o={o} v={v} X={X} seed={seed} frag={F} cbno={cbno} "
            f"eta=({eta_o:.2e}, {eta_v:.2e})")
        Co, eo, Cv, ev, lam_o, lam_v = S.oracle_space(F, eta_o, eta_v, cbno)
        Uo, Uv = S.U(F)
        sp = L.local_space(S.Lao, S.C, S.eo, S.ev, Uo, Uv, eta_occ=eta_o, eta_vir=eta_v,
                           cbno=cbno)
        assert (sp.C_occ.shape[1], sp.C_vir.shape[1]) == (Co.shape[1], Cv.shape[1])
        assert sp.n_int_occ == o - lam_o.size and sp.n_int_vir == v - lam_v.size
        np.testing.assert_allclose(host(sp.eps_occ), eo, rtol=0, atol=1e-10)
        np.testing.assert_allclose(host(sp.eps_vir), ev, rtol=0, atol=1e-10)
        for got, ref in ((host(sp.lambda_occ), lam_o), (host(sp.lambda_vir), lam_v)):
            if ref.size:
                np.testing.assert_allclose(got, ref, rtol=0, atol=1e-10 * np.abs(ref).max())
        Cgo, Cgv = host(sp.C_occ), host(sp.C_vir)
        np.testing.assert_allclose(Cgo @ Cgo.T, Co @ Co.T, rtol=0, atol=1e-8)
        np.testing.assert_allclose(Cgv @ Cgv.T, Cv @ Cv.T, rtol=0, atol=1e-8)
        np.testing.assert_allclose(Cgo.T @ Cgo, np.eye(Cgo.shape[1]), rtol=0, atol=1e-12)
        np.testing.assert_allclose(Cgv.T @ np.diag(s.eps_vir) @ Cgv, np.diag(host(sp.eps_vir)),
                                   rtol=0, atol=1e-11)
        UF = Co.T @ s.U_occ[:, F]
        Ua = host(sp.U_act)
        np.testing.assert_allclose(Ua.T @ Ua, UF.T @ UF, rtol=0, atol=1e-10)


def test_thresholds_bracket_the_sizes():
    """eta = 0 keeps everything; eta above every |lambda| keeps the internal
    orbitals only (the limits of Eq. 26)."""
    s = make_system(5, 30, 90, 26, nfrag=3)
    S = Sys(s)
    Uo, _ = S.U(s.fragments[0])
    say("thresholds o=5 v=30")
    sp = L.local_space(S.Lao, S.C, S.eo, S.ev, Uo, None, eta_occ=0.0, eta_vir=0.0)
    assert (sp.C_occ.shape[1], sp.C_vir.shape[1]) == (5, 30)
    np.testing.assert_allclose(np.sort(host(sp.eps_occ)), s.eps_occ, atol=1e-12)
    sp = L.local_space(S.Lao, S.C, S.eo, S.ev, Uo, None, eta_occ=1e3, eta_vir=1e3)
    assert (sp.C_occ.shape[1], sp.C_vir.shape[1]) == (len(s.fragments[0]), 0)


@pytest.mark.parametrize("o,v,X,seed,n_occ,n_vir", [(6, 41, 120, 31, 4, 17), (3, 8, 24, 32, 3, 8),
                                                    (10, 89, 260, 33, 1, 50)])
def test_local_hamiltonian_matches_oracle(o, v, X, seed, n_occ, n_vir):
    say(f"local Hamiltonian o={o} v={v} X={X} active=({n_occ}, {n_vir})")
    s = make_system(o, v, X, seed)
    Co = random_orthonormal(o, n_occ, seed + 1)
    Cv = random_orthonormal(v, n_vir, seed + 2)
    S = Sys(s)
    B = host(L.local_hamiltonian(S.Lao, S.C, S.eo, S.ev, dev(Co), dev(Cv)))
    Cact = np.zeros((s.n, n_occ + n_vir))
    Cact[:o, :n_occ] = Co
    Cact[o:, n_occ:] = Cv
    ref = lno.df_transform(s.Lao, s.C @ Cact)
    np.testing.assert_allclose(B, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("o,v,X,seed", [(4, 20, 72, 41), (7, 53, 90, 42), (13, 61, 150, 43),
                                        (1, 5, 9, 44)])
def test_fragment_mp2_matches_oracle(o, v, X, seed):
    say(f"MP2 o={o} v={v} X={X}")
    f = make_fragment(o, v, X, seed)
    t2_ref, e_ref = occ.mp2(f.B, f.eps_occ, f.eps_vir)
    Bd, eod, evd = dev(f.B), dev(f.eps_occ), dev(f.eps_vir)
    e, t2 = L.fragment_mp2(Bd, eod, evd)
    assert abs(e - e_ref) <= 1e-12 * abs(e_ref)
    np.testing.assert_allclose(host(t2), t2_ref, rtol=0, atol=1e-13 * np.abs(t2_ref).max())
    # energy only, through a workspace of one row and of a few rows
    fs = L.make_fragment_struct(Bd, eod, evd, None, None, 1e-8)
    st, nmin = L.lnocc_mp2_workspace_bytes(fs)
    assert st == L.LNOCC_OK
    ws = L.Workspace(DEV)
    for rows in (1, 3):
        buf = ws.ensure(nmin + (rows - 1) * o * v * v * 8)
        opt = L.make_options()
        opt.workspace, opt.workspace_bytes = buf.data_ptr(), nmin + (rows - 1) * o * v * v * 8
        opt.stream = torch.cuda.current_stream().cuda_stream
        assert L.lnocc_fragment_mp2(fs, opt) == L.LNOCC_OK, L.lnocc_last_error()
        assert abs(fs.e_mp2 - e_ref) <= 1e-12 * abs(e_ref)


def _project(Bd, eod, evd, t1d, t2d, Ud, triples):
    """lnocc_fragment_pair_energies: projected (CCSD, (T)) energies summed over the LOs."""
    o, nlo = eod.numel(), Ud.shape[1]
    z = lambda *sh: torch.zeros(sh, dtype=torch.float64, device=DEV)  # noqa: E731
    Ecc, Et, pc, pt = z(o, o), z(o, o), z(nlo), z(nlo)
    f = L.make_fragment_struct(Bd, eod, evd, t1d, t2d, 1e-8)
    opt = L.make_options()
    st, nbytes = L.lnocc_pair_workspace_bytes(f, opt)
    assert st == L.LNOCC_OK
    buf = L.Workspace(DEV).ensure(nbytes)
    opt.workspace, opt.workspace_bytes = buf.data_ptr(), buf.numel()
    opt.stream = torch.cuda.current_stream().cuda_stream
    st = L.lnocc_fragment_pair_energies(f, opt, Ecc.data_ptr(), Et.data_ptr() if triples else None,
                                        Ud.data_ptr(), nlo, pc.data_ptr(),
                                        pt.data_ptr() if triples else None)
    assert st == L.LNOCC_OK, L.lnocc_last_error()
    return float(pc.sum()), float(pt.sum()) if triples else 0.0


def _gpu_chain(S, etas, cbno):
    """Every fragment through the library: active space, local Hamiltonian,
    CCSD(T), projected CCSD / (T) / MP2 energies; then the full-system MP2."""
    e_cc = e_t = 0.0
    frag_mp2 = []
    for F, (eta_o, eta_v) in zip(S.s.fragments, etas):
        Uo, Uv = S.U(F)
        sp = L.local_space(S.Lao, S.C, S.eo, S.ev, Uo, Uv, eta_occ=eta_o, eta_vir=eta_v, cbno=cbno)
        BF = L.local_hamiltonian(S.Lao, S.C, S.eo, S.ev, sp.C_occ, sp.C_vir)
        r = L.solve(BF, sp.eps_occ, sp.eps_vir, conv_tol=1e-10)
        assert r.status == L.LNOCC_OK
        c, t = _project(BF, sp.eps_occ, sp.eps_vir, r.t1, r.t2, sp.U_act, True)
        e_cc += c
        e_t += t
        _, t2m = L.fragment_mp2(BF, sp.eps_occ, sp.eps_vir)
        t1z = torch.zeros_like(r.t1)
        frag_mp2.append(_project(BF, sp.eps_occ, sp.eps_vir, t1z, t2m, sp.U_act, False)[0])
    o, v = S.s.nocc, S.s.nvir
    Bfull = L.local_hamiltonian(S.Lao, S.C, S.eo, S.ev, torch.eye(o, dtype=torch.float64, device=DEV),
                                torch.eye(v, dtype=torch.float64, device=DEV))
    e_full, _ = L.fragment_mp2(Bfull, S.eo, S.ev, want_t2=False)
    return e_cc, e_t, sum(frag_mp2), L.lnocc_mp2_composite(e_full, frag_mp2)


def _oracle_chain(S, etas, cbno):
    s = S.s
    e_cc = e_t = e_mp2 = 0.0
    for F, (eta_o, eta_v) in zip(s.fragments, etas):
        Co, eo, Cv, ev, _, _ = S.oracle_space(F, eta_o, eta_v, cbno)
        no, nv = Co.shape[1], Cv.shape[1]
        Cact = np.zeros((s.n, no + nv))
        Cact[:s.nocc, :no] = Co
        Cact[s.nocc:, no:] = Cv
        BF = lno.df_transform(s.Lao, s.C @ Cact)
        UF = Co.T @ s.U_occ[:, F]
        r = occ.ccsd(BF, eo, ev, conv_tol=1e-11)
        assert r.converged
        e_cc += opr.project(opr.ccsd_pair_matrix(BF, no, r.t1, r.t2), UF).sum()
        e_t += opr.project(opr.triples_pair_matrix(BF, eo, ev, r.t1, r.t2), UF).sum()
        t2m, _ = occ.mp2(BF, eo, ev)
        e_mp2 += opr.project(opr.ccsd_pair_matrix(BF, no, np.zeros((no, nv)), t2m), UF).sum()
    _, e_full = occ.mp2(s.B, s.eps_occ, s.eps_vir)
    return e_cc, e_t, e_mp2, lno.mp2_composite(e_full, [e_mp2])


@pytest.mark.parametrize("cbno", [False, True])
def test_lno_chain_matches_oracle(cbno):
    """The whole LNO-CCSD(T) chain on the library matches the oracle's chain at
    thresholds that truncate both spaces, and at eta = 0 it recovers the
    canonical energies of the whole system (composite correction 0)."""
    s = make_system(5, 24, 90, 51, nlo_vir=2, nfrag=2)
    S = Sys(s)
    etas = [S.etas(F, cbno) for F in s.fragments]
    say(f"LNO chain cbno={cbno} etas={etas}")
    gpu = _gpu_chain(S, etas, cbno)
    ref = _oracle_chain(S, etas, cbno)
    say(f"  gpu {gpu}  oracle {ref}")
    for g, r in zip(gpu, ref):
        assert abs(g - r) < 1e-8, (gpu, ref)
    assert abs(gpu[3]) > 1e-6        # the truncation leaves a visible correction
    say("LNO chain at eta = 0")
    gpu0 = _gpu_chain(S, [(0.0, 0.0)] * len(s.fragments), cbno)
    ref_cc = occ.ccsd(s.B, s.eps_occ, s.eps_vir, conv_tol=1e-11)
    ref_t = otr.e_triples_full(s.B, s.eps_occ, s.eps_vir, ref_cc.t1, ref_cc.t2)
    assert abs(gpu0[0] - ref_cc.e_ccsd) < 1e-8
    assert abs(gpu0[1] - ref_t) < 1e-9
    assert abs(gpu0[3]) < 1e-11
