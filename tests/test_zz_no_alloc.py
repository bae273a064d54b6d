"""GPU: the no-allocation entry point lnocc_fragment_ccsd_static against
lnocc_fragment_ccsd on the same inputs, two calls in a row (the second on a
smaller fragment, so that the static array holds the first call's data).

Both run the same kernels in the same order on FP64 data, so energies and
amplitudes must agree to FP64 rounding (checked at 1e-12 absolute, the parity
bar of the FP64 path being 1e-8 Eh against the oracle).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2407_11258_amd import lnocc as L  # noqa: E402
from synth import make_fragment  # noqa: E402

DEV = "cuda:0"


def _solve(entry, f, precision):
    o, v = f.nocc, f.nvir
    B = torch.tensor(f.B, device=DEV)
    eo = torch.tensor(f.eps_occ, device=DEV)
    ev = torch.tensor(f.eps_vir, device=DEV)
    t1 = torch.full((o, v), float("nan"), dtype=torch.float64, device=DEV)
    t2 = torch.full((o, o, v, v), float("nan"), dtype=torch.float64, device=DEV)
    fs = L.make_fragment_struct(B, eo, ev, t1, t2, 1e-10)
    opt = L.make_options(precision=precision)
    if entry == "workspace":
        L.Workspace(DEV).attach([fs], opt)
        st = L.lnocc_fragment_ccsd(fs, opt)
    else:
        opt.stream = torch.cuda.current_stream().cuda_stream
        st = L.lnocc_fragment_ccsd_static(fs, opt)
    torch.cuda.synchronize()
    return st, fs, t1.cpu().numpy(), t2.cpu().numpy()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_entry_point_matches_workspace_entry_point(precision):
    for shape in [(4, 20, 72, 0), (3, 14, 50, 7)]:   # second call smaller than the first
        print(f"[gpu-case] static scratch {precision} shape {shape}", file=sys.stderr, flush=True)
        f = make_fragment(*shape)
        st_s, fs_s, t1_s, t2_s = _solve("static", f, precision)
        st_w, fs_w, t1_w, t2_w = _solve("workspace", f, precision)
        assert st_s == L.LNOCC_OK, L.lnocc_last_error()
        assert st_w == L.LNOCC_OK
        assert fs_s.n_iter == fs_w.n_iter
        assert abs(fs_s.e_ccsd - fs_w.e_ccsd) < 1e-12
        assert abs(fs_s.e_t - fs_w.e_t) < 1e-12
        assert abs(fs_s.e_mp2 - fs_w.e_mp2) < 1e-12
        np.testing.assert_allclose(t1_s, t1_w, rtol=0, atol=1e-12)
        np.testing.assert_allclose(t2_s, t2_w, rtol=0, atol=1e-12)


def test_static_entry_point_refuses_large_fragments():
    f = make_fragment(8, 40, 150, 3)
    st, fs, _, _ = _solve("static", f, "fp64")
    assert st == L.LNOCC_ENOMEM
    assert "static array" in L.lnocc_last_error()
