"""Host-side checks of the C ABI (no GPU needed).

* the library loads and exports every function include/lnocc.h declares;
* the ctypes mirrors have the C layout (sizes and offsets from gcc);
* argument validation answers before any device work;
* validation mode runs the whole launch sequence of a solve, every
  contraction checked to stay inside the workspace and the caller's arrays,
  for the named workloads and precisions (pointers are never dereferenced).
"""
import ctypes as C
import os
import pathlib
import re
import subprocess
import tempfile

import pytest

from paper_2407_11258_amd import lnocc as L
from synth import CONFIG_SHAPES, batch_shapes

ROOT = pathlib.Path(__file__).resolve().parent.parent
HEADER = ROOT / "include" / "lnocc.h"


def declared_functions():
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lnocc_\w+)\s*\(", text)))


def test_every_declared_function_is_exported():
    names = declared_functions()
    assert "lnocc_fragment_ccsd" in names and "lnocc_batch_solve" in names
    lib = C.CDLL(str(L._LIB_PATH))
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(L.EXPORTS)


def test_struct_layouts_match_the_header():
    structs = {"lnocc_fragment_t": L.lnocc_fragment_t, "lnocc_options_t": L.lnocc_options_t,
               "lnocc_operand_t": L.lnocc_operand_t, "lnocc_contract_t": L.lnocc_contract_t,
               "lnocc_kernel_stats_t": L.lnocc_kernel_stats_t,
               "lnocc_system_t": L.lnocc_system_t, "lnocc_local_space_t": L.lnocc_local_space_t}
    lines = ['#include <stdio.h>', '#include <stddef.h>', f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    with tempfile.TemporaryDirectory() as td:
        src, exe = os.path.join(td, "l.c"), os.path.join(td, "l")
        open(src, "w").write("\n".join(lines))
        subprocess.run(["gcc", "-std=c11", src, "-o", exe], check=True)
        out = subprocess.run([exe], check=True, capture_output=True, text=True).stdout
    for line in out.splitlines():
        cname, what, val = line.split()
        py = structs[cname]
        if what == "size":
            assert C.sizeof(py) == int(val), cname
        else:
            assert getattr(py, what).offset == int(val), (cname, what)


def test_defaults_and_status_strings():
    opt = L.lnocc_default_options()
    assert (opt.precision, opt.guess, opt.do_triples, opt.max_iter, opt.diis_space,
            opt.diis_start) == (L.LNOCC_FP64, L.LNOCC_GUESS_MP2, 1, 100, 16, 1)
    for st in (0, 1, -1, -2, -3, -4):
        assert L.lnocc_status_string(st).startswith("LNOCC")
    assert "unknown" in L.lnocc_status_string(42)


def test_argument_errors_need_no_device():
    opt = L.lnocc_default_options()
    f = L.lnocc_fragment_t()
    assert L.lnocc_workspace_bytes([f], opt) == (L.LNOCC_EINVAL, 0)       # nocc = 0
    f.nocc, f.nvir, f.naux = 4, 20, 72
    st, n = L.lnocc_workspace_bytes([f], opt)
    assert st == L.LNOCC_OK and n > 0
    assert L._lib.lnocc_fragment_ccsd(None, C.byref(opt)) == L.LNOCC_EINVAL
    assert L.lnocc_fragment_ccsd(f, opt) == L.LNOCC_EINVAL                  # null B
    bad = L.lnocc_default_options()
    bad.diis_space = 0
    assert L.lnocc_workspace_bytes([f], bad)[0] == L.LNOCC_EINVAL
    bad.diis_space = 17
    assert L.lnocc_workspace_bytes([f], bad)[0] == L.LNOCC_EINVAL
    bad.diis_space = 16
    assert L.lnocc_workspace_bytes([f], bad)[0] == L.LNOCC_OK
    bad = L.lnocc_default_options()
    bad.precision = 7
    assert L.lnocc_workspace_bytes([f], bad)[0] == L.LNOCC_EINVAL
    f.nocc = 2000                                                            # beyond limits
    assert L.lnocc_workspace_bytes([f], opt)[0] == L.LNOCC_EINVAL


def _fake_fragment(o, v, X):
    """Pointer values in disjoint ranges; never dereferenced in validation mode."""
    f = L.lnocc_fragment_t()
    f.nocc, f.nvir, f.naux = o, v, X
    n = o + v
    base = 1 << 44
    f.B = base
    f.eps_occ = base + X * n * n * 8 + 4096
    f.eps_vir = f.eps_occ + o * 8 + 4096
    f.t1 = f.eps_vir + v * 8 + 4096
    f.t2 = f.t1 + o * v * 8 + 4096
    f.conv_tol = 1e-8
    return f


@pytest.fixture
def validation_mode():
    L.lnocc_set_validation_mode(True)
    yield
    L.lnocc_set_validation_mode(False)


SHAPES = [v[:3] for v in CONFIG_SHAPES.values()] + [(1, 1, 1), (2, 37, 61), (1, 10, 20),
                                                    (6, 45, 100)] + [s[:3] for s in batch_shapes()[:6]]


@pytest.mark.parametrize("ladder", ["stored", "on_the_fly"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "bf16"])
@pytest.mark.parametrize("o,v,X", SHAPES)
def test_launch_sequence_stays_in_bounds(validation_mode, o, v, X, precision, ladder):
    opt = L.make_options(precision=precision, ladder=ladder)
    f = _fake_fragment(o, v, X)
    st, nbytes = L.lnocc_workspace_bytes([f], opt)
    assert st == L.LNOCC_OK
    opt.workspace, opt.workspace_bytes = 1 << 45, nbytes
    assert L.lnocc_fragment_ccsd(f, opt) == L.LNOCC_OK
    assert L.lnocc_fragment_triples(f, opt) == L.LNOCC_OK
    assert L.lnocc_ccsd_residuals(f, opt, 1 << 46, (1 << 46) + (1 << 40)) == L.LNOCC_OK
    # a workspace one byte short is refused before anything runs
    opt.workspace_bytes = nbytes - 1
    assert L.lnocc_fragment_ccsd(f, opt) == L.LNOCC_ENOMEM


def test_small_ladder_blocks_and_triple_batches(validation_mode):
    opt = L.make_options(ladder_chunk_bytes=1 << 20, triples_batch=5, ladder="on_the_fly")
    f = _fake_fragment(7, 53, 90)
    st, nbytes = L.lnocc_workspace_bytes([f], opt)
    opt.workspace, opt.workspace_bytes = 1 << 45, nbytes
    assert L.lnocc_fragment_ccsd(f, opt) == L.LNOCC_OK


def test_tune_cache_is_read_and_a_missing_file_skipped(validation_mode, tmp_path):
    """opt.tune_cache: the plan file is read before the call's first contraction;
    a missing file is no error; nothing is rewritten when no plan was added."""
    plan = tmp_path / "plans.txt"
    plan.write_text("0.0.0|16.1.16.1|1.1.0.1.1|160.1:160.0.1.0:160.0.1.0|16.0.1.0 3 4\n")
    opt = L.make_options(tune_cache=plan, autotune=True)
    f = _fake_fragment(2, 5, 9)
    st, nbytes = L.lnocc_workspace_bytes([f], opt)
    assert st == L.LNOCC_OK
    opt.workspace, opt.workspace_bytes = 1 << 45, nbytes
    L.lnocc_autotune_clear()
    try:
        assert L.lnocc_fragment_ccsd(f, opt) == L.LNOCC_OK
        out = tmp_path / "out.txt"
        assert L.lnocc_autotune_save(out) == 1
        assert out.read_text() == plan.read_text()
        opt.tune_cache = str(tmp_path / "missing.txt").encode()
        assert L.lnocc_fragment_ccsd(f, opt) == L.LNOCC_OK
        assert not (tmp_path / "missing.txt").exists()
    finally:
        L.lnocc_autotune_clear()


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_triples_partials_fit_every_batch(validation_mode, precision):
    """The (T) energy launch of every batch of triples, the short last one
    included, writes no more partial sums than the workspace holds (the launcher
    refuses one that would)."""
    shapes = [s[:3] for s in batch_shapes()] + [(9, 202, 633), (13, 207, 660), (18, 214, 696),
                                                 (5, 30, 60), (40, 40, 240)]
    for (o, v, X) in shapes:
        for nb in (0, 3, 7, 31):
            opt = L.make_options(precision=precision, triples_batch=nb)
            f = _fake_fragment(o, v, X)
            st, nbytes = L.lnocc_workspace_bytes([f], opt)
            assert st == L.LNOCC_OK
            opt.workspace, opt.workspace_bytes = 1 << 45, nbytes
            assert L.lnocc_fragment_triples(f, opt) == L.LNOCC_OK, (o, v, X, nb,
                                                                    L.lnocc_last_error())


@pytest.mark.parametrize("o,v,X", [(4, 20, 72), (3, 13, 40), (6, 45, 100), (1, 5, 9)])
def test_pair_energy_launches_stay_in_bounds(validation_mode, o, v, X):
    """Every launch of the pair energies (CCSD and (T) pair matrices, projection)
    stays inside the workspace and the caller's arrays; a workspace one byte short
    is refused before anything runs."""
    opt = L.make_options()
    f = _fake_fragment(o, v, X)
    st, nbytes = L.lnocc_pair_workspace_bytes(f, opt)
    assert st == L.LNOCC_OK
    assert nbytes >= L.lnocc_workspace_bytes([f], opt)[1]
    opt.workspace, opt.workspace_bytes = 1 << 45, nbytes
    out = 1 << 46
    nlo = o + 2
    args = (out, out + (1 << 30), out + (2 << 30), nlo, out + (3 << 30), out + (4 << 30))
    assert L.lnocc_fragment_pair_energies(f, opt, *args) == L.LNOCC_OK, L.lnocc_last_error()
    assert L.lnocc_fragment_pair_energies(f, opt, out, None, None, 0, None, None) == L.LNOCC_OK
    opt.workspace_bytes = nbytes - 1
    assert L.lnocc_fragment_pair_energies(f, opt, *args) == L.LNOCC_ENOMEM
    opt.workspace_bytes = nbytes
    assert L.lnocc_fragment_pair_energies(f, opt, out, None, out + (2 << 30), 0, out, None) == L.LNOCC_EINVAL


def _fake_system(o, v, X):
    s = L.lnocc_system_t()
    s.nocc, s.nvir, s.naux = o, v, X
    n = o + v
    base = 1 << 44
    s.Lao = base
    s.C = base + X * n * n * 8 + 4096
    s.eps_occ = s.C + n * n * 8 + 4096
    s.eps_vir = s.eps_occ + o * 8 + 4096
    return s


def _fake_space(o, v, nlo, cbno, with_vir):
    sp = L.lnocc_local_space_t()
    out = 1 << 46
    sp.U_occ = out
    sp.U_vir = out + (1 << 36) if with_vir else None
    sp.nlo, sp.cbno, sp.eta_occ, sp.eta_vir = nlo, int(cbno), 1e-5, 1e-6
    for k, name in enumerate(("C_occ", "eps_occ", "C_vir", "eps_vir", "lambda_occ",
                              "lambda_vir", "U_act")):
        setattr(sp, name, out + ((k + 2) << 36))
    return sp


LNO_SHAPES = [(4, 10, 30, 2), (3, 5, 18, 8), (1, 1, 1, 1), (16, 160, 528, 3), (7, 53, 90, 40),
              (32, 400, 1300, 2)]


@pytest.mark.parametrize("with_vir", [False, True])
@pytest.mark.parametrize("cbno", [False, True])
@pytest.mark.parametrize("o,v,X,nlo", LNO_SHAPES)
def test_local_space_launches_stay_in_bounds(validation_mode, o, v, X, nlo, cbno, with_vir):
    """Every launch of the active-space construction (Sec. II.C-E) and of the
    local Hamiltonian's DF transform (Eq. 27b) stays inside the workspace and the
    caller's arrays (validation mode keeps every internal orbital and every LNO,
    the largest sizes); a workspace one byte short is refused."""
    sysd = _fake_system(o, v, X)
    st, nbytes = L.lnocc_local_space_workspace_bytes(sysd, nlo, cbno)
    assert st == L.LNOCC_OK and nbytes > 0
    sp = _fake_space(o, v, nlo, cbno, with_vir)
    ws = 1 << 45
    assert L.lnocc_local_space(sysd, sp, ws, nbytes) == L.LNOCC_OK, L.lnocc_last_error()
    assert (sp.n_int_occ, sp.n_occ) == (min(nlo, o), o)
    assert (sp.n_int_vir, sp.n_vir) == ((min(nlo, v) if with_vir else 0), v)
    assert L.lnocc_local_space(sysd, sp, ws, nbytes - 1) == L.LNOCC_ENOMEM
    st, hb = L.lnocc_local_hamiltonian_workspace_bytes(sysd, sp.n_occ, sp.n_vir)
    assert st == L.LNOCC_OK
    B = 1 << 47
    assert L.lnocc_local_hamiltonian(sysd, sp.C_occ, sp.n_occ, sp.C_vir, sp.n_vir, B, ws,
                                     hb) == L.LNOCC_OK, L.lnocc_last_error()
    assert L.lnocc_local_hamiltonian(sysd, sp.C_occ, sp.n_occ, sp.C_vir, sp.n_vir, B, ws,
                                     hb - 1) == L.LNOCC_ENOMEM
    if o > 1 and v > 1:   # a truncated space
        st, hb = L.lnocc_local_hamiltonian_workspace_bytes(sysd, o - 1, v // 2)
        assert L.lnocc_local_hamiltonian(sysd, sp.C_occ, o - 1, sp.C_vir, v // 2, B, ws,
                                         hb) == L.LNOCC_OK


def test_local_space_argument_errors():
    sysd = _fake_system(4, 10, 30)
    assert L.lnocc_local_space_workspace_bytes(sysd, 0, False)[0] == L.LNOCC_EINVAL
    big = _fake_system(4, 2049, 30)
    assert L.lnocc_local_space_workspace_bytes(big, 2, False)[0] == L.LNOCC_EINVAL
    st, nbytes = L.lnocc_local_space_workspace_bytes(sysd, 2, False)
    for field, value in (("eta_occ", -1.0), ("eta_vir", float("nan")), ("nlo", 0),
                         ("U_occ", None), ("C_vir", None)):
        sp = _fake_space(4, 10, 2, False, False)
        setattr(sp, field, value)
        assert L.lnocc_local_space(sysd, sp, 1 << 45, nbytes) == L.LNOCC_EINVAL, field
    assert L.lnocc_local_hamiltonian_workspace_bytes(sysd, 5, 3)[0] == L.LNOCC_EINVAL
    assert L.lnocc_local_hamiltonian_workspace_bytes(sysd, 0, 0)[0] == L.LNOCC_EINVAL
    assert L.lnocc_mp2_composite(-1.0, [-0.25, -0.5]) == pytest.approx(-0.25, abs=0)


@pytest.mark.parametrize("o,v,X", [(4, 20, 72), (1, 1, 1), (6, 45, 100), (16, 160, 528)])
def test_mp2_launches_stay_in_bounds(validation_mode, o, v, X):
    """The MP2 entry point (whole amplitudes, or energy only through a workspace
    of one or a few occupied rows) stays in bounds; a short workspace is refused."""
    opt = L.make_options()
    f = _fake_fragment(o, v, X)
    st, nbytes = L.lnocc_mp2_workspace_bytes(f)
    assert st == L.LNOCC_OK
    opt.workspace, opt.workspace_bytes = 1 << 45, nbytes
    assert L.lnocc_fragment_mp2(f, opt) == L.LNOCC_OK, L.lnocc_last_error()
    opt.workspace_bytes = nbytes - 1
    assert L.lnocc_fragment_mp2(f, opt) == L.LNOCC_ENOMEM
    f.t2 = None
    st, n1 = L.lnocc_mp2_workspace_bytes(f)
    assert n1 > nbytes
    for extra in (0, 3 * o * v * v * 8 // 2):
        opt.workspace_bytes = n1 + extra
        assert L.lnocc_fragment_mp2(f, opt) == L.LNOCC_OK, L.lnocc_last_error()


def test_static_scratch_entry_point(validation_mode):
    """The no-allocation variant ignores the caller's workspace, runs the same
    launch sequence inside its static array and refuses a fragment that needs
    more than the array holds, naming the sizes."""
    opt = L.make_options(precision="fp64")
    opt.workspace, opt.workspace_bytes = 0, 0
    for shp in [(4, 20, 72), (3, 14, 50), (6, 30, 100)]:
        f = _fake_fragment(*shp)
        need = L.lnocc_workspace_bytes([f], opt)[1]
        assert need <= L.LNOCC_STATIC_SCRATCH_BYTES
        assert L.lnocc_fragment_ccsd_static(f, opt) == L.LNOCC_OK, L.lnocc_last_error()
    f = _fake_fragment(16, 160, 528)
    assert L.lnocc_fragment_ccsd_static(f, opt) == L.LNOCC_ENOMEM
    assert "static array" in L.lnocc_last_error()
    assert f.status == L.LNOCC_ENOMEM
    f = _fake_fragment(4, 20, 72)
    f.conv_tol = 0.0
    assert L.lnocc_fragment_ccsd_static(f, opt) == L.LNOCC_EINVAL


def _batch(shapes):
    arr = (L.lnocc_fragment_t * len(shapes))()
    for k, (o, v, X) in enumerate(shapes):
        arr[k] = _fake_fragment(o, v, X)
    return arr


@pytest.mark.parametrize("streams", [1, 3, 0])
def test_batch_schedule_stays_in_bounds(validation_mode, streams):
    shapes = [s[:3] for s in batch_shapes()[:7]] + [(1, 1, 1)]
    arr = _batch(shapes)
    opt = L.make_options(precision="fp32", batch_slots=streams, batch_streams=2)
    st, nbytes = L.lnocc_workspace_bytes(arr, opt)
    assert st == L.LNOCC_OK
    single = max(L.lnocc_workspace_bytes([arr[k]], opt)[1] for k in range(len(arr)))
    slots = min(len(arr), streams or 4)
    assert nbytes >= slots * single
    opt.workspace, opt.workspace_bytes = 1 << 45, nbytes
    assert L.lnocc_batch_solve(arr, opt) == L.LNOCC_OK
    assert all(arr[k].status == L.LNOCC_OK for k in range(len(arr)))
    # a workspace of one slice runs the fragments one at a time
    opt.workspace_bytes = single + 255
    assert L.lnocc_batch_solve(arr, opt) == L.LNOCC_OK


def test_batch_errors_are_per_fragment(validation_mode):
    arr = _batch([(4, 20, 72), (3, 15, 40), (2, 9, 30)])
    arr[1].conv_tol = 0.0                       # rejected on the host
    opt = L.make_options(batch_slots=2)
    st, nbytes = L.lnocc_workspace_bytes(arr, opt)
    opt.workspace, opt.workspace_bytes = 1 << 45, nbytes
    assert L.lnocc_batch_solve(arr, opt) == L.LNOCC_EINVAL
    assert [arr[k].status for k in range(3)] == [L.LNOCC_OK, L.LNOCC_EINVAL, L.LNOCC_OK]
    arr[1].conv_tol = 1e-8
    opt.workspace_bytes = 1024                  # no slice fits
    assert L.lnocc_batch_solve(arr, opt) == L.LNOCC_ENOMEM
    assert all(arr[k].status == L.LNOCC_ENOMEM for k in range(3))
    assert L._lib.lnocc_batch_solve(arr, 0, C.byref(opt)) == L.LNOCC_EINVAL


FAKE_MODEL = 1 << 47


@pytest.mark.parametrize("o,v,X", [(4, 20, 72), (1, 1, 1), (6, 45, 100), (16, 160, 528)])
def test_learned_guess_launches_stay_in_bounds(validation_mode, o, v, X):
    opt = L.make_options(guess=L.LNOCC_GUESS_MLP, mlp=FAKE_MODEL)
    f = _fake_fragment(o, v, X)
    st, nbytes = L.lnocc_workspace_bytes([f], opt)
    assert st == L.LNOCC_OK
    plain = L.lnocc_workspace_bytes([f], L.make_options())[1]
    assert nbytes >= plain                      # the network scratch and the fallback step
    opt.workspace, opt.workspace_bytes = 1 << 45, nbytes
    assert L.lnocc_fragment_ccsd(f, opt) == L.LNOCC_OK
    assert f.guess_used == L.LNOCC_GUESS_MLP and f.n_iter == 2
    opt.mlp = None
    assert L.lnocc_fragment_ccsd(f, opt) == L.LNOCC_EINVAL      # no model
    opt.mlp = FAKE_MODEL + 4
    assert L.lnocc_fragment_ccsd(f, opt) == L.LNOCC_EINVAL      # misaligned model


def test_network_calls_stay_in_bounds(validation_mode):
    base = 1 << 46
    blob, X, Y, out, grad, adam = (base + k * (1 << 36) for k in range(6))
    n = 5000
    for training, rows in ((False, 1 << 17), (True, 4096)):
        st, nbytes = L.lnocc_mlp_workspace_bytes(rows, training)
        assert st == L.LNOCC_OK and nbytes > rows * 4 * 256
    opt = L.lnocc_default_options()
    opt.workspace = 1 << 45
    opt.workspace_bytes = L.lnocc_mlp_workspace_bytes(n, True)[1]
    assert L.lnocc_mlp_init(blob, X, Y, n, 7, opt) == L.LNOCC_OK
    assert L.lnocc_mlp_predict(blob, X, 3 * n + 17, out, opt) == L.LNOCC_OK
    st, loss = L.lnocc_mlp_loss_grad(blob, X, Y, n, grad, opt)
    assert st == L.LNOCC_OK
    st, losses = L.lnocc_mlp_train(blob, adam, 0, 70, X, Y, 10 * n, n, 1e-3, 3, opt)
    assert st == L.LNOCC_OK and len(losses) == 70
    # a batch larger than the workspace holds, bad arguments
    assert L.lnocc_mlp_loss_grad(blob, X, Y, 2 * n, grad, opt)[0] == L.LNOCC_ENOMEM
    assert L.lnocc_mlp_train(blob, adam, 0, 1, X, Y, n, n, -1.0, 3, opt)[0] == L.LNOCC_EINVAL
    assert L.lnocc_mlp_predict(blob, X + 4, n, out, opt) == L.LNOCC_EINVAL
    assert L.lnocc_mlp_workspace_bytes(0, False)[0] == L.LNOCC_EINVAL
    f = _fake_fragment(5, 30, 70)
    o2 = L.make_options()
    o2.workspace, o2.workspace_bytes = 1 << 45, L.lnocc_workspace_bytes([f], o2)[1]
    assert L.lnocc_mlp_samples(f, o2, base, 1000, X, Y) == L.LNOCC_OK


def test_ladder_mode_changes_the_workspace():
    f = _fake_fragment(16, 160, 528)
    st_a, auto = L.lnocc_workspace_bytes([f], L.make_options())
    st_s, stored = L.lnocc_workspace_bytes([f], L.make_options(ladder="stored"))
    st_f, fly = L.lnocc_workspace_bytes([f], L.make_options(ladder="on_the_fly"))
    assert st_a == st_s == st_f == L.LNOCC_OK
    assert auto == stored > fly                 # v^4 / 2 of stored integrals fit the 32 GiB cap
    big = _fake_fragment(32, 400, 1300)
    assert L.lnocc_workspace_bytes([big], L.make_options())[1] == \
        L.lnocc_workspace_bytes([big], L.make_options(ladder="on_the_fly"))[1]


def test_one_hip_runtime_in_the_process():
    """The binding loads torch first, so liblnocc binds to torch's HIP runtime
    instead of mapping a second one (which would find no device)."""
    maps = pathlib.Path("/proc/self/maps").read_text().splitlines()
    hip = {ln.split()[-1] for ln in maps if "libamdhip64" in ln}
    hsa = {ln.split()[-1] for ln in maps if "libhsa-runtime64" in ln}
    assert len(hip) == 1 and len(hsa) == 1, (hip, hsa)


def test_options_are_checked():
    f = _fake_fragment(2, 5, 9)
    for field, bad in (("batch_streams", -1), ("batch_streams", 65), ("batch_slots", -2),
                       ("ladder_mode", 3), ("ladder_mode", -1)):
        opt = L.make_options()
        setattr(opt, field, bad)
        assert L.lnocc_workspace_bytes([f], opt)[0] == L.LNOCC_EINVAL, field


def test_missing_library_fails_loudly(tmp_path):
    with pytest.raises(RuntimeError):
        L.load_library(tmp_path / "nope.so")
