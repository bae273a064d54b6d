"""ctypes binding of liblnocc (include/lnocc.h), same names as the C ABI.

Argument marshalling only: every step of the fragment solve runs in the HIP
library.  PyTorch supplies device memory (tensors, the workspace) and the
stream.  Importing this module fails loudly when the library is missing.
"""
from __future__ import annotations

import ctypes as C
import dataclasses
import os
import pathlib

_PKG = pathlib.Path(__file__).resolve().parent
_LIB_PATH = _PKG / "liblnocc.so"

LNOCC_OK = 0
LNOCC_NOT_CONVERGED = 1
LNOCC_EINVAL = -1
LNOCC_ENOMEM = -2
LNOCC_EDEVICE = -3
LNOCC_ENUMERIC = -4

LNOCC_FP64, LNOCC_FP32, LNOCC_BF16, LNOCC_FP32_SPLIT, LNOCC_FP64_SPLIT = 0, 1, 2, 3, 4
LNOCC_GUESS_MP2, LNOCC_GUESS_USER, LNOCC_GUESS_MLP = 0, 1, 2
LNOCC_MLP_FEATURES, LNOCC_MLP_HIDDEN, LNOCC_MLP_HEADER, LNOCC_MLP_PARAMS = 16, 256, 64, 136256
LNOCC_MLP_BLOB = LNOCC_MLP_HEADER + LNOCC_MLP_PARAMS

PRECISIONS = {"fp64": LNOCC_FP64, "fp32": LNOCC_FP32, "bf16": LNOCC_BF16}
LNOCC_LADDER_AUTO, LNOCC_LADDER_STORED, LNOCC_LADDER_ON_THE_FLY = 0, 1, 2
LADDER_MODES = {"auto": 0, "stored": 1, "on_the_fly": 2}


class lnocc_fragment_t(C.Structure):
    _fields_ = [
        ("nocc", C.c_int32), ("nvir", C.c_int32), ("naux", C.c_int32), ("reserved0", C.c_int32),
        ("B", C.c_void_p), ("eps_occ", C.c_void_p), ("eps_vir", C.c_void_p),
        ("conv_tol", C.c_double),
        ("t1", C.c_void_p), ("t2", C.c_void_p),
        ("e_mp2", C.c_double), ("e_ccsd", C.c_double), ("e_t", C.c_double),
        ("residual", C.c_double),
        ("n_iter", C.c_int32), ("status", C.c_int32),
        ("guess_used", C.c_int32), ("reserved1", C.c_int32),
    ]


# lnocc_iter_fn: (fragment, iteration, energy, step norm, user)
lnocc_iter_fn = C.CFUNCTYPE(None, C.POINTER(lnocc_fragment_t), C.c_int32, C.c_double,
                            C.c_double, C.c_void_p)


class lnocc_options_t(C.Structure):
    _fields_ = [
        ("precision", C.c_int32), ("guess", C.c_int32), ("do_triples", C.c_int32),
        ("max_iter", C.c_int32), ("diis_space", C.c_int32), ("diis_start", C.c_int32),
        ("stream", C.c_void_p), ("workspace", C.c_void_p), ("workspace_bytes", C.c_size_t),
        ("ladder_chunk_bytes", C.c_size_t), ("triples_batch", C.c_int32),
        ("batch_slots", C.c_int32), ("level_shift", C.c_double),
        ("batch_streams", C.c_int32), ("ladder_mode", C.c_int32),
        ("mlp", C.c_void_p), ("graphs", C.c_int32), ("autotune", C.c_int32),
        ("tune_cache", C.c_char_p), ("on_iter", lnocc_iter_fn), ("user", C.c_void_p),
    ]


class lnocc_operand_t(C.Structure):
    _fields_ = [("p", C.c_void_p), ("s_ro", C.c_int64), ("s_ri", C.c_int64),
                ("s_ko", C.c_int64), ("s_ki", C.c_int64), ("b0", C.c_int64),
                ("b1", C.c_int64), ("bid", C.c_int64)]


class lnocc_contract_t(C.Structure):
    _fields_ = [
        ("M", C.c_int32), ("Mi", C.c_int32), ("N", C.c_int32), ("Ni", C.c_int32),
        ("nseg", C.c_int32), ("K", C.c_int32 * 4), ("Ki", C.c_int32 * 4),
        ("scale", C.c_double * 4), ("a", lnocc_operand_t * 4), ("b", lnocc_operand_t * 4),
        ("c", C.c_void_p), ("c_mo", C.c_int64), ("c_mi", C.c_int64), ("c_no", C.c_int64),
        ("c_ni", C.c_int64), ("c_b0", C.c_int64), ("c_b1", C.c_int64), ("c_bid", C.c_int64),
        ("beta", C.c_double), ("batch", C.c_int32), ("nb1", C.c_int32),
        ("precision", C.c_int32), ("tile", C.c_int32),
    ]


class lnocc_system_t(C.Structure):
    _fields_ = [("nocc", C.c_int32), ("nvir", C.c_int32), ("naux", C.c_int32),
                ("reserved0", C.c_int32), ("Lao", C.c_void_p), ("C", C.c_void_p),
                ("eps_occ", C.c_void_p), ("eps_vir", C.c_void_p)]


class lnocc_local_space_t(C.Structure):
    _fields_ = [("U_occ", C.c_void_p), ("U_vir", C.c_void_p), ("nlo", C.c_int32),
                ("cbno", C.c_int32), ("eta_occ", C.c_double), ("eta_vir", C.c_double),
                ("C_occ", C.c_void_p), ("eps_occ", C.c_void_p), ("C_vir", C.c_void_p),
                ("eps_vir", C.c_void_p), ("lambda_occ", C.c_void_p), ("lambda_vir", C.c_void_p),
                ("U_act", C.c_void_p), ("n_occ", C.c_int32), ("n_vir", C.c_int32), ("n_int_occ", C.c_int32),
                ("n_int_vir", C.c_int32)]


class lnocc_kernel_stats_t(C.Structure):
    _fields_ = [("launches", C.c_int64), ("ms", C.c_double), ("flops", C.c_double)]


LNOCC_KERNEL_CLASSES = 7
KERNEL_CLASS_NAMES = ("other", "ladder_build", "ladder_contract", "triples_w", "mlp", "ring",
                      "split")

EXPORTS = ("lnocc_default_options", "lnocc_status_string", "lnocc_last_error",
           "lnocc_workspace_bytes",
           "lnocc_fragment_ccsd", "lnocc_fragment_ccsd_static", "lnocc_fragment_triples",
           "lnocc_ccsd_residuals", "lnocc_pair_workspace_bytes", "lnocc_fragment_pair_energies",
           "lnocc_batch_solve", "lnocc_contract", "lnocc_profile_enable",
           "lnocc_profile_collect", "lnocc_set_validation_mode", "lnocc_mlp_workspace_bytes",
           "lnocc_mlp_samples", "lnocc_mlp_init", "lnocc_mlp_predict", "lnocc_mlp_loss_grad",
           "lnocc_mlp_train", "lnocc_autotune_save", "lnocc_autotune_load",
           "lnocc_autotune_clear", "lnocc_local_space_workspace_bytes", "lnocc_local_space",
           "lnocc_local_hamiltonian_workspace_bytes", "lnocc_local_hamiltonian",
           "lnocc_mp2_workspace_bytes", "lnocc_fragment_mp2", "lnocc_mp2_composite")


def load_library(path: str | os.PathLike | None = None) -> C.CDLL:
    # LNOCC_LIBRARY names another build of the same library (the host-sanitized
    # one of the CPU checks); the default is the in-tree build
    path = path or os.environ.get("LNOCC_LIBRARY") or None
    p = pathlib.Path(path) if path else _LIB_PATH
    if not p.exists():
        raise RuntimeError(f"liblnocc not built ({p}); run paper_2407_11258_amd.build_lib.build()")
    # One HIP runtime per process: PyTorch ships its own libamdhip64 (same
    # soname as the system one liblnocc links).  Loading torch first makes the
    # library bind to that runtime; loading liblnocc first would bring in a
    # second runtime, which then finds no device once torch owns it.
    import torch  # noqa: F401
    lib = C.CDLL(str(p))
    FP, OP = C.POINTER(lnocc_fragment_t), C.POINTER(lnocc_options_t)
    lib.lnocc_default_options.argtypes = [OP]
    lib.lnocc_default_options.restype = None
    lib.lnocc_status_string.argtypes = [C.c_int]
    lib.lnocc_status_string.restype = C.c_char_p
    lib.lnocc_last_error.argtypes = []
    lib.lnocc_last_error.restype = C.c_char_p
    lib.lnocc_workspace_bytes.argtypes = [FP, C.c_int32, OP, C.POINTER(C.c_size_t)]
    lib.lnocc_workspace_bytes.restype = C.c_int
    for name in ("lnocc_fragment_ccsd", "lnocc_fragment_ccsd_static", "lnocc_fragment_triples"):
        getattr(lib, name).argtypes = [FP, OP]
        getattr(lib, name).restype = C.c_int
    lib.lnocc_pair_workspace_bytes.argtypes = [FP, OP, C.POINTER(C.c_size_t)]
    lib.lnocc_pair_workspace_bytes.restype = C.c_int
    lib.lnocc_fragment_pair_energies.argtypes = [FP, OP, C.c_void_p, C.c_void_p, C.c_void_p,
                                                 C.c_int32, C.c_void_p, C.c_void_p]
    lib.lnocc_fragment_pair_energies.restype = C.c_int
    lib.lnocc_ccsd_residuals.argtypes = [FP, OP, C.c_void_p, C.c_void_p]
    lib.lnocc_ccsd_residuals.restype = C.c_int
    lib.lnocc_batch_solve.argtypes = [FP, C.c_int32, OP]
    lib.lnocc_batch_solve.restype = C.c_int
    lib.lnocc_contract.argtypes = [C.POINTER(lnocc_contract_t), C.c_void_p]
    lib.lnocc_contract.restype = C.c_int
    lib.lnocc_profile_enable.argtypes = [C.c_int]
    lib.lnocc_profile_enable.restype = None
    lib.lnocc_profile_collect.argtypes = [C.POINTER(lnocc_kernel_stats_t)]
    lib.lnocc_profile_collect.restype = None
    lib.lnocc_set_validation_mode.argtypes = [C.c_int]
    lib.lnocc_set_validation_mode.restype = None
    P, I64 = C.c_void_p, C.c_int64
    lib.lnocc_mlp_workspace_bytes.argtypes = [I64, C.c_int32, C.POINTER(C.c_size_t)]
    lib.lnocc_mlp_samples.argtypes = [FP, OP, P, I64, P, P]
    lib.lnocc_mlp_init.argtypes = [P, P, P, I64, C.c_uint64, OP]
    lib.lnocc_mlp_predict.argtypes = [P, P, I64, P, OP]
    lib.lnocc_mlp_loss_grad.argtypes = [P, P, P, I64, P, C.POINTER(C.c_double), OP]
    lib.lnocc_mlp_train.argtypes = [P, P, I64, C.c_int32, P, P, I64, C.c_int32, C.c_float,
                                    C.c_uint64, C.POINTER(C.c_double), OP]
    lib.lnocc_autotune_save.argtypes = [C.c_char_p]
    lib.lnocc_autotune_save.restype = C.c_int
    lib.lnocc_autotune_load.argtypes = [C.c_char_p]
    lib.lnocc_autotune_load.restype = C.c_int
    lib.lnocc_autotune_clear.argtypes = []
    lib.lnocc_autotune_clear.restype = None
    SP, LP = C.POINTER(lnocc_system_t), C.POINTER(lnocc_local_space_t)
    SZ = C.POINTER(C.c_size_t)
    lib.lnocc_local_space_workspace_bytes.argtypes = [SP, C.c_int32, C.c_int32, SZ]
    lib.lnocc_local_space.argtypes = [SP, LP, P, C.c_size_t, P]
    lib.lnocc_local_hamiltonian_workspace_bytes.argtypes = [SP, C.c_int32, C.c_int32, SZ]
    lib.lnocc_local_hamiltonian.argtypes = [SP, P, C.c_int32, P, C.c_int32, P, P, C.c_size_t, P]
    lib.lnocc_mp2_workspace_bytes.argtypes = [FP, SZ]
    lib.lnocc_fragment_mp2.argtypes = [FP, OP]
    lib.lnocc_mp2_composite.argtypes = [C.c_double, C.POINTER(C.c_double), C.c_int32]
    lib.lnocc_mp2_composite.restype = C.c_double
    for name in ("lnocc_local_space_workspace_bytes", "lnocc_local_space",
                 "lnocc_local_hamiltonian_workspace_bytes", "lnocc_local_hamiltonian",
                 "lnocc_mp2_workspace_bytes", "lnocc_fragment_mp2"):
        getattr(lib, name).restype = C.c_int
    for name in ("lnocc_mlp_workspace_bytes", "lnocc_mlp_samples", "lnocc_mlp_init",
                 "lnocc_mlp_predict", "lnocc_mlp_loss_grad", "lnocc_mlp_train"):
        getattr(lib, name).restype = C.c_int
    return lib


_lib = load_library()


# ------------------------------------------------------------ same-name wrappers
def lnocc_default_options() -> lnocc_options_t:
    opt = lnocc_options_t()
    _lib.lnocc_default_options(C.byref(opt))
    return opt


def lnocc_status_string(status: int) -> str:
    return _lib.lnocc_status_string(int(status)).decode()


def lnocc_autotune_save(path) -> int:
    return _lib.lnocc_autotune_save(str(path).encode())


def lnocc_autotune_load(path) -> int:
    return _lib.lnocc_autotune_load(str(path).encode())


def lnocc_autotune_clear() -> None:
    _lib.lnocc_autotune_clear()


def lnocc_last_error() -> str:
    return _lib.lnocc_last_error().decode()


def lnocc_workspace_bytes(frags, opt: lnocc_options_t) -> tuple[int, int]:
    arr = (lnocc_fragment_t * len(frags))(*frags)
    out = C.c_size_t(0)
    st = _lib.lnocc_workspace_bytes(arr, len(frags), C.byref(opt), C.byref(out))
    return st, out.value


def lnocc_fragment_ccsd(frag: lnocc_fragment_t, opt: lnocc_options_t) -> int:
    return _lib.lnocc_fragment_ccsd(C.byref(frag), C.byref(opt))


LNOCC_STATIC_SCRATCH_BYTES = 64 << 20


def lnocc_fragment_ccsd_static(frag: lnocc_fragment_t, opt: lnocc_options_t) -> int:
    return _lib.lnocc_fragment_ccsd_static(C.byref(frag), C.byref(opt))


def lnocc_pair_workspace_bytes(frag: lnocc_fragment_t, opt: lnocc_options_t) -> tuple[int, int]:
    out = C.c_size_t(0)
    st = _lib.lnocc_pair_workspace_bytes(C.byref(frag), C.byref(opt), C.byref(out))
    return st, out.value


def lnocc_fragment_pair_energies(frag: lnocc_fragment_t, opt: lnocc_options_t, pair_ccsd: int,
                                 pair_t: int | None, U: int | None, nlo: int,
                                 proj_ccsd: int | None, proj_t: int | None) -> int:
    return _lib.lnocc_fragment_pair_energies(C.byref(frag), C.byref(opt), pair_ccsd, pair_t, U,
                                             nlo, proj_ccsd, proj_t)


def lnocc_fragment_triples(frag: lnocc_fragment_t, opt: lnocc_options_t) -> int:
    return _lib.lnocc_fragment_triples(C.byref(frag), C.byref(opt))


def lnocc_ccsd_residuals(frag: lnocc_fragment_t, opt: lnocc_options_t, r1_ptr: int,
                         r2_ptr: int) -> int:
    return _lib.lnocc_ccsd_residuals(C.byref(frag), C.byref(opt), r1_ptr, r2_ptr)


def lnocc_batch_solve(frags, opt: lnocc_options_t) -> int:
    """frags: ctypes array of lnocc_fragment_t (results are written into it)."""
    return _lib.lnocc_batch_solve(frags, len(frags), C.byref(opt))


def lnocc_contract(desc: lnocc_contract_t, stream: int = 0) -> int:
    return _lib.lnocc_contract(C.byref(desc), C.c_void_p(stream))


def lnocc_profile_enable(on: bool) -> None:
    _lib.lnocc_profile_enable(int(bool(on)))


def lnocc_profile_collect() -> dict:
    arr = (lnocc_kernel_stats_t * LNOCC_KERNEL_CLASSES)()
    _lib.lnocc_profile_collect(arr)
    return {KERNEL_CLASS_NAMES[k]: {"launches": arr[k].launches, "ms": arr[k].ms,
                                    "flops": arr[k].flops} for k in range(LNOCC_KERNEL_CLASSES)}


def lnocc_set_validation_mode(on: bool) -> None:
    _lib.lnocc_set_validation_mode(int(bool(on)))


def lnocc_mlp_workspace_bytes(rows: int, training: bool) -> tuple[int, int]:
    out = C.c_size_t(0)
    st = _lib.lnocc_mlp_workspace_bytes(int(rows), int(bool(training)), C.byref(out))
    return st, out.value


def lnocc_mlp_samples(frag: lnocc_fragment_t, opt: lnocc_options_t, idx_ptr: int, n: int,
                      x_ptr: int, y_ptr: int | None) -> int:
    return _lib.lnocc_mlp_samples(C.byref(frag), C.byref(opt), idx_ptr, n, x_ptr, y_ptr)


def lnocc_mlp_init(blob_ptr: int, x_ptr: int, y_ptr: int, n: int, seed: int,
                   opt: lnocc_options_t) -> int:
    return _lib.lnocc_mlp_init(blob_ptr, x_ptr, y_ptr, n, seed, C.byref(opt))


def lnocc_mlp_predict(blob_ptr: int, x_ptr: int, n: int, out_ptr: int, opt: lnocc_options_t) -> int:
    return _lib.lnocc_mlp_predict(blob_ptr, x_ptr, n, out_ptr, C.byref(opt))


def lnocc_mlp_loss_grad(blob_ptr: int, x_ptr: int, y_ptr: int, n: int, grad_ptr: int,
                        opt: lnocc_options_t) -> tuple[int, float]:
    loss = C.c_double(0.0)
    st = _lib.lnocc_mlp_loss_grad(blob_ptr, x_ptr, y_ptr, n, grad_ptr, C.byref(loss), C.byref(opt))
    return st, loss.value


def lnocc_mlp_train(blob_ptr: int, adam_ptr: int, step0: int, nsteps: int, x_ptr: int,
                    y_ptr: int, n: int, batch: int, lr: float, seed: int,
                    opt: lnocc_options_t, want_losses: bool = True) -> tuple[int, list]:
    losses = (C.c_double * max(1, nsteps))() if want_losses else None
    st = _lib.lnocc_mlp_train(blob_ptr, adam_ptr, step0, nsteps, x_ptr, y_ptr, n, batch, lr, seed,
                              losses, C.byref(opt))
    return st, (list(losses)[:nsteps] if want_losses else [])


def lnocc_local_space_workspace_bytes(sys: lnocc_system_t, nlo: int, cbno: bool) -> tuple[int, int]:
    out = C.c_size_t(0)
    st = _lib.lnocc_local_space_workspace_bytes(C.byref(sys), nlo, int(bool(cbno)), C.byref(out))
    return st, out.value


def lnocc_local_space(sys: lnocc_system_t, sp: lnocc_local_space_t, workspace: int,
                      workspace_bytes: int, stream: int = 0) -> int:
    return _lib.lnocc_local_space(C.byref(sys), C.byref(sp), workspace, workspace_bytes, stream)


def lnocc_local_hamiltonian_workspace_bytes(sys: lnocc_system_t, n_occ: int,
                                            n_vir: int) -> tuple[int, int]:
    out = C.c_size_t(0)
    st = _lib.lnocc_local_hamiltonian_workspace_bytes(C.byref(sys), n_occ, n_vir, C.byref(out))
    return st, out.value


def lnocc_local_hamiltonian(sys: lnocc_system_t, C_occ: int | None, n_occ: int,
                            C_vir: int | None, n_vir: int, B: int, workspace: int,
                            workspace_bytes: int, stream: int = 0) -> int:
    return _lib.lnocc_local_hamiltonian(C.byref(sys), C_occ, n_occ, C_vir, n_vir, B, workspace,
                                        workspace_bytes, stream)


def lnocc_mp2_workspace_bytes(frag: lnocc_fragment_t) -> tuple[int, int]:
    out = C.c_size_t(0)
    st = _lib.lnocc_mp2_workspace_bytes(C.byref(frag), C.byref(out))
    return st, out.value


def lnocc_fragment_mp2(frag: lnocc_fragment_t, opt: lnocc_options_t) -> int:
    return _lib.lnocc_fragment_mp2(C.byref(frag), C.byref(opt))


def lnocc_mp2_composite(e_mp2_full: float, e_mp2_fragments) -> float:
    arr = (C.c_double * max(1, len(e_mp2_fragments)))(*e_mp2_fragments)
    return _lib.lnocc_mp2_composite(e_mp2_full, arr, len(e_mp2_fragments))


# ------------------------------------------------------------ torch helpers
@dataclasses.dataclass
class Result:
    status: int
    e_mp2: float
    e_ccsd: float
    e_t: float
    n_iter: int
    residual: float
    t1: object
    t2: object
    guess_used: int = 0


def _torch():
    import torch
    return torch


def _stream_handle(torch):
    return torch.cuda.current_stream().cuda_stream


def make_fragment_struct(B, eps_occ, eps_vir, t1, t2, conv_tol: float) -> lnocc_fragment_t:
    f = lnocc_fragment_t()
    f.nocc, f.nvir, f.naux = eps_occ.numel(), eps_vir.numel(), B.shape[0]
    f.B, f.eps_occ, f.eps_vir = B.data_ptr(), eps_occ.data_ptr(), eps_vir.data_ptr()
    f.conv_tol = conv_tol
    f.t1 = t1.data_ptr() if t1 is not None else None
    f.t2 = t2.data_ptr() if t2 is not None else None
    return f


def make_options(precision: str = "fp64", do_triples: bool = True, max_iter: int = 100,
                 diis_space: int = 16, diis_start: int = 1, guess: int = LNOCC_GUESS_MP2,
                 ladder_chunk_bytes: int = 0, triples_batch: int = 0,
                 level_shift: float = 0.0, batch_slots: int = 0,
                 batch_streams: int = 0, mlp=None, ladder: str = "auto",
                 graphs: bool = True, autotune: bool = False, tune_cache=None,
                 on_iter=None) -> lnocc_options_t:
    """Options struct.  on_iter, if given, is called as on_iter(fragment_index, it,
    energy, residual) after every CCSD iteration, where fragment_index counts the
    fragments of the call's array; tune_cache is a plan-file path."""
    opt = lnocc_default_options()
    opt.precision = PRECISIONS[precision]
    opt.do_triples = int(do_triples)
    opt.max_iter = max_iter
    opt.diis_space = diis_space
    opt.diis_start = diis_start
    opt.guess = guess
    opt.ladder_chunk_bytes = ladder_chunk_bytes
    opt.triples_batch = triples_batch
    opt.level_shift = level_shift
    opt.batch_slots = batch_slots
    opt.batch_streams = batch_streams
    opt.ladder_mode = LADDER_MODES[ladder]
    opt.graphs = int(bool(graphs))
    opt.autotune = int(bool(autotune))
    if tune_cache is not None:
        opt.tune_cache = str(tune_cache).encode()
    if on_iter is not None:
        def _tramp(frag, it, e, r, user, _cb=on_iter):
            # the fragment's position in the call's array: its address relative to
            # the first element, registered in opt.user
            base = user or 0
            _cb((C.addressof(frag.contents) - base) // C.sizeof(lnocc_fragment_t), it, e, r)
        opt.on_iter = lnocc_iter_fn(_tramp)
    if mlp is not None:
        opt.mlp = mlp if isinstance(mlp, int) else mlp.data_ptr()
    return opt


class Workspace:
    """A torch-allocated device buffer that grows on demand."""

    def __init__(self, device="cuda"):
        self.device = device
        self.buf = None

    def ensure(self, nbytes: int):
        torch = _torch()
        if self.buf is None or self.buf.numel() < nbytes:
            self.buf = None
            self.buf = torch.empty(max(nbytes, 256), dtype=torch.uint8, device=self.device)
        return self.buf

    def attach(self, frags, opt: lnocc_options_t):
        st, nbytes = lnocc_workspace_bytes(frags, opt)
        if st != LNOCC_OK:
            raise ValueError(lnocc_status_string(st))
        buf = self.ensure(nbytes)
        opt.workspace = buf.data_ptr()
        opt.workspace_bytes = buf.numel()
        opt.stream = _stream_handle(_torch())
        return opt


def solve(B, eps_occ, eps_vir, *, conv_tol=1e-8, t1=None, t2=None, workspace=None, **kw) -> Result:
    """Fragment CCSD(T) on device tensors (FP64). Returns energies and amplitudes."""
    torch = _torch()
    o, v = eps_occ.numel(), eps_vir.numel()
    if t1 is None:
        t1 = torch.empty((o, v), dtype=torch.float64, device=B.device)
    if t2 is None:
        t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=B.device)
    opt = make_options(**kw)
    f = make_fragment_struct(B, eps_occ, eps_vir, t1, t2, conv_tol)
    if opt.on_iter:
        opt.user = C.addressof(f)
    ws = workspace or Workspace(B.device)
    ws.attach([f], opt)
    st = lnocc_fragment_ccsd(f, opt)
    return Result(st, f.e_mp2, f.e_ccsd, f.e_t, f.n_iter, f.residual, t1, t2, f.guess_used)


def solve_batch(fragments, *, conv_tol=1e-8, workspace=None, **kw) -> list[Result]:
    """lnocc_batch_solve over [(B, eps_occ, eps_vir), ...] device tensors (FP64).
    Allocates the amplitudes; returns one Result per fragment, in input order."""
    torch = _torch()
    amps = []
    arr = (lnocc_fragment_t * len(fragments))()
    for k, (B, eo, ev) in enumerate(fragments):
        o, v = eo.numel(), ev.numel()
        t1 = torch.empty((o, v), dtype=torch.float64, device=B.device)
        t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=B.device)
        amps.append((t1, t2))
        arr[k] = make_fragment_struct(B, eo, ev, t1, t2, conv_tol)
    opt = make_options(**kw)
    if opt.on_iter:
        opt.user = C.addressof(arr)
    ws = workspace or Workspace(fragments[0][0].device)
    ws.attach(list(arr), opt)
    lnocc_batch_solve(arr, opt)
    return [Result(arr[k].status, arr[k].e_mp2, arr[k].e_ccsd, arr[k].e_t, arr[k].n_iter,
                   arr[k].residual, *amps[k], arr[k].guess_used) for k in range(len(fragments))]


# ------------------------------------------------------------ local active spaces
@dataclasses.dataclass
class ActiveSpace:
    status: int
    C_occ: object        # [nocc, n_occ] active occupied orbitals on the canonical ones
    eps_occ: object      # [n_occ]
    C_vir: object        # [nvir, n_vir]
    eps_vir: object      # [n_vir]
    lambda_occ: object   # external occupied eigenvalues, descending |lambda|
    lambda_vir: object
    U_act: object        # [n_occ, nlo] the fragment's LOs on the active occupied orbitals
    n_int_occ: int
    n_int_vir: int


def make_system_struct(Lao, Cmo, eps_occ, eps_vir) -> lnocc_system_t:
    s = lnocc_system_t()
    s.nocc, s.nvir, s.naux = eps_occ.numel(), eps_vir.numel(), Lao.shape[0]
    s.Lao, s.C = Lao.data_ptr(), Cmo.data_ptr()
    s.eps_occ, s.eps_vir = eps_occ.data_ptr(), eps_vir.data_ptr()
    return s


def local_space(Lao, Cmo, eps_occ, eps_vir, U_occ, U_vir=None, *, eta_occ=0.0, eta_vir=0.0,
                cbno=False, workspace=None) -> ActiveSpace:
    """lnocc_local_space on device tensors (FP64); returns views of the active
    columns."""
    torch = _torch()
    dev = Lao.device
    sysd = make_system_struct(Lao, Cmo, eps_occ, eps_vir)
    no, nv = sysd.nocc, sysd.nvir
    nlo = U_occ.shape[1]
    sp = lnocc_local_space_t()
    sp.U_occ = U_occ.data_ptr()
    sp.U_vir = U_vir.data_ptr() if U_vir is not None else None
    sp.nlo, sp.cbno, sp.eta_occ, sp.eta_vir = nlo, int(bool(cbno)), eta_occ, eta_vir
    f64 = dict(dtype=torch.float64, device=dev)
    Co, Cv = torch.zeros((no, no), **f64), torch.zeros((nv, nv), **f64)
    eo, ev = torch.zeros(no, **f64), torch.zeros(nv, **f64)
    lo, lv = torch.zeros(no, **f64), torch.zeros(nv, **f64)
    sp.C_occ, sp.eps_occ, sp.C_vir, sp.eps_vir = (Co.data_ptr(), eo.data_ptr(), Cv.data_ptr(),
                                                  ev.data_ptr())
    sp.lambda_occ, sp.lambda_vir = lo.data_ptr(), lv.data_ptr()
    Ua = torch.zeros((no, nlo), **f64)
    sp.U_act = Ua.data_ptr()
    st, nbytes = lnocc_local_space_workspace_bytes(sysd, nlo, cbno)
    if st != LNOCC_OK:
        raise ValueError(lnocc_status_string(st))
    ws = (workspace or Workspace(dev)).ensure(nbytes)
    st = lnocc_local_space(sysd, sp, ws.data_ptr(), ws.numel(), _stream_handle(torch))
    if st < 0:
        raise RuntimeError(f"lnocc_local_space: {lnocc_status_string(st)} {lnocc_last_error()}")
    return ActiveSpace(st, Co[:, :sp.n_occ], eo[:sp.n_occ], Cv[:, :sp.n_vir], ev[:sp.n_vir],
                       lo[:no - sp.n_int_occ], lv[:nv - sp.n_int_vir], Ua[:sp.n_occ],
                       sp.n_int_occ, sp.n_int_vir)


def local_hamiltonian(Lao, Cmo, eps_occ, eps_vir, C_occ, C_vir, workspace=None):
    """lnocc_local_hamiltonian: B [naux, na, na] of the active orbitals C_occ
    [nocc, n_occ] and C_vir [nvir, n_vir] (copied into the [nocc][nocc] /
    [nvir][nvir] arrays the C call reads)."""
    torch = _torch()
    dev = Lao.device
    sysd = make_system_struct(Lao, Cmo, eps_occ, eps_vir)
    no, nv = sysd.nocc, sysd.nvir
    n_occ, n_vir = C_occ.shape[1], C_vir.shape[1]
    Co = torch.zeros((no, no), dtype=torch.float64, device=dev)
    Cv = torch.zeros((nv, nv), dtype=torch.float64, device=dev)
    Co[:, :n_occ] = C_occ
    Cv[:, :n_vir] = C_vir
    na = n_occ + n_vir
    B = torch.empty((sysd.naux, na, na), dtype=torch.float64, device=dev)
    st, nbytes = lnocc_local_hamiltonian_workspace_bytes(sysd, n_occ, n_vir)
    if st != LNOCC_OK:
        raise ValueError(lnocc_status_string(st))
    ws = (workspace or Workspace(dev)).ensure(nbytes)
    st = lnocc_local_hamiltonian(sysd, Co.data_ptr(), n_occ, Cv.data_ptr(), n_vir, B.data_ptr(),
                                 ws.data_ptr(), ws.numel(), _stream_handle(torch))
    if st != LNOCC_OK:
        raise RuntimeError(f"lnocc_local_hamiltonian: {lnocc_status_string(st)} {lnocc_last_error()}")
    return B


def fragment_mp2(B, eps_occ, eps_vir, *, want_t2=True, workspace=None):
    """lnocc_fragment_mp2: (E_MP2, t2 or None)."""
    torch = _torch()
    o, v = eps_occ.numel(), eps_vir.numel()
    t2 = torch.empty((o, o, v, v), dtype=torch.float64, device=B.device) if want_t2 else None
    f = make_fragment_struct(B, eps_occ, eps_vir, None, t2, 1e-8)
    st, nbytes = lnocc_mp2_workspace_bytes(f)
    if st != LNOCC_OK:
        raise ValueError(lnocc_status_string(st))
    opt = make_options()
    ws = (workspace or Workspace(B.device)).ensure(nbytes)
    opt.workspace, opt.workspace_bytes = ws.data_ptr(), ws.numel()
    opt.stream = _stream_handle(torch)
    st = lnocc_fragment_mp2(f, opt)
    if st != LNOCC_OK:
        raise RuntimeError(f"lnocc_fragment_mp2: {lnocc_status_string(st)} {lnocc_last_error()}")
    return f.e_mp2, t2
