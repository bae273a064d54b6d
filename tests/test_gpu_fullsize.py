"""GPU: full-size workloads against stored oracle values.

* (T) at the large workload's virtual and auxiliary size (nvir=400, naux=1300,
  nocc=6) on seeded amplitudes, with batches of 4 triples so that the launch
  shapes of the large workload's (T) run.  The amplitudes are random (scale
  1e-2), which makes E_(T) about -113 Eh; the bound is relative: FP64 products
  1e-11 of |E|, FP32 products (FP32 rounding of the W sums over ~400 terms,
  FP64 energy sum) 1e-6 of |E|.
* fragments of the batched workload (nocc 6..24, nvir 60..214) solved through
  lnocc_batch_solve in the benchmark's configuration (4 slots on 4 streams)
  against converged oracle CCSD and (T) values: FP64 within 1e-8 Eh and 1e-7 on
  256 sampled amplitudes, FP32 within 1e-6 Eh and 1e-6.
Values come from tests/golden/make_golden.py (oracle only).
"""
import json
import pathlib
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2407_11258_amd import lnocc as L  # noqa: E402
from synth import batch_shapes, make_fragment, random_amplitudes  # noqa: E402

DEV = "cuda:0"
GOLDEN = pathlib.Path(__file__).resolve().parent / "golden"


def say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def _golden(name):
    path = GOLDEN / f"{name}.json"
    if not path.exists():
        pytest.skip(f"{path.name} not generated")
    return json.loads(path.read_text())


def dev(x):
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=DEV)


@pytest.mark.parametrize("precision,rtol", [("fp64", 1e-11), ("fp32", 1e-6)])
def test_large_virtual_triples_against_stored_oracle(precision, rtol):
    g = _golden("large_triples")
    o, v, X, seed, aseed = g["nocc"], g["nvir"], g["naux"], g["seed"], g["amplitude_seed"]
    say(f"(T) nocc={o} nvir={v} naux={X} {precision}, batches of 4 triples")
    f = make_fragment(o, v, X, seed)
    assert f.sha256() == g["input_sha256"]
    t1, t2 = random_amplitudes(o, v, aseed)
    B, eo, ev = dev(f.B), dev(f.eps_occ), dev(f.eps_vir)
    del f
    t1d, t2d = dev(t1), dev(t2)
    opt = L.make_options(precision=precision, triples_batch=4)
    fs = L.make_fragment_struct(B, eo, ev, t1d, t2d, 1e-8)
    ws = L.Workspace(DEV)
    ws.attach([fs], opt)
    st = L.lnocc_fragment_triples(fs, opt)
    assert st == L.LNOCC_OK, L.lnocc_last_error()
    d = fs.e_t - g["e_t"]
    say(f"  E_(T) {fs.e_t:.10f} oracle {g['e_t']:.10f} relative difference {abs(d) / abs(g['e_t']):.1e}")
    assert abs(d) <= rtol * abs(g["e_t"])
    del ws, B, t2d
    torch.cuda.empty_cache()


@pytest.mark.parametrize("precision,tol_e,tol_t", [("fp64", 1e-8, 1e-7), ("fp32", 1e-6, 1e-6)])
def test_batch_fragments_against_stored_oracle(precision, tol_e, tol_t):
    g = _golden("batch_ccsd")
    shapes = batch_shapes()
    frags = []
    for ent in g["fragments"]:
        o, v, X, seed = shapes[ent["index"]]
        assert (o, v, X, seed) == (ent["nocc"], ent["nvir"], ent["naux"], ent["seed"])
        f = make_fragment(o, v, X, seed)
        assert f.sha256() == ent["input_sha256"]
        frags.append((dev(f.B), dev(f.eps_occ), dev(f.eps_vir)))
    say(f"batch of {len(frags)} oracle-checked fragments, {precision}, 4 slots x 4 streams")
    conv = 1e-10 if precision == "fp64" else 1e-8
    res = L.solve_batch(frags, conv_tol=conv, precision=precision, batch_slots=4,
                        batch_streams=4, max_iter=150)
    for ent, r in zip(g["fragments"], res):
        de, dt = r.e_ccsd - ent["e_ccsd"], r.e_t - ent["e_t"]
        idx = np.array(ent["t2_index"])
        T2 = r.t2.cpu().numpy()
        damp = np.abs(T2[idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]] - ent["t2_value"]).max()
        i1 = np.array(ent["t1_index"])
        T1 = r.t1.cpu().numpy()
        damp1 = np.abs(T1[i1[:, 0], i1[:, 1]] - ent["t1_value"]).max()
        say(f"  ({ent['nocc']}, {ent['nvir']}, {ent['naux']}): status {r.status} iters {r.n_iter} "
            f"dE_CCSD {de:.1e} dE_(T) {dt:.1e} max|dT2| {damp:.1e} max|dT1| {damp1:.1e}")
        assert r.status == L.LNOCC_OK
        assert abs(r.e_mp2 - ent["e_mp2"]) < 1e-10
        assert abs(de) < tol_e and abs(dt) < tol_e
        assert damp < tol_t and damp1 < tol_t
