"""GPU: the batched solve (several fragments in flight, on the caller's
stream or spread over streams of their own) against one-at-a-time solves and
the FP64 oracle.

Each fragment of a batch runs the same kernels with the same launch shapes as
a lone lnocc_fragment_ccsd call, so results must agree bit for bit; energies
against the oracle follow the single-fragment tolerances (1e-8 Eh at FP64,
1e-6 Eh with FP32 ladder and (T) products).
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2407_11258_amd import lnocc as L  # noqa: E402
from oracle import ccsd as occ, triples as otr  # noqa: E402
from synth import make_fragment  # noqa: E402

DEV = "cuda:0"
SHAPES = [(4, 20, 72, 40), (2, 13, 45, 41), (5, 26, 93, 42), (3, 31, 102, 43), (1, 9, 30, 44),
          (6, 17, 69, 45), (4, 38, 126, 46)]


def say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def _on_device(f):
    return tuple(torch.tensor(x, dtype=torch.float64, device=DEV)
                 for x in (f.B, f.eps_occ, f.eps_vir))


@pytest.mark.parametrize("slots,streams", [(3, 0), (8, 0), (3, 3), (8, 4)])
def test_batch_equals_one_at_a_time(slots, streams):
    say(f"batch vs sequential, {len(SHAPES)} fragments, {slots} slots, {streams} streams")
    frags = [make_fragment(*s) for s in SHAPES]
    dev = [_on_device(f) for f in frags]
    batch = L.solve_batch(dev, conv_tol=1e-9, batch_slots=slots, batch_streams=streams)
    say(f"  statuses {[r.status for r in batch]} last error '{L.lnocc_last_error()}'")
    for k, (B, eo, ev) in enumerate(dev):
        one = L.solve(B, eo, ev, conv_tol=1e-9)
        b = batch[k]
        say(f"  fragment {k} {SHAPES[k][:3]}: iters {b.n_iter} status {b.status}")
        assert b.status == one.status == L.LNOCC_OK
        assert (b.e_mp2, b.e_ccsd, b.e_t, b.n_iter) == (one.e_mp2, one.e_ccsd, one.e_t, one.n_iter)
        assert torch.equal(b.t2, one.t2) and torch.equal(b.t1, one.t1)


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-8), ("fp32", 1e-6)])
def test_batch_matches_oracle(precision, tol):
    say(f"batch vs oracle {precision}")
    frags = [make_fragment(*s) for s in SHAPES[:4]]
    res = L.solve_batch([_on_device(f) for f in frags], conv_tol=1e-9, precision=precision,
                        batch_slots=4, batch_streams=2)
    say(f"  statuses {[r.status for r in res]} last error '{L.lnocc_last_error()}'")
    for f, r in zip(frags, res):
        ref = occ.ccsd(f.B, f.eps_occ, f.eps_vir, conv_tol=1e-10)
        ref_t = otr.e_triples_restricted(f.B, f.eps_occ, f.eps_vir, ref.t1, ref.t2)
        say(f"  o={f.nocc} v={f.nvir}: dE_ccsd={r.e_ccsd - ref.e_ccsd:.2e} dE_t={r.e_t - ref_t:.2e}")
        assert r.status == L.LNOCC_OK
        assert abs(r.e_mp2 - ref.e_mp2) < 1e-12
        assert abs(r.e_ccsd - ref.e_ccsd) < tol
        assert abs(r.e_t - ref_t) < tol


def test_batch_reports_per_fragment_errors():
    say("batch with a rejected fragment")
    frags = [make_fragment(*s) for s in SHAPES[:3]]
    dev = [_on_device(f) for f in frags]
    B, eo, ev = dev[1]
    bad = ev.clone()
    bad[0] = eo.max()                           # no gap: rejected on the host
    dev[1] = (B, eo, bad)
    res = L.solve_batch(dev, conv_tol=1e-8, batch_slots=2, do_triples=False)
    assert [r.status for r in res] == [L.LNOCC_OK, L.LNOCC_EINVAL, L.LNOCC_OK]
    one = L.solve(*dev[2], conv_tol=1e-8, do_triples=False)
    assert res[2].e_ccsd == one.e_ccsd and res[2].e_t == 0.0


def test_batch_workload_start_at_full_size():
    """The 64 fragments of the batched workload (nocc 6..24, nvir 60..220,
    naux = 3 (nocc + nvir)) through lnocc_batch_solve in the launch configuration
    the benchmark times (FP32 mode, 4 slots on 4 streams, graphs) with
    max_iter = 0: every fragment's MP2 energy (Eq. 7 at the MP1 amplitudes of
    Eq. 21), the energy of that start, the MP1 amplitude norm and 8 sampled
    amplitudes against oracle values stored by tests/golden/make_golden.py
    (batch:mp2)."""
    import json
    import pathlib
    path = pathlib.Path(__file__).resolve().parent / "golden" / "batch_mp2.json"
    if not path.exists():
        pytest.skip(f"{path.name} not generated")
    frs = json.loads(path.read_text())["fragments"]
    say(f"batch workload at full size: {len(frs)} fragments, MP2 start")
    dev = []
    for x in frs:
        f = make_fragment(*x["shape"])
        assert f.sha256() == x["input_sha256"]
        dev.append(_on_device(f))
    res = L.solve_batch(dev, precision="fp32", batch_slots=4, batch_streams=4, max_iter=0,
                        do_triples=False)
    worst = 0.0
    for k, (r, x) in enumerate(zip(res, frs)):
        assert r.status == L.LNOCC_OK, (k, x["shape"], L.lnocc_last_error())
        worst = max(worst, abs(r.e_mp2 - x["e_mp2"]))
        assert abs(r.e_mp2 - x["e_mp2"]) < 1e-10, (k, x["shape"])
        assert abs(r.e_ccsd - r.e_mp2) < 1e-12
        idx = np.array(x["t2_index"])
        got = r.t2[idx[:, 0], idx[:, 1], idx[:, 2], idx[:, 3]].cpu().numpy()
        np.testing.assert_allclose(got, x["t2_value"], rtol=0, atol=1e-13)
        assert abs(float(torch.linalg.vector_norm(r.t2)) - x["t2_norm"]) < 1e-12 * x["t2_norm"]
    say(f"  worst |dE_mp2| {worst:.1e}")
    del dev, res
    torch.cuda.empty_cache()
