"""GPU: the progress callback and the plan-file option of lnocc_options_t.

The callback is called once per CCSD iteration of every fragment, with that
fragment's step norm (its last call carries the residual the solve reports) and
the CCSD energy of the amplitudes entering the iteration (E_MP2 at the first);
the plan file is written after a call whose autotuning added plans and read by
a later call.
"""
import sys

import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from paper_2407_11258_amd import lnocc as L  # noqa: E402
from synth import make_fragment  # noqa: E402

DEV = "cuda:0"


def say(msg):
    print(f"[gpu-case] {msg}", file=sys.stderr, flush=True)


def _on_device(f):
    return tuple(torch.tensor(x, dtype=torch.float64, device=DEV)
                 for x in (f.B, f.eps_occ, f.eps_vir))


def test_progress_callback_single_fragment():
    say("on_iter, single fragment (4, 20, 72)")
    calls = []
    r = L.solve(*_on_device(make_fragment(4, 20, 72, 40)), conv_tol=1e-9,
                on_iter=lambda k, it, e, res: calls.append((k, it, e, res)))
    assert r.status == L.LNOCC_OK
    assert [c[1] for c in calls] == list(range(1, r.n_iter + 1))
    assert all(c[0] == 0 for c in calls)
    assert calls[0][2] == r.e_mp2
    assert calls[-1][3] == r.residual
    assert all(res > 1e-9 for _, _, _, res in calls[:-1])
    assert abs(calls[-1][2] - r.e_ccsd) < 1e-8


def test_progress_callback_batch():
    shapes = [(4, 20, 72, 40), (2, 13, 45, 41), (5, 26, 93, 42)]
    say("on_iter, batch of 3 over 2 streams")
    frags = [_on_device(make_fragment(*s)) for s in shapes]
    calls = {}
    res = L.solve_batch(frags, conv_tol=1e-9, batch_slots=2, batch_streams=2,
                        on_iter=lambda k, it, e, r: calls.setdefault(k, []).append((it, r)))
    for k, r in enumerate(res):
        assert r.status == L.LNOCC_OK
        assert [it for it, _ in calls[k]] == list(range(1, r.n_iter + 1))
        assert calls[k][-1][1] == r.residual


def test_tune_cache_written_and_read(tmp_path):
    path = tmp_path / "plans.txt"
    frag = _on_device(make_fragment(4, 20, 72, 40))
    L.lnocc_autotune_clear()
    try:
        say("tune_cache: autotuned solve writes the plan file")
        r = L.solve(*frag, autotune=True, tune_cache=path)
        assert r.status == L.LNOCC_OK
        lines = path.read_text().splitlines()
        assert lines and all(len(x.split()) == 3 for x in lines)
        say(f"  {len(lines)} plans; a fresh process state reads them back")
        L.lnocc_autotune_clear()
        r2 = L.solve(*frag, tune_cache=path)
        assert r2.status == L.LNOCC_OK
        again = tmp_path / "again.txt"
        assert L.lnocc_autotune_save(again) == len(lines)
        assert sorted(again.read_text().splitlines()) == sorted(lines)
        assert abs(r2.e_ccsd - r.e_ccsd) < 1e-12
    finally:
        L.lnocc_autotune_clear()
