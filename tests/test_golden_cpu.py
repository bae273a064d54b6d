"""Stored oracle values (tests/golden/*.json, written by make_golden.py from
oracle/ only) are reproduced by the oracle as it stands, and describe the
inputs the generator draws today."""
import json
import pathlib

import numpy as np
import pytest

from synth import CONFIG_SHAPES, make_fragment

GOLDEN = pathlib.Path(__file__).resolve().parent / "golden"


def test_small_golden_is_reproduced():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", GOLDEN / "make_golden.py")
    mg = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mg)
    stored = json.loads((GOLDEN / "single_small.json").read_text())
    fresh = mg.golden("single_small")
    for key in ("input_sha256", "n_iter"):
        assert fresh[key] == stored[key]
    for key in ("e_mp2", "e_ccsd", "e_t", "t1_norm", "t2_norm"):
        assert abs(fresh[key] - stored[key]) < 1e-12, key
    np.testing.assert_allclose(fresh["t2_value"], stored["t2_value"], atol=1e-12, rtol=0)


@pytest.mark.parametrize("name", ["single_small", "single_realistic"])
def test_golden_inputs_match_generator(name):
    path = GOLDEN / f"{name}.json"
    if not path.exists():
        pytest.skip(f"{path.name} not generated")
    g = json.loads(path.read_text())
    o, v, X, seed = CONFIG_SHAPES[name]
    assert (g["nocc"], g["nvir"], g["naux"], g["seed"]) == (o, v, X, seed)
    assert make_fragment(o, v, X, seed).sha256() == g["input_sha256"]
    assert g["converged"]
