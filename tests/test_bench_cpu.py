"""Host logic of bench.py: the roofline's traffic lookup (one entry per workload,
ladder path, precision and kernel class, used only while the kernel sources are
the ones it was measured on) and the refusal of more than one GPU."""
import importlib.util
import json
import pathlib
import subprocess
import sys

ROOT = pathlib.Path(__file__).resolve().parents[1]


def load_bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", ROOT / "bench.py")
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def split_prof():
    zero = {"ms": 0.0, "flops": 0.0, "launches": 0}
    return {"other": dict(zero), "triples_w": dict(zero),
            "split": {"ms": 10.0, "flops": 1e12, "launches": 40}}


def test_traffic_entries_are_kept_per_ladder_path():
    bench = load_bench()
    table = json.loads((ROOT / "profiles" / "traffic.json").read_text())
    current = bench.kernel_sources_hash()
    for wkey in ("single_realistic", "single_realistic_otf"):
        r = bench.roofline(split_prof(), "fp32", wkey)
        assert r["kernel"] == "split" and r["precision"] == "split_bf16x6"
        assert abs(r["achieved"] - 1e12 / 10.0 / 1e9) < 1e-9
        assert abs(r["frac"] - r["achieved"] / r["peak"]) < 1e-12
        ent = table.get(f"{wkey}:split_bf16x6:split")
        if ent and ent.get("sources") == current:
            assert r["traffic"] == ent["bytes_per_launch"]
        else:
            assert r["traffic"] is None
    # the two paths run different kernels: their entries must not coincide
    a = table.get("single_realistic:split_bf16x6:split")
    b = table.get("single_realistic_otf:split_bf16x6:split")
    if a and b:
        assert a["kernels"] != b["kernels"]


def test_unknown_workload_has_no_traffic():
    bench = load_bench()
    assert bench.roofline(split_prof(), "fp32", "no_such_workload")["traffic"] is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, str(ROOT / "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "--gpus 1" in r.stderr
