"""Host code under AddressSanitizer and UBSan: the CPU ABI checks
(tests/test_abi_cpu.py: argument validation, struct layouts, and every launch
sequence in validation mode, where every host code path runs without a device)
repeated in a child process against liblnocc_asan.so, the build with the
host code sanitized, with the sanitizer runtime preloaded.  Any report aborts
the child (halt_on_error) and fails this test."""
import os
import pathlib
import subprocess
import sys

import pytest

from paper_2407_11258_amd import build_lib

ROOT = pathlib.Path(__file__).resolve().parent.parent


def test_abi_checks_under_sanitizers():
    rt = build_lib.sanitizer_runtime()
    if not build_lib.SAN_LIB.exists() or rt is None:
        pytest.skip("liblnocc_asan.so not built (build_lib.build_sanitized())")
    env = dict(os.environ)
    env.update(LNOCC_LIBRARY=str(build_lib.SAN_LIB), LD_PRELOAD=str(rt),
               ASAN_OPTIONS="detect_leaks=0:alloc_dealloc_mismatch=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu", str(ROOT / "tests" / "test_abi_cpu.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout, tail
