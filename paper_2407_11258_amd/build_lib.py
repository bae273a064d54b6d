"""Compiles liblnocc.so (HIP, gfx950) in place with hipcc.

Usage: python -m paper_2407_11258_amd.build_lib   (or call build()).
Objects go to paper_2407_11258_amd/_build/, the library to
paper_2407_11258_amd/liblnocc.so.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import pathlib
import shutil
import subprocess

PKG = pathlib.Path(__file__).resolve().parent
SRC = PKG / "csrc"
OUT = PKG / "_build"
LIB = PKG / "liblnocc.so"
SOURCES = ["gett.hip", "kernels.hip", "triples.hip", "pairs.hip", "mlp.hip", "lno.hip", "solver.hip",
           "abi.hip", "abi_lno.hip"]

# -packed-fp32-ops: no v_pk_*_f32 generation (see the numerics notes of the design).
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found; ROCm is required to build liblnocc")
    return exe


# Host-sanitized variant for the CPU checks of the ABI (validation mode runs
# every host code path without a device): AddressSanitizer and UBSan on the
# host code only; the device code is built as usual.
SAN_OUT = PKG / "_build_asan"
SAN_LIB = PKG / "liblnocc_asan.so"
SAN_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: pathlib.Path, obj: pathlib.Path, flags) -> None:
    cmd = [hipcc(), *flags, "-c", str(src), "-o", str(obj)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src.name}:\n{r.stderr}")


def _build(out: pathlib.Path, lib: pathlib.Path, flags, link_flags, jobs: int) -> pathlib.Path:
    out.mkdir(exist_ok=True)
    objs = [out / (s.replace(".hip", ".o")) for s in SOURCES]
    with cf.ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda so: _compile(SRC / so[0], so[1], flags), zip(SOURCES, objs)))
    tmp = lib.with_suffix(".so.tmp")
    cmd = [hipcc(), "--offload-arch=gfx950", "-shared", "-fPIC", *link_flags, *map(str, objs),
           "-o", str(tmp)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed:\n{r.stderr}")
    os.replace(tmp, lib)
    return lib


def build(jobs: int = 4) -> pathlib.Path:
    return _build(OUT, LIB, FLAGS, [], jobs)


def build_sanitized(jobs: int = 4) -> pathlib.Path:
    flags = [f for f in FLAGS if f != "-O3"] + ["-O1", "-g"] + SAN_HOST
    return _build(SAN_OUT, SAN_LIB, flags, SAN_HOST[:4] + ["-shared-libsan"], jobs)


def sanitizer_runtime() -> pathlib.Path | None:
    """The compiler's AddressSanitizer runtime (preloaded by the sanitized checks)."""
    for c in sorted(pathlib.Path("/opt/rocm").glob("lib/llvm/lib/clang/*/lib/linux/"
                                                  "libclang_rt.asan-x86_64.so")):
        return c
    return None


if __name__ == "__main__":
    print(build())
    print(build_sanitized())
