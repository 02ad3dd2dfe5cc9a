"""Build the HIP library libinla_bta.so for gfx950 in place (hipcc, no JIT cache)."""
from __future__ import annotations

import glob
import hashlib
import os
import shutil
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libinla_bta.so")
SOURCES = ["bta_kernels.hip", "model_kernels.hip", "engine.cpp", "optimizer.cpp", "integrate.cpp", "nongauss.cpp"]
ARCH = os.environ.get("INLA_OFFLOAD_ARCH", "gfx950")


def source_files() -> list[str]:
    """Every file the library is compiled from: the sources, the internal
    headers and the public header."""
    files = [os.path.join(CSRC, s) for s in SOURCES]
    files += sorted(glob.glob(os.path.join(CSRC, "*.h")))
    files.append(os.path.join(ROOT, "include", "inla_bta.h"))
    return files


def source_hash() -> str:
    """SHA-256 (first 16 hex digits) over the library's source files, in a
    fixed order, with their names: the build id the library reports through
    inla_build_id() and the binding checks before any call."""
    h = hashlib.sha256()
    for path in source_files():
        h.update(os.path.basename(path).encode() + b"\0")
        with open(path, "rb") as fh:
            h.update(fh.read())
        h.update(b"\0")
    return h.hexdigest()[:16]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_command(out: str = LIB) -> list[str]:
    return [
        hipcc(), f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
        # keep packed FP32 instructions out of the generated code
        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
        "-I" + os.path.join(ROOT, "include"),
        f'-DINLA_SOURCE_HASH="{source_hash()}"',
        *[os.path.join(CSRC, s) for s in SOURCES],
        "-o", out,
    ]


def build(verbose: bool = False) -> str:
    """Compile every source into libinla_bta.so (always recompiles)."""
    tmp = LIB + ".tmp"
    cmd = compile_command(tmp)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + res.stdout + res.stderr)
    if verbose:
        print(" ".join(cmd))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
