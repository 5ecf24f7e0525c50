"""Build of the gfx950 library libslsht.so (in-tree, next to this file).

hipcc compiles the kernels for gfx950 only, with packed FP32 instructions
disabled for device code, and links the host core into one shared library
whose exported C ABI is declared in include/slsht.h.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libslsht.so")
SOURCES = ["slsht_kernels.hip", "slsht_synth.hip", "slsht_energy.hip", "slsht_slepian.hip",
           "slsht_factored.hip", "slsht_modsht.hip", "slsht_noalloc.hip", "slsht_staged.hip",
           "slsht_geom.cpp", "slsht_api.cpp", "slsht_server.cpp"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def compile_cmd(out: str = LIB, extra: list[str] | None = None) -> list[str]:
    return [hipcc(), "-O3", "--offload-arch=gfx950", "-std=c++17", "-fPIC", "-shared",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-Wno-unused-command-line-argument",
            "-I", os.path.join(ROOT, "include"),
            *[os.path.join(CSRC, s) for s in SOURCES],
            *(extra or []), "-lpthread", "-o", out]


def build(verbose: bool = False) -> str:
    """Compile libslsht.so; returns its path.  Writes to a temporary name first
    so that a failed build never leaves a half-written library behind."""
    tmp = LIB + ".tmp"
    cmd = compile_cmd(tmp)
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed with status {res.returncode}")
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
