"""Builds libblm.so (all HIP sources under csrc/) for gfx950 with hipcc.

Usage: python -m paper_1702_01481_amd.build_lib   (or build() from Python)
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libblm.so")
# the input generator of the banded-G synthetic model (not part of libblm)
SYNTHGEN_SRC = os.path.join(HERE, "synthgen", "synth_gen.hip")
SYNTHGEN_LIB = os.path.join(HERE, "synthgen", "libsynthgen.so")

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    # no packed FP32 instructions in device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def sources():
    return sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))


def _compile(srcs, out, includes, verbose):
    tmp = out + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *[a for inc in includes for a in ("-I", inc)], *srcs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compiles every HIP source of csrc/ into libblm.so, and the sample
    generator into synthgen/libsynthgen.so; returns libblm's path."""
    _compile(sources(), LIB, [INCLUDE, CSRC], verbose)
    _compile([SYNTHGEN_SRC], SYNTHGEN_LIB, [], verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
    print(LIB)
