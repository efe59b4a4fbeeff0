"""Builds libblm.so (all HIP sources under csrc/) for gfx950 with hipcc.

Usage: python -m paper_1702_01481_amd.build_lib   (or build() from Python)
       python -m paper_1702_01481_amd.build_lib --sanitize   (libblm_san.so, host code under ASan/UBSan)
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


# host code under AddressSanitizer and UndefinedBehaviorSanitizer (device
# code is built as usual): a CPU check of the library's host logic, loaded
# by a Python started with the sanitizer runtime preloaded and
# BLM_LIBRARY pointing at it
SAN_LIB = os.path.join(HERE, "libblm_san.so")
SAN_FLAGS = ["-O1", "-g", "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
             "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined",
             "-shared-libsan"]


def asan_runtime() -> str:
    """Path of the sanitizer runtime to preload (clang's, which hipcc links against)."""
    out = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    path = out.stdout.strip()
    if not os.path.isabs(path) or not os.path.exists(path):
        import glob
        cands = glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
        if not cands:
            raise RuntimeError("clang's AddressSanitizer runtime not found")
        path = cands[0]
    return path


def build_sanitized(verbose: bool = False) -> str:
    """libblm_san.so: the library with its host code under ASan and UBSan."""
    tmp = SAN_LIB + ".tmp"
    flags = [f for f in HIPCC_FLAGS if f != "-O3"] + SAN_FLAGS
    cmd = [hipcc(), *flags, "-I", INCLUDE, "-I", CSRC, *sources(), "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, SAN_LIB)
    return SAN_LIB


def build(verbose: bool = False) -> str:
    """Compiles every HIP source of csrc/ into libblm.so, and the sample
    generator into synthgen/libsynthgen.so; returns libblm's path."""
    _compile(sources(), LIB, [INCLUDE, CSRC], verbose)
    _compile([SYNTHGEN_SRC], SYNTHGEN_LIB, [], verbose)
    return LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_sanitized(verbose="-v" in sys.argv))
    else:
        build(verbose="-v" in sys.argv)
        print(LIB)
