"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(libblm_san.so, built by build() beside libblm.so; device code as usual):
the CPU checks of the host logic (exports, configuration checks and sizing,
workspace planning, the allocation-free entry point's argument checks) run
in a child Python with the sanitizer runtime preloaded and the binding
pointed at the sanitized build.  Any report fails the child (UBSan reports
do not recover)."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def _stale(lib, srcs):
    return not os.path.exists(lib) or any(os.path.getmtime(s) > os.path.getmtime(lib) for s in srcs)


def test_host_checks_under_asan_and_ubsan():
    from paper_1702_01481_amd import build_lib
    srcs = build_lib.sources() + [os.path.join(build_lib.INCLUDE, "blm.h"),
                                  os.path.join(build_lib.CSRC, "blm_internal.h")]
    if _stale(build_lib.SAN_LIB, srcs):
        pytest.skip("libblm_san.so is missing or older than the sources: run build() first")
    env = dict(os.environ, LD_PRELOAD=build_lib.asan_runtime(), BLM_LIBRARY=build_lib.SAN_LIB,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1")
    probe = ("from paper_1702_01481_amd import blm; lib = blm.load(); "
             "assert blm.LIB_PATH.endswith('libblm_san.so') and hasattr(lib, '__asan_report_load8')")
    subprocess.run([sys.executable, "-c", probe], env=env, cwd=ROOT, check=True, timeout=300)
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_lib_cpu.py")],
                       env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    print(r.stdout[-2000:], r.stderr[-2000:])
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr
