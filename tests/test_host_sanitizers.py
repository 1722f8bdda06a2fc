"""Host code of liblens.so under AddressSanitizer and UndefinedBehaviorSanitizer.

Opt-in (LENS_SANITIZE=1; the instrumented build takes a few minutes):
builds liblens_asan.so (host code instrumented, device code as usual), then
runs the host-only tests of the ABI and the binding -- descriptor checks,
null and mis-sized arguments of every entry point, rejected arrays -- in a
subprocess with the sanitizer runtime preloaded and LENS_LIB pointing at
that library.  No call there reaches the GPU; paths past validation are
covered by the GPU parity tests instead.
"""
import glob
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.skipif(os.environ.get("LENS_SANITIZE") != "1",
                                reason="opt-in host sanitizer run: LENS_SANITIZE=1")

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _asan_runtime():
    found = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not found:
        pytest.skip("no clang AddressSanitizer runtime under /opt/rocm/llvm")
    return found[-1]


def test_host_validation_clean_under_asan_and_ubsan():
    from paper_2606_30633_amd import build as B
    lib = B.build_library(force=False, sanitize=True)
    env = dict(os.environ, LD_PRELOAD=_asan_runtime(), LENS_LIB=lib, LENS_SANITIZE="0",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_abi.py", "tests/test_binding_checks.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    report = r.stdout[-4000:] + r.stderr[-4000:]
    assert r.returncode == 0, report
    assert "AddressSanitizer" not in r.stderr and "runtime error:" not in r.stderr, report
    assert " passed" in r.stdout, report
