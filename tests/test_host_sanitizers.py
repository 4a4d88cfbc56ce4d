"""The library's host code under the address and undefined-behaviour
sanitizers (CPU only).

The host sources (plan, macro-tile plan, C API, eigen-solvers, launchers)
are built a second time with -fsanitize=address,undefined on the host side
(libdmrg_san.so), and the host tests that drive them -- the C-ABI checks
(plans, layouts, error paths, the host eigen-solvers and LDOS) and the
driver's host bookkeeping -- are run again against that build in a child
process with the sanitizer runtime preloaded; any report fails the run.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_host_code_under_sanitizers():
    from paper_0902_3185_amd import build as B
    rt = B.asan_runtime()
    if rt is None:
        pytest.skip("the compiler's address-sanitizer runtime is not installed")
    lib = B.build_sanitized()
    env = dict(os.environ, DMRG_LIB=lib, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_abi_host.py", "tests/test_driver_host.py",
                        "tests/test_driver_orchestration.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=1200)
    tail = (r.stdout[-4000:] + "\n" + r.stderr[-4000:])
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail
