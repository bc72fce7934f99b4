"""The host-side setup code (CSR to stencil, Galerkin coarsening, boundary
classes, dense coarse inverse, LDU coefficient matrices) under
AddressSanitizer and UndefinedBehaviorSanitizer: the host-library tests of
``test_host_abi.py`` run in a child process against ``libirk_host_asan.so``
(g++ -fsanitize=address,undefined, built by ``build()``), with the ASan
runtime preloaded; any report aborts the child."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ASAN_LIB = os.path.join(ROOT, "paper_2010_11377_amd", "libirk_host_asan.so")


def _runtime():
    try:
        p = subprocess.run(["g++", "-print-file-name=libasan.so"], capture_output=True, text=True,
                           check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_host_setup_under_sanitizers():
    rt = _runtime()
    if rt is None or not os.path.exists(ASAN_LIB):
        pytest.skip("sanitizer runtime or libirk_host_asan.so missing")
    with open(ASAN_LIB, "rb") as f:
        assert b"__asan_report" in f.read(), "the sanitized library is not instrumented"
    env = dict(os.environ, IRK_HOST_TEST_LIB=ASAN_LIB, LD_PRELOAD=rt,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_host_abi.py"), "-q",
           "-p", "no:cacheprovider", "-k",
           "stencil or galerkin or classes or dense_inverse or coefficient"]
    p = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    out = p.stdout + p.stderr
    assert p.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out and " skipped" not in out, out[-2000:]
