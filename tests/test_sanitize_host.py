"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer,
on the CPU: the library is rebuilt with host-side instrumentation
(_build.build_library(sanitize=True); device code unchanged), and the host-level
tests -- argument validation of every entry point, the lattice construction and
enumeration, the detection threshold -- run against it in a child process with
the sanitizer runtime preloaded.  Any report aborts the child."""
import os
import subprocess
import sys

import pytest

from paper_1003_0844_amd import _build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

pytestmark = pytest.mark.slow


@pytest.fixture(scope="module")
def sanitized_lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("san") / "libfstat_san.so")
    return _build.build_library(sanitize=True, out=out)


def test_host_code_is_clean_under_asan_and_ubsan(sanitized_lib):
    env = dict(os.environ)
    env.update(LD_PRELOAD=_build.sanitizer_runtime(), FSTAT_LIBRARY=sanitized_lib,
               ASAN_OPTIONS="detect_leaks=0:verify_asan_link_order=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    check = ("import ctypes; from paper_1003_0844_amd import fstat; L = fstat.lib(); "
             "assert fstat.LIB_PATH == %r; "
             "ctypes.CDLL(None).__asan_init; print('sanitized library loaded')" % sanitized_lib)
    r = subprocess.run([sys.executable, "-c", check], cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "sanitized library loaded" in r.stdout, r.stdout + r.stderr[-3000:]
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu",
                        "tests/test_abi.py", "tests/test_lattice_host.py", "tests/test_search_host.py"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = r.stdout[-3000:] + r.stderr[-3000:]
    assert r.returncode == 0, tail
    assert "passed" in r.stdout and "ERROR: AddressSanitizer" not in tail and "runtime error" not in tail, tail
