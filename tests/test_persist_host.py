"""The persistent launch's work queue on the CPU: the library's schedule
(csrc/persist_sched.h) of a three-segment call is checked to be in dependency
order, and a threaded emulation of the kernel's claim / wait / signal logic
runs every tile exactly once, for several workgroup counts, spill-slot
counts and claim sizes (no GPU).  The emulation is built with the host sanitizers (AddressSanitizer,
UndefinedBehaviorSanitizer) over the schedule code."""
import os
import subprocess

import pytest

from paper_1003_0844_amd import _build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("emu") / "persist_queue_emu")
    hipcc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc")
    cmd = [hipcc, "-O1", "-std=c++17", *_build.SANITIZE_HOST, "-I" + os.path.join(ROOT, "include"),
           "-I" + os.path.join(ROOT, "paper_1003_0844_amd", "csrc"), os.path.join(ROOT, "tests", "persist_queue_emu.hip"),
           "-o", exe, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    return exe


@pytest.mark.parametrize("threads,slots,chunk", [(16, 3, 1), (64, 8, 1), (768, 8, 1), (256, 5, 4), (100, 3, 16),
                                                 (768, 32, 16), (768, 8, 64), (33, 4, 8)])
def test_queue_runs_every_tile_once(emu, threads, slots, chunk):
    r = subprocess.run([emu, str(threads), str(slots), str(chunk)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ordered 1" in r.stdout
    assert "error 0, items never run 0, run twice 0, bad tiles 0" in r.stdout, r.stdout
