"""Build of the HIP library libfstat.so (gfx950), in-tree beside this file.

    python -m paper_1003_0844_amd._build

compiles every source under csrc/ with hipcc into one shared object.  Packed
FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libfstat.so")
SOURCES = ["api.hip", "sky.hip", "grid.hip", "prep.hip", "grad.hip", "search.hip", "probe.hip", "grad_static.hip", "persist.hip", "lattice.cpp"]
ARCH = os.environ.get("FSTAT_OFFLOAD_ARCH", "gfx950")


def _hipcc() -> str:
    for c in (os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "bin", "hipcc"), "hipcc"):
        if os.path.sep not in c or os.path.exists(c):
            return c
    return "hipcc"


def common_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


def build_library(verbose: bool = False) -> str:
    os.makedirs(os.path.join(HERE, "_objs"), exist_ok=True)
    hipcc = _hipcc()

    def compile_one(src):
        obj = os.path.join(HERE, "_objs", os.path.splitext(src)[0] + ".o")
        if src.endswith(".cpp"):   # host-only C++
            cmd = [hipcc, "-x", "c++", "-O3", "-std=c++17", "-fPIC", "-I" + os.path.join(ROOT, "include"),
                   "-I" + CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
        else:
            cmd = [hipcc, *common_flags(), "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr[-6000:]))
        if verbose and r.stderr.strip():
            print(r.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
