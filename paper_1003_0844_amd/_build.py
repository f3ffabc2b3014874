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


# -ffp-contract=on: a multiply and an add are fused only within one source
# expression, so that the rounding of the shared tile code does not depend on
# the kernel it is inlined into (the persistent launch and the pass kernels
# give bit-identical maps); across statements the default would fuse as the
# surrounding code allows.
def common_flags():
    return ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=on",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


# Host-side AddressSanitizer + UndefinedBehaviorSanitizer instrumentation (the
# device code is built as usual): a CPU-only check of the library's host code.
SANITIZE_HOST = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]


def _clangxx() -> str:
    return os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib", "llvm", "bin", "clang++")


def build_library(verbose: bool = False, sanitize: bool = False, out: str = "") -> str:
    """Compile every source into LIB (or `out`).  sanitize: instrument the host
    code with AddressSanitizer and UndefinedBehaviorSanitizer (loading the
    result needs the sanitizer runtime preloaded)."""
    objdir = os.path.join(HERE, "_objs_san" if sanitize else "_objs")
    os.makedirs(objdir, exist_ok=True)
    hipcc = _hipcc()
    lib = out or LIB

    def compile_one(src):
        obj = os.path.join(objdir, os.path.splitext(src)[0] + ".o")
        if src.endswith(".cpp"):   # host-only C++
            cc = _clangxx() if sanitize else hipcc
            cmd = [cc, "-x", "c++", "-O3" if not sanitize else "-O1", "-std=c++17", "-fPIC",
                   "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-c", os.path.join(CSRC, src), "-o", obj]
            if sanitize:
                cmd[1:1] = [f.replace("-Xarch_host", "") for f in SANITIZE_HOST if f != "-Xarch_host"]
        else:
            cmd = [hipcc, *common_flags(), *(SANITIZE_HOST if sanitize else []), "-c", os.path.join(CSRC, src),
                   "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("compile failed for %s:\n%s" % (src, r.stderr[-6000:]))
        if verbose and r.stderr.strip():
            print(r.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=min(len(SOURCES), 8)) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = lib + ".tmp%d" % os.getpid()
    rocm_lib = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "lib")
    # roctx: the ranges the library marks around its calls
    libs = ["-L" + rocm_lib, "-lrocprofiler-sdk-roctx", "-Wl,-rpath," + rocm_lib]
    if sanitize:
        cmd = [_clangxx(), "-shared", "-fPIC", "-shared-libasan", "-fsanitize=address,undefined", *objs,
               "-lamdhip64", *libs, "-o", tmp]
    else:
        cmd = [hipcc, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, *libs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr[-4000:])
    os.replace(tmp, lib)
    return lib


def sanitizer_runtime() -> str:
    """The AddressSanitizer runtime of the ROCm clang (to preload)."""
    import glob
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    hits = sorted(glob.glob(os.path.join(rocm, "lib", "llvm", "lib", "clang", "*", "lib", "linux",
                                         "libclang_rt.asan-x86_64.so")))
    if not hits:
        raise RuntimeError("no libclang_rt.asan-x86_64.so under " + rocm)
    return hits[-1]


if __name__ == "__main__":
    print(build_library(verbose="-v" in sys.argv))
