"""Every workgroup barrier of the library's kernels sits in uniform control
flow as compiled for gfx950: no s_barrier inside a loop whose latch is
exec-masked (tests/asm_barriers.py says why that matters).  Each HIP source
of the library is compiled to assembly with the library's own flags (CPU
only, nothing runs).  The checker itself is pinned on two small work-queue
kernels: the form whose claim and completion are thread-0 blocks on either
side of the loop latch, with a break on a flag read from LDS, is flagged; the
form with the completion deferred to the claim and the flags read as
wave-uniform values is not."""
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_1003_0844_amd import _build
from tests import asm_barriers

HIP_SOURCES = [s for s in _build.SOURCES if s.endswith(".hip")]


def _asm(src_path, out_path, flags):
    cmd = [_build._hipcc(), *flags, "--cuda-device-only", "-S", "-o", out_path, src_path]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    with open(out_path) as f:
        return asm_barriers.parse(f.read())


@pytest.fixture(scope="module")
def library_asm(tmp_path_factory):
    d = tmp_path_factory.mktemp("asm")
    flags = _build.common_flags()
    with ThreadPoolExecutor(max_workers=min(len(HIP_SOURCES), 8)) as ex:
        res = list(ex.map(lambda s: _asm(os.path.join(_build.CSRC, s), str(d / (s + ".s")), flags), HIP_SOURCES))
    return dict(zip(HIP_SOURCES, res))


def test_no_barrier_in_an_exec_masked_loop(library_asm):
    bad = {s: asm_barriers.barriers_in_masked_loops(f) for s, f in library_asm.items()}
    assert all(not v for v in bad.values()), {s: v for s, v in bad.items() if v}


def test_the_work_queue_and_simplex_loops_are_seen(library_asm):
    # the kernels whose loops hold barriers are parsed, with their barriers
    assert asm_barriers.barrier_count(library_asm["persist.hip"], "k_persist") > 0
    assert asm_barriers.barrier_count(library_asm["search.hip"], "k_nelder_mead") > 0
    assert asm_barriers.barrier_count(library_asm["grid.hip"], "k_pass1") > 0


QUEUE_DIVERGENT = r"""
#include <hip/hip_runtime.h>
__global__ void k_queue(unsigned long long* head, long long n, unsigned* cnt, float* out) {
  __shared__ unsigned long long s_item;
  __shared__ int s_ok;
  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(head, 1ull);
    __syncthreads();
    const long long item = (long long)s_item;
    if (item >= n) break;
    if (threadIdx.x == 0) s_ok = cnt[item] < 5u;
    __syncthreads();
    if (!s_ok) break;
    out[item * 256 + threadIdx.x] += 1.f;
    __syncthreads();
    if (threadIdx.x == 0) atomicAdd(cnt + item, 1u);
  }
}
"""

QUEUE_UNIFORM = r"""
#include <hip/hip_runtime.h>
__global__ void k_queue(unsigned long long* head, long long n, unsigned* cnt, float* out) {
  __shared__ unsigned long long s_item;
  __shared__ int s_ok;
  unsigned* pend = nullptr;
  for (;;) {
    if (threadIdx.x == 0) {
      if (pend) atomicAdd(pend, 1u);
      s_item = atomicAdd(head, 1ull);
    }
    pend = nullptr;
    __syncthreads();
    const unsigned long long v = s_item;
    const long long item = (long long)(((unsigned long long)(unsigned)__builtin_amdgcn_readfirstlane((int)(v >> 32)) << 32) |
                                       (unsigned)__builtin_amdgcn_readfirstlane((int)(unsigned)v));
    if (item >= n) break;
    if (threadIdx.x == 0) s_ok = cnt[item] < 5u;
    __syncthreads();
    if (__builtin_amdgcn_readfirstlane(s_ok) == 0) break;
    out[item * 256 + threadIdx.x] += 1.f;
    __syncthreads();
    pend = cnt + item;
  }
  if (threadIdx.x == 0 && pend) atomicAdd(pend, 1u);
}
"""


@pytest.mark.parametrize("src,flagged", [(QUEUE_DIVERGENT, True), (QUEUE_UNIFORM, False)])
def test_checker_on_two_queue_loops(tmp_path, src, flagged):
    p = tmp_path / "queue.hip"
    p.write_text(src)
    f = _asm(str(p), str(tmp_path / "queue.s"), _build.common_flags())
    assert asm_barriers.barrier_count(f, "k_queue") == 3
    assert bool(asm_barriers.barriers_in_masked_loops(f)) == flagged
