"""The C-ABI library on the CPU: it loads, exports every entry point the header
declares, and rejects bad arguments before any device work (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_1003_0844_amd import fstat

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fstat.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fstat_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = fstat.lib()
    names = _declared()
    assert "fstat_plan" in names and "fstat_grid" in names and "fstat_grad" in names
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(fstat.EXPORTS)


def test_library_marks_its_calls_with_roctx_ranges():
    # the plan / grid / graph / gradient entry points push and pop a roctx range
    # (rocprofv3 --marker-trace); the library links the roctx library for it
    import subprocess
    out = subprocess.run(["nm", "-D", fstat.LIB_PATH], capture_output=True, text=True, check=True).stdout
    undefined = {line.split()[-1] for line in out.splitlines() if " U " in line}
    assert {"roctxRangePushA", "roctxRangePop"} <= undefined


def test_strerror():
    L = fstat.lib()
    assert L.fstat_strerror(0) == b"ok"
    assert b"sidereal" in L.fstat_strerror(-2)
    assert L.fstat_strerror(-99) == b"unknown status"


def _plan_status(n=43082, dt=2.0, days=1, nfft=0, interp=1, prec=0, x=None, det=None):
    L = fstat.lib()
    x = np.zeros(n) if x is None else x
    seg = fstat._Segment()
    seg.x = x.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    seg.n, seg.dt, seg.n_sidereal_days, seg.f_ref_hz, seg.sigma2, seg.nfft = n, dt, days, 435.1875, 1.0, nfft
    d = det or fstat.default_detector()
    dd = fstat._Detector(d.lat, d.lon, d.gamma, d.zeta, d.radius)
    e = fstat.Ephemeris()
    ee = fstat._Ephemeris(e.obliquity, e.orbit_radius, e.orbit_omega, e.orbit_phase0, e.sidereal_day, e.gmst0)
    o = fstat._Options(interp, prec, 0, 0, 0, 0)
    h = ctypes.c_void_p()
    return L.fstat_plan(ctypes.byref(seg), 1, ctypes.byref(dd), ctypes.byref(ee), ctypes.byref(o), ctypes.byref(h))


def test_plan_rejects_non_integer_sidereal_days():
    assert _plan_status(n=43000) == fstat.ENOTINTDAYS
    assert _plan_status(n=43082, days=2) == fstat.ENOTINTDAYS


def test_plan_rejects_bad_sizes():
    assert _plan_status(nfft=3 << 14) == fstat.EUNSUPPORTED        # not a power of two
    assert _plan_status(nfft=1 << 15) == fstat.EUNSUPPORTED        # below n
    assert _plan_status(nfft=1 << 23) == fstat.EUNSUPPORTED        # above 2^22
    assert _plan_status(n=8, dt=86164.0 / 8) == fstat.EUNSUPPORTED  # n < 16


def test_plan_rejects_bad_values():
    assert _plan_status(interp=3) == fstat.EINVAL
    assert _plan_status(prec=2) == fstat.EINVAL
    x = np.zeros(43082)
    x[7] = math.nan
    assert _plan_status(x=x) == fstat.EINVAL
    assert _plan_status(dt=-2.0) == fstat.EINVAL
    L = fstat.lib()
    h = ctypes.c_void_p()
    assert L.fstat_plan(None, 1, None, None, None, ctypes.byref(h)) == fstat.EINVAL


def test_calls_on_null_plan_are_rejected():
    L = fstat.lib()
    nodes = fstat.nodes_array([0.0], [0.0], [0.0])
    out = fstat._Out(mode=0, k_lo=0, k_hi=10, F=1)
    assert L.fstat_grid(None, nodes.ctypes.data_as(ctypes.c_void_p), 1, ctypes.byref(out), None) == fstat.EINVAL
    assert L.fstat_eval(None, None, None, 1, None, None, None) == fstat.EINVAL
    assert L.fstat_grad(None, None, None, 1, None, None, None) == fstat.EINVAL
    assert L.fstat_adjoint(None, None, None, 1, None, None, None, None) == fstat.EINVAL
    assert L.fstat_plan_info(None, 0, None, None, None, None, None) == fstat.EINVAL
    assert L.fstat_eval_exact(None, None, None, 1, None, None) == fstat.EINVAL
    assert L.fstat_refine(None, None, None, 1, None, None, None, None, None) == fstat.EINVAL
    assert L.fstat_amplitudes(None, None, None, 1, None, None, None) == fstat.EINVAL
    assert L.fstat_graph_create(None, None, 1, None, None) == fstat.EINVAL
    assert L.fstat_graph_launch(None, None) == fstat.EINVAL
    k = np.zeros(1, dtype=np.int64)
    params = np.zeros((1, 4))
    assert L.fstat_bin_params(None, nodes.ctypes.data_as(ctypes.c_void_p), k.ctypes.data_as(ctypes.c_void_p), 1, 0,
                              params.ctypes.data_as(ctypes.c_void_p), None) == fstat.EINVAL
    assert L.fstat_plan_status(None) == fstat.EINVAL
    L.fstat_graph_destroy(None)
    L.fstat_destroy(None)


def test_node_record_layout_matches_header():
    # fstat_node: 3 doubles, an int32 and a float = 32 bytes; fstat_crossing: 24 bytes
    assert fstat.NODE_DTYPE.itemsize == 32
    assert fstat.NODE_DTYPE.fields["bin_offset"][1] == 28
    assert fstat.CROSSING_DTYPE.itemsize == 24
    assert ctypes.sizeof(fstat._Segment) == 72
    assert ctypes.sizeof(fstat._Out) == 80
    # fstat_refine_options: 4 + 1 doubles, 2 int32
    assert ctypes.sizeof(fstat._RefineOptions) == 48
    # fstat_lattice: 2 x 16 + 8 doubles, 2 int32; fstat_lattice_region: 6 doubles, 2 int32
    assert ctypes.sizeof(fstat._Lattice) == 328
    assert ctypes.sizeof(fstat._LatticeRegion) == 56


def test_copy_probe_rejects_bad_arguments():
    # checked before any device work: misaligned, odd sizes, overlap, NULL
    L = fstat.lib()
    vp = ctypes.c_void_p
    assert L.fstat_copy_probe(vp(4096), vp(1 << 20), 0, 0, None) == fstat.EINVAL
    assert L.fstat_copy_probe(vp(4096), vp(1 << 20), 24, 0, None) == fstat.EINVAL
    assert L.fstat_copy_probe(vp(4100), vp(1 << 20), 32, 0, None) == fstat.EINVAL
    assert L.fstat_copy_probe(vp(4096), vp(4096 + 16), 64, 0, None) == fstat.EINVAL
    assert L.fstat_copy_probe(None, vp(1 << 20), 64, 0, None) == fstat.EINVAL
    assert L.fstat_copy_probe(vp(4096), vp(1 << 20), 64, -1, None) == fstat.EINVAL


def test_spill_write_probe_rejects_bad_arguments():
    # checked before any device work: NULL or misaligned buffer, node count,
    # first-pass length, block width
    L = fstat.lib()
    vp = ctypes.c_void_p
    assert L.fstat_spill_write_probe(None, 1, 8, 1024, 16, None) == fstat.EINVAL
    assert L.fstat_spill_write_probe(vp(4100), 1, 8, 1024, 16, None) == fstat.EINVAL
    assert L.fstat_spill_write_probe(vp(4096), 0, 8, 1024, 16, None) == fstat.EINVAL
    assert L.fstat_spill_write_probe(vp(4096), 65536, 8, 1024, 16, None) == fstat.EINVAL
    assert L.fstat_spill_write_probe(vp(4096), 1, 0, 1024, 16, None) == fstat.EINVAL
    assert L.fstat_spill_write_probe(vp(4096), 1, 8, 512, 16, None) == fstat.EINVAL
    assert L.fstat_spill_write_probe(vp(4096), 1, 8, 1024, 12, None) == fstat.EINVAL
    assert L.fstat_spill_write_probe(vp(4096), 1, 8, 1024, 2048, None) == fstat.EINVAL
    assert L.fstat_spill_write_probe(vp(4096), 1, 8, 1024, -1, None) == fstat.EINVAL
