"""The library's lattice grid (Sec. IV) through the C ABI, on the CPU (host
computations, no device): the reduced Fisher matrix, the constrained lattice
and its node enumeration against the oracle."""
import ctypes
import math

import numpy as np
import pytest

from oracle import lattice as L
from oracle import method, model
from paper_1003_0844_amd import fstat
from tests.common import DET, EPH

FDET = fstat.default_detector()
FEPH = fstat.Ephemeris()


def _pair(days=2, dt=0.5, t0=3.7e6, mask=None, nfft=0):
    n = int(round(days * model.SIDEREAL_DAY / dt))
    x = np.zeros(n)
    return (fstat.SegmentSpec(x=x, dt=dt, n_days=days, t0=t0, mask=mask, nfft=nfft),
            method.Segment(x=x, dt=dt, n_days=days, t0=t0, mask=mask, nfft=nfft))


def _scaled_diff(A, B):
    s = np.sqrt(np.outer(np.diag(B), np.diag(B)))
    return float(np.max(np.abs(A - B) / s))


@pytest.mark.parametrize("case", ["2d", "1d_gaps", "6d_late"])
def test_fisher_matches_oracle(case):
    if case == "2d":
        spec, seg = _pair()
    elif case == "1d_gaps":
        n = int(round(model.SIDEREAL_DAY / 2.0))
        mask = np.ones(n, np.uint8)
        mask[5000:9000] = 0
        mask[30000:30500] = 0
        spec, seg = _pair(days=1, dt=2.0, t0=1.0e5, mask=mask)
    else:
        spec, seg = _pair(days=6, dt=4.0, t0=2.5e7)
    G = fstat.lattice_fisher(spec, FDET, FEPH)
    Go = L.segment_fisher(seg, DET, EPH)
    assert np.array_equal(G, G.T)
    assert _scaled_diff(G, Go) < 1e-12


@pytest.fixture(scope="module")
def both():
    spec, seg = _pair()
    lat = fstat.Lattice.for_segment(spec, FDET, FEPH, c0=0.75)
    lo = L.constrained_lattice(L.segment_fisher(seg, DET, EPH), lat.dp0, 0.75)
    return lat, lo


def test_lattice_numbers_match_oracle(both):
    lat, lo = both
    # fstat_lattice_segment: the segment's Fisher matrix and the resolution of
    # its default FFT length nextpow2(2n) = 2^20, the same as the two calls
    assert lat.dp0 == 2 * math.pi / ((1 << 20) * 0.5)
    spec, _ = _pair()
    lat2 = fstat.Lattice.build(fstat.lattice_fisher(spec, FDET, FEPH), 2 * math.pi / ((1 << 20) * 0.5), 0.75)
    assert np.array_equal(lat.basis, lat2.basis) and lat.theta == lat2.theta
    for name in ("mu", "nu", "theta", "R"):
        assert abs(getattr(lat, name) - lo[name]) < 1e-12 * abs(lo[name]), name
    m1, ma = L.margins(lat.gamma, lat.R)
    assert abs(lat.margin_w1 - m1) < 1e-9 * m1 and abs(lat.margin_sky - ma) < 1e-9 * ma
    # the same lattice up to a rotation that keeps a0: the same cell volume
    assert abs(abs(np.linalg.det(lat.basis)) / abs(np.linalg.det(lo["basis"])) - 1) < 1e-9


def test_library_lattice_is_a_constrained_covering(both):
    lat, lo = both
    B = lat.basis
    assert B[0, 0] == lat.dp0 and np.all(B[0, 1:] == 0)         # Eq. (avec)
    assert np.all(B[1, 2:] == 0) and B[1, 1] != 0               # Eq. (constraint2)
    # covering radius in whitened coordinates (the oracle's whitening)
    X = np.linalg.solve(lo["M"], B.T).T
    assert L.covering_radius(X) <= lat.R * (1 + 1e-9)
    assert abs(L.thickness(X, lat.R) - L.thickness(L.generator_a4star(lat.R), lat.R) * lat.theta / L.THETA_A4STAR) \
        < 1e-9
    # the stated reduction of the basis
    u, v = B[2, 2:], B[3, 2:]
    assert u @ u <= v @ v * (1 + 1e-12) and abs(u @ v) <= 0.5 * (u @ u) * (1 + 1e-12)
    assert np.all(np.abs(B[2:, 1]) <= 0.5 * abs(B[1, 1]) * (1 + 1e-12))
    assert np.all(np.abs(B[1:, 0]) <= 0.5 * B[0, 0] * (1 + 1e-12))


def test_virgo_thickness_through_the_library():
    spec, seg = _pair()
    G = fstat.lattice_fisher(spec, FDET, FEPH)
    lat = fstat.Lattice.build(G, math.pi / (len(spec.x) * spec.dt), 0.75)
    assert abs(lat.theta - 2.1) < 0.05 and abs(lat.theta / 1.7655 - 1.2) < 0.03


def _key_set(nodes, k):
    return {(int(a), int(b), int(c), round(float(al), 9), round(float(de), 9))
            for (a, b, c), al, de in zip(k, nodes["alpha"], nodes["delta"])}


@pytest.mark.parametrize("region", ["patch", "full", "north", "south"])
def test_nodes_match_oracle_enumeration(both, region):
    lat, _ = both
    f_sky = 436.0 if region == "patch" else 30.0
    om = 2 * math.pi * f_sky
    sky = (0.3 * om, -0.4 * om, 150.0) if region == "patch" else None
    hemi = {"north": 1, "south": -1}.get(region, 0)
    nodes, k = lat.nodes(f_sky, -8e-10, 1e-10, FEPH, sky=sky, hemisphere=hemi, seg=3, coef=True)
    recs = L.lattice_nodes(lat.basis, lat.gamma, lat.R, f_sky, -8e-10, 1e-10, EPH.obliquity, sky=sky,
                           hemisphere=hemi, seg=3)
    assert len(nodes) == len(recs) > 0
    want = {(r[5][0], r[5][1], r[5][2], round(r[0], 9), round(r[1], 9)) for r in recs}
    assert _key_set(nodes, k) == want
    assert np.all(nodes["seg"] == 3)
    # each node's fdot and bin offset follow from its lattice coefficients
    B = lat.basis
    tau = k[:, 0:1] * B[1] + k[:, 1:2] * B[2] + k[:, 2:3] * B[3]
    assert np.allclose(nodes["fdot"], tau[:, 1] / (2 * math.pi), rtol=1e-12, atol=1e-24)
    frac = np.mod(tau[:, 0] / B[0, 0], 1.0).astype(np.float32)
    frac[frac >= np.float32(1.0)] = 0.0
    assert np.array_equal(nodes["bin_offset"], frac)
    assert np.all((nodes["bin_offset"] >= 0) & (nodes["bin_offset"] < 1))
    if hemi:
        ce, se = math.cos(EPH.obliquity), math.sin(EPH.obliquity)
        nz = -np.sin(nodes["alpha"]) * np.cos(nodes["delta"]) * se + np.sin(nodes["delta"]) * ce
        assert np.all(hemi * nz >= -1e-12)


def test_node_capacity_and_counts(both):
    lat, _ = both
    L_ = fstat.lib()
    reg = fstat._LatticeRegion(30.0, -1e-10, 0.0, 0.0, 0.0, 0.0, 0, 0)
    e = fstat._eph_struct(FEPH)
    n = ctypes.c_int64()
    assert L_.fstat_lattice_nodes(ctypes.byref(lat._raw), ctypes.byref(reg), ctypes.byref(e), None, None, 0,
                                  ctypes.byref(n)) == fstat.OK
    total = n.value
    part = np.zeros(5, dtype=fstat.NODE_DTYPE)
    assert L_.fstat_lattice_nodes(ctypes.byref(lat._raw), ctypes.byref(reg), ctypes.byref(e),
                                  part.ctypes.data_as(ctypes.c_void_p), None, 5, ctypes.byref(n)) == fstat.OK
    assert n.value == total
    full = lat.nodes(30.0, -1e-10, 0.0, FEPH)
    assert np.array_equal(part, full[:5])


def test_lattice_argument_checks(both):
    lat, _ = both
    L_ = fstat.lib()
    g = np.ascontiguousarray(lat.gamma.reshape(16))
    out = fstat._Lattice()
    gp = g.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    assert L_.fstat_lattice_build(gp, lat.dp0, 0.75, 0, ctypes.byref(out)) == fstat.OK
    assert L_.fstat_lattice_build(gp, lat.dp0, 1.0, 0, ctypes.byref(out)) == fstat.EINVAL
    assert L_.fstat_lattice_build(gp, lat.dp0, 0.0, 0, ctypes.byref(out)) == fstat.EINVAL
    assert L_.fstat_lattice_build(gp, -lat.dp0, 0.75, 0, ctypes.byref(out)) == fstat.EINVAL
    assert L_.fstat_lattice_build(gp, lat.dp0, 0.75, 0, None) == fstat.EINVAL
    bad = g.copy()
    bad[1] *= 1.5                                   # not symmetric
    assert L_.fstat_lattice_build(bad.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), lat.dp0, 0.75, 0,
                                  ctypes.byref(out)) == fstat.EINVAL
    indef = np.diag([1.0, 1.0, 1.0, -1.0]).reshape(16)
    assert L_.fstat_lattice_build(indef.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1.0, 0.75, 0,
                                  ctypes.byref(out)) == fstat.EINVAL
    sing = np.ones(16)                               # rank one
    assert L_.fstat_lattice_build(sing.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), 1.0, 0.75, 0,
                                  ctypes.byref(out)) == fstat.EINVAL
    e = fstat._eph_struct(FEPH)
    n = ctypes.c_int64()
    for reg in (fstat._LatticeRegion(30.0, 0.0, -1e-10, 0, 0, 0, 0, 0),      # fdot_lo > fdot_hi
                fstat._LatticeRegion(0.0, -1e-10, 0.0, 0, 0, 0, 0, 0),       # f_sky <= 0
                fstat._LatticeRegion(30.0, -1e-10, 0.0, 0, 0, 0, 2, 0)):     # hemisphere
        assert L_.fstat_lattice_nodes(ctypes.byref(lat._raw), ctypes.byref(reg), ctypes.byref(e), None, None, 0,
                                      ctypes.byref(n)) == fstat.EINVAL
    reg = fstat._LatticeRegion(30.0, -1e-10, 0.0, 0, 0, 0, 0, 0)
    assert L_.fstat_lattice_nodes(ctypes.byref(lat._raw), ctypes.byref(reg), ctypes.byref(e), None, None, 3,
                                  ctypes.byref(n)) == fstat.EINVAL          # capacity without a buffer
    spec, _ = _pair(days=1, dt=2.0)
    s = fstat._segment_struct(spec, [])
    s.n = 1
    d = fstat._Detector(FDET.lat, FDET.lon, FDET.gamma, FDET.zeta, FDET.radius)
    gbuf = (ctypes.c_double * 16)()
    assert L_.fstat_lattice_fisher(ctypes.byref(s), ctypes.byref(d), ctypes.byref(e), gbuf) == fstat.EINVAL


@pytest.mark.parametrize("days,dt,t0", [(1, 13.0, 0.0), (1, 2.0, 0.0), (2, 13.0, 0.0), (6, 4.0, 2.5e7)])
def test_lattice_for_several_segments(days, dt, t0):
    # whitening rows span many decades for short segments: the library must
    # still solve e0 = M^-1 a0 and agree with the oracle
    spec, seg = _pair(days=days, dt=dt, t0=t0)
    lat = fstat.Lattice.for_segment(spec, FDET, FEPH, c0=0.75)
    lo = L.constrained_lattice(L.segment_fisher(seg, DET, EPH), lat.dp0, 0.75)
    for name in ("mu", "nu", "theta"):
        assert abs(getattr(lat, name) - lo[name]) < 1e-10 * abs(lo[name]), name
    X = np.linalg.solve(lo["M"], lat.basis.T).T
    assert L.covering_radius(X) <= lat.R * (1 + 1e-9)


def test_covering_rule_matches_oracle(both):
    lat0, _ = both
    lat = fstat.Lattice.build(lat0.gamma, lat0.dp0, 0.75, rule=fstat.NU_COVERING)
    assert lat.rule == fstat.NU_COVERING
    lo = L.constrained_lattice(lat0.gamma, lat0.dp0, 0.75, rule="covering")
    for name in ("mu", "nu", "theta"):
        assert abs(getattr(lat, name) - lo[name]) < 1e-9 * abs(lo[name]), name
    X = np.linalg.solve(lo["M"], lat.basis.T).T
    cr = L.covering_radius(X)
    assert lat.R * (1 - 1e-9) <= cr <= lat.R * (1 + 1e-9)
    assert lat.theta < lat0.theta
    g = np.ascontiguousarray(lat0.gamma.reshape(16))
    out = fstat._Lattice()
    assert fstat.lib().fstat_lattice_build(g.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), lat0.dp0, 0.75, 2,
                                           ctypes.byref(out)) == fstat.EINVAL
