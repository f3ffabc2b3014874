"""Pins of the oracle's geometry (Sec. II, Eqs. pha4-pha5) and amplitude
modulation (Eq. patt) against routes that do not share its formulas."""
import math

import numpy as np
import pytest

from oracle import method, model
from tests.common import DET, EPH

RNG = np.random.default_rng(12345)


def _rot_eps(eps):
    # the obliquity rotation matrix of Eqs. (pha4)/(pha5)
    return np.array([[1, 0, 0], [0, math.cos(eps), math.sin(eps)], [0, -math.sin(eps), math.cos(eps)]])


def _roemer_matrix_route(T, alpha, delta, det, eph):
    """n0 . r_d / c built from the two matrix equations, vector by vector."""
    n_eq = np.array([math.cos(alpha) * math.cos(delta), math.sin(alpha) * math.cos(delta), math.sin(delta)])
    n0 = _rot_eps(eph.obliquity) @ n_eq
    out = []
    for tt in np.atleast_1d(T):
        ang = eph.orbit_omega * tt + eph.orbit_phase0
        r_es = eph.orbit_radius * np.array([math.cos(ang), math.sin(ang), 0.0])
        th = eph.gmst0 + det.lon + 2 * math.pi * tt / eph.sidereal_day
        r_e = det.radius * np.array([math.cos(det.lat) * math.cos(th),
                                     math.cos(det.lat) * math.sin(th), math.sin(det.lat)])
        r_d = r_es + _rot_eps(eph.obliquity) @ r_e
        out.append(n0 @ r_d / model.C_LIGHT)
    return np.array(out)


def test_roemer_delay_matches_matrix_form():
    T = RNG.uniform(0, 3.2e7, 40)
    for _ in range(20):
        al, de = RNG.uniform(0, 2 * math.pi), math.asin(RNG.uniform(-1, 1))
        got = model.roemer_delay(T, al, de, DET, EPH)
        ref = _roemer_matrix_route(T, al, de, DET, EPH)
        assert np.max(np.abs(got - ref)) < 1e-10  # seconds; |phi_m| ~ 500 s


def test_roemer_delay_bounds_and_ecliptic_pole():
    T = np.linspace(0, 3.2e7, 2001)
    lim = (EPH.orbit_radius + DET.radius) / model.C_LIGHT
    for _ in range(10):
        al, de = RNG.uniform(0, 2 * math.pi), math.asin(RNG.uniform(-1, 1))
        assert np.max(np.abs(model.roemer_delay(T, al, de, DET, EPH))) <= lim
    # a source at the ecliptic north pole sees no orbital delay at all
    pole_a, pole_d = 1.5 * math.pi, 0.5 * math.pi - EPH.obliquity
    pm = model.roemer_delay(T, pole_a, pole_d, DET, EPH)
    assert np.max(np.abs(pm)) <= DET.radius / model.C_LIGHT * (1 + 1e-12)
    # a source in the ecliptic plane sees the full orbital delay, AU/c ~ 499 s
    pm = model.roemer_delay(T, 0.0, 0.0, DET, EPH)
    assert abs(np.max(np.abs(pm)) - EPH.orbit_radius / model.C_LIGHT) < 0.03


def test_roemer_rate_is_orbital_plus_diurnal_velocity():
    # |d phi_m/dt| <= (v_orbit + v_diurnal)/c ~ 9.93e-5 + 1.12e-6
    v_orb = EPH.orbit_radius * EPH.orbit_omega / model.C_LIGHT
    v_rot = DET.radius * math.cos(DET.lat) * 2 * math.pi / EPH.sidereal_day / model.C_LIGHT
    assert abs(v_orb - 9.93e-5) < 2e-7
    T = np.linspace(0, 3.2e7, 20001)
    h = 1.0
    for al, de in [(0.3, 0.1), (2.0, -0.7), (4.0, 1.2)]:
        d = (model.roemer_delay(T + h, al, de, DET, EPH) - model.roemer_delay(T - h, al, de, DET, EPH)) / (2 * h)
        assert np.max(np.abs(d)) <= v_orb + v_rot + 1e-12


def test_roemer_partials_match_finite_differences():
    T = RNG.uniform(0, 3.2e7, 50)
    al, de = 1.1, -0.4
    pm, d_al, d_de, d_T = method._roemer_partials(T, al, de, DET, EPH)
    h = 1e-6
    fd_al = (model.roemer_delay(T, al + h, de, DET, EPH) - model.roemer_delay(T, al - h, de, DET, EPH)) / (2 * h)
    fd_de = (model.roemer_delay(T, al, de + h, DET, EPH) - model.roemer_delay(T, al, de - h, DET, EPH)) / (2 * h)
    fd_T = (model.roemer_delay(T + 1.0, al, de, DET, EPH) - model.roemer_delay(T - 1.0, al, de, DET, EPH)) / 2.0
    assert np.max(np.abs(d_al - fd_al)) < 1e-6
    assert np.max(np.abs(d_de - fd_de)) < 1e-6
    assert np.max(np.abs(d_T - fd_T)) < 1e-12


# --------------------------------------------------------------------------
# a(t), b(t)
# --------------------------------------------------------------------------
def _tensor_ab(T, alpha, delta, det, eph):
    """a, b from the detector tensor D = (u1 u1^T - u2 u2^T)/2 contracted with
    the plus/cross polarisation tensors at psi = 0 (Eq. patt with zeta = 90
    deg).  Wave basis: p along d n/d alpha, q = p x n."""
    out_a, out_b = [], []
    for tt in np.atleast_1d(T):
        th = eph.gmst0 + det.lon + 2 * math.pi * tt / eph.sidereal_day
        lam, g = det.lat, det.gamma
        e_e = np.array([-math.sin(th), math.cos(th), 0.0])
        e_n = np.array([-math.sin(lam) * math.cos(th), -math.sin(lam) * math.sin(th), math.cos(lam)])
        u1 = math.cos(g - math.pi / 4) * e_e + math.sin(g - math.pi / 4) * e_n
        u2 = math.cos(g + math.pi / 4) * e_e + math.sin(g + math.pi / 4) * e_n
        D = 0.5 * (np.outer(u1, u1) - np.outer(u2, u2))
        n = np.array([math.cos(delta) * math.cos(alpha), math.cos(delta) * math.sin(alpha), math.sin(delta)])
        p = np.array([-math.sin(alpha), math.cos(alpha), 0.0])
        q = np.cross(p, n)
        out_a.append(np.sum(D * (np.outer(p, p) - np.outer(q, q))))
        out_b.append(np.sum(D * (np.outer(p, q) + np.outer(q, p))))
    return np.array(out_a), np.array(out_b)


def test_ab_match_detector_tensor():
    for _ in range(25):
        det = model.Detector(lat=math.asin(RNG.uniform(-1, 1)), lon=RNG.uniform(0, 2 * math.pi),
                             gamma=RNG.uniform(0, math.pi))
        al, de = RNG.uniform(0, 2 * math.pi), math.asin(RNG.uniform(-1, 1))
        T = RNG.uniform(0, 1e6, 8)
        a, b = model.amplitude_modulation(T, al, de, det, EPH)
        ta, tb = _tensor_ab(T, al, de, det, EPH)
        assert np.max(np.abs(a - ta)) < 1e-14
        assert np.max(np.abs(b - tb)) < 1e-14


def test_ab_at_zenith():
    # source overhead (delta = latitude, on the local meridian)
    T = 3600.0
    th = float(model.sidereal_angle(T, DET, EPH))
    a, b = model.amplitude_modulation(T, th, DET.lat, DET, EPH)
    assert abs(a - math.sin(2 * DET.gamma)) < 1e-14
    assert abs(b - math.cos(2 * DET.gamma)) < 1e-14
    assert abs(a * a + b * b - 1.0) < 1e-14


def test_ab_uncorrelated_over_whole_sidereal_days():
    # Sec. III A: T_o a whole number of sidereal days => <ab> = 0
    dt = 26.0
    for days in (1, 2, 3):
        t = np.arange(int(days * EPH.sidereal_day / dt)) * dt
        for _ in range(5):
            al, de = RNG.uniform(0, 2 * math.pi), math.asin(RNG.uniform(-1, 1))
            a, b = model.amplitude_modulation(t, al, de, DET, EPH)
            assert abs(np.mean(a * b)) < 1e-15
    # ... and the check has teeth: over 0.3 day it does not vanish
    t = np.arange(1000) * dt
    a, b = model.amplitude_modulation(t, 1.0, 0.5, DET, EPH)
    assert abs(np.mean(a * b)) > 1e-3


def test_ab_sky_and_time_average_is_two_fifths():
    # the textbook 2/5 = sky- and polarisation-average of F+^2 + Fx^2 for a
    # 90-degree interferometer
    g = np.random.default_rng(3)
    al = g.uniform(0, 2 * math.pi, 4000)
    de = np.arcsin(g.uniform(-1, 1, 4000))
    t = np.arange(0, EPH.sidereal_day, 600.0)
    tot = 0.0
    for a_, d_ in zip(al, de):
        a, b = model.amplitude_modulation(t, a_, d_, DET, EPH)
        tot += np.mean(a * a + b * b)
    assert abs(tot / al.size - 0.4) < 0.004


def test_ab_partials_match_finite_differences():
    T = RNG.uniform(0, 1e6, 30)
    al, de = 0.7, 0.3
    a, b, ax, bx, ad, bd = method._ab_partials(T, al, de, DET, EPH)
    h = 1e-6
    ap, bp = model.amplitude_modulation(T, al + h, de, DET, EPH)
    am, bm = model.amplitude_modulation(T, al - h, de, DET, EPH)
    assert np.max(np.abs(ax - (ap - am) / (2 * h))) < 1e-8
    assert np.max(np.abs(bx - (bp - bm) / (2 * h))) < 1e-8
    ap, bp = model.amplitude_modulation(T, al, de + h, DET, EPH)
    am, bm = model.amplitude_modulation(T, al, de - h, DET, EPH)
    assert np.max(np.abs(ad - (ap - am) / (2 * h))) < 1e-8
    assert np.max(np.abs(bd - (bp - bm) / (2 * h))) < 1e-8


def test_earth_rotation_rate_matches_paper():
    import json, os
    gold = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))
    # the workloads take a sidereal day of exactly 86164 s; the paper's NOVAS
    # rate corresponds to 86164.0989 s -- within 1.2e-6 relative
    w = 2 * math.pi / EPH.sidereal_day
    assert abs(w / gold["earth_rotation_rate"]["value"] - 1) < 1.2e-6


def test_extended_precision_delay_matches_matrix_form():
    # the extended-precision copy used for the f_ref phi_m phase
    T = RNG.uniform(0, 3.2e7, 20)
    for _ in range(5):
        al, de = RNG.uniform(0, 2 * math.pi), math.asin(RNG.uniform(-1, 1))
        got = model.roemer_delay_ext(T, al, de, DET, EPH)
        assert got.dtype == np.longdouble
        assert np.max(np.abs(got.astype(np.float64) - _roemer_matrix_route(T, al, de, DET, EPH))) < 1e-10
        # and it resolves differences FP64 cannot: relative to phi_m(0) the
        # two agree to the FP64 rounding of a ~500 s quantity
        d_ext = (got - model.roemer_delay_ext(0.0, al, de, DET, EPH)).astype(np.float64)
        d_64 = model.roemer_delay(T, al, de, DET, EPH) - model.roemer_delay(0.0, al, de, DET, EPH)
        assert np.max(np.abs(d_ext - d_64)) < 1e-12
