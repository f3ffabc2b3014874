"""Signal model and detector geometry in FP64 (oracle; test infrastructure only).

Paper: Sec. II ("Response of a detector to a periodic gravitational wave").

Readings where the paper is silent:

* The detector's position w.r.t. the SSB comes from an analytic ephemeris: the
  Earth's centre moves on a circle of radius ``orbit_radius`` in the ecliptic
  plane, and the site rotates on a sphere of radius ``radius`` at the sidereal
  rate.  This replaces the DE405-based astrometry of Sec. V, and keeps the
  structure of Eq. (pha5): an SSB->Earth vector with no ecliptic-normal
  component plus an Earth->site vector given in the celestial (equatorial)
  frame.
* a(t), b(t) are not printed in the paper (Sec. II defers to the
  interferometer formulas of an earlier paper in the series).  We use the
  standard interferometer form, with gamma the angle of the arm bisector
  measured counter-clockwise from local East and x = alpha - (local sidereal
  angle).  It is pinned in the tests by an independent detector-tensor
  computation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

C_LIGHT = 299_792_458.0            # m/s
AU = 1.495978707e11                # m
R_EARTH = 6.378140e6               # m (equatorial radius used in Sec. V)
SIDEREAL_DAY = 86164.0             # s; T_o is a whole number of these
YEAR = 365.256363004 * 86400.0     # s, sidereal year


@dataclass(frozen=True)
class Detector:
    """Interferometer site.  Angles in radians."""
    lat: float
    lon: float
    gamma: float                   # arm bisector, ccw from local East
    zeta: float = math.pi / 2      # angle between the arms
    radius: float = R_EARTH


@dataclass(frozen=True)
class Ephemeris:
    """Analytic circular-orbit ephemeris (see module docstring)."""
    obliquity: float = math.radians(23.44)
    orbit_radius: float = AU
    orbit_omega: float = 2.0 * math.pi / YEAR
    orbit_phase0: float = 0.0
    sidereal_day: float = SIDEREAL_DAY
    gmst0: float = 0.0


def default_detector() -> Detector:
    """The synthetic site of the workloads: latitude 43.63 deg, longitude 10.5
    deg, arm azimuth 19.4 deg with 90-deg arms.  Reading of the azimuth: the
    first arm points 19.4 deg east of North, so the bisector of the two arms
    is 115.6 deg counter-clockwise from East (the other arm choice flips the
    sign of both a and b and leaves F unchanged)."""
    return Detector(lat=math.radians(43.63), lon=math.radians(10.5),
                    gamma=math.radians(115.6))


# --------------------------------------------------------------------------
# Geometry (Eqs. pha4, pha5)
# --------------------------------------------------------------------------
def earth_center(T, eph: Ephemeris):
    """SSB -> Earth-centre vector (R^x_ES, R^y_ES, 0), SSB ecliptic frame."""
    ang = eph.orbit_omega * np.asarray(T, dtype=np.float64) + eph.orbit_phase0
    return eph.orbit_radius * np.cos(ang), eph.orbit_radius * np.sin(ang)


def sidereal_angle(T, det: Detector, eph: Ephemeris):
    """Local sidereal angle of the site's meridian, radians."""
    return eph.gmst0 + det.lon + 2.0 * math.pi * np.asarray(T, dtype=np.float64) / eph.sidereal_day


def site_vector(T, det: Detector, eph: Ephemeris):
    """Earth-centre -> detector vector (R^x_E, R^y_E, R^z_E), celestial frame."""
    th = sidereal_angle(T, det, eph)
    cl = math.cos(det.lat)
    return (det.radius * cl * np.cos(th), det.radius * cl * np.sin(th),
            det.radius * math.sin(det.lat) * np.ones_like(th))


def roemer_delay(T, alpha, delta, det: Detector, eph: Ephemeris):
    """phi_m = n0 . r_d / c, in seconds: the explicit scalar product that
    follows Eqs. (pha4)-(pha5) in Sec. II."""
    xes, yes = earth_center(T, eph)
    xe, ye, ze = site_vector(T, det, eph)
    ca, sa = math.cos(alpha), math.sin(alpha)
    cd, sd = math.cos(delta), math.sin(delta)
    ce, se = math.cos(eph.obliquity), math.sin(eph.obliquity)
    dot = (ca * cd * (xes + xe)
           + (sa * cd * ce + sd * se) * yes
           + sa * cd * ye + sd * ze)
    return dot / C_LIGHT


def roemer_delay_ext(T, alpha, delta, det: Detector, eph: Ephemeris):
    """The same scalar product in extended precision (numpy longdouble, a
    64-bit mantissa on x86-64).  Used where the delay is multiplied by f_ref:
    f_ref phi_m reaches ~2e5 turns, where FP64 rounding alone would leave
    ~1e-11 turn of error."""
    L = np.longdouble
    T = np.asarray(T, dtype=L)
    two_pi = 2 * L(np.pi)
    ang = L(eph.orbit_omega) * T + L(eph.orbit_phase0)
    xes, yes = L(eph.orbit_radius) * np.cos(ang), L(eph.orbit_radius) * np.sin(ang)
    th = L(eph.gmst0) + L(det.lon) + two_pi * T / L(eph.sidereal_day)
    rc = L(det.radius) * np.cos(L(det.lat))
    xe, ye, ze = rc * np.cos(th), rc * np.sin(th), L(det.radius) * np.sin(L(det.lat))
    a, d, e = L(alpha), L(delta), L(eph.obliquity)
    ca, sa, cd, sd, ce, se = np.cos(a), np.sin(a), np.cos(d), np.sin(d), np.cos(e), np.sin(e)
    dot = ca * cd * (xes + xe) + (sa * cd * ce + sd * se) * yes + sa * cd * ye + sd * ze
    return dot / L(C_LIGHT)


# --------------------------------------------------------------------------
# Amplitude modulation (Sec. II, Eq. patt)
# --------------------------------------------------------------------------
def _ab_coeffs(delta, det: Detector):
    """Fourier coefficients in x = alpha - sidereal angle:
    a = a2c cos2x + a2s sin2x + a1c cos x + a1s sin x + a0,
    b = b2c cos2x + b2s sin2x + b1c cos x + b1s sin x."""
    g2, lam = 2.0 * det.gamma, det.lat
    s2g, c2g = math.sin(g2), math.cos(g2)
    sl, cl = math.sin(lam), math.cos(lam)
    s2l, c2l = math.sin(2 * lam), math.cos(2 * lam)
    sd, cd = math.sin(delta), math.cos(delta)
    s2d, c2d = math.sin(2 * delta), math.cos(2 * delta)
    a = dict(a2c=s2g * (3 - c2l) * (3 - c2d) / 16.0,
             a2s=-c2g * sl * (3 - c2d) / 4.0,
             a1c=s2g * s2l * s2d / 4.0,
             a1s=-c2g * cl * s2d / 2.0,
             a0=0.75 * s2g * cl * cl * cd * cd)
    b = dict(b2c=c2g * sl * sd,
             b2s=s2g * (3 - c2l) * sd / 4.0,
             b1c=c2g * cl * cd,
             b1s=s2g * s2l * cd / 2.0)
    return a, b


def amplitude_modulation(T, alpha, delta, det: Detector, eph: Ephemeris):
    """a(t), b(t) of the interferometer (sin(zeta) factored out, Eq. patt)."""
    x = alpha - sidereal_angle(T, det, eph)
    ca, cb = _ab_coeffs(delta, det)
    a = (ca["a2c"] * np.cos(2 * x) + ca["a2s"] * np.sin(2 * x)
         + ca["a1c"] * np.cos(x) + ca["a1s"] * np.sin(x) + ca["a0"])
    b = (cb["b2c"] * np.cos(2 * x) + cb["b2s"] * np.sin(2 * x)
         + cb["b1c"] * np.cos(x) + cb["b1s"] * np.sin(x))
    return a, b


# --------------------------------------------------------------------------
# Phase (Eq. pha3, split as Eqs. pham/phas) in the band-relative frame
# --------------------------------------------------------------------------
def baseband_phase_cycles(t, T0, f, fdot, alpha, delta, f_ref, det, eph):
    """Phase of Eq. (pha3) with one spindown, omega_0 = 2 pi (f_ref + f),
    omega_1 = 2 pi fdot, minus the heterodyne 2 pi f_ref t, in cycles.

    t is segment time (spindown reference at t = 0, as in Eq. pha3); T0 is the
    segment start on the ephemeris clock.  With phi_m = n0.r_d/c:
        phase/2pi = f (t + phi_m) + f_ref phi_m + fdot (t^2/2 + phi_m t).
    """
    t = np.asarray(t, dtype=np.float64)
    pm = roemer_delay(T0 + t, alpha, delta, det, eph)
    return f * (t + pm) + f_ref * pm + fdot * (0.5 * t * t + pm * t)


# --------------------------------------------------------------------------
# Signal for injections (Eqs. resp, patt, hphc, h0iota)
# --------------------------------------------------------------------------
def signal(t, T0, f, fdot, alpha, delta, h0, cosi, psi, phi0, f_ref, det, eph):
    """Detector response h(t) of Eq. (resp) with beam patterns of Eq. (patt),
    polarisations of Eq. (hphc) and amplitudes of Eq. (h0iota), evaluated on
    the band-relative phase (the heterodyne is already applied to the data)."""
    a, b = amplitude_modulation(T0 + np.asarray(t, dtype=np.float64), alpha, delta, det, eph)
    ph = 2.0 * math.pi * baseband_phase_cycles(t, T0, f, fdot, alpha, delta, f_ref, det, eph)
    h0p = 0.5 * h0 * (1.0 + cosi * cosi)
    h0x = h0 * cosi
    sz = math.sin(det.zeta)
    fp = sz * (a * math.cos(2 * psi) + b * math.sin(2 * psi))
    fx = sz * (b * math.cos(2 * psi) - a * math.sin(2 * psi))
    return fp * h0p * np.cos(ph + phi0) + fx * h0x * np.sin(ph + phi0)


def injection(n, dt, T0, params, f_ref, sigma2, det, eph, mask=None):
    """Signal scaled to the requested optimal SNR: sum(m h^2)/sigma^2 = snr^2
    (Eq. snr-def with the time-domain scalar product of Eq. approx1).

    params: dict with f, fdot, alpha, delta, cosi, psi, phi0, snr."""
    t = np.arange(n, dtype=np.float64) * dt
    h = signal(t, T0, params["f"], params["fdot"], params["alpha"], params["delta"],
               1.0, params["cosi"], params["psi"], params["phi0"], f_ref, det, eph)
    m = np.ones(n) if mask is None else np.asarray(mask, dtype=np.float64)
    rho1 = math.sqrt(np.sum(m * h * h) / sigma2)
    return h * (params["snr"] / rho1) * m
