// Detector geometry on the device, FP64 (Sec. II).
//
// Angles of the analytic ephemeris are carried in cycles (turns) and turned
// into sines and cosines with sincospi, so no reduction by 2 pi is needed:
//   orbital angle   Theta_o(t) = orb_c0 + t * orb_rate_c      (turns)
//   sidereal angle  theta(t)   = sid_c0 + t * sid_rate_c      (turns)
// with t the segment time (global time T = t0 + t); the host folds t0 into the
// two start phases.  The per-sample paths work with the Roemer delay relative
// to the segment start, dphi_m(t) = phi_m(t) - phi_m(0): the constant
// phi_m(0) (up to 500 s, i.e. ~2e5 turns at f_ref) only adds a common phase to
// both correlations, which F does not see.  The Roemer delay n0.r_d/c is the explicit scalar product
// that follows Eqs. (pha4)-(pha5); a(t), b(t) are the interferometer
// amplitude-modulation functions (standard form, gamma = arm bisector measured
// counter-clockwise from local East, x = alpha - theta).
#pragma once
#include <hip/hip_runtime.h>

struct SegGeo {
  double orb_r;       // orbit radius / c  [s]
  double orb_c0;      // orbital angle at segment start [turns, in [0,1)]
  double orb_rate_c;  // orbital rate [turns/s]
  double site_rc;     // R cos(lat) / c [s]
  double site_rz;     // R sin(lat) / c [s]
  double sid_c0;      // local sidereal angle at segment start [turns, in [0,1)]
  double sid_rate_c;  // 1 / sidereal day [turns/s]
  double ceps, seps;  // obliquity
  double s2g, c2g;    // sin, cos of 2 gamma
  double sl, cl;      // sin, cos of latitude
  double s2l, c2l;    // sin, cos of 2 latitude
  double cth0, sth0;  // cos, sin of the sidereal angle at t = 0
  double sin_zeta;    // sin of the angle between the arms (scales the amplitudes)
};

// Everything about one sky position that the per-sample loops need.
struct SkyConst {
  double nx, nye, ny, nz;        // n0 components entering n0.r_d (see roemer)
  double ca, sa;                 // cos, sin alpha
  double a2c, a2s, a1c, a1s, a0; // a = a2c cos2x + a2s sin2x + a1c cos x + a1s sin x + a0
  double b2c, b2s, b1c, b1s;     // b = b2c cos2x + b2s sin2x + b1c cos x + b1s sin x
  // partials of the coefficients w.r.t. delta (used by the gradient)
  double da2c, da2s, da1c, da1s, da0, db2c, db2s, db1c, db1s;
  // partials of the n0 components w.r.t. alpha and delta
  double nx_a, nye_a, ny_a, nz_a, nx_d, nye_d, ny_d, nz_d;
  double tb0;                    // barycentric time of t = 0: phi_m(0)
  double pad[3];
};

__device__ __forceinline__ void sky_const(double alpha, double delta, const SegGeo& g, SkyConst& k) {
  double sa, ca, sd, cd, s2d, c2d;
  sincos(alpha, &sa, &ca);
  sincos(delta, &sd, &cd);
  sincos(2.0 * delta, &s2d, &c2d);
  k.ca = ca;
  k.sa = sa;
  k.nx = ca * cd;
  k.nye = sa * cd * g.ceps + sd * g.seps;
  k.ny = sa * cd;
  k.nz = sd;
  k.nx_a = -sa * cd;
  k.nye_a = ca * cd * g.ceps;
  k.ny_a = ca * cd;
  k.nz_a = 0.0;
  k.nx_d = -ca * sd;
  k.nye_d = -sa * sd * g.ceps + cd * g.seps;
  k.ny_d = -sa * sd;
  k.nz_d = cd;
  const double s2g = g.s2g, c2g = g.c2g, sl = g.sl, cl = g.cl, s2l = g.s2l, c2l = g.c2l;
  k.a2c = s2g * (3.0 - c2l) * (3.0 - c2d) / 16.0;
  k.a2s = -c2g * sl * (3.0 - c2d) / 4.0;
  k.a1c = s2g * s2l * s2d / 4.0;
  k.a1s = -c2g * cl * s2d / 2.0;
  k.a0 = 0.75 * s2g * cl * cl * cd * cd;
  k.b2c = c2g * sl * sd;
  k.b2s = s2g * (3.0 - c2l) * sd / 4.0;
  k.b1c = c2g * cl * cd;
  k.b1s = s2g * s2l * cd / 2.0;
  k.da2c = s2g * (3.0 - c2l) * 2.0 * s2d / 16.0;
  k.da2s = -c2g * sl * 2.0 * s2d / 4.0;
  k.da1c = s2g * s2l * 2.0 * c2d / 4.0;
  k.da1s = -c2g * cl * 2.0 * c2d / 2.0;
  k.da0 = -0.75 * s2g * cl * cl * s2d;
  k.db2c = c2g * sl * cd;
  k.db2s = s2g * (3.0 - c2l) * cd / 4.0;
  k.db1c = -c2g * cl * sd;
  k.db1s = -s2g * s2l * sd / 2.0;
  k.tb0 = 0.0;
}

struct Ephem {  // positions (in light-seconds) and the sidereal angle at one time
  double xes, yes;    // SSB -> Earth centre, ecliptic frame
  double xe, ye, ze;  // Earth centre -> site, celestial frame
  double cth, sth;    // cos, sin of the local sidereal angle
  double cor, sor;    // cos, sin of the orbital angle
};

__device__ __forceinline__ Ephem ephem(const SegGeo& g, double t) {
  Ephem e;
  double co = g.orb_c0 + t * g.orb_rate_c;
  double cs = g.sid_c0 + t * g.sid_rate_c;
  co -= rint(co);
  cs -= rint(cs);
  sincospi(2.0 * co, &e.sor, &e.cor);
  sincospi(2.0 * cs, &e.sth, &e.cth);
  e.xes = g.orb_r * e.cor;
  e.yes = g.orb_r * e.sor;
  e.xe = g.site_rc * e.cth;
  e.ye = g.site_rc * e.sth;
  e.ze = g.site_rz;
  return e;
}

// phi_m = n0 . r_d / c  [s]
__device__ __forceinline__ double roemer(const SkyConst& k, const Ephem& e) {
  return k.nx * (e.xes + e.xe) + k.nye * e.yes + k.ny * e.ye + k.nz * e.ze;
}

// Change of the detector position since t = 0, in light-seconds, and the
// sidereal angle at t.  The orbital part uses the half-angle forms
//   cos(T0 + d) - cos T0 = -2 sin(T0 + d/2) sin(d/2)
//   sin(T0 + d) - sin T0 =  2 cos(T0 + d/2) sin(d/2)
// so the ~500 s orbital delay never appears as a large number that is then
// differenced: dphi_m keeps FP64 relative accuracy on its own (small) size.
struct EphemD {
  double dxes, dyes;  // change of the SSB -> Earth-centre vector
  double dxe, dye;    // change of the Earth-centre -> site vector
  double cth, sth;    // cos, sin of the local sidereal angle at t
};

__device__ __forceinline__ EphemD ephem_delta(const SegGeo& g, double t) {
  EphemD e;
  const double h = t * g.orb_rate_c;  // orbital advance, turns
  double mid = g.orb_c0 + 0.5 * h;
  mid -= rint(mid);
  double sm, cm;
  sincospi(2.0 * mid, &sm, &cm);
  const double sh = sinpi(h);
  e.dxes = -2.0 * g.orb_r * sm * sh;
  e.dyes = 2.0 * g.orb_r * cm * sh;
  double cs = g.sid_c0 + t * g.sid_rate_c;
  cs -= rint(cs);
  sincospi(2.0 * cs, &e.sth, &e.cth);
  e.dxe = g.site_rc * (e.cth - g.cth0);
  e.dye = g.site_rc * (e.sth - g.sth0);
  return e;
}

// dphi_m(t) = phi_m(t) - phi_m(0)  [s]
__device__ __forceinline__ double roemer_delta(const SkyConst& k, const EphemD& e) {
  return k.nx * (e.dxes + e.dxe) + k.nye * e.dyes + k.ny * e.dye;
}

// cos, sin of x = alpha - theta and of 2x
struct HourAngle {
  double c1, s1, c2, s2;
};
__device__ __forceinline__ HourAngle hour_angle(const SkyConst& k, double cth, double sth) {
  HourAngle h;
  h.c1 = k.ca * cth + k.sa * sth;
  h.s1 = k.sa * cth - k.ca * sth;
  h.c2 = h.c1 * h.c1 - h.s1 * h.s1;
  h.s2 = 2.0 * h.s1 * h.c1;
  return h;
}
__device__ __forceinline__ HourAngle hour_angle(const SkyConst& k, const Ephem& e) {
  return hour_angle(k, e.cth, e.sth);
}

__device__ __forceinline__ void amp_ab(const SkyConst& k, const HourAngle& h, double& a, double& b) {
  a = k.a2c * h.c2 + k.a2s * h.s2 + k.a1c * h.c1 + k.a1s * h.s1 + k.a0;
  b = k.b2c * h.c2 + k.b2s * h.s2 + k.b1c * h.c1 + k.b1s * h.s1;
}

// Detector time t of the barycentric grid point t_b0 + j dt (t_b0 = phi_m(0)),
// i.e. the solution of t + dphi_m(t) = j dt.  Fixed point t <- j dt - dphi_m(t)
// from t = j dt; |d phi_m/dt| < 1.1e-4, so four steps take an initial error of
// a minute below 1e-14 s.  Returns t, the ephemeris change at t and
// dpm = dphi_m(t).
__device__ __forceinline__ double ssb_to_detector(const SegGeo& g, const SkyConst& k, double jdt, EphemD& e,
                                                  double& dpm) {
  double t = jdt;
#pragma unroll 1
  for (int it = 0; it < 4; ++it) {
    e = ephem_delta(g, t);
    t = jdt - roemer_delta(k, e);
  }
  e = ephem_delta(g, t);
  dpm = roemer_delta(k, e);
  return t;
}

// ---------------------------------------------------------------------------
// The ephemeris of one sample time by angle addition (the grid's sky
// preparation and the candidate kernels): the three angles at j dt are turned
// into sines and cosines once; the ephemeris at the detector time t = j dt - d
// (|d| below 1000 s) follows from small rotations of them.
// ---------------------------------------------------------------------------
// sin and cos of a small angle (|x| < 0.2) by their Taylor polynomials through
// x^11 and x^12: remainders below 1e-17 relative.
__device__ __forceinline__ void small_sincos(double x, double& s, double& c) {
  const double x2 = x * x;
  s = x * (1.0 - x2 * (1.0 / 6.0) *
                     (1.0 - x2 * (1.0 / 20.0) *
                                (1.0 - x2 * (1.0 / 42.0) * (1.0 - x2 * (1.0 / 72.0) * (1.0 - x2 * (1.0 / 110.0))))));
  c = 1.0 - x2 * 0.5 *
                (1.0 - x2 * (1.0 / 12.0) *
                           (1.0 - x2 * (1.0 / 30.0) *
                                      (1.0 - x2 * (1.0 / 56.0) *
                                                 (1.0 - x2 * (1.0 / 90.0) * (1.0 - x2 * (1.0 / 132.0))))));
}

// The analytic ephemeris at one time t: the angles of ephem_delta as sines and
// cosines, from which the ephemeris at any nearby time t - d follows by angle
// addition.
struct EphemBase {
  double sm, cm;    // 2 pi (orb_c0 + h/2), h = t orb_rate_c
  double sh, ch;    // pi h
  double sth, cth;  // local sidereal angle
};

__device__ __forceinline__ EphemBase ephem_base(const SegGeo& g, double t) {
  EphemBase b;
  const double h = t * g.orb_rate_c;
  double mid = g.orb_c0 + 0.5 * h;
  mid -= rint(mid);
  sincospi(2.0 * mid, &b.sm, &b.cm);
  sincospi(h, &b.sh, &b.ch);
  double cs = g.sid_c0 + t * g.sid_rate_c;
  cs -= rint(cs);
  sincospi(2.0 * cs, &b.sth, &b.cth);
  return b;
}

// dphi_m at t - d and its time derivative (the same quantities as
// roemer_delta(ephem_delta(t - d))): the orbital angles move by
// pi orb_rate_c d, the sidereal angle by 2 pi sid_rate_c d.  |d| <= 1000 s
// (twice the orbit's light time), so both angles stay below 0.08 rad.
__device__ __forceinline__ void roemer_at(const SegGeo& g, const SkyConst& k, const EphemBase& b, double d,
                                          double& dpm, double& ddpm) {
  constexpr double PI = 3.14159265358979323846;
  const double wo = PI * g.orb_rate_c, ws = 2.0 * PI * g.sid_rate_c;
  double so, co, ss, cs;
  small_sincos(wo * d, so, co);
  small_sincos(ws * d, ss, cs);
  const double sm = b.sm * co - b.cm * so, cm = b.cm * co + b.sm * so;
  const double sh = b.sh * co - b.ch * so, ch = b.ch * co + b.sh * so;
  const double sth = b.sth * cs - b.cth * ss, cth = b.cth * cs + b.sth * ss;
  const double dxes = -2.0 * g.orb_r * sm * sh, dyes = 2.0 * g.orb_r * cm * sh;
  const double dxe = g.site_rc * (cth - g.cth0), dye = g.site_rc * (sth - g.sth0);
  dpm = k.nx * (dxes + dxe) + k.nye * dyes + k.ny * dye;
  const double vxes = -2.0 * g.orb_r * wo * (cm * sh + sm * ch), vyes = 2.0 * g.orb_r * wo * (cm * ch - sm * sh);
  const double vxe = -g.site_rc * ws * sth, vye = g.site_rc * ws * cth;
  ddpm = k.nx * (vxes + vxe) + k.nye * vyes + k.ny * vye;
}

// The detector time t of the barycentric grid point t_b0 + j dt, i.e. the
// solution of t + dphi_m(t) = j dt, and the ephemeris there.  d0 = dphi_m(j dt)
// is within |dphi_m'| x 500 s ~ 0.05 s of dphi_m(t); one step of the fixed-point
// relation linearised at t1 = j dt - d0,
//   dphi_m(t) = (dphi_m(t1) + dphi_m'(t1) d0) / (1 + dphi_m'(t1)),
// leaves ~1e-13 s (the curvature of dphi_m is below 1e-10 s/s^2).  The
// sidereal and orbital angles at t follow by one more small rotation.
struct SampleGeo {
  double t, dpm;    // detector time, dphi_m(t)
  double cth, sth;  // local sidereal angle at t
  double cor, sor;  // orbital angle at t
};

__device__ __forceinline__ SampleGeo sample_geo(const SegGeo& g, const SkyConst& k, double jdt) {
  constexpr double PI = 3.14159265358979323846;
  const EphemBase b = ephem_base(g, jdt);
  double d, dd, v, dv;
  roemer_at(g, k, b, 0.0, d, dd);
  roemer_at(g, k, b, d, v, dv);
  SampleGeo s;
  s.dpm = (v + dv * d) / (1.0 + dv);
  s.t = jdt - s.dpm;
  double so, co, ss, cs;
  small_sincos(PI * g.orb_rate_c * s.dpm, so, co);
  small_sincos(2.0 * PI * g.sid_rate_c * s.dpm, ss, cs);
  s.sth = b.sth * cs - b.cth * ss;
  s.cth = b.cth * cs + b.sth * ss;
  // orbital angle = (half-way angle) + (half advance), both rotated back
  const double sm = b.sm * co - b.cm * so, cm = b.cm * co + b.sm * so;
  const double sh = b.sh * co - b.ch * so, ch = b.ch * co + b.sh * so;
  s.cor = cm * ch - sm * sh;
  s.sor = sm * ch + cm * sh;
  return s;
}

// The absolute ephemeris at the sample's detector time.
__device__ __forceinline__ Ephem ephem_of(const SegGeo& g, const SampleGeo& s) {
  Ephem e;
  e.cor = s.cor;
  e.sor = s.sor;
  e.cth = s.cth;
  e.sth = s.sth;
  e.xes = g.orb_r * s.cor;
  e.yes = g.orb_r * s.sor;
  e.xe = g.site_rc * s.cth;
  e.ye = g.site_rc * s.sth;
  e.ze = g.site_rz;
  return e;
}
