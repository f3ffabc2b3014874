// Device helpers for F at continuous candidate parameters (f, fdot, alpha,
// delta): block reductions, the interpolant with its derivative, the sky set-up
// and the per-sample terms of the correlations, by the resampling method of
// Sec. VI A on the barycentric grid and exactly on the detector samples.
#pragma once
#include "demod.h"
#include "internal.h"
#include "moments.h"

namespace {

constexpr int GB = 256;
constexpr double TWO_PI = 6.283185307179586476925286766559;

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// fixed-order block sum of NV values; results valid in thread 0
template <int NV>
__device__ __forceinline__ void block_sums(double (&v)[NV], double* sh) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wsum(v[i]);
  if ((tid & 63) == 0)
#pragma unroll
    for (int i = 0; i < NV; ++i) sh[(tid >> 6) * NV + i] = v[i];
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = 0.0;
      for (int w = 0; w < GB / 64; ++w) s += sh[w * NV + i];
      v[i] = s;
    }
  }
}

// interpolated x and dx/du at the fractional sample position u = j + off
// (integer j, small offset off = -dphi_m/dt: the weight carries the rounding of
// off only)
__device__ __forceinline__ void interp_d(const SegDev& sg, int64_t j, double off, double& xr, double& dxdu) {
  xr = 0.0;
  dxdu = 0.0;
  const int64_t n = sg.n;
  const double lo = -(double)j, hi = (double)(n - 1 - j);
  if (!(off >= lo - SPAN_EPS && off <= hi + SPAN_EPS)) return;
  off = fmin(fmax(off, lo), hi);
  if (sg.interp == 0) {
    xr = sg.x[j + (int64_t)floor(off + 0.5)];
    return;
  }
  const double w = 2.0 * off;
  const double fl = floor(w);
  int64_t i = 2 * j + (int64_t)fl;
  if (i > 2 * n - 2) i = 2 * n - 2;
  const double s = w - fl;
  const double y0 = sg.y[i], y1 = sg.y[i + 1];
  if (sg.interp == 1) {
    xr = (1.0 - s) * y0 + s * y1;
    dxdu = 2.0 * (y1 - y0);
  } else {
    const double m0 = sg.M[i], m1 = sg.M[i + 1], r = 1.0 - s;
    xr = r * y0 + s * y1 + ((r * r * r - r) * m0 + (s * s * s - s) * m1) / 6.0;
    dxdu = 2.0 * (y1 - y0 + ((1.0 - 3.0 * r * r) * m0 + (3.0 * s * s - 1.0) * m1) / 6.0);
  }
}

struct Cand {
  double f, fdot, alpha, delta;
};

__device__ __forceinline__ void setup_sky(const SegDev& sg, const Cand& c, SkyConst& k) {
  sky_const(c.alpha, c.delta, sg.geo, k);
  k.tb0 = roemer(k, ephem(sg.geo, 0.0));
}

// Terms of sample j of S_a, S_b by the resampling method: barycentric grid
// t_b_j = t_b0 + j dt, detector time t_j from the angle-addition ephemeris and
// one linearised fixed-point step (sample_geo), cyc_j = f_ref dphi_m(t_j) +
// fdot (t_j^2/2 + phi_m(t_j) t_j) + f j dt:  acc += (Re S_a, Im S_a, Re S_b,
// Im S_b).  A, B, C come from the mask moments (abc_moments).
__device__ __forceinline__ void method_terms(const SegDev& sg, const SkyConst& k, const Cand& c, int64_t j,
                                             double (&acc)[4]) {
  const SampleGeo s = sample_geo(sg.geo, k, (double)j * sg.dt);
  const double t = s.t, dpm = s.dpm;
  const double pm = k.tb0 + dpm;
  double xr, dxdu;
  interp_d(sg, j, -dpm / sg.dt, xr, dxdu);
  double a, b;
  amp_ab(k, hour_angle(k, s.cth, s.sth), a, b);
  double cyc = sg.f_ref * dpm + c.fdot * (0.5 * t * t + pm * t) + c.f * ((double)j * sg.dt);
  cyc -= rint(cyc);
  double sn, co;
  sincospi(2.0 * cyc, &sn, &co);
  acc[0] += xr * a * co;
  acc[1] -= xr * a * sn;
  acc[2] += xr * b * co;
  acc[3] -= xr * b * sn;
}

// A, B, C of a sky position over the segment's detector samples outside gaps,
// from its mask moments.
__device__ __forceinline__ void abc_moments(const SegDev& sg, const SkyConst& k, double& A, double& B, double& C) {
  AbPoly fa, fb;
  ab_poly(k, fa, fb);
  A = moment_sum(fa.v, fa.v, sg.mom);
  B = moment_sum(fb.v, fb.v, sg.mom);
  C = moment_sum(fa.v, fb.v, sg.mom);
}

// The same terms without resampling (Eqs. OS-Fab summed on the detector
// samples t_i = i dt, as the paper's fine search): the phase of Eq. (pha3)
// less the heterodyne, f (t + phi_m) + f_ref phi_m + fdot (t^2/2 + phi_m t), at
// the detector time itself; x is the masked data.
__device__ __forceinline__ void exact_terms(const SegDev& sg, const SkyConst& k, const Cand& c, int64_t i,
                                            double (&acc)[7]) {
  const double t = (double)i * sg.dt;
  const Ephem e = ephem(sg.geo, t);
  const double pm = roemer(k, e);
  double a, b;
  amp_ab(k, hour_angle(k, e), a, b);
  double c1 = c.f * (t + pm);
  c1 -= rint(c1);
  double c2 = sg.f_ref * pm;
  c2 -= rint(c2);
  double cyc = c1 + c2 + c.fdot * (0.5 * t * t + pm * t);
  cyc -= rint(cyc);
  double s, co;
  sincospi(2.0 * cyc, &s, &co);
  const double x = sg.x[i];
  acc[0] += x * a * co;
  acc[1] -= x * a * s;
  acc[2] += x * b * co;
  acc[3] -= x * b * s;
  const double m = sg.mask ? (sg.mask[i] ? 1.0 : 0.0) : 1.0;
  acc[4] += m * a * a;
  acc[5] += m * b * b;
  acc[6] += m * a * b;
}

__device__ __forceinline__ double combine_F(const double (&acc)[7], double sigma2) {
  const double Sar = acc[0], Sai = acc[1], Sbr = acc[2], Sbi = acc[3];
  const double A = acc[4], B = acc[5], C = acc[6];
  // F of Eq. OS with C != 0 (gaps): (B|S_a|^2 + A|S_b|^2 - 2C Re(S_a S_b*)) / (sigma^2 (AB - C^2))
  const double num = B * (Sar * Sar + Sai * Sai) + A * (Sbr * Sbr + Sbi * Sbi) - 2.0 * C * (Sar * Sbr + Sai * Sbi);
  return num / (sigma2 * (A * B - C * C));
}

}  // namespace
