// A, B, C (the sums of a^2, b^2, a b over the detector samples outside gaps)
// and their derivatives in alpha and delta from the nine mask moments of a
// segment, M_k = sum_i m_i e^{i k theta_i} (k = 0..4, theta_i the local
// sidereal angle of sample i).
//
// a and b are trigonometric polynomials of degree 2 in the hour angle
// H = alpha - theta (Sec. II), so in z = e^{i theta}
//   a = sum_{h=-2..2} a_h z^h,  a_0 = a0,  a_h = conj(w)^h (c_h + i s_h) / 2,
//   a_{-h} = conj(a_h),  w = e^{i alpha},
// with c_h, s_h the cos hH and sin hH coefficients (b alike, b_0 = 0).  For two
// such real polynomials f, g the coefficients of f g are
// (fg)_k = sum_h f_h g_{k-h}, |k| <= 4, and
//   sum_i m_i f(theta_i) g(theta_i) = (fg)_0 M_0 + 2 Re sum_{k=1..4} (fg)_k M_k:
// the direct sum over the samples rearranged, no approximation.  The sums are
// bilinear, so a derivative moves onto one factor: d/dalpha multiplies a_h by
// -i h (w^h depends on alpha), d/ddelta replaces the coefficients by their
// delta derivatives.
#pragma once
#include "cplx.h"
#include "geometry.h"

// the coefficients f_0, f_1, f_2 of a degree-2 polynomial in z (f_{-h} = conj f_h)
struct AbPoly {
  cpx<double> v[3];
};

__device__ __forceinline__ cpx<double> cpow_conj(const SkyConst& k, int h) {
  const cpx<double> w{k.ca, -k.sa};  // conj(e^{i alpha})
  return h == 1 ? w : cmul(w, w);
}

// a and b as polynomials in z
__device__ __forceinline__ void ab_poly(const SkyConst& k, AbPoly& fa, AbPoly& fb) {
  const cpx<double> w1 = cpow_conj(k, 1), w2 = cpow_conj(k, 2);
  fa.v[0] = {k.a0, 0.0};
  fa.v[1] = cmul(w1, cpx<double>{0.5 * k.a1c, 0.5 * k.a1s});
  fa.v[2] = cmul(w2, cpx<double>{0.5 * k.a2c, 0.5 * k.a2s});
  fb.v[0] = {0.0, 0.0};
  fb.v[1] = cmul(w1, cpx<double>{0.5 * k.b1c, 0.5 * k.b1s});
  fb.v[2] = cmul(w2, cpx<double>{0.5 * k.b2c, 0.5 * k.b2s});
}

// their derivatives in alpha (f_h -> -i h f_h) and in delta
__device__ __forceinline__ void ab_poly_partials(const SkyConst& k, const AbPoly& fa, const AbPoly& fb, AbPoly& fa_al,
                                                 AbPoly& fb_al, AbPoly& fa_de, AbPoly& fb_de) {
#pragma unroll
  for (int h = 0; h < 3; ++h) {
    fa_al.v[h] = {h * fa.v[h].y, -h * fa.v[h].x};
    fb_al.v[h] = {h * fb.v[h].y, -h * fb.v[h].x};
  }
  const cpx<double> w1 = cpow_conj(k, 1), w2 = cpow_conj(k, 2);
  fa_de.v[0] = {k.da0, 0.0};
  fa_de.v[1] = cmul(w1, cpx<double>{0.5 * k.da1c, 0.5 * k.da1s});
  fa_de.v[2] = cmul(w2, cpx<double>{0.5 * k.da2c, 0.5 * k.da2s});
  fb_de.v[0] = {0.0, 0.0};
  fb_de.v[1] = cmul(w1, cpx<double>{0.5 * k.db1c, 0.5 * k.db1s});
  fb_de.v[2] = cmul(w2, cpx<double>{0.5 * k.db2c, 0.5 * k.db2s});
}

// sum_i m_i f(theta_i) g(theta_i)
__device__ __forceinline__ double moment_sum(const cpx<double> (&f)[3], const cpx<double> (&g)[3],
                                             const double* __restrict__ mom) {
  auto coef = [&](const cpx<double> (&c)[3], int h) -> cpx<double> { return h >= 0 ? c[h] : cconj(c[-h]); };
  double acc = 0.0;
#pragma unroll
  for (int kk = 0; kk <= 4; ++kk) {
    cpx<double> fg{0.0, 0.0};
#pragma unroll
    for (int h = -2; h <= 2; ++h) {
      const int h2 = kk - h;
      if (h2 < -2 || h2 > 2) continue;
      fg = cadd(fg, cmul(coef(f, h), coef(g, h2)));
    }
    const cpx<double> m{mom[2 * kk], mom[2 * kk + 1]};
    const double re = fg.x * m.x - fg.y * m.y;  // Re(fg M_k)
    acc += kk == 0 ? re : 2.0 * re;
  }
  return acc;
}
