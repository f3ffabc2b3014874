// The per-sample demodulation of one grid node (Sec. VI A, Eqs. pham/phas/ia).
//
// On the barycentric grid t_b_j = t_b0 + j dt (t_b0 = phi_m(0)) the detector
// time is t_j = j dt - dphi_m(t_j), dphi_m = phi_m - phi_m(0).  The
// frequency-independent part of the phase is, in turns,
//   f_ref dphi_m(t_j) + fdot (t_j^2/2 + phi_m(t_j) t_j)
// (the spindown phase of Eq. phas plus the part of omega_0 phi_m that the
// band-relative FFT does not absorb, less the constant f_ref phi_m(0) that is
// common to both correlations).  The sky-only first term comes precomputed
// (reduced to [-1/2, 1/2]) in Quad::p0; the spindown term is evaluated here in
// FP64 and the total is reduced before it reaches the sine/cosine, which run
// in the working precision T.
#pragma once
#include "internal.h"

// FP32 path: the hardware sine/cosine take their argument in turns
// (sin(2 pi x)); x is already reduced to [-1/2, 1/2].
__device__ __forceinline__ void sincos_turns(double x, float& s, float& c) {
  const float xf = (float)x;
  s = __builtin_amdgcn_sinf(xf);
  c = __builtin_amdgcn_cosf(xf);
}
__device__ __forceinline__ void sincos_turns(double x, double& s, double& c) {
  sincospi(2.0 * x, &s, &c);
}

// J: the sample index type (int inside one FFT pass, where j < nfft <= 2^22,
// converts to double in one instruction; int64_t elsewhere).
template <typename T, typename J>
__device__ __forceinline__ Pair<T> demod_elem(const Quad<T>& q, double tb0, J j, double dt,
                                              double fdot, double fshift) {
  const double dd = (double)q.dd;  // phi_m(t_j) - phi_m(0)
  const double t = (double)j * dt - dd;
  // fshift j moves the transform's bins by a fraction of a bin (lattice lines)
  double cyc = (double)q.p0 + fdot * (t * (0.5 * t + tb0 + dd)) + fshift * (double)j;
  cyc -= rint(cyc);
  T s, c;
  sincos_turns(cyc, s, c);
  // x a e^{-i phi}, x b e^{-i phi}
  return {{q.wa * c, -q.wa * s}, {q.wb * c, -q.wb * s}};
}
