// F at continuous parameters and its adjoint (candidate refinement off the
// grid, after the coarse search of Sec. VI C), all FP64.
//
// Forward, per candidate (f, fdot, alpha, delta), over the barycentric grid
// t_b_j = t_b0 + j dt (the method of Sec. VI A with the FFT kernel replaced by
// e^{-2 pi i f j dt}):
//   S_a = sum_j w_a,j e_j,  w_a,j = x(t_j) a(t_j),  e_j = e^{-2 pi i cyc_j},
//   cyc_j = f_ref dphi_m(t_j) + fdot (t_j^2/2 + phi_m(t_j) t_j) + f j dt,
// (dphi_m = phi_m - phi_m(0); the constant f_ref phi_m(0) is a common phase),
// likewise S_b, and A, B, C over the detector samples; F as in fstat_grid.
//
// Adjoint: with F = num / D, num = B|S_a|^2 + A|S_b|^2 - 2C Re(S_a S_b*),
// D = sigma^2 (AB - C^2), a change dS_a moves F by Re(conj(g_a) dS_a) with
// g_a = 2 (B S_a - C S_b)/D (and g_b = 2 (A S_b - C S_a)/D).  Per sample,
//   dF/dtheta += dw_a Re(E_a) + 2 pi w_a dcyc Im(E_a) + (same for b),
//   E_a = conj(g_a) e_j,
// plus F_A dA/dtheta + F_B dB/dtheta + F_C dC/dtheta from the detector-grid
// sums.  The sample-level derivatives go through t_j by implicit
// differentiation of t_j + phi_m(t_j) = t_b0(alpha, delta) + j dt:
//   dt_j/dtheta = (dt_b0/dtheta - dphi_m/dtheta(t_j)) / (1 + phi_m'(t_j)).
// The forward state (S_a, S_b, A, B, C) is kept; the resampled series is
// recomputed, never stored.
#include "candidate.h"

namespace {

__global__ void __launch_bounds__(GB)
k_eval(const SegDev* __restrict__ segs, int nseg, const int32_t* __restrict__ segi,
       const double* __restrict__ params, double* __restrict__ Fout, double* __restrict__ state) {
  __shared__ double sh[(GB / 64) * 4];
  const int64_t ci = blockIdx.x;
  const int si = segi ? segi[ci] : 0;
  if (si < 0 || si >= nseg) {  // invalid segment index: NaN result, nothing read
    if (threadIdx.x == 0) Fout[ci + threadIdx.x] = __builtin_nan("");
    return;
  }
  const SegDev sg = segs[si];
  const Cand c{params[4 * ci], params[4 * ci + 1], params[4 * ci + 2], params[4 * ci + 3]};
  SkyConst k;
  setup_sky(sg, c, k);
  double acc[4] = {0, 0, 0, 0};
  for (int64_t j = threadIdx.x; j < sg.n; j += GB) method_terms(sg, k, c, j, acc);
  block_sums<4>(acc, sh);
  if (threadIdx.x == 0) {
    const double Sar = acc[0], Sai = acc[1], Sbr = acc[2], Sbi = acc[3];
    double A, B, C;
    abc_moments(sg, k, A, B, C);
    const double num = B * (Sar * Sar + Sai * Sai) + A * (Sbr * Sbr + Sbi * Sbi) - 2.0 * C * (Sar * Sbr + Sai * Sbi);
    Fout[ci + threadIdx.x] = num / (sg.sigma2 * (A * B - C * C));
    if (state) {
      double* st = state + FSTATE * ci + threadIdx.x;
      st[0] = Sar;
      st[1] = Sai;
      st[2] = Sbr;
      st[3] = Sbi;
      st[4] = A;
      st[5] = B;
      st[6] = C;
      st[7] = 0.0;
    }
  }
}

struct Partials {  // phi_m partials w.r.t. alpha, delta, and time derivative
  double al, de, T;
};
__device__ __forceinline__ Partials roemer_partials(const SegDev& sg, const SkyConst& k, const Ephem& e) {
  const SegGeo& g = sg.geo;
  const double wo = TWO_PI * g.orb_rate_c, wr = TWO_PI * g.sid_rate_c;
  Partials p;
  p.al = k.nx_a * (e.xes + e.xe) + k.nye_a * e.yes + k.ny_a * e.ye + k.nz_a * e.ze;
  p.de = k.nx_d * (e.xes + e.xe) + k.nye_d * e.yes + k.ny_d * e.ye + k.nz_d * e.ze;
  const double dxes = -g.orb_r * wo * e.sor, dyes = g.orb_r * wo * e.cor;
  const double dxe = -g.site_rc * wr * e.sth, dye = g.site_rc * wr * e.cth;
  p.T = k.nx * (dxes + dxe) + k.nye * dyes + k.ny * dye;
  return p;
}

struct AbPartials {
  double a, b, ax, bx, ad, bd;  // values, d/dx (x = alpha - sidereal angle), d/ddelta
};
__device__ __forceinline__ AbPartials ab_partials(const SkyConst& k, const HourAngle& h) {
  AbPartials r;
  amp_ab(k, h, r.a, r.b);
  r.ax = -2.0 * k.a2c * h.s2 + 2.0 * k.a2s * h.c2 - k.a1c * h.s1 + k.a1s * h.c1;
  r.bx = -2.0 * k.b2c * h.s2 + 2.0 * k.b2s * h.c2 - k.b1c * h.s1 + k.b1s * h.c1;
  r.ad = k.da2c * h.c2 + k.da2s * h.s2 + k.da1c * h.c1 + k.da1s * h.s1 + k.da0;
  r.bd = k.db2c * h.c2 + k.db2s * h.s2 + k.db1c * h.c1 + k.db1s * h.s1;
  return r;
}

__global__ void __launch_bounds__(GB)
k_adjoint(const SegDev* __restrict__ segs, int nseg, const int32_t* __restrict__ segi,
          const double* __restrict__ params, const double* __restrict__ state, const double* __restrict__ gF,
          double* __restrict__ dp) {
  __shared__ double sh[(GB / 64) * 4];
  const int64_t ci = blockIdx.x;
  const int si = segi ? segi[ci] : 0;
  if (si < 0 || si >= nseg) {
    if (threadIdx.x < 4) dp[4 * ci + threadIdx.x] = __builtin_nan("");
    return;
  }
  const SegDev sg = segs[si];
  const Cand c{params[4 * ci], params[4 * ci + 1], params[4 * ci + 2], params[4 * ci + 3]};
  SkyConst k;
  setup_sky(sg, c, k);
  const double* st = state + FSTATE * ci;
  const double Sar = st[0], Sai = st[1], Sbr = st[2], Sbi = st[3], A = st[4], B = st[5], C = st[6];
  const double s2 = sg.sigma2;
  const double D = s2 * (A * B - C * C);
  const double Sa2 = Sar * Sar + Sai * Sai, Sb2 = Sbr * Sbr + Sbi * Sbi, Rab = Sar * Sbr + Sai * Sbi;
  const double num = B * Sa2 + A * Sb2 - 2.0 * C * Rab;
  // adjoint weights of S_a, S_b and partials of F w.r.t. A, B, C
  const double gar = 2.0 * (B * Sar - C * Sbr) / D, gai = 2.0 * (B * Sai - C * Sbi) / D;
  const double gbr = 2.0 * (A * Sbr - C * Sar) / D, gbi = 2.0 * (A * Sbi - C * Sai) / D;
  const double FA = Sb2 / D - num * s2 * B / (D * D);
  const double FB = Sa2 / D - num * s2 * A / (D * D);
  const double FC = -2.0 * Rab / D + num * s2 * 2.0 * C / (D * D);
  const double wr = TWO_PI * sg.geo.sid_rate_c;
  const Partials p0 = roemer_partials(sg, k, ephem(sg.geo, 0.0));  // d t_b0 / d(alpha, delta)

  double acc[4] = {0, 0, 0, 0};
  for (int64_t j = threadIdx.x; j < sg.n; j += GB) {
    const double jdt = (double)j * sg.dt;
    const SampleGeo sgeo = sample_geo(sg.geo, k, jdt);
    const double t = sgeo.t, dpm = sgeo.dpm;
    const double pm = k.tb0 + dpm;
    double xr, dxdu;
    interp_d(sg, j, -dpm / sg.dt, xr, dxdu);
    const AbPartials ab = ab_partials(k, hour_angle(k, sgeo.cth, sgeo.sth));
    const Partials pp = roemer_partials(sg, k, ephem_of(sg.geo, sgeo));  // absolute positions at t
    double cyc = sg.f_ref * dpm + c.fdot * (0.5 * t * t + pm * t) + c.f * jdt;
    cyc -= rint(cyc);
    double s, co;
    sincospi(2.0 * cyc, &s, &co);
    // E = conj(g) e, e = (co, -s)
    const double Ear = gar * co - gai * s, Eai = -gar * s - gai * co;
    const double Ebr = gbr * co - gbi * s, Ebi = -gbr * s - gbi * co;
    const double wa = xr * ab.a, wb = xr * ab.b;
    // f and fdot: phase only
    acc[0] += TWO_PI * jdt * (wa * Eai + wb * Ebi);
    const double Q = 0.5 * t * t + pm * t;
    acc[1] += TWO_PI * Q * (wa * Eai + wb * Ebi);
    // alpha, delta
    const double den = 1.0 + pp.T;
#pragma unroll
    for (int th = 0; th < 2; ++th) {
      const double dtb0 = th == 0 ? p0.al : p0.de;
      const double dpmx = th == 0 ? pp.al : pp.de;
      const double dtj = (dtb0 - dpmx) / den;
      const double dxr = dxdu * dtj / sg.dt;
      const double dx = (th == 0 ? 1.0 : 0.0) - wr * dtj;
      const double da = ab.ax * dx + (th == 1 ? ab.ad : 0.0);
      const double db = ab.bx * dx + (th == 1 ? ab.bd : 0.0);
      const double dpm_th = dpmx + pp.T * dtj;
      const double dcyc = sg.f_ref * dpm_th + c.fdot * (t * dtj + dpm_th * t + pm * dtj);
      const double dwa = dxr * ab.a + xr * da, dwb = dxr * ab.b + xr * db;
      acc[2 + th] += dwa * Ear + TWO_PI * wa * dcyc * Eai + dwb * Ebr + TWO_PI * wb * dcyc * Ebi;
    }
  }
  block_sums<4>(acc, sh);
  if (threadIdx.x == 0) {
    // A, B, C on the detector samples: their alpha and delta derivatives from
    // the mask moments
    AbPoly fa, fb, fa_al, fb_al, fa_de, fb_de;
    ab_poly(k, fa, fb);
    ab_poly_partials(k, fa, fb, fa_al, fb_al, fa_de, fb_de);
    const double* mom = sg.mom;
    const double dA_al = 2.0 * moment_sum(fa.v, fa_al.v, mom), dA_de = 2.0 * moment_sum(fa.v, fa_de.v, mom);
    const double dB_al = 2.0 * moment_sum(fb.v, fb_al.v, mom), dB_de = 2.0 * moment_sum(fb.v, fb_de.v, mom);
    const double dC_al = moment_sum(fa_al.v, fb.v, mom) + moment_sum(fa.v, fb_al.v, mom);
    const double dC_de = moment_sum(fa_de.v, fb.v, mom) + moment_sum(fa.v, fb_de.v, mom);
    acc[2] += FA * dA_al + FB * dB_al + FC * dC_al;
    acc[3] += FA * dA_de + FB * dB_de + FC * dC_de;
    const double w = gF ? gF[ci] : 1.0;
    double* o = dp + 4 * ci + threadIdx.x;
    o[0] = w * acc[0];
    o[1] = w * acc[1];
    o[2] = w * acc[2];
    o[3] = w * acc[3];
  }
}

// Second step of the ML estimation (Sec. III): the amplitudes of Eq. (ampone)
// from the correlations of k_eval, and their inversion.  One thread per
// candidate.  The correlations leave out the phase 2 pi (f_ref + f) phi_m(0)
// common to S_a and S_b; it is restored first.  With h1..h4 = a cos, b cos,
// a sin, b sin of the phase the normal equations are
//   [A C; C B] (A1, A2) = 2 (Re S_a, Re S_b),  [A C; C B] (A3, A4) = -2 (Im S_a, Im S_b)
// (Eq. amle0 when C = 0).  Inversion: z1 = A1 + i A2, z2 = A4 - i A3 satisfy
// z1 +- z2 = (h0+ +- h0x) e^{i(2 psi +- phi0)}; h0 = h0+ + sqrt(h0+^2 - h0x^2),
// cos iota = h0x / h0 (Eq. h0iota).  psi in [0, pi/2), phi0 in [0, 2 pi).
__global__ void k_amplitudes(const SegDev* __restrict__ segs, int nseg, const int32_t* __restrict__ segi,
                             const double* __restrict__ params, const double* __restrict__ state, int64_t n,
                             double* __restrict__ out) {
  const int64_t ci = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ci >= n) return;
  double* o = out + 8 * ci;
  const int si = segi ? segi[ci] : 0;
  if (si < 0 || si >= nseg) {
    for (int q = 0; q < 8; ++q) o[q] = __builtin_nan("");
    return;
  }
  const SegDev sg = segs[si];
  const Cand c{params[4 * ci], params[4 * ci + 1], params[4 * ci + 2], params[4 * ci + 3]};
  SkyConst k;
  setup_sky(sg, c, k);
  const double* st = state + FSTATE * ci;
  double turns = (sg.f_ref + c.f) * k.tb0;
  turns -= rint(turns);
  double sn, cs;
  sincospi(2.0 * turns, &sn, &cs);
  // S e^{-i theta0}
  const double sar = st[0] * cs + st[1] * sn, sai = st[1] * cs - st[0] * sn;
  const double sbr = st[2] * cs + st[3] * sn, sbi = st[3] * cs - st[2] * sn;
  const double A = st[4], B = st[5], C = st[6];
  const double w = 2.0 / ((A * B - C * C) * sg.geo.sin_zeta);
  const double a1 = w * (B * sar - C * sbr), a2 = w * (A * sbr - C * sar);
  const double a3 = -w * (B * sai - C * sbi), a4 = -w * (A * sbi - C * sai);
  const double zpr = a1 + a4, zpi = a2 - a3, zmr = a1 - a4, zmi = a2 + a3;
  const double mp = sqrt(zpr * zpr + zpi * zpi), mm = sqrt(zmr * zmr + zmi * zmi);
  const double hp = 0.5 * (mp + mm), hx = 0.5 * (mp - mm);
  const double h0 = hp + sqrt(mp * mm);
  const double ap = mp > 0.0 ? atan2(zpi, zpr) : 0.0;
  const double am = mm > 0.0 ? atan2(zmi, zmr) : 0.0;
  const double half_pi = 1.5707963267948966192313216916398;
  double psi = 0.25 * (ap + am), phi0 = 0.5 * (ap - am);
  const double shift = floor(psi / half_pi);
  psi -= shift * half_pi;
  phi0 -= shift * 2.0 * half_pi;
  phi0 -= floor(phi0 / (4.0 * half_pi)) * (4.0 * half_pi);
  o[0] = a1;
  o[1] = a2;
  o[2] = a3;
  o[3] = a4;
  o[4] = h0;
  o[5] = h0 > 0.0 ? hx / h0 : 0.0;
  o[6] = psi;
  o[7] = phi0;
}

}  // namespace

namespace fsk {

hipError_t amplitudes(const SegDev* d_segs, int nseg, const int32_t* d_seg, const double* d_params, int64_t n,
                      const double* d_state, double* d_out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_amplitudes, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, st, d_segs, nseg, d_seg,
                     d_params, d_state, n, d_out);
  return hipGetLastError();
}


hipError_t grad_forward(const SegDev* d_segs, int nseg, const int32_t* d_seg, const double* d_params, int64_t n,
                        double* d_F, double* d_state, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_eval, dim3((unsigned)n), dim3(GB), 0, st, d_segs, nseg, d_seg, d_params, d_F, d_state);
  return hipGetLastError();
}

hipError_t grad_adjoint(const SegDev* d_segs, int nseg, const int32_t* d_seg, const double* d_params, int64_t n,
                        const double* d_state, const double* d_gF, double* d_dp, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_adjoint, dim3((unsigned)n), dim3(GB), 0, st, d_segs, nseg, d_seg, d_params, d_state, d_gF,
                     d_dp);
  return hipGetLastError();
}

}  // namespace fsk
