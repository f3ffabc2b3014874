// Sky-level preparation, shared by all spindowns of a sky position
// (Sec. IV: the spindown basis vectors of the grid carry no sky components, so
// the resampling is done once per sky position and reused).
//
//   sky_setup     per sky: n0 components, a/b coefficients, t_b0 = phi_m(0)
//   sky_prep      per (sky, sample): invert t_b -> t (FP64), interpolate the
//                 data at t (Sec. VI A), a(t), b(t), Roemer delay; the
//                 ephemeris of a sample is shared by a group of sky positions
//   sky_finalize  per sky: the detector-grid sums A, B, C of the F combination
//                 from the segment's mask moments, and the combination
//                 coefficients
//   mask_moments  per segment (plan time): M_k = sum_i m_i e^{i k theta_i},
//                 k = 0..4, theta_i the sidereal angle of detector sample i
//
// A, B, C from moments: a and b are trigonometric polynomials of degree 2 in
// the hour angle H = alpha - theta (Sec. II), so in z = e^{i theta}
//   a = sum_{h=-2..2} a_h z^h,  a_0 = a0,  a_h = conj(w)^h (c_h + i s_h) / 2,
//   a_{-h} = conj(a_h),  w = e^{i alpha},
// with c_h, s_h the cos hH and sin hH coefficients (b alike, b_0 = 0).  The
// product of two such polynomials f g has coefficients
// (fg)_k = sum_h f_h g_{k-h}, |k| <= 4, and, both being real,
//   sum_i m_i f(theta_i) g(theta_i) = (fg)_0 M_0 + 2 Re sum_{k=1..4} (fg)_k M_k.
// This is the direct sum over the samples rearranged (no approximation); the
// moments are shared by every sky position of the segment.
#include "demod.h"
#include "internal.h"

namespace {

constexpr int SKY_BLOCK = 256;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// Fixed-order block sum; result valid in thread 0.
template <int BLOCK>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  const int tid = threadIdx.x;
  v = wave_sum(v);
  __syncthreads();
  if ((tid & 63) == 0) sh[tid >> 6] = v;
  __syncthreads();
  v = 0.0;
  if (tid < 64) {
    v = (tid < BLOCK / 64) ? sh[tid] : 0.0;
    v = wave_sum(v);
  }
  return v;
}

__global__ void k_sky_setup(const double* __restrict__ ad, int nsky, SegGeo g, SkyConst* __restrict__ out) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsky) return;
  SkyConst k;
  sky_const(ad[2 * s], ad[2 * s + 1], g, k);
  const Ephem e = ephem(g, 0.0);
  k.tb0 = roemer(k, e);
  out[s] = k;
}

template <typename T> struct DataPtrs;
template <> struct DataPtrs<float> {
  static __device__ __forceinline__ const float* x(const SegDev& s) { return s.xf; }
  static __device__ __forceinline__ const float* y(const SegDev& s) { return s.yf; }
  static __device__ __forceinline__ const float* M(const SegDev& s) { return s.Mf; }
};
template <> struct DataPtrs<double> {
  static __device__ __forceinline__ const double* x(const SegDev& s) { return s.x; }
  static __device__ __forceinline__ const double* y(const SegDev& s) { return s.y; }
  static __device__ __forceinline__ const double* M(const SegDev& s) { return s.M; }
};

// x at the fractional sample position u = j + off, 0 outside [0, N-1].  The
// position is carried as the integer j plus the small offset off = -dphi_m/dt
// (a few hundred samples at most), so the interpolation weight holds only the
// rounding of off, not that of the absolute time j dt.
// The first barycentric sample lands exactly on t = 0 (t_b0 = phi_m(0)); a
// margin of SPAN_EPS samples keeps its last rounding bit from deciding whether
// it is inside the data span.  Positions within the margin are clamped.
template <typename T, int INTERP>
__device__ __forceinline__ T interp_at(const SegDev& sg, int64_t j, double off) {
  const int64_t n = sg.n;
  const double lo = -(double)j, hi = (double)(n - 1 - j);  // exact integers
  if (!(off >= lo - SPAN_EPS && off <= hi + SPAN_EPS)) return (T)0;
  off = fmin(fmax(off, lo), hi);
  if constexpr (INTERP == 0) {
    const int64_t i = j + (int64_t)floor(off + 0.5);
    return DataPtrs<T>::x(sg)[i];
  } else {
    const double w = 2.0 * off;
    const double fl = floor(w);
    int64_t i = 2 * j + (int64_t)fl;
    if (i > 2 * n - 2) i = 2 * n - 2;
    const T s = (T)(w - fl);
    const T* y = DataPtrs<T>::y(sg);
    const T y0 = y[i], y1 = y[i + 1];
    if constexpr (INTERP == 1) {
      return ((T)1 - s) * y0 + s * y1;
    } else {
      const T* M = DataPtrs<T>::M(sg);
      const T r = (T)1 - s;
      return r * y0 + s * y1 + ((r * r * r - r) * M[i] + (s * s * s - s) * M[i + 1]) * (T)(1.0 / 6.0);
    }
  }
}

// Sky positions per thread of k_sky_prep: the ephemeris at a sample's time is
// shared by all of them.
constexpr int SKY_GROUP = 8;

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

// Per (sky, sample j): the detector time t of the barycentric grid point
// t_b0 + j dt, i.e. t = j dt - d with d = dphi_m(t), then x(t) by
// interpolation, a(t), b(t) and the demodulation record.  d is found from
// d0 = dphi_m(j dt) by one step of the fixed-point relation linearised at d0:
// d = (dphi_m(t1) + dphi_m'(t1) d0) / (1 + dphi_m'(t1)), t1 = j dt - d0.  d0
// is within |dphi_m'| x 500 s ~ 0.05 s of the solution and the curvature of
// dphi_m is below 1e-10 s/s^2, so the step leaves ~1e-13 s (a phase error of
// 5e-11 turns at 435 Hz); a second step would change rounding only.  A
// thread takes one sample for SKY_GROUP sky positions.
template <typename T, int INTERP>
__global__ void __launch_bounds__(SKY_BLOCK)
k_sky_prep(SegDev sg, const SkyConst* __restrict__ skies, int nsky, Quad<T>* __restrict__ out,
           int64_t stride) {
  const int s0 = blockIdx.y * SKY_GROUP;
  const int ng = min(SKY_GROUP, nsky - s0);
  const int64_t pos = (int64_t)blockIdx.x * SKY_BLOCK + threadIdx.x;
  const int64_t total = (int64_t)sg.R * sg.Ceff;
  constexpr double TWO_PI = 6.28318530717958647692;

  if (pos < total) {
    const int64_t r = pos / sg.Ceff;
    const int64_t c = pos - r * sg.Ceff;
    const int64_t j = r + (int64_t)sg.R * c;
    if (j < sg.n) {
      const EphemBase b = ephem_base(sg.geo, (double)j * sg.dt);
      for (int g = 0; g < ng; ++g) {
        const SkyConst& k = skies[s0 + g];
        double d, dd, v, dv;
        roemer_at(sg.geo, k, b, 0.0, d, dd);
        roemer_at(sg.geo, k, b, d, v, dv);
        const double dpm = (v + dv * d) / (1.0 + dv);
        double ss, cs;
        small_sincos(TWO_PI * sg.geo.sid_rate_c * dpm, ss, cs);
        const double sth = b.sth * cs - b.cth * ss, cth = b.cth * cs + b.sth * ss;
        const T xr = interp_at<T, INTERP>(sg, j, -dpm / sg.dt);
        double a, bb;
        amp_ab(k, hour_angle(k, cth, sth), a, bb);
        double p = sg.f_ref * dpm;
        p -= rint(p);
        Quad<T> q;
        q.wa = xr * (T)a;
        q.wb = xr * (T)bb;
        q.p0 = (T)p;
        q.dd = (T)dpm;
        out[(int64_t)(s0 + g) * stride + pos] = q;
      }
    } else {
      for (int g = 0; g < ng; ++g) out[(int64_t)(s0 + g) * stride + pos] = Quad<T>{(T)0, (T)0, (T)0, (T)0};
    }
  }
}

// per sky (one thread): A, B, C from the mask moments, then the coefficients
// of the F combination
__device__ __forceinline__ cpx<double> cpow_conj(const SkyConst& k, int h) {
  const cpx<double> w{k.ca, -k.sa};  // conj(e^{i alpha})
  return h == 1 ? w : cmul(w, w);
}

// sum_i m_i f(theta_i) g(theta_i) for f, g given by their coefficients in
// z^h, h = 0..2 (negative h: conjugates)
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

__global__ void k_sky_finalize(const SkyConst* __restrict__ sky, int nsky, const double* __restrict__ mom,
                               double sigma2, SkyCoef* __restrict__ coef) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= nsky) return;
  const SkyConst& k = sky[s];
  const cpx<double> w1 = cpow_conj(k, 1), w2 = cpow_conj(k, 2);
  const cpx<double> fa[3] = {{k.a0, 0.0}, cmul(w1, cpx<double>{0.5 * k.a1c, 0.5 * k.a1s}),
                             cmul(w2, cpx<double>{0.5 * k.a2c, 0.5 * k.a2s})};
  const cpx<double> fb[3] = {{0.0, 0.0}, cmul(w1, cpx<double>{0.5 * k.b1c, 0.5 * k.b1s}),
                             cmul(w2, cpx<double>{0.5 * k.b2c, 0.5 * k.b2s})};
  const double A = moment_sum(fa, fa, mom);
  const double B = moment_sum(fb, fb, mom);
  const double C = moment_sum(fa, fb, mom);
  const double D = sigma2 * (A * B - C * C);
  SkyCoef o;
  o.A = A;
  o.B = B;
  o.C = C;
  o.cB = B / D;
  o.cA = A / D;
  o.cC = 2.0 * C / D;
  coef[s] = o;
}

constexpr int MOM_BLOCKS_MAX = 256;

// per workgroup: partial moments over a grid-stride share of the samples
__global__ void __launch_bounds__(SKY_BLOCK) k_mask_moments(SegDev sg, double* __restrict__ part) {
  __shared__ double sh[SKY_BLOCK / 64];
  double acc[9];
#pragma unroll
  for (int q = 0; q < 9; ++q) acc[q] = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * SKY_BLOCK + threadIdx.x; i < sg.n; i += (int64_t)gridDim.x * SKY_BLOCK) {
    const double m = sg.mask ? (sg.mask[i] ? 1.0 : 0.0) : 1.0;
    double cs = sg.geo.sid_c0 + (double)i * sg.dt * sg.geo.sid_rate_c;  // theta_i / 2 pi
    cs -= rint(cs);
    acc[0] += m;
#pragma unroll
    for (int kk = 1; kk <= 4; ++kk) {
      double sn, cn;
      sincospi(2.0 * kk * cs, &sn, &cn);
      acc[2 * kk - 1] += m * cn;
      acc[2 * kk] += m * sn;
    }
  }
#pragma unroll
  for (int q = 0; q < 9; ++q) {
    const double v = block_sum<SKY_BLOCK>(acc[q], sh);
    if (threadIdx.x == 0) part[(int64_t)blockIdx.x * 9 + q] = v;
  }
}

// fixed-order sum of the partials (one thread per moment component)
__global__ void k_mask_moments_sum(const double* __restrict__ part, int nblk, double* __restrict__ mom) {
  const int q = threadIdx.x;
  if (q >= 9) return;
  double v = 0.0;
  for (int b = 0; b < nblk; ++b) v += part[(int64_t)b * 9 + q];
  // layout (Re, Im) per k: M_0 = (v0, 0), M_k = (v_{2k-1}, v_{2k})
  if (q == 0) {
    mom[0] = v;
    mom[1] = 0.0;
  } else {
    mom[q + 1] = v;
  }
}

template <typename T>
__global__ void k_demod_series(SegDev sg, const SkyConst* __restrict__ sky, const Quad<T>* __restrict__ q,
                               double fdot, double fshift, double* __restrict__ out) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= sg.n) return;
  const int64_t r = j % sg.R, c = j / sg.R;
  const Pair<T> z = demod_elem<T>(q[r * sg.Ceff + c], sky[0].tb0, j, sg.dt, fdot, fshift);
  out[4 * j] = (double)z.a.x;
  out[4 * j + 1] = (double)z.a.y;
  out[4 * j + 2] = (double)z.b.x;
  out[4 * j + 3] = (double)z.b.y;
}

}  // namespace

namespace fsk {

hipError_t sky_setup(const double* d_ad, int nsky, const SegDev& seg, SkyConst* d_out, hipStream_t st) {
  if (nsky <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sky_setup, dim3((nsky + 63) / 64), dim3(64), 0, st, d_ad, nsky, seg.geo, d_out);
  return hipGetLastError();
}

int sky_prep_blocks(const SegDev& seg) {
  const int64_t total = (int64_t)seg.R * seg.Ceff;
  return (int)((total + SKY_BLOCK - 1) / SKY_BLOCK);
}

hipError_t sky_prep(int prec, const SegDev& seg, const SkyConst* d_sky, int nsky, void* d_quads,
                    int64_t stride, hipStream_t st) {
  if (nsky <= 0) return hipSuccess;
  dim3 grid(sky_prep_blocks(seg), (nsky + SKY_GROUP - 1) / SKY_GROUP), block(SKY_BLOCK);
#define SKY_CASE(T, I) \
  hipLaunchKernelGGL((k_sky_prep<T, I>), grid, block, 0, st, seg, d_sky, nsky, (Quad<T>*)d_quads, stride)
  if (prec == 0) {
    if (seg.interp == 0) SKY_CASE(float, 0);
    else if (seg.interp == 1) SKY_CASE(float, 1);
    else SKY_CASE(float, 2);
  } else {
    if (seg.interp == 0) SKY_CASE(double, 0);
    else if (seg.interp == 1) SKY_CASE(double, 1);
    else SKY_CASE(double, 2);
  }
#undef SKY_CASE
  return hipGetLastError();
}

hipError_t sky_finalize(const SegDev& seg, const SkyConst* d_sky, int nsky, SkyCoef* d_coef, hipStream_t st) {
  if (nsky <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sky_finalize, dim3((nsky + 63) / 64), dim3(64), 0, st, d_sky, nsky, seg.mom, seg.sigma2,
                     d_coef);
  return hipGetLastError();
}

int mask_moment_blocks(const SegDev& seg) {
  const int64_t b = (seg.n + SKY_BLOCK - 1) / SKY_BLOCK;
  return (int)(b < MOM_BLOCKS_MAX ? b : MOM_BLOCKS_MAX);
}

hipError_t mask_moments(const SegDev& seg, double* d_part, double* d_mom, hipStream_t st) {
  const int nblk = mask_moment_blocks(seg);
  hipLaunchKernelGGL(k_mask_moments, dim3(nblk), dim3(SKY_BLOCK), 0, st, seg, d_part);
  hipLaunchKernelGGL(k_mask_moments_sum, dim3(1), dim3(64), 0, st, (const double*)d_part, nblk, d_mom);
  return hipGetLastError();
}

hipError_t demod_series(int prec, const SegDev& seg, const SkyConst* d_sky, const void* d_quads, int64_t,
                        double fdot, double fshift, double* d_out, hipStream_t st) {
  dim3 grid((unsigned)((seg.n + 255) / 256)), block(256);
  if (prec == 0)
    hipLaunchKernelGGL(k_demod_series<float>, grid, block, 0, st, seg, d_sky, (const Quad<float>*)d_quads, fdot,
                       fshift, d_out);
  else
    hipLaunchKernelGGL(k_demod_series<double>, grid, block, 0, st, seg, d_sky, (const Quad<double>*)d_quads,
                       fdot, fshift, d_out);
  return hipGetLastError();
}

}  // namespace fsk
