// Sky-level preparation, shared by all spindowns of a sky position
// (Sec. IV: the spindown basis vectors of the grid carry no sky components, so
// the resampling is done once per sky position and reused).
//
//   sky_setup     per sky: n0 components, a/b coefficients, t_b0 = phi_m(0)
//   sky_prep      per (sky, sample): invert t_b -> t (FP64), interpolate the
//                 data at t (Sec. VI A), a(t), b(t), Roemer delay; plus the
//                 detector-grid sums A, B, C of the F combination
//   sky_finalize  per sky: fixed-order sum of the A, B, C partials and the
//                 combination coefficients
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

template <typename T, int INTERP>
__global__ void __launch_bounds__(SKY_BLOCK)
k_sky_prep(SegDev sg, const SkyConst* __restrict__ skies, Quad<T>* __restrict__ out, int64_t stride,
           double* __restrict__ abc_part) {
  __shared__ double sh[SKY_BLOCK / 64];
  const int s = blockIdx.y;
  const SkyConst k = skies[s];
  const int64_t pos = (int64_t)blockIdx.x * SKY_BLOCK + threadIdx.x;
  const int64_t total = (int64_t)sg.R * sg.Ceff;

  if (pos < total) {
    const int64_t r = pos / sg.Ceff;
    const int64_t c = pos - r * sg.Ceff;
    const int64_t j = r + (int64_t)sg.R * c;
    Quad<T> q = {(T)0, (T)0, (T)0, (T)0};
    if (j < sg.n) {
      EphemD e;
      double dpm;
      (void)ssb_to_detector(sg.geo, k, (double)j * sg.dt, e, dpm);
      const T xr = interp_at<T, INTERP>(sg, j, -dpm / sg.dt);
      double a, b;
      amp_ab(k, hour_angle(k, e.cth, e.sth), a, b);
      double p = sg.f_ref * dpm;
      p -= rint(p);
      q.wa = xr * (T)a;
      q.wb = xr * (T)b;
      q.p0 = (T)p;
      q.dd = (T)dpm;
    }
    out[(int64_t)s * stride + pos] = q;
  }

  // A, B, C on the detector samples t_i = i dt
  double aa = 0.0, bb = 0.0, ab = 0.0;
  if (pos < sg.n) {
    const Ephem e = ephem(sg.geo, (double)pos * sg.dt);
    double a, b;
    amp_ab(k, hour_angle(k, e), a, b);
    const double m = sg.mask ? (sg.mask[pos] ? 1.0 : 0.0) : 1.0;
    aa = m * a * a;
    bb = m * b * b;
    ab = m * a * b;
  }
  aa = block_sum<SKY_BLOCK>(aa, sh);
  bb = block_sum<SKY_BLOCK>(bb, sh);
  ab = block_sum<SKY_BLOCK>(ab, sh);
  if (threadIdx.x == 0) {
    double* p = abc_part + ((int64_t)s * gridDim.x + blockIdx.x) * 3;
    p[0] = aa;
    p[1] = bb;
    p[2] = ab;
  }
}

// one workgroup per sky: fixed-order sum of the per-block partials
__global__ void __launch_bounds__(SKY_BLOCK)
k_sky_finalize(const double* __restrict__ part, int nblk, double sigma2, SkyCoef* __restrict__ coef) {
  __shared__ double sh[SKY_BLOCK / 64];
  const int s = blockIdx.x;
  const double* p = part + (int64_t)s * nblk * 3;
  double A = 0.0, B = 0.0, C = 0.0;
  for (int i = threadIdx.x; i < nblk; i += SKY_BLOCK) {
    A += p[3 * i];
    B += p[3 * i + 1];
    C += p[3 * i + 2];
  }
  A = block_sum<SKY_BLOCK>(A, sh);
  B = block_sum<SKY_BLOCK>(B, sh);
  C = block_sum<SKY_BLOCK>(C, sh);
  if (threadIdx.x == 0) {
    const double D = sigma2 * (A * B - C * C);
    SkyCoef o;
    o.A = A;
    o.B = B;
    o.C = C;
    o.cB = B / D;
    o.cA = A / D;
    o.cC = 2.0 * C / D;
    coef[s + threadIdx.x] = o;
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
                    int64_t stride, double* d_abc_part, int nblk, hipStream_t st) {
  if (nsky <= 0) return hipSuccess;
  dim3 grid(nblk, nsky), block(SKY_BLOCK);
#define SKY_CASE(T, I) \
  hipLaunchKernelGGL((k_sky_prep<T, I>), grid, block, 0, st, seg, d_sky, (Quad<T>*)d_quads, stride, d_abc_part)
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

hipError_t sky_finalize(const SegDev& seg, const double* d_part, int nblk, int nsky, SkyCoef* d_coef,
                        hipStream_t st) {
  if (nsky <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sky_finalize, dim3(nsky), dim3(SKY_BLOCK), 0, st, d_part, nblk, seg.sigma2, d_coef);
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
