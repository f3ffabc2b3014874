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
#include "tiles.h"

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
  if (s < nsky) out[s] = sky_setup_one(ad[2 * s], ad[2 * s + 1], g);
}

template <typename T, int INTERP>
__global__ void __launch_bounds__(SKY_BLOCK)
k_sky_prep(SegDev sg, const SkyConst* __restrict__ skies, int nsky, Quad<T>* __restrict__ out,
           int64_t stride) {
  const int s0 = blockIdx.y * SKY_GROUP;
  sky_prep_pos<T, INTERP>(sg, skies + s0, min(SKY_GROUP, nsky - s0), (int64_t)blockIdx.x * SKY_BLOCK + threadIdx.x,
                          out + (int64_t)s0 * stride, stride);
}

// per sky (one thread): A, B, C from the mask moments, then the coefficients
// of the F combination
__global__ void k_sky_finalize(const SkyConst* __restrict__ sky, int nsky, const double* __restrict__ mom,
                               double sigma2, SkyCoef* __restrict__ coef) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s < nsky) coef[s] = sky_coef_one(sky[s], mom, sigma2);
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
