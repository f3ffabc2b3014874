// Plan-time preparation of a data segment (node-independent, FP64):
//   * gap mask applied, FP32 copy;
//   * noise variance (unbiased, outside gaps) when the caller gives none;
//   * the first step of the two-step resampling (Sec. VI A): 2x upsampling by
//     zero-padding the DFT of the data, and for the cubic variant the second
//     derivatives of the periodic cubic spline through the 2N-point series.
//
// With X the N-point DFT of x and kappa_k the signed frequency of bin k
// (k, or k - N above N/2; the Nyquist bin of an even N is split evenly between
// +N/2 and -N/2), the 2N-point band-limited series is
//   y(s) = (1/N) sum_k X_k e^{2 pi i kappa_k s / N},  y[2m] = x[m],
// and its odd samples are an N-point inverse DFT:
//   y[2m+1] = IDFT_N( P X )[m],   P_k = e^{i pi kappa_k / N}  (0 at Nyquist).
// The periodic spline through (n, y_n), n < 2N, has second derivatives
//   M_n = (1/N) sum_k G_k X_k e^{2 pi i kappa_k (n/2) / N},
//   G_k = 6 (2 cos(pi kappa_k/N) - 2) / (4 + 2 cos(pi kappa_k/N)),
// which is the cyclic tridiagonal system M_{n-1} + 4 M_n + M_{n+1} =
// 6 (y_{n-1} - 2 y_n + y_{n+1}) solved in its eigenbasis.  Hence
//   M[2m] = IDFT_N(G X)[m],  M[2m+1] = IDFT_N(G P X)[m].
// All spectra are Hermitian, so y_odd and M_even share one complex IDFT.
//
// N is arbitrary (the workloads have N = 2^a 13 1657 ...), so the N-point DFTs
// use Bluestein's chirp-z identity, jk = (j^2 + k^2 - (k-j)^2)/2, with
// power-of-two FFTs of length L >= 2N - 1.
#include "fft_block.h"
#include "internal.h"

namespace {

constexpr int gen_block(int nb) { return nb < 64 ? 64 : (nb > 256 ? 256 : nb); }
constexpr int GEN_CMAX = 4096;                 // longest single-workgroup FP64 transform
constexpr int gen_ncol(int R) { return 2048 / R < 32 ? (2048 / R < 1 ? 1 : 2048 / R) : 32; }

__global__ void k_twiddles_f64(cpx<double>* __restrict__ tab, int64_t denom, int64_t count, int64_t step) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= count) return;
  double s, c;
  sincospi(-2.0 * (double)((m * step) % denom) / (double)denom, &s, &c);
  tab[m] = cpx<double>{c, s};
}
__global__ void k_twiddles_f32(cpx<float>* __restrict__ tab, int64_t denom, int64_t count, int64_t step) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= count) return;
  double s, c;
  sincospi(-2.0 * (double)((m * step) % denom) / (double)denom, &s, &c);
  tab[m] = cpx<float>{(float)c, (float)s};
}

// ---------------------------------------------------------------------------
// generic power-of-two complex FFT in FP64 (plan time only)
// ---------------------------------------------------------------------------
template <int L, int DIR>
__global__ void __launch_bounds__(gen_block(L / 16))
k_fft_small(cpx<double>* __restrict__ data, const cpx<double>* __restrict__ tw) {
  __shared__ cpx<double> lds[lds_slots(L, 1)];
  auto load = [&](int i, int) -> cpx<double> { return data[i]; };
  auto store = [&](int i, int, auto& v, auto str) {
    constexpr int RS = std::extent<std::remove_reference_t<decltype(v)>>::value;
#pragma unroll
    for (int q = 0; q < RS; ++q) data[i + q * decltype(str)::value] = v[q];
  };
  block_fft<cpx<double>, L, 1, gen_block(L / 16), DIR>(lds, tw, load, store);
}

// pass A: column r (stride R) -> length-C FFT -> twiddle e^{DIR 2 pi i r k2/(R C)} -> tmp[r][k2]
template <int C, int DIR>
__global__ void __launch_bounds__(gen_block(C / 16))
k_fft_passA(const cpx<double>* __restrict__ in, cpx<double>* __restrict__ tmp, int R,
            const cpx<double>* __restrict__ tw) {
  __shared__ cpx<double> lds[lds_slots(C, 1)];
  const int r = blockIdx.x;
  const int64_t L = (int64_t)R * C;
  auto load = [&](int c, int) -> cpx<double> { return in[r + (int64_t)R * c]; };
  auto store = [&](int i, int, auto& v, auto str) {
    constexpr int RS = std::extent<std::remove_reference_t<decltype(v)>>::value;
#pragma unroll
    for (int q = 0; q < RS; ++q) {
      const int k2 = i + q * decltype(str)::value;
      double s, co;
      sincospi((double)DIR * 2.0 * (double)((int64_t)r * k2) / (double)L, &s, &co);
      tmp[(int64_t)r * C + k2] = cmul(v[q], cpx<double>{co, s});
    }
  };
  block_fft<cpx<double>, C, 1, gen_block(C / 16), DIR>(lds, tw, load, store);
}

// pass B: a block of NCOL columns k2 -> length-R FFTs -> out[C k1 + k2]
template <int R, int DIR>
__global__ void __launch_bounds__(gen_block(gen_ncol(R) * R / 16))
k_fft_passB(const cpx<double>* __restrict__ tmp, cpx<double>* __restrict__ out, int C,
            const cpx<double>* __restrict__ tw) {
  constexpr int NCOL = gen_ncol(R);
  __shared__ cpx<double> lds[lds_slots(R, NCOL)];
  const int cb = blockIdx.x;
  auto load = [&](int r, int col) -> cpx<double> { return tmp[(int64_t)r * C + (int64_t)cb * NCOL + col]; };
  auto store = [&](int i, int col, auto& v, auto str) {
    constexpr int RS = std::extent<std::remove_reference_t<decltype(v)>>::value;
#pragma unroll
    for (int q = 0; q < RS; ++q)
      out[(int64_t)C * (i + q * decltype(str)::value) + (int64_t)cb * NCOL + col] = v[q];
  };
  block_fft<cpx<double>, R, NCOL, gen_block(NCOL * R / 16), DIR>(lds, tw, load, store);
}

template <int DIR>
hipError_t fft_generic(cpx<double>* data, int64_t L, cpx<double>* tmp, cpx<double>* twtab, hipStream_t st) {
  // twtab has room for L entries; holds e^{-2 pi i m / len} for the block lengths in use
  auto twid = [&](cpx<double>* tab, int64_t len) {
    hipLaunchKernelGGL(k_twiddles_f64, dim3((unsigned)((len + 255) / 256)), dim3(256), 0, st, tab, len, len,
                       (int64_t)1);
  };
  if (L <= GEN_CMAX) {
    twid(twtab, L);
#define FS(LL)                                                                                   \
  case LL:                                                                                       \
    hipLaunchKernelGGL((k_fft_small<LL, DIR>), dim3(1), dim3(gen_block(LL / 16)), 0, st, data, twtab); \
    break;
    switch (L) {
      FS(2) FS(4) FS(8) FS(16) FS(32) FS(64) FS(128) FS(256) FS(512) FS(1024) FS(2048) FS(4096)
      default: return hipErrorInvalidValue;
    }
#undef FS
    return hipGetLastError();
  }
  const int C = GEN_CMAX;
  const int R = (int)(L / C);
  cpx<double>* twC = twtab;
  cpx<double>* twR = twtab + C;
  twid(twC, C);
  twid(twR, R);
  hipLaunchKernelGGL((k_fft_passA<GEN_CMAX, DIR>), dim3(R), dim3(gen_block(GEN_CMAX / 16)), 0, st, data, tmp, R,
                     twC);
#define FB(RR)                                                                                      \
  case RR:                                                                                          \
    hipLaunchKernelGGL((k_fft_passB<RR, DIR>), dim3(C / gen_ncol(RR)), dim3(gen_block(gen_ncol(RR) * RR / 16)), \
                       0, st, tmp, data, C, twR);                                                   \
    break;
  switch (R) {
    FB(2) FB(4) FB(8) FB(16) FB(32) FB(64) FB(128) FB(256) FB(512) FB(1024) FB(2048)
    default: return hipErrorInvalidValue;
  }
#undef FB
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Bluestein DFT of arbitrary length N (FP64)
// ---------------------------------------------------------------------------
// chirp w_n = e^{-i pi n^2 / N}, with n^2 reduced mod 2N in integers
__device__ __forceinline__ cpx<double> chirp(int64_t n, int64_t N) {
  const int64_t m = (n * n) % (2 * N);  // n < N <= 2^22: n^2 fits
  double s, c;
  sincospi((double)m / (double)N, &s, &c);
  return cpx<double>{c, -s};
}

// a[n] = z[n] w_n (n < N), 0 elsewhere; b = conj(w) wrapped around
__global__ void k_blue_fill(const cpx<double>* __restrict__ z, int64_t N, int64_t L, cpx<double>* __restrict__ a,
                            cpx<double>* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= L) return;
  a[i] = (i < N) ? cmul(z[i], chirp(i, N)) : cpx<double>{0.0, 0.0};
  if (i < N) b[i] = cconj(chirp(i, N));
  else if (i > L - N) b[i] = cconj(chirp(L - i, N));
  else b[i] = cpx<double>{0.0, 0.0};
}
__global__ void k_cmul_inplace(cpx<double>* __restrict__ a, const cpx<double>* __restrict__ b, int64_t L) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < L) a[i] = cmul(a[i], b[i]);
}
// X[k] = w_k c[k] / L
__global__ void k_blue_out(const cpx<double>* __restrict__ c, int64_t N, int64_t L, cpx<double>* __restrict__ X) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  X[k] = cscale(cmul(c[k], chirp(k, N)), 1.0 / (double)L);
}

inline int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

struct BlueWork {
  cpx<double>*a, *b, *tmp, *tw;
  int64_t L;
};
inline BlueWork blue_carve(void* work, int64_t N) {
  BlueWork w;
  w.L = next_pow2(2 * N - 1 < 2 ? 2 : 2 * N - 1);
  cpx<double>* p = (cpx<double>*)work;
  w.a = p;
  w.b = p + w.L;
  w.tmp = p + 2 * w.L;
  w.tw = p + 3 * w.L;
  return w;
}
inline size_t blue_bytes(int64_t N) {
  const int64_t L = next_pow2(2 * N - 1 < 2 ? 2 : 2 * N - 1);
  return (size_t)(4 * L) * sizeof(cpx<double>);
}

// forward DFT of z (length N) into X, using the work area
hipError_t dft_bluestein(const cpx<double>* z, int64_t N, cpx<double>* X, void* work, hipStream_t st) {
  BlueWork w = blue_carve(work, N);
  const unsigned gL = (unsigned)((w.L + 255) / 256);
  hipLaunchKernelGGL(k_blue_fill, dim3(gL), dim3(256), 0, st, z, N, w.L, w.a, w.b);
  hipError_t e;
  if ((e = fft_generic<-1>(w.a, w.L, w.tmp, w.tw, st)) != hipSuccess) return e;
  if ((e = fft_generic<-1>(w.b, w.L, w.tmp, w.tw, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_cmul_inplace, dim3(gL), dim3(256), 0, st, w.a, w.b, w.L);
  if ((e = fft_generic<1>(w.a, w.L, w.tmp, w.tw, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_blue_out, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, st, w.a, N, w.L, X);
  return hipGetLastError();
}

__global__ void k_conj_scale(cpx<double>* __restrict__ v, int64_t n, double s) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) v[i] = cpx<double>{v[i].x * s, -v[i].y * s};
}

// IDFT_N(V) = conj(DFT_N(conj V)) / N, in place on V (uses out as scratch)
hipError_t idft_bluestein(cpx<double>* V, int64_t N, cpx<double>* out, void* work, hipStream_t st) {
  const unsigned g = (unsigned)((N + 255) / 256);
  hipLaunchKernelGGL(k_conj_scale, dim3(g), dim3(256), 0, st, V, N, 1.0);
  hipError_t e = dft_bluestein(V, N, out, work, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_conj_scale, dim3(g), dim3(256), 0, st, out, N, 1.0 / (double)N);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// segment preparation kernels
// ---------------------------------------------------------------------------
__global__ void k_mask(const double* __restrict__ xraw, const uint8_t* __restrict__ mask, int64_t n,
                       double* __restrict__ x, float* __restrict__ xf) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double v = (mask && !mask[i]) ? 0.0 : xraw[i];
  x[i] = v;
  xf[i] = (float)v;
}

__global__ void k_real_to_cpx(const double* __restrict__ x, int64_t n, cpx<double>* __restrict__ z) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) z[i] = cpx<double>{x[i], 0.0};
}

// unbiased variance of the samples outside gaps, one workgroup, fixed order
__global__ void __launch_bounds__(1024)
k_variance(const double* __restrict__ xraw, const uint8_t* __restrict__ mask, int64_t n, double* __restrict__ out) {
  __shared__ double sh[16];
  __shared__ double mean_s;
  const int tid = threadIdx.x;
  auto bsum = [&](double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
    __syncthreads();
    if ((tid & 63) == 0) sh[tid >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (tid == 0)
      for (int w = 0; w < 16; ++w) t += sh[w];
    return t;
  };
  double s = 0.0, c = 0.0;
  for (int64_t i = tid; i < n; i += 1024) {
    const double m = (mask && !mask[i]) ? 0.0 : 1.0;
    s += m * xraw[i];
    c += m;
  }
  const double S = bsum(s);
  const double Cn = bsum(c);
  if (tid == 0) mean_s = S / Cn;
  __syncthreads();
  const double mu = mean_s;
  double q = 0.0;
  for (int64_t i = tid; i < n; i += 1024) {
    const double m = (mask && !mask[i]) ? 0.0 : 1.0;
    const double d = xraw[i] - mu;
    q += m * d * d;
  }
  const double Q = bsum(q);
  if (tid == 0) out[tid] = Q / (Cn - 1.0);
}

// spectra for the odd samples and the spline: V1 = P X (+ i G X), V2 = G P X
__global__ void k_up_spectra(const cpx<double>* __restrict__ X, int64_t N, int cubic, cpx<double>* __restrict__ V1,
                             cpx<double>* __restrict__ V2) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= N) return;
  const bool nyq = (N % 2 == 0) && (k == N / 2);
  const int64_t kap = nyq ? N / 2 : ((2 * k < N) ? k : k - N);
  double sp, cp;
  sincospi((double)kap / (double)N, &sp, &cp);
  const cpx<double> P = nyq ? cpx<double>{0.0, 0.0} : cpx<double>{cp, sp};
  const cpx<double> PX = cmul(P, X[k]);
  if (!cubic) {
    V1[k] = PX;
    return;
  }
  const double G = 6.0 * (2.0 * cp - 2.0) / (4.0 + 2.0 * cp);
  const cpx<double> GX = cscale(X[k], G);
  V1[k] = cpx<double>{PX.x - GX.y, PX.y + GX.x};  // P X + i G X
  V2[k] = cscale(PX, G);
}

__global__ void k_up_assemble(const double* __restrict__ x, const cpx<double>* __restrict__ o1,
                              const cpx<double>* __restrict__ o2, int64_t N, int cubic, double* __restrict__ y,
                              float* __restrict__ yf, double* __restrict__ M, float* __restrict__ Mf) {
  const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= N) return;
  const double ye = x[m], yo = o1[m].x;
  y[2 * m] = ye;
  y[2 * m + 1] = yo;
  yf[2 * m] = (float)ye;
  yf[2 * m + 1] = (float)yo;
  if (cubic) {
    const double me = o1[m].y, mo = o2[m].x;
    M[2 * m] = me;
    M[2 * m + 1] = mo;
    Mf[2 * m] = (float)me;
    Mf[2 * m + 1] = (float)mo;
  }
}

}  // namespace

namespace fsk {

hipError_t make_twiddles(int prec, int64_t denom, int64_t count, int64_t step, void* d_tab, hipStream_t st) {
  const unsigned g = (unsigned)((count + 255) / 256);
  if (prec == 0)
    hipLaunchKernelGGL(k_twiddles_f32, dim3(g), dim3(256), 0, st, (cpx<float>*)d_tab, denom, count, step);
  else
    hipLaunchKernelGGL(k_twiddles_f64, dim3(g), dim3(256), 0, st, (cpx<double>*)d_tab, denom, count, step);
  return hipGetLastError();
}

hipError_t fft_c2c_f64(cpx<double>* data, int64_t L, int dir, cpx<double>* tmp, cpx<double>* twtab, hipStream_t st) {
  return dir < 0 ? fft_generic<-1>(data, L, tmp, twtab, st) : fft_generic<1>(data, L, tmp, twtab, st);
}

size_t prep_work_bytes(int64_t n) {
  // X, V1, V2, o1, o2 (N each) + z (N) + Bluestein area
  return (size_t)(6 * n) * sizeof(cpx<double>) + blue_bytes(n) + 256;
}

hipError_t prep_mask(const double* xraw, const uint8_t* mask, int64_t n, double* x, float* xf, hipStream_t st) {
  hipLaunchKernelGGL(k_mask, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, xraw, mask, n, x, xf);
  return hipGetLastError();
}

hipError_t prep_variance(const double* xraw, const uint8_t* mask, int64_t n, double* d_out, hipStream_t st) {
  hipLaunchKernelGGL(k_variance, dim3(1), dim3(1024), 0, st, xraw, mask, n, d_out);
  return hipGetLastError();
}

hipError_t prep_upsample(const double* x, int64_t n, int interp, double* y, float* yf, double* M, float* Mf,
                         void* work, hipStream_t st) {
  cpx<double>* p = (cpx<double>*)work;
  cpx<double>* z = p;
  cpx<double>* X = p + n;
  cpx<double>* V1 = p + 2 * n;
  cpx<double>* V2 = p + 3 * n;
  cpx<double>* o1 = p + 4 * n;
  cpx<double>* o2 = p + 5 * n;
  void* blue = (void*)(p + 6 * n);
  const int cubic = (interp == 2);
  const unsigned g = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_real_to_cpx, dim3(g), dim3(256), 0, st, x, n, z);
  hipError_t e = dft_bluestein(z, n, X, blue, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_up_spectra, dim3(g), dim3(256), 0, st, X, n, cubic, V1, V2);
  if ((e = idft_bluestein(V1, n, o1, blue, st)) != hipSuccess) return e;
  if (cubic && (e = idft_bluestein(V2, n, o2, blue, st)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_up_assemble, dim3(g), dim3(256), 0, st, x, o1, o2, n, cubic, y, yf, M, Mf);
  return hipGetLastError();
}

}  // namespace fsk
