// Tile functions shared by the launch-per-pass kernels (sky.hip, grid.hip) and
// the persistent grid kernel (persist.hip): one workgroup's share of a pass,
// written once so that both launch shapes compute bit-identical results.
//
//   sky_setup_one   per sky: n0 components, a/b coefficients, t_b0 = phi_m(0)
//   sky_prep_pos    per (sample position, group of sky positions): the
//                   resampled, a/b-weighted record of Sec. VI A
//   sky_coef_one    per sky: A, B, C from the mask moments and the
//                   coefficients of the F combination (Eq. OS)
//   pass1_tile      one column of the first FFT pass of a node
//   pass2_tile      one column block of the second FFT pass and the
//                   F combination
#pragma once
#include "demod.h"
#include "fft_block.h"
#include "internal.h"
#include "moments.h"

namespace {

template <typename T>
constexpr int cfg_B2(int R) {
  return sizeof(T) == 4 ? (4096 / R < 64 ? 4096 / R : 64) : (2048 / R < 32 ? 2048 / R : 32);
}
constexpr int cfg_block(int nb) { return nb < 64 ? 64 : (nb > 256 ? 256 : nb); }

// The spill layout for pass 2 blocks of B2 columns (see above).
template <typename T>
constexpr bool spill_blocked(int B2) {
  return B2 * (int)sizeof(Pair<T>) < 512;
}

// Position of spill element (r, k2) within a node's nfft elements in the
// blocked layout; lb2 = log2(B2).  A bijection onto [0, R C) when B2 divides C.
__device__ __forceinline__ int64_t spill_index(int r, int k2, int R, int lb2) {
  const int B2 = 1 << lb2;
  return ((int64_t)(k2 >> lb2) * R + r) * B2 + (k2 & (B2 - 1));
}

// Pass 1 for column r of one node: dst is the node's nfft spill elements,
// lds lds_slots(C, 1) slots.
template <typename T, int C, bool BLK>
__device__ __forceinline__ void pass1_tile(const SegDev& sg, const Quad<T>* __restrict__ quads, int64_t qstride,
                                           const SkyConst* __restrict__ skies, const NodeDev& node, int r,
                                           const cpx<T>* __restrict__ twC, const cpx<T>* __restrict__ twlo,
                                           const cpx<T>* __restrict__ twhi, Pair<T>* __restrict__ dst,
                                           lds_t<Pair<T>>* __restrict__ lds) {
  constexpr int BLOCK = cfg_block(C / 16);
  const Quad<T>* __restrict__ col = quads + (int64_t)node.sky * qstride + (int64_t)r * sg.Ceff;
  const double tb0 = skies[node.sky].tb0;
  const double fdot = node.fdot;
  const double fshift = node.fshift;
  const int ceff = sg.Ceff;
  const int R = sg.R;
  const double dt = sg.dt;
  // columns c >= ceff are the zero padding
  auto make = [&](const Quad<T>& q, int c, int) -> Pair<T> {
    if (c < ceff) return demod_elem<T>(q, tb0, r + R * c, dt, fdot, fshift);
    return Pair<T>{{(T)0, (T)0}, {(T)0, (T)0}};
  };
  const int lb2 = BLK ? __builtin_ctz(cfg_B2<T>(R)) : 0;  // log2 of pass 2's B2 (BLK = spill_blocked)
  // inter-pass twiddle e^{-2 pi i r k2/nfft} for the outputs k2 = i + q STR of a
  // butterfly: (table value at r i) x (table value at r STR)^q
  auto store = [&](int i, int, auto& v, auto str) {
    constexpr int RS = std::extent<std::remove_reference_t<decltype(v)>>::value;
    constexpr int STR = decltype(str)::value;
    const int m0 = r * i, ms = r * STR;  // both < nfft, exact
    const cpx<T> base = cmul(twhi[m0 >> 12], twlo[m0 & 4095]);
    const cpx<T> step = cmul(twhi[ms >> 12], twlo[ms & 4095]);
    cpx<T> pw[RS];
    powers<RS>(step, pw);
#pragma unroll
    for (int q = 0; q < RS; ++q) {
      const int k2 = i + q * STR;
      int64_t at;
      if constexpr (BLK) at = spill_index(r, k2, R, lb2);
      else at = (int64_t)r * C + k2;
      store_stream(&dst[at], twmul(v[q], cmul(base, pw[q])));
    }
  };
  if constexpr (C >= 1024) {
    // all sky-record reads of a thread in flight together (the interbinned
    // 2-day grid: pass 1 ~20 % faster); the reads of padding columns are
    // clamped to the row's last record (ceff >= 1)
    auto read = [&](int c, int) -> Quad<T> { return col[c < ceff ? c : ceff - 1]; };
    block_fft_split<Pair<T>, C, 1, BLOCK, -1>(lds, twC, read, make, store);
  } else {
    // short rows: one read per element; the split form would double the
    // registers of these 64-thread workgroups
    auto load = [&](int c, int) -> Pair<T> {
      return c < ceff ? make(col[c], c, 0) : Pair<T>{{(T)0, (T)0}, {(T)0, (T)0}};
    };
    block_fft<Pair<T>, C, 1, BLOCK, -1>(lds, twC, load, store);
  }
}

// Pass 2 for the column block cb (B2 adjacent k2) of one node: src is the
// node's spill, lds lds_slots(R, B2) slots.  Mode 1: the block's largest F
// and its bin (ties to the lowest bin; k = INT64_MAX if no bin of the block
// lies in [k_lo, k_hi)) are returned in thread 0, and stored at part[cb]
// unless part is null.
template <typename T, int R, int MODE>
__device__ __forceinline__ MaxPartial pass2_tile(const SegDev& sg, const Pair<T>* __restrict__ spill_node,
                                           const NodeDev& node, const SkyCoef& cf, const cpx<T>* __restrict__ twR,
                                           const GridOut& out, int cb, MaxPartial* __restrict__ part,
                                           lds_t<Pair<T>>* __restrict__ lds) {
  constexpr int B2 = cfg_B2<T>(R);
  constexpr int BLOCK = cfg_block(B2 * R / 16);
  const int C = sg.C;
  // blocked: the workgroup's R x B2 elements are contiguous; row-major: rows
  // of B2 elements at stride C
  constexpr bool BLK = spill_blocked<T>(B2);
  const Pair<T>* __restrict__ src = spill_node + (BLK ? (int64_t)cb * R * B2 : (int64_t)cb * B2);
  auto load = [&](int r, int col) -> Pair<T> {
    if constexpr (BLK) return load_stream(&src[r * B2 + col]);
    else return load_stream(&src[(int64_t)r * C + col]);
  };
  const T cB = (T)cf.cB, cA = (T)cf.cA, cC = (T)cf.cC;
  const int64_t klo = out.k_lo, khi = out.k_hi;
  double best = -1.0;
  int64_t bestk = INT64_MAX;
  auto store1 = [&](int k1, int col, const Pair<T>& v) {
    if (k1 >= R / 2) return;
    const int64_t k = (int64_t)C * k1 + (int64_t)cb * B2 + col;
    if (k < klo || k >= khi) return;
    // explicit fused operations: every output mode rounds identically
    const T pa = fma(v.a.x, v.a.x, v.a.y * v.a.y);
    const T pb = fma(v.b.x, v.b.x, v.b.y * v.b.y);
    const T re = fma(v.a.x, v.b.x, v.a.y * v.b.y);
    const T F = fma(cB, pa, fma(cA, pb, -(cC * re)));
    if constexpr (MODE == 0) {
      store_stream(&((T*)out.F)[(int64_t)node.row * (khi - klo) + (k - klo)], F);
    } else if constexpr (MODE == 1) {
      const double f = (double)F;
      if (f > best || (f == best && k < bestk)) {
        best = f;
        bestk = k;
      }
    } else {
      if ((double)F > out.threshold) {
        const unsigned long long i = atomicAdd(out.n_xing, 1ull);
        if ((int64_t)i < out.max_xing) ((Crossing*)out.xing)[i] = Crossing{node.row, k, (double)F};
      }
    }
  };
  auto store = [&](int i, int col, auto& v, auto str) {
    constexpr int RS = std::extent<std::remove_reference_t<decltype(v)>>::value;
    constexpr int STR = decltype(str)::value;
#pragma unroll
    for (int q = 0; q < RS; ++q) store1(i + q * STR, col, v[q]);
  };
  block_fft<Pair<T>, R, B2, BLOCK, -1>(lds, twR, load, store);
  if constexpr (MODE == 1) {
    // block arg-max, ties to the lowest bin
    __shared__ double sf[BLOCK / 64];
    __shared__ int64_t sk[BLOCK / 64];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const double f2 = __shfl_down(best, o, 64);
      const int64_t k2 = __shfl_down(bestk, o, 64);
      if (f2 > best || (f2 == best && k2 < bestk)) {
        best = f2;
        bestk = k2;
      }
    }
    if ((threadIdx.x & 63) == 0) {
      sf[threadIdx.x >> 6] = best;
      sk[threadIdx.x >> 6] = bestk;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int w = 1; w < BLOCK / 64; ++w)
        if (sf[w] > best || (sf[w] == best && sk[w] < bestk)) {
          best = sf[w];
          bestk = sk[w];
        }
      if (part) part[cb] = MaxPartial{best, bestk};
    }
  }
  return MaxPartial{best, bestk};
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

// Per (sky, sample j): the detector time t of the barycentric grid point
// t_b0 + j dt, i.e. t = j dt - d with d = dphi_m(t), then x(t) by
// interpolation, a(t), b(t) and the demodulation record.  d is found from
// d0 = dphi_m(j dt) by one step of the fixed-point relation linearised at d0:
// d = (dphi_m(t1) + dphi_m'(t1) d0) / (1 + dphi_m'(t1)), t1 = j dt - d0.  d0
// is within |dphi_m'| x 500 s ~ 0.05 s of the solution and the curvature of
// dphi_m is below 1e-10 s/s^2, so the step leaves ~1e-13 s (a phase error of
// 5e-11 turns at 435 Hz); a second step would change rounding only.  One call
// takes one sample position (column-major record index pos) for ng <= SKY_GROUP
// sky positions: skies and out point at the group's first sky.
template <typename T, int INTERP>
__device__ __forceinline__ void sky_prep_pos(const SegDev& sg, const SkyConst* __restrict__ skies, int ng, int64_t pos,
                                             Quad<T>* __restrict__ out, int64_t stride) {
  const int64_t total = (int64_t)sg.R * sg.Ceff;
  constexpr double TWO_PI = 6.28318530717958647692;
  if (pos >= total) return;
  const int64_t r = pos / sg.Ceff;
  const int64_t c = pos - r * sg.Ceff;
  const int64_t j = r + (int64_t)sg.R * c;
  if (j < sg.n) {
    const EphemBase b = ephem_base(sg.geo, (double)j * sg.dt);
    for (int g = 0; g < ng; ++g) {
      const SkyConst& k = skies[g];
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
      out[(int64_t)g * stride + pos] = q;
    }
  } else {
    for (int g = 0; g < ng; ++g) out[(int64_t)g * stride + pos] = Quad<T>{(T)0, (T)0, (T)0, (T)0};
  }
}

// The per-sky constants at (alpha, delta) and t_b0 = phi_m(0).
__device__ __forceinline__ SkyConst sky_setup_one(double alpha, double delta, const SegGeo& g) {
  SkyConst k;
  sky_const(alpha, delta, g, k);
  const Ephem e = ephem(g, 0.0);
  k.tb0 = roemer(k, e);
  return k;
}

// A, B, C from the mask moments, then the coefficients of the F combination.
__device__ __forceinline__ SkyCoef sky_coef_one(const SkyConst& k, const double* __restrict__ mom, double sigma2) {
  AbPoly fa, fb;
  ab_poly(k, fa, fb);
  const double A = moment_sum(fa.v, fa.v, mom);
  const double B = moment_sum(fb.v, fb.v, mom);
  const double C = moment_sum(fa.v, fb.v, mom);
  const double D = sigma2 * (A * B - C * C);
  SkyCoef o;
  o.A = A;
  o.B = B;
  o.C = C;
  o.cB = B / D;
  o.cA = A / D;
  o.cC = 2.0 * C / D;
  return o;
}

// "Largest F, ties to the lowest bin" (associative and commutative): a wave
// reduction of (best, bestk) held by the 64 lanes; the result in lane 0.
__device__ __forceinline__ void wave_argmax(double& best, int64_t& bk) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double f2 = __shfl_down(best, o, 64);
    const int64_t k2 = __shfl_down(bk, o, 64);
    if (f2 > best || (f2 == best && k2 < bk)) {
      best = f2;
      bk = k2;
    }
  }
}

}  // namespace
