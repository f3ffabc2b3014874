// Structures shared by the host orchestration and the kernels.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cplx.h"
#include "geometry.h"

// Per-sample record of one sky position on the barycentric grid, laid out
// column-major for the first FFT pass (sample j = r + R c at r*Ceff + c):
//   wa = x(t_j) a(t_j), wb = x(t_j) b(t_j)    (resampled, a/b-weighted data)
//   p0 = frac(f_ref dphi_m(t_j))              (turns)
//   dd = dphi_m(t_j) = phi_m(t_j) - phi_m(0)  (s)
template <typename T>
struct Quad {
  T wa, wb, p0, dd;
};

// Per-sky combination coefficients of F (B/D, A/D, 2C/D with
// D = sigma^2 (AB - C^2)) and the raw sums.
struct SkyCoef {
  double cB, cA, cC;  // B/D, A/D, 2C/D
  double A, B, C;
};

// One node of a grid batch.
struct NodeDev {
  double fdot;
  double fshift;  // bin offset / nfft: cycles per sample added to the demodulation phase
  int32_t sky;    // index into the sky batch
  int32_t row;    // output row (the caller's node index)
};

// Everything about a segment that the kernels need.
struct SegDev {
  SegGeo geo;
  int64_t n;         // samples
  double dt;
  double f_ref;
  double sigma2;
  int64_t nfft;
  int32_t R, C, Ceff; // nfft = R*C; first pass transforms R columns of length C
  int32_t interp;    // 0 nearest, 1 linear on the 2x series, 2 cubic on the 2x series
  const double* x;   // masked data [n]
  const float* xf;
  const double* y;   // 2x upsampled [2n]
  const float* yf;
  const double* M;   // periodic spline second derivatives [2n]
  const float* Mf;
  const uint8_t* mask;  // [n] or null
  const double* mom;    // [10]: M_k = sum_i m_i e^{i k theta_i}, k = 0..4, (Re, Im); theta_i the
                        // sidereal angle of detector sample i, m_i its mask value
};

struct GridOut {
  int32_t mode;        // 0 map, 1 per-node max, 2 crossings
  int32_t interbin;    // 1: also the half bins k + 1/2 (output index 2k + h)
  int64_t k_lo, k_hi;
  double threshold;
  void* F;             // mode 0: [rows][k_hi-k_lo] of T
  void* Fmax;          // mode 1: [rows] of T
  int64_t* kmax;       // mode 1
  void* xing;          // mode 2: records
  unsigned long long* n_xing;
  int64_t max_xing;
};

struct Crossing {
  int64_t node;
  int64_t k;
  double F;
};

struct MaxPartial {
  double F;
  int64_t k;
};

constexpr double SPAN_EPS = 1e-6;  // margin of the data-span test, in samples
constexpr int FSTATE = 8;  // doubles of forward state per candidate: S_a, S_b, A, B, C, pad

// ---- launchers (defined in the .hip files) ----
namespace fsk {
// sky.hip
hipError_t sky_setup(const double* d_alpha_delta, int nsky, const SegDev& seg, SkyConst* d_out, hipStream_t st);
int sky_prep_blocks(const SegDev& seg);
hipError_t sky_prep(int prec, const SegDev& seg, const SkyConst* d_sky, int nsky, void* d_quads,
                    int64_t quad_stride, hipStream_t st);
hipError_t sky_finalize(const SegDev& seg, const SkyConst* d_sky, int nsky, SkyCoef* d_coef, hipStream_t st);
// the segment's mask moments (SegDev::mom) into d_mom[10]; d_part: scratch of
// mask_moment_blocks(seg) x 9 doubles
int mask_moment_blocks(const SegDev& seg);
hipError_t mask_moments(const SegDev& seg, double* d_part, double* d_mom, hipStream_t st);
hipError_t demod_series(int prec, const SegDev& seg, const SkyConst* d_sky, const void* d_quads,
                        int64_t quad_stride, double fdot, double fshift, double* d_out, hipStream_t st);
// grid.hip
int pass2_b2(int prec, int R);
hipError_t grid_pass1(int prec, int C, const SegDev& seg, const void* d_quads, int64_t quad_stride,
                      const SkyConst* d_sky, const NodeDev* d_nodes, int nnodes, const void* tw_C,
                      const void* tw_lo, const void* tw_hi, void* d_spill, hipStream_t st);
hipError_t grid_pass2(int prec, int R, const SegDev& seg, const void* d_spill, const NodeDev* d_nodes, int nnodes,
                      const SkyCoef* d_coef, const void* tw_R, const GridOut& out, MaxPartial* d_part,
                      hipStream_t st);
hipError_t max_finalize(const MaxPartial* d_part, int nparts, const NodeDev* d_nodes, int nnodes, int prec,
                        const GridOut& out, hipStream_t st);
hipError_t zero_u64(unsigned long long* p, hipStream_t st);
// prep.hip
hipError_t make_twiddles(int prec, int64_t denom, int64_t count, int64_t step, void* d_tab, hipStream_t st);
hipError_t fft_c2c_f64(cpx<double>* d_data, int64_t L, int dir, cpx<double>* d_tmp, cpx<double>* d_twtab,
                       hipStream_t st);
size_t prep_work_bytes(int64_t n);
hipError_t prep_mask(const double* d_xraw, const uint8_t* d_mask, int64_t n, double* d_x, float* d_xf,
                     hipStream_t st);
hipError_t prep_variance(const double* d_xraw, const uint8_t* d_mask, int64_t n, double* d_out, hipStream_t st);
hipError_t prep_upsample(const double* d_x, int64_t n, int interp, double* d_y, float* d_yf, double* d_M,
                         float* d_Mf, void* d_work, hipStream_t st);
// grad.hip
hipError_t grad_forward(const SegDev* d_segs, int nseg, const int32_t* d_seg, const double* d_params, int64_t n,
                        double* d_F, double* d_state, hipStream_t st);
hipError_t grad_adjoint(const SegDev* d_segs, int nseg, const int32_t* d_seg, const double* d_params, int64_t n,
                        const double* d_state, const double* d_gF, double* d_dp, hipStream_t st);
hipError_t amplitudes(const SegDev* d_segs, int nseg, const int32_t* d_seg, const double* d_params, int64_t n,
                      const double* d_state, double* d_out, hipStream_t st);
// search.hip
hipError_t eval_exact(const SegDev* d_segs, int nseg, const int32_t* d_seg, const double* d_params, int64_t n,
                      double* d_F, hipStream_t st);
hipError_t nelder_mead(const SegDev* d_segs, int nseg, const int32_t* d_seg, const double* d_params, int64_t n,
                       const double* scale, double tol, int max_evals, int exact, double* d_pout, double* d_F,
                       int32_t* d_evals, hipStream_t st);
}  // namespace fsk
