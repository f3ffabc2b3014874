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

// ---- the persistent grid launch (persist.hip) ----
// The work of a whole grid call as one queue of tiles, each one workgroup's
// share of a stage: the sky preparation of a batch of sky positions
// (set-up, record tiles, combination coefficients), pass 1 of a node (its R
// columns), pass 2 of a node (its C/B2 = R column blocks at C = 4096).  The
// queue is cut into units of PUNIT consecutive tiles of one stage; a unit
// record says which.
constexpr int PUNIT = 64;
constexpr int PREP_POS = 4;  // sample positions per thread of a sky-preparation tile
enum : int32_t { PU_SKY = 0, PU_P1 = 1, PU_P2 = 2 };
struct PUnit {
  int32_t kind;  // PU_SKY / PU_P1 / PU_P2
  int32_t id;    // batch (PU_SKY) or node (PU_P1, PU_P2) of the call
  int32_t sub;   // the unit's place in its stage: tile = sub * PUNIT + item % PUNIT
  int32_t pad;
};
// A batch of sky positions of one segment and the nodes that use them.
struct PBatch {
  int32_t seg, set;      // segment; sky set (0 / 1) that holds its records
  int32_t sky0, nsky;    // into the call's (alpha, delta) list
  int32_t node0, nnode;  // into the call's node list
  int32_t nblk;          // sample blocks of PREP_POS x 256 positions
  int32_t nprep;         // record tiles: ceil(nsky / SKY_GROUP) x nblk
};
struct PSegTw {  // twiddle tables of a segment
  const void *twC, *twR, *twlo, *twhi;
};
struct PersistArgs {
  const SegDev* segs;
  const PSegTw* tw;
  const PUnit* units;
  int64_t nitems;             // tiles in the queue (units x PUNIT)
  const PBatch* batches;
  int32_t nbatch, nslots;     // batches; spill slots
  const int32_t* node_batch;  // batch of each node
  const NodeDev* nodes;       // the call's nodes, grouped by batch
  const double* sky_ad;       // (alpha, delta) of the call's sky positions
  void* quads[2];             // sky sets: records of up to 64 skies, stride R Ceff of the batch's segment
  SkyConst* sky[2];
  SkyCoef* coef[2];
  void* spill;                // nslots x slot_elems spill elements; node n uses slot n % nslots
  int64_t slot_elems;
  unsigned long long* best;   // max mode, per node: the largest F so far as an ordered key (max_key)
  GridOut out;
  unsigned long long* head;   // tiles claimed
  int32_t chunk;              // tiles a workgroup claims at once (a divisor of PUNIT)
  uint32_t* cnt;              // completion counters: 4 per batch, then 2 per node
  uint32_t* error;            // sticky flag: a wait outlived spin_ticks
  uint64_t spin_ticks;        // wall-clock ticks a wait may last
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
// persist.hip: the whole grid call in one launch (FP32, C = 4096, 64 <= R <=
// 1024, no interbinning); counters, head and spill must be zeroed / sized by
// the caller (persist_zero clears the n32 words of counters and per-node
// maximum keys at cnt, and head)
int persistent_blocks(int mode);
hipError_t persist_zero(uint32_t* cnt, int64_t n32, unsigned long long* head, hipStream_t st);
hipError_t grid_persistent(const PersistArgs& a, int mode, int blocks, hipStream_t st);
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
