// Fine search (Sec. VI C): F at continuous parameters evaluated exactly, by
// direct summation of Eqs. (OS)-(Fab) on the detector samples, and a
// Nelder-Mead simplex search for the maximum of F starting from coarse-grid
// candidates, one workgroup per candidate.
//
// Nelder-Mead (Nelder & Mead 1965; reflection 1, expansion 2, contraction 1/2,
// shrink 1/2), on g = -F in scaled coordinates u (theta = theta_start + u
// scale), initial simplex theta_start plus one unit step along each axis.
// Every thread of the workgroup runs the same simplex logic on the same values;
// each F evaluation is a block-wide sum.  The loop ends when every vertex lies
// within tol (in scale units, per axis) of the best one or after max_evals
// evaluations.
#include "candidate.h"

namespace {

constexpr int NP = 4;         // parameters
constexpr int NV = NP + 1;    // simplex vertices

// A double that thread 0 left in LDS, read as a wave-uniform value.  Every
// thread then takes the same branches of the simplex logic, and the compiler
// sees those branches (and the loops around the block-wide sums, with their
// barriers) as uniform.
__device__ __forceinline__ double uniform_f64(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)u);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// A decision of the simplex logic, taken as a wave-uniform branch: every
// thread holds the same values, so the first lane's outcome is every lane's.
__device__ __forceinline__ bool uniform_if(bool c) { return __builtin_amdgcn_readfirstlane((int)c) != 0; }

template <bool EXACT>
__device__ double block_F(const SegDev& sg, const Cand& c, double* sh, double* shF) {
  SkyConst k;
  setup_sky(sg, c, k);
  double acc[7] = {0, 0, 0, 0, 0, 0, 0};
  if constexpr (EXACT) {
    for (int64_t j = threadIdx.x; j < sg.n; j += GB) exact_terms(sg, k, c, j, acc);
    block_sums<7>(acc, sh);
  } else {
    double acc4[4] = {0, 0, 0, 0};
    for (int64_t j = threadIdx.x; j < sg.n; j += GB) method_terms(sg, k, c, j, acc4);
    block_sums<4>(acc4, sh);
#pragma unroll
    for (int i = 0; i < 4; ++i) acc[i] = acc4[i];
    if (threadIdx.x == 0) abc_moments(sg, k, acc[4], acc[5], acc[6]);
  }
  if (threadIdx.x == 0) *shF = combine_F(acc, sg.sigma2);
  __syncthreads();
  const double F = uniform_f64(*shF);
  __syncthreads();  // every thread has read shF and sh before the next evaluation writes them
  return F;
}

__global__ void __launch_bounds__(GB)
k_eval_exact(const SegDev* __restrict__ segs, int nseg, const int32_t* __restrict__ segi,
             const double* __restrict__ params, double* __restrict__ Fout) {
  __shared__ double sh[(GB / 64) * 7];
  __shared__ double shF;
  const int64_t ci = blockIdx.x;
  const int si = segi ? segi[ci] : 0;
  if (si < 0 || si >= nseg) {
    if (threadIdx.x == 0) Fout[ci] = __builtin_nan("");
    return;
  }
  const SegDev sg = segs[si];
  const Cand c{params[4 * ci], params[4 * ci + 1], params[4 * ci + 2], params[4 * ci + 3]};
  const double F = block_F<true>(sg, c, sh, &shF);
  if (threadIdx.x == 0) Fout[ci] = F;
}

struct NMArgs {
  double scale[NP];
  double tol;
  int max_evals;
};

template <bool EXACT>
__global__ void __launch_bounds__(GB)
k_nelder_mead(const SegDev* __restrict__ segs, int nseg, const int32_t* __restrict__ segi,
              const double* __restrict__ p0, NMArgs o, double* __restrict__ pout, double* __restrict__ Fout,
              int32_t* __restrict__ evals) {
  __shared__ double sh[(GB / 64) * 7];
  __shared__ double shF;
  const int64_t ci = blockIdx.x;
  const int si = segi ? segi[ci] : 0;
  if (si < 0 || si >= nseg) {
    if (threadIdx.x == 0) {
      for (int d = 0; d < NP; ++d) pout[NP * ci + d] = __builtin_nan("");
      Fout[ci] = __builtin_nan("");
      if (evals) evals[ci] = 0;
    }
    return;
  }
  const SegDev sg = segs[si];
  double base[NP];
  for (int d = 0; d < NP; ++d) base[d] = p0[NP * ci + d];
  int nev = 0;
  auto g_at = [&](const double (&u)[NP]) -> double {
    const Cand c{base[0] + u[0] * o.scale[0], base[1] + u[1] * o.scale[1], base[2] + u[2] * o.scale[2],
                 base[3] + u[3] * o.scale[3]};
    ++nev;
    return -block_F<EXACT>(sg, c, sh, &shF);
  };
  double v[NV][NP], g[NV];
  for (int i = 0; i < NV; ++i) {
    for (int d = 0; d < NP; ++d) v[i][d] = (i == d + 1) ? 1.0 : 0.0;
    g[i] = g_at(v[i]);
  }
  while (uniform_if(nev < o.max_evals)) {
    // order the vertices by g (insertion sort, ties keep their order), with
    // every compare-exchange spelled out: once vertex i has settled, the
    // remaining comparisons below it find the prefix ordered and swap nothing,
    // and the fixed indices keep v and g in registers
#pragma unroll
    for (int i = 1; i < NV; ++i)
#pragma unroll
      for (int j = i; j > 0; --j)
        if (uniform_if(g[j] < g[j - 1])) {
          const double tg = g[j];
          g[j] = g[j - 1];
          g[j - 1] = tg;
#pragma unroll
          for (int d = 0; d < NP; ++d) {
            const double tv = v[j][d];
            v[j][d] = v[j - 1][d];
            v[j - 1][d] = tv;
          }
        }
    double diam = 0.0;
    for (int i = 1; i < NV; ++i)
      for (int d = 0; d < NP; ++d) diam = fmax(diam, fabs(v[i][d] - v[0][d]));
    if (uniform_if(diam < o.tol)) break;
    double cen[NP];
    for (int d = 0; d < NP; ++d) {
      double sum = 0.0;
      for (int i = 0; i < NV - 1; ++i) sum += v[i][d];
      cen[d] = sum / (double)(NV - 1);
    }
    double xr[NP];
    for (int d = 0; d < NP; ++d) xr[d] = cen[d] + (cen[d] - v[NV - 1][d]);
    const double gr = g_at(xr);
    bool shrink = false;
    if (uniform_if(gr < g[0])) {
      double xe[NP];
      for (int d = 0; d < NP; ++d) xe[d] = cen[d] + 2.0 * (xr[d] - cen[d]);
      const double ge = g_at(xe);
      if (uniform_if(ge < gr)) {
        for (int d = 0; d < NP; ++d) v[NV - 1][d] = xe[d];
        g[NV - 1] = ge;
      } else {
        for (int d = 0; d < NP; ++d) v[NV - 1][d] = xr[d];
        g[NV - 1] = gr;
      }
    } else if (uniform_if(gr < g[NV - 2])) {
      for (int d = 0; d < NP; ++d) v[NV - 1][d] = xr[d];
      g[NV - 1] = gr;
    } else if (uniform_if(gr < g[NV - 1])) {
      double xc[NP];  // outside contraction
      for (int d = 0; d < NP; ++d) xc[d] = cen[d] + 0.5 * (xr[d] - cen[d]);
      const double gc = g_at(xc);
      if (uniform_if(gc <= gr)) {
        for (int d = 0; d < NP; ++d) v[NV - 1][d] = xc[d];
        g[NV - 1] = gc;
      } else {
        shrink = true;
      }
    } else {
      double xc[NP];  // inside contraction
      for (int d = 0; d < NP; ++d) xc[d] = cen[d] + 0.5 * (v[NV - 1][d] - cen[d]);
      const double gc = g_at(xc);
      if (uniform_if(gc < g[NV - 1])) {
        for (int d = 0; d < NP; ++d) v[NV - 1][d] = xc[d];
        g[NV - 1] = gc;
      } else {
        shrink = true;
      }
    }
    if (uniform_if(shrink)) {
      for (int i = 1; i < NV; ++i) {
        for (int d = 0; d < NP; ++d) v[i][d] = v[0][d] + 0.5 * (v[i][d] - v[0][d]);
        g[i] = g_at(v[i]);
      }
    }
  }
  int b = 0;
  for (int i = 1; i < NV; ++i)
    if (g[i] < g[b]) b = i;
  if (threadIdx.x == 0) {
    for (int d = 0; d < NP; ++d) pout[NP * ci + d] = base[d] + v[b][d] * o.scale[d];
    Fout[ci] = -g[b];
    if (evals) evals[ci] = nev;
  }
}

}  // namespace

namespace fsk {

hipError_t eval_exact(const SegDev* d_segs, int nseg, const int32_t* d_seg, const double* d_params, int64_t n,
                      double* d_F, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_eval_exact, dim3((unsigned)n), dim3(GB), 0, st, d_segs, nseg, d_seg, d_params, d_F);
  return hipGetLastError();
}

hipError_t nelder_mead(const SegDev* d_segs, int nseg, const int32_t* d_seg, const double* d_params, int64_t n,
                       const double* scale, double tol, int max_evals, int exact, double* d_pout, double* d_F,
                       int32_t* d_evals, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  NMArgs o{};
  for (int d = 0; d < NP; ++d) o.scale[d] = scale[d];
  o.tol = tol;
  o.max_evals = max_evals;
  if (exact)
    hipLaunchKernelGGL(k_nelder_mead<true>, dim3((unsigned)n), dim3(GB), 0, st, d_segs, nseg, d_seg, d_params, o,
                       d_pout, d_F, d_evals);
  else
    hipLaunchKernelGGL(k_nelder_mead<false>, dim3((unsigned)n), dim3(GB), 0, st, d_segs, nseg, d_seg, d_params, o,
                       d_pout, d_F, d_evals);
  return hipGetLastError();
}

}  // namespace fsk
