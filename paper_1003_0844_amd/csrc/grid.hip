// The per-node hot path: demodulation fused into the first FFT pass, the
// second pass fused with the F combination (Sec. VI A-B, Eqs. ia, DFT, OS).
//
// nfft = R * C.  Sample j = r + R c (r < R, c < C), bin k = C k1 + k2
// (k1 < R, k2 < C):
//   X[C k1 + k2] = sum_r e^{-2 pi i r k1/R} [ e^{-2 pi i r k2/nfft}
//                                             sum_c x[r + R c] e^{-2 pi i c k2/C} ]
// Pass 1 (one workgroup per column r of one node): build x_j for the a- and
//   b-weighted series on the fly from the sky record and the node's spindown,
//   length-C FFT in LDS, inter-pass twiddle, store Z (a and b interleaved,
//   16 B per element in FP32).
// Pass 2 (one workgroup per block of B2 adjacent k2 of one node): length-R FFT
//   of each column, keep the bins k < nfft/2 (k1 < R/2), combine
//   F = (B|S_a|^2 + A|S_b|^2 - 2C Re(S_a S_b*)) / (sigma^2 (AB - C^2)) and write
//   the map row, the per-node maximum or the threshold crossings.
// The inter-pass spill Z is the only HBM round trip of a node:
// 2 x 8 B x nfft written and read in FP32.  Where a row of pass 2's column
// block is shorter than 512 B (B2 elements), Z is stored blocked,
// Z[k2 / B2][r][k2 % B2], so that pass 2 reads one contiguous R x B2 block
// per workgroup; otherwise row-major, Z[r][k2].  Measured on the 2-day grid:
// with 256 B rows (nfft = 2^20, B2 = 16) the blocked layout makes pass 2
// 13 % faster and pass 1 6 % slower (step +3.5 %); with 512 B rows (nfft =
// 2^19, B2 = 32) pass 2 gains 1 % and pass 1 loses 3 %.
#include "tiles.h"

namespace {

// Map the hardware workgroup id so that consecutive logical column blocks run
// on the same XCD (the dispatcher deals workgroups round-robin over 8 XCDs):
// adjacent blocks then share L2 lines of the output rows.
__device__ __forceinline__ int xcd_local(int bid, int nblk) {
  if (nblk % 8 != 0) return bid;
  return (bid % 8) * (nblk / 8) + bid / 8;
}

template <typename T, int C, bool BLK>
__global__ void __launch_bounds__(cfg_block(C / 16))
k_pass1(SegDev sg, const Quad<T>* __restrict__ quads, int64_t qstride, const SkyConst* __restrict__ skies,
        const NodeDev* __restrict__ nodes, const cpx<T>* __restrict__ twC, const cpx<T>* __restrict__ twlo,
        const cpx<T>* __restrict__ twhi, Pair<T>* __restrict__ spill) {
  __shared__ lds_t<Pair<T>> lds[lds_slots(C, 1)];
  const int nd = blockIdx.y;
  pass1_tile<T, C, BLK>(sg, quads, qstride, skies, nodes[nd], blockIdx.x, twC, twlo, twhi,
                        spill + (int64_t)nd * sg.nfft, lds);
}

template <typename T, int R, int MODE>
__global__ void __launch_bounds__(cfg_block(cfg_B2<T>(R) * R / 16))
k_pass2(SegDev sg, const Pair<T>* __restrict__ spill, const NodeDev* __restrict__ nodes,
        const SkyCoef* __restrict__ coef, const cpx<T>* __restrict__ twR, GridOut out,
        MaxPartial* __restrict__ part) {
  constexpr int B2 = cfg_B2<T>(R);
  __shared__ lds_t<Pair<T>> lds[lds_slots(R, B2)];
  const int nd = blockIdx.y;
  const NodeDev node = nodes[nd];
  pass2_tile<T, R, MODE>(sg, spill + (int64_t)nd * sg.nfft, node, coef[node.sky], twR, out,
                         xcd_local(blockIdx.x, gridDim.x), part + (int64_t)nd * gridDim.x, lds);
}

constexpr int cmax(int a, int b) { return a > b ? a : b; }

// Pass 2 with interbinning (Eq. intbin): F at the Fourier bins k and at the
// half bins k + 1/2, with S(k + 1/2) ~ (S(k+1) - S(k)) / sqrt(2) for S_a and
// S_b.  The workgroup transforms one column more than it owns, k2_0 + B2 (or
// column 0 for the last block, whose outputs at k1 + 1 continue the band), so
// that the right neighbour of every owned bin is local.  The final spectra
// (rows k1 <= R/2) are staged in LDS; the epilogue reads each bin and its
// neighbour from there.  Output index 2k + h, h = 1 for the half bin.
template <typename T>
constexpr int ib_block(int R) {
  const int nb = (cfg_B2<T>(R) + 1) * R / 16;
  const int b = (nb + 63) / 64 * 64;
  return b > 1024 ? 1024 : b;
}
constexpr int ib_slots(int R, int ncol) { return cmax(lds_slots(R, ncol), 2 * (R / 2 + 1) * ncol); }

template <typename T, int R, int MODE>
__global__ void __launch_bounds__(ib_block<T>(R))
k_pass2_ib(SegDev sg, const Pair<T>* __restrict__ spill, const NodeDev* __restrict__ nodes,
           const SkyCoef* __restrict__ coef, const cpx<T>* __restrict__ twR, GridOut out,
           MaxPartial* __restrict__ part) {
  constexpr int B2 = cfg_B2<T>(R);
  constexpr int NCOL = B2 + 1;
  constexpr int BLOCK = ib_block<T>(R);
  using GL = StageShape<R, NCOL, BLOCK, fft_nstages(R) - 1>;
  __shared__ lds_t<Pair<T>> lds[ib_slots(R, NCOL)];
  const int nd = blockIdx.y;
  const int cb = xcd_local(blockIdx.x, gridDim.x);
  const NodeDev node = nodes[nd];
  const int C = sg.C;
  const int k2_0 = cb * B2;
  const bool wrap = k2_0 + B2 == C;
  const int k2_x = wrap ? 0 : k2_0 + B2;
  // the own B2 columns and column k2_x, in the spill layout of this B2;
  // ordinary loads: the extra column is read by the neighbouring workgroup
  // too, and with streaming loads this kernel runs 25-30 % slower (measured)
  constexpr bool BLK = spill_blocked<T>(B2);
  const Pair<T>* __restrict__ src = spill + (int64_t)nd * sg.nfft;
  auto load = [&](int r, int col) -> Pair<T> {
    if constexpr (BLK) {
      const int k2 = col < B2 ? k2_0 + col : k2_x;
      return src[((int64_t)(k2 / B2) * R + r) * B2 + (k2 % B2)];
    } else {
      return src[(int64_t)r * C + (col < B2 ? k2_0 + col : k2_x)];
    }
  };
  Pair<T> fin[GL::PER][GL::Rs];
  auto keep = [&](int, int, auto& v, auto, int m) {
#pragma unroll
    for (int q = 0; q < GL::Rs; ++q) fin[m][q] = v[q];
  };
  block_fft<Pair<T>, R, NCOL, BLOCK, -1>(lds, twR, load, keep);
  __syncthreads();  // every thread is past the last exchange
  Pair<T>* __restrict__ stg = reinterpret_cast<Pair<T>*>(lds);  // [k1][col], k1 <= R/2
#pragma unroll
  for (int m = 0; m < GL::PER; ++m) {
    const int b = (int)threadIdx.x + m * BLOCK;
    if (GL::NB % BLOCK == 0 || b < GL::NB) {
      const int col = b % NCOL;
      const int i = b / NCOL;
#pragma unroll
      for (int q = 0; q < GL::Rs; ++q) {
        const int k1 = i + q * (R / GL::Rs);
        if (k1 <= R / 2) stg[k1 * NCOL + col] = fin[m][q];
      }
    }
  }
  __syncthreads();
  const SkyCoef cf = coef[node.sky];
  const T cB = (T)cf.cB, cA = (T)cf.cA, cC = (T)cf.cC;
  const T rs2 = (T)0.70710678118654752440084436210485;
  const int64_t klo = out.k_lo, khi = out.k_hi;
  double best = -1.0;
  int64_t bestk = INT64_MAX;
  // explicit fused operations: every output mode rounds identically
  auto fcomb = [&](const cpx<T>& a, const cpx<T>& b) -> T {
    const T pa = fma(a.x, a.x, a.y * a.y);
    const T pb = fma(b.x, b.x, b.y * b.y);
    const T re = fma(a.x, b.x, a.y * b.y);
    return fma(cB, pa, fma(cA, pb, -(cC * re)));
  };
  auto emit = [&](int64_t k, int h, T F) {
    const int64_t kh = 2 * k + h;
    if constexpr (MODE == 0) {
      store_stream(&((T*)out.F)[(int64_t)node.row * 2 * (khi - klo) + (kh - 2 * klo)], F);
    } else if constexpr (MODE == 1) {
      const double f = (double)F;
      if (f > best || (f == best && kh < bestk)) {
        best = f;
        bestk = kh;
      }
    } else {
      if ((double)F > out.threshold) {
        const unsigned long long n = atomicAdd(out.n_xing, 1ull);
        if ((int64_t)n < out.max_xing) ((Crossing*)out.xing)[n] = Crossing{node.row, kh, (double)F};
      }
    }
  };
  for (int o = threadIdx.x; o < (R / 2) * B2; o += BLOCK) {
    const int col = o % B2;
    const int k1 = o / B2;
    const int64_t k = (int64_t)C * k1 + k2_0 + col;
    if (k < klo || k >= khi) continue;
    const Pair<T> s0 = stg[k1 * NCOL + col];
    const Pair<T> s1 = col + 1 < B2 ? stg[k1 * NCOL + col + 1] : stg[(wrap ? k1 + 1 : k1) * NCOL + B2];
    const cpx<T> ha{(s1.a.x - s0.a.x) * rs2, (s1.a.y - s0.a.y) * rs2};
    const cpx<T> hb{(s1.b.x - s0.b.x) * rs2, (s1.b.y - s0.b.y) * rs2};
    emit(k, 0, fcomb(s0.a, s0.b));
    emit(k, 1, fcomb(ha, hb));
  }
  if constexpr (MODE == 1) {
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
      part[(int64_t)nd * gridDim.x + cb] = MaxPartial{best, bestk};
    }
  }
}

// One wave per node: each lane scans a strided share of the node's partials,
// then the wave reduces.  "Largest F, ties to the lowest bin" is associative
// and commutative, so the result equals that of a sequential scan.
template <typename T>
__global__ void __launch_bounds__(64) k_max_finalize(const MaxPartial* __restrict__ part, int nparts,
                                                    const NodeDev* __restrict__ nodes, T* __restrict__ Fmax,
                                                    int64_t* __restrict__ kmax) {
  const int nd = blockIdx.x;
  const MaxPartial* __restrict__ p = part + (int64_t)nd * nparts;
  double best = -1.0;
  int64_t bk = INT64_MAX;
  for (int i = threadIdx.x; i < nparts; i += 64) {
    const MaxPartial q = p[i];
    if (q.F > best || (q.F == best && q.k < bk)) {
      best = q.F;
      bk = q.k;
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    const double f2 = __shfl_down(best, o, 64);
    const int64_t k2 = __shfl_down(bk, o, 64);
    if (f2 > best || (f2 == best && k2 < bk)) {
      best = f2;
      bk = k2;
    }
  }
  if (threadIdx.x == 0) {
    Fmax[nodes[nd].row] = (T)best;
    kmax[nodes[nd].row] = bk;
  }
}

__global__ void k_zero_u64(unsigned long long* p) {
  if (threadIdx.x == 0) p[threadIdx.x] = 0ull;
}

template <typename T>
hipError_t launch_pass1(int C, const SegDev& seg, const void* quads, int64_t qstride, const SkyConst* sky,
                        const NodeDev* nodes, int nnodes, const void* twC, const void* twlo, const void* twhi,
                        void* spill, hipStream_t st) {
  dim3 grid(seg.R, nnodes);
  const bool blk = spill_blocked<T>(cfg_B2<T>(seg.R));  // the layout pass 2 reads
#define P1(CC)                                                                                                  \
  case CC:                                                                                                      \
    if (blk)                                                                                                    \
      hipLaunchKernelGGL((k_pass1<T, CC, true>), grid, dim3(cfg_block(CC / 16)), 0, st, seg,                    \
                         (const Quad<T>*)quads, qstride, sky, nodes, (const cpx<T>*)twC, (const cpx<T>*)twlo,   \
                         (const cpx<T>*)twhi, (Pair<T>*)spill);                                                 \
    else                                                                                                        \
      hipLaunchKernelGGL((k_pass1<T, CC, false>), grid, dim3(cfg_block(CC / 16)), 0, st, seg,                   \
                         (const Quad<T>*)quads, qstride, sky, nodes, (const cpx<T>*)twC, (const cpx<T>*)twlo,   \
                         (const cpx<T>*)twhi, (Pair<T>*)spill);                                                 \
    break;
  switch (C) {
    P1(64) P1(128) P1(256) P1(512) P1(1024) P1(2048) P1(4096)
    default: return hipErrorInvalidValue;
  }
#undef P1
  return hipGetLastError();
}

template <typename T, int MODE>
hipError_t launch_pass2_mode(int R, const SegDev& seg, const void* spill, const NodeDev* nodes, int nnodes,
                             const SkyCoef* coef, const void* twR, const GridOut& out, MaxPartial* part,
                             hipStream_t st) {
#define P2(RR)                                                                                        \
  case RR: {                                                                                          \
    constexpr int B2 = cfg_B2<T>(RR);                                                                 \
    dim3 grid(seg.C / B2, nnodes);                                                                    \
    if (out.interbin)                                                                                 \
      hipLaunchKernelGGL((k_pass2_ib<T, RR, MODE>), grid, dim3(ib_block<T>(RR)), 0, st, seg,          \
                         (const Pair<T>*)spill, nodes, coef, (const cpx<T>*)twR, out, part);          \
    else                                                                                              \
      hipLaunchKernelGGL((k_pass2<T, RR, MODE>), grid, dim3(cfg_block(B2 * RR / 16)), 0, st, seg,     \
                         (const Pair<T>*)spill, nodes, coef, (const cpx<T>*)twR, out, part);          \
  } break;
  switch (R) {
    P2(16) P2(32) P2(64) P2(128) P2(256) P2(512) P2(1024)
    default: return hipErrorInvalidValue;
  }
#undef P2
  return hipGetLastError();
}

}  // namespace

namespace fsk {

int pass2_b2(int prec, int R) { return prec == 0 ? cfg_B2<float>(R) : cfg_B2<double>(R); }

hipError_t grid_pass1(int prec, int C, const SegDev& seg, const void* quads, int64_t qstride, const SkyConst* sky,
                      const NodeDev* nodes, int nnodes, const void* twC, const void* twlo, const void* twhi,
                      void* spill, hipStream_t st) {
  if (nnodes <= 0) return hipSuccess;
  if (prec == 0) return launch_pass1<float>(C, seg, quads, qstride, sky, nodes, nnodes, twC, twlo, twhi, spill, st);
  return launch_pass1<double>(C, seg, quads, qstride, sky, nodes, nnodes, twC, twlo, twhi, spill, st);
}

hipError_t grid_pass2(int prec, int R, const SegDev& seg, const void* spill, const NodeDev* nodes, int nnodes,
                      const SkyCoef* coef, const void* twR, const GridOut& out, MaxPartial* part, hipStream_t st) {
  if (nnodes <= 0) return hipSuccess;
  if (prec == 0) {
    if (out.mode == 0) return launch_pass2_mode<float, 0>(R, seg, spill, nodes, nnodes, coef, twR, out, part, st);
    if (out.mode == 1) return launch_pass2_mode<float, 1>(R, seg, spill, nodes, nnodes, coef, twR, out, part, st);
    return launch_pass2_mode<float, 2>(R, seg, spill, nodes, nnodes, coef, twR, out, part, st);
  }
  if (out.mode == 0) return launch_pass2_mode<double, 0>(R, seg, spill, nodes, nnodes, coef, twR, out, part, st);
  if (out.mode == 1) return launch_pass2_mode<double, 1>(R, seg, spill, nodes, nnodes, coef, twR, out, part, st);
  return launch_pass2_mode<double, 2>(R, seg, spill, nodes, nnodes, coef, twR, out, part, st);
}

hipError_t max_finalize(const MaxPartial* part, int nparts, const NodeDev* nodes, int nnodes, int prec,
                        const GridOut& out, hipStream_t st) {
  if (nnodes <= 0) return hipSuccess;
  dim3 grid(nnodes), block(64);
  if (prec == 0)
    hipLaunchKernelGGL(k_max_finalize<float>, grid, block, 0, st, part, nparts, nodes, (float*)out.Fmax, out.kmax);
  else
    hipLaunchKernelGGL(k_max_finalize<double>, grid, block, 0, st, part, nparts, nodes, (double*)out.Fmax,
                       out.kmax);
  return hipGetLastError();
}

hipError_t zero_u64(unsigned long long* p, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(1), dim3(1), 0, st, p);
  return hipGetLastError();
}

}  // namespace fsk
