// Workgroup-level Stockham FFT for gfx950.
//
// One workgroup transforms NCOL independent columns of length L (a power of
// two).  Stages are radix 16 except the last (16, 8, 4 or 2).  The first stage
// reads its inputs through a Load functor (global memory, or values computed
// on the fly), the last stage hands each butterfly's Rs outputs to the Store
// functor as store(i, col, v, integral_constant STRIDE): v[q] is output
// i + q STRIDE;
// the stages
// in between exchange through LDS, in place, one barrier before and one after
// each write phase.
//
// Stockham stage with span Ns and radix Rs (butterfly i, k = i mod Ns):
//   inputs  x[i + q L/Rs]            q < Rs
//   twiddle x_q *= w^{q k}           w = exp(DIR 2 pi i / (Ns Rs))
//   radix-Rs DFT
//   outputs y[(i div Ns) Ns Rs + k + q Ns]
// which leaves the transform in natural order.  In the last stage
// Ns Rs = L and the outputs are y[i + q L/Rs].
//
// LDS element (idx, col) lives at lin + (lin >> 4), lin = idx*NCOL + col:
// one pad slot per 16 elements breaks the power-of-two strides of the write
// phase.  Threads map column-fastest (col = b mod NCOL) so that global loads
// and stores of NCOL adjacent columns are contiguous.
#pragma once
#include <type_traits>

#include "cplx.h"

constexpr int fft_nstages(int L) {
  int s = 0;
  long l = 1;
  while (l < L) {
    l *= 16;
    ++s;
  }
  return s < 1 ? 1 : s;
}
constexpr int fft_radix(int L, int s) {
  const int S = fft_nstages(L);
  if (s < S - 1) return 16;
  int p = 1;
  for (int i = 0; i < S - 1; ++i) p *= 16;
  return L / p;
}
constexpr int fft_span(int L, int s) {
  int p = 1;
  for (int i = 0; i < s; ++i) p *= fft_radix(L, i);
  return p;
}
// p[q] = w^q, q < R: squares for even q, one more factor w for odd q
// (at most six products deep for R = 16)
template <int R, typename T>
__device__ __forceinline__ void powers(cpx<T> w, cpx<T> (&p)[R]) {
  p[0] = cpx<T>{(T)1, (T)0};
  if constexpr (R > 1) p[1] = w;
#pragma unroll
  for (int q = 2; q < R; ++q) p[q] = (q % 2 == 0) ? cmul(p[q / 2], p[q / 2]) : cmul(p[q - 1], w);
}

constexpr int lds_slots(int L, int NCOL) { return L * NCOL + ((L * NCOL) >> 4); }

__device__ __forceinline__ int lds_addr(int idx, int col, int ncol) {
  const int lin = idx * ncol + col;
  return lin + (lin >> 4);
}

template <typename E, int L, int NCOL, int BLOCK, int DIR, int S, class Load, class Store>
__device__ __forceinline__ void fft_stage(E* __restrict__ lds,
                                          const cpx<typename elem_traits<E>::real>* __restrict__ tw,
                                          Load& load, Store& store) {
  using T = typename elem_traits<E>::real;
  constexpr int NS = fft_nstages(L);
  constexpr int Rs = fft_radix(L, S);
  constexpr int Ns = fft_span(L, S);
  constexpr int NB = NCOL * (L / Rs);
  constexpr int PER = (NB + BLOCK - 1) / BLOCK;
  constexpr int TWS = L / (Ns * Rs);  // table stride: table holds exp(-2 pi i m / L)
  const int tid = threadIdx.x;

  E v[PER][Rs];
#pragma unroll
  for (int m = 0; m < PER; ++m) {
    const int b = tid + m * BLOCK;
    if (NB % BLOCK == 0 || b < NB) {
      const int col = b % NCOL;
      const int i = b / NCOL;
      const int k = i % Ns;
#pragma unroll
      for (int q = 0; q < Rs; ++q) {
        const int idx = i + q * (L / Rs);
        if constexpr (S == 0) v[m][q] = load(idx, col);
        else v[m][q] = lds[lds_addr(idx, col, NCOL)];
      }
      if constexpr (S > 0) {
        // one table load per butterfly, the other powers by multiplication
        cpx<T> w = tw[k * TWS];
        if constexpr (DIR > 0) w.y = -w.y;
        cpx<T> pw[Rs];
        powers<Rs>(w, pw);
#pragma unroll
        for (int q = 1; q < Rs; ++q) v[m][q] = twmul(v[m][q], pw[q]);
      }
      dft<Rs, DIR>(v[m]);
    }
  }

  if constexpr (S == NS - 1) {
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int b = tid + m * BLOCK;
      if (NB % BLOCK == 0 || b < NB) {
        const int col = b % NCOL;
        const int i = b / NCOL;
        store(i, col, v[m], std::integral_constant<int, L / Rs>());
      }
    }
  } else {
    if constexpr (S > 0) __syncthreads();
#pragma unroll
    for (int m = 0; m < PER; ++m) {
      const int b = tid + m * BLOCK;
      if (NB % BLOCK == 0 || b < NB) {
        const int col = b % NCOL;
        const int i = b / NCOL;
        const int k = i % Ns;
        const int base = (i / Ns) * Ns * Rs + k;
#pragma unroll
        for (int q = 0; q < Rs; ++q) lds[lds_addr(base + q * Ns, col, NCOL)] = v[m][q];
      }
    }
    __syncthreads();
    fft_stage<E, L, NCOL, BLOCK, DIR, S + 1>(lds, tw, load, store);
  }
}

// Transform NCOL columns of length L.  tw: exp(-2 pi i m / L), m < L.
template <typename E, int L, int NCOL, int BLOCK, int DIR, class Load, class Store>
__device__ __forceinline__ void block_fft(E* __restrict__ lds,
                                          const cpx<typename elem_traits<E>::real>* __restrict__ tw,
                                          Load& load, Store& store) {
  fft_stage<E, L, NCOL, BLOCK, DIR, 0>(lds, tw, load, store);
}
