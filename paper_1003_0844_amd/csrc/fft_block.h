// Workgroup-level Stockham FFT for gfx950.
//
// One workgroup transforms NCOL independent columns of length L (a power of
// two).  Stages are radix 16 except the last (16, 8, 4 or 2).  The first stage
// reads its inputs through a Load functor (global memory, or values computed
// on the fly), the last stage hands each butterfly's Rs outputs to the Store
// functor as store(i, col, v, integral_constant STRIDE): v[q] is output
// i + q STRIDE.  Consecutive stages exchange their data through LDS.
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
//
// Pair elements (the a- and b-weighted series of one node) cross the LDS in
// two rounds, a halves first, then b halves, through a buffer of single
// complex values: the workgroup needs half the LDS, so twice as many
// workgroups fit on a CU, at the price of two more barriers per exchange.
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

template <int L, int NCOL, int BLOCK, int S>
struct StageShape {
  static constexpr int Rs = fft_radix(L, S);
  static constexpr int Ns = fft_span(L, S);
  static constexpr int NB = NCOL * (L / Rs);       // butterflies of the stage
  static constexpr int PER = (NB + BLOCK - 1) / BLOCK;  // butterflies per thread
};

// p[q] = w^q, q < R: squares for even q, one more factor w for odd q
// (at most six products deep for R = 16)
template <int R, typename T>
__device__ __forceinline__ void powers(cpx<T> w, cpx<T> (&p)[R]) {
  p[0] = cpx<T>{(T)1, (T)0};
  if constexpr (R > 1) p[1] = w;
#pragma unroll
  for (int q = 2; q < R; ++q) p[q] = (q % 2 == 0) ? cmul(p[q / 2], p[q / 2]) : cmul(p[q - 1], w);
}

// Thread index as an opaque value: index arithmetic derived from it is redone
// per transform instead of being kept live across a loop of transforms.
__device__ __forceinline__ int fft_tid() {
  int t = threadIdx.x;
  asm volatile("" : "+v"(t));
  return t;
}

constexpr int lds_slots(int L, int NCOL) { return L * NCOL + ((L * NCOL) >> 4); }

__device__ __forceinline__ int lds_addr(int idx, int col, int ncol) {
  const int lin = idx * ncol + col;
  return lin + (lin >> 4);
}

// LDS slot type of an element type: pairs are exchanged half by half.
template <typename E>
struct lds_of {
  using type = E;
  static constexpr int rounds = 1;
};
template <typename T>
struct lds_of<Pair<T>> {
  using type = cpx<T>;
  static constexpr int rounds = 2;
};
template <typename E>
using lds_t = typename lds_of<E>::type;

template <int H, typename T>
__device__ __forceinline__ cpx<T>& part(Pair<T>& e) {
  if constexpr (H == 0) return e.a;
  else return e.b;
}
template <int H, typename T>
__device__ __forceinline__ cpx<T>& part(cpx<T>& e) {
  return e;
}

// Outputs of stage S (registers v) become the inputs of stage S+1 (registers
// u) through LDS.  The leading barrier protects the previous exchange's reads.
template <typename E, int L, int NCOL, int BLOCK, int S, int PV, int RV, int PU, int RU>
__device__ __forceinline__ void exchange(lds_t<E>* __restrict__ lds, E (&v)[PV][RV], E (&u)[PU][RU]) {
  using G0 = StageShape<L, NCOL, BLOCK, S>;
  using G1 = StageShape<L, NCOL, BLOCK, S + 1>;
  const int tid = fft_tid();
  auto put = [&](auto h) {
    constexpr int H = decltype(h)::value;
#pragma unroll
    for (int m = 0; m < PV; ++m) {
      const int b = tid + m * BLOCK;
      if (G0::NB % BLOCK == 0 || b < G0::NB) {
        const int col = b % NCOL;
        const int i = b / NCOL;
        const int k = i % G0::Ns;
        const int base = (i / G0::Ns) * G0::Ns * G0::Rs + k;
#pragma unroll
        for (int q = 0; q < RV; ++q) lds[lds_addr(base + q * G0::Ns, col, NCOL)] = part<H>(v[m][q]);
      }
    }
  };
  auto get = [&](auto h) {
    constexpr int H = decltype(h)::value;
#pragma unroll
    for (int m = 0; m < PU; ++m) {
      const int b = tid + m * BLOCK;
      if (G1::NB % BLOCK == 0 || b < G1::NB) {
        const int col = b % NCOL;
        const int i = b / NCOL;
#pragma unroll
        for (int q = 0; q < RU; ++q) part<H>(u[m][q]) = lds[lds_addr(i + q * (L / G1::Rs), col, NCOL)];
      }
    }
  };
  if constexpr (S > 0) __syncthreads();
  put(std::integral_constant<int, 0>());
  __syncthreads();
  get(std::integral_constant<int, 0>());
  if constexpr (lds_of<E>::rounds == 2) {
    __syncthreads();
    put(std::integral_constant<int, 1>());
    __syncthreads();
    get(std::integral_constant<int, 1>());
  }
}

// Issue the stage-0 loads of one transform into v.
template <typename E, int L, int NCOL, int BLOCK, class Load>
__device__ __forceinline__ void fft_fetch(Load& load,
                                          E (&v)[StageShape<L, NCOL, BLOCK, 0>::PER][StageShape<L, NCOL, BLOCK, 0>::Rs]) {
  using G = StageShape<L, NCOL, BLOCK, 0>;
  const int tid = fft_tid();
#pragma unroll
  for (int m = 0; m < G::PER; ++m) {
    const int b = tid + m * BLOCK;
    if (G::NB % BLOCK == 0 || b < G::NB) {
#pragma unroll
      for (int q = 0; q < G::Rs; ++q) v[m][q] = load(b / NCOL + q * (L / G::Rs), b % NCOL);
    }
  }
}

// Stage twiddle bases w^k, k = i mod Ns, read from the table
// exp(-2 pi i m / L) as each butterfly needs them (one load per butterfly).
template <typename T, int L>
struct TwTable {
  const cpx<T>* __restrict__ tab;
  template <int S>
  __device__ __forceinline__ cpx<T> operator()(std::integral_constant<int, S>, int, int k) const {
    return tab[k * (L / (fft_span(L, S) * fft_radix(L, S)))];
  }
};

// Stage S on the registers v (the inputs of the stage).
template <typename E, int L, int NCOL, int BLOCK, int DIR, int S, class TwF, class Store>
__device__ __forceinline__ void fft_stage(lds_t<E>* __restrict__ lds, const TwF& twf, Store& store,
                                          E (&v)[StageShape<L, NCOL, BLOCK, S>::PER][StageShape<L, NCOL, BLOCK, S>::Rs]) {
  using T = typename elem_traits<E>::real;
  using G = StageShape<L, NCOL, BLOCK, S>;
  constexpr int NS = fft_nstages(L);
  constexpr int Rs = G::Rs;
  const int tid = fft_tid();

#pragma unroll
  for (int m = 0; m < G::PER; ++m) {
    const int b = tid + m * BLOCK;
    if (G::NB % BLOCK == 0 || b < G::NB) {
      if constexpr (S > 0) {
        // one twiddle base per butterfly, the other powers by multiplication
        cpx<T> w = twf(std::integral_constant<int, S>(), m, (b / NCOL) % G::Ns);
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
    for (int m = 0; m < G::PER; ++m) {
      const int b = tid + m * BLOCK;
      if (G::NB % BLOCK == 0 || b < G::NB) {
        // store(i, col, v, STRIDE) or, when it takes one more argument, also the
        // thread's butterfly slot m of the last stage
        if constexpr (std::is_invocable_v<Store&, int, int, E (&)[Rs], std::integral_constant<int, L / Rs>, int>)
          store(b / NCOL, b % NCOL, v[m], std::integral_constant<int, L / Rs>(), m);
        else
          store(b / NCOL, b % NCOL, v[m], std::integral_constant<int, L / Rs>());
      }
    }
  } else {
    using G1 = StageShape<L, NCOL, BLOCK, S + 1>;
    E u[G1::PER][G1::Rs];
    exchange<E, L, NCOL, BLOCK, S>(lds, v, u);
    fft_stage<E, L, NCOL, BLOCK, DIR, S + 1>(lds, twf, store, u);
  }
}

// Transform NCOL columns of length L.  tw: exp(-2 pi i m / L), m < L.
// lds: lds_slots(L, NCOL) slots of lds_t<E>.
template <typename E, int L, int NCOL, int BLOCK, int DIR, class Load, class Store>
__device__ __forceinline__ void block_fft(lds_t<E>* __restrict__ lds,
                                          const cpx<typename elem_traits<E>::real>* __restrict__ tw,
                                          Load& load, Store& store) {
  using G = StageShape<L, NCOL, BLOCK, 0>;
  E v[G::PER][G::Rs];
  fft_fetch<E, L, NCOL, BLOCK>(load, v);
  fft_stage<E, L, NCOL, BLOCK, DIR, 0>(lds, TwTable<typename elem_traits<E>::real, L>{tw}, store, v);
}

// As block_fft, with each stage-0 input made in two steps: read(i, col)
// returns what element i of column col needs from memory, make(raw, i, col)
// turns that into the element.  All reads of a thread are issued before the
// first element is made, so they are in flight together; a Load functor that
// reads under a per-element condition keeps each read in its own branch, and
// the thread then waits for one read after another.
template <typename E, int L, int NCOL, int BLOCK, int DIR, class Read, class Make, class Store>
__device__ __forceinline__ void block_fft_split(lds_t<E>* __restrict__ lds,
                                                const cpx<typename elem_traits<E>::real>* __restrict__ tw,
                                                Read& read, Make& make, Store& store) {
  using G = StageShape<L, NCOL, BLOCK, 0>;
  using Raw = decltype(read(0, 0));
  const int tid = fft_tid();
  Raw raw[G::PER][G::Rs];
#pragma unroll
  for (int m = 0; m < G::PER; ++m) {
    const int b = tid + m * BLOCK;
    if (G::NB % BLOCK == 0 || b < G::NB) {
#pragma unroll
      for (int q = 0; q < G::Rs; ++q) raw[m][q] = read(b / NCOL + q * (L / G::Rs), b % NCOL);
    }
  }
  E v[G::PER][G::Rs];
#pragma unroll
  for (int m = 0; m < G::PER; ++m) {
    const int b = tid + m * BLOCK;
    if (G::NB % BLOCK == 0 || b < G::NB) {
#pragma unroll
      for (int q = 0; q < G::Rs; ++q) v[m][q] = make(raw[m][q], b / NCOL + q * (L / G::Rs), b % NCOL);
    }
  }
  fft_stage<E, L, NCOL, BLOCK, DIR, 0>(lds, TwTable<typename elem_traits<E>::real, L>{tw}, store, v);
}
