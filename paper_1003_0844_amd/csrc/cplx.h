// Complex arithmetic and in-register radix-2/4/8/16 DFTs for the Stockham
// FFT kernels (gfx950, wave64).  DIR = -1 is the forward transform
// (kernel e^{-2 pi i jk/n}, the DFT of Sec. VI B), DIR = +1 the inverse
// (unnormalised).
#pragma once
#include <hip/hip_runtime.h>

template <typename T>
struct cpx {
  T x, y;
};

template <typename T>
__device__ __forceinline__ cpx<T> cadd(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> csub(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cmul(cpx<T> a, cpx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T>
__device__ __forceinline__ cpx<T> cconj(cpx<T> a) { return {a.x, -a.y}; }
template <typename T>
__device__ __forceinline__ cpx<T> cscale(cpx<T> a, T s) { return {a.x * s, a.y * s}; }

// multiply by DIR * i  (forward: -i, inverse: +i)
template <int DIR, typename T>
__device__ __forceinline__ cpx<T> rot90(cpx<T> a) {
  if constexpr (DIR < 0) return {a.y, -a.x};
  else return {-a.y, a.x};
}

// Two complex values sharing every index and twiddle: the a- and b-weighted
// series of one grid node travel together through the FFT.
template <typename T>
struct Pair {
  cpx<T> a, b;
};

template <typename T>
__device__ __forceinline__ cpx<T> twmul(cpx<T> v, cpx<T> w) { return cmul(v, w); }

// Streaming (non-temporal) access for data a pass touches once: the
// inter-pass spill written by pass 1 and read once by pass 2, and the F map.
// With both passes in flight this keeps them from displacing each other's
// cached lines (the 2-day grid: +9 % at equal batch, +16 % with the larger
// batches it makes the best choice).
template <typename T>
__device__ __forceinline__ Pair<T> load_stream(const Pair<T>* p) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  const v4 w = __builtin_nontemporal_load(reinterpret_cast<const v4*>(p));
  return Pair<T>{{w.x, w.y}, {w.z, w.w}};
}
template <typename T>
__device__ __forceinline__ void store_stream(Pair<T>* p, const Pair<T>& v) {
  typedef T v4 __attribute__((ext_vector_type(4)));
  v4 w;
  w.x = v.a.x;
  w.y = v.a.y;
  w.z = v.b.x;
  w.w = v.b.y;
  __builtin_nontemporal_store(w, reinterpret_cast<v4*>(p));
}
template <typename T>
__device__ __forceinline__ void store_stream(T* p, T v) {
  __builtin_nontemporal_store(v, p);
}
template <typename T>
__device__ __forceinline__ Pair<T> twmul(Pair<T> v, cpx<T> w) { return {cmul(v.a, w), cmul(v.b, w)}; }

template <typename E> struct elem_traits;
template <typename T> struct elem_traits<cpx<T>> { using real = T; };
template <typename T> struct elem_traits<Pair<T>> { using real = T; };

// ---------------------------------------------------------------------------
// In-register DFTs of size 2, 4, 8, 16 on cpx<T>, natural order in and out.
// ---------------------------------------------------------------------------
template <int DIR, typename T>
__device__ __forceinline__ void dft2(cpx<T>& a, cpx<T>& b) {
  cpx<T> t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft4(cpx<T>& v0, cpx<T>& v1, cpx<T>& v2, cpx<T>& v3) {
  cpx<T> t0 = cadd(v0, v2), t1 = csub(v0, v2);
  cpx<T> t2 = cadd(v1, v3), t3 = rot90<DIR>(csub(v1, v3));
  v0 = cadd(t0, t2);
  v2 = csub(t0, t2);
  v1 = cadd(t1, t3);
  v3 = csub(t1, t3);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft8(cpx<T> (&v)[8]) {
  const T h = (T)0.70710678118654752440084436210485;
  cpx<T> e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  cpx<T> o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<DIR>(e0, e1, e2, e3);
  dft4<DIR>(o0, o1, o2, o3);
  // w8^k = (cos(pi k/4), DIR sin(pi k/4))
  o1 = cmul(o1, cpx<T>{h, (T)DIR * h});
  o2 = rot90<DIR>(o2);
  o3 = cmul(o3, cpx<T>{-h, (T)DIR * h});
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

template <int DIR, typename T>
__device__ __forceinline__ void dft16(cpx<T> (&v)[16]) {
  const T c1 = (T)0.92387953251128675612818318939679;  // cos(pi/8)
  const T s1 = (T)0.38268343236508977172845998403040;  // sin(pi/8)
  const T h = (T)0.70710678118654752440084436210485;
  cpx<T> e[8], o[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    e[i] = v[2 * i];
    o[i] = v[2 * i + 1];
  }
  dft8<DIR>(e);
  dft8<DIR>(o);
  // w16^k = (cos(pi k/8), DIR sin(pi k/8)), k = 1..7
  o[1] = cmul(o[1], cpx<T>{c1, (T)DIR * s1});
  o[2] = cmul(o[2], cpx<T>{h, (T)DIR * h});
  o[3] = cmul(o[3], cpx<T>{s1, (T)DIR * c1});
  o[4] = rot90<DIR>(o[4]);
  o[5] = cmul(o[5], cpx<T>{-s1, (T)DIR * c1});
  o[6] = cmul(o[6], cpx<T>{-h, (T)DIR * h});
  o[7] = cmul(o[7], cpx<T>{-c1, (T)DIR * s1});
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    v[i] = cadd(e[i], o[i]);
    v[i + 8] = csub(e[i], o[i]);
  }
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(cpx<T> (&v)[R]) {
  static_assert(R == 1 || R == 2 || R == 4 || R == 8 || R == 16, "radix");
  if constexpr (R == 2) dft2<DIR>(v[0], v[1]);
  else if constexpr (R == 4) dft4<DIR>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<DIR>(v);
  else if constexpr (R == 16) dft16<DIR>(v);
}

template <int R, int DIR, typename T>
__device__ __forceinline__ void dft(Pair<T> (&v)[R]) {
  cpx<T> a[R], b[R];
#pragma unroll
  for (int i = 0; i < R; ++i) {
    a[i] = v[i].a;
    b[i] = v[i].b;
  }
  dft<R, DIR>(a);
  dft<R, DIR>(b);
#pragma unroll
  for (int i = 0; i < R; ++i) v[i] = {a[i], b[i]};
}
