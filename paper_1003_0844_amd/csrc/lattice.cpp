// The grid of Sec. IV on the host: the reduced Fisher matrix of the linear
// phase model (Sec. III B, Eqs. philin, albe, siglin, redFm-def), a lattice
// covering of the four phase parameters (omega_0, omega_1, alpha_1, alpha_2)
// built from A4* (Eq. gen) with one basis vector on the frequency axis and one
// without sky components (Eqs. avec, constraint2, opt, opt2), and the
// enumeration of its grid nodes over a sky region and a spindown range.
//
// Plan-time work of a few milliseconds: plain C++ in FP64, no device calls.
//
// Construction (the paper leaves several steps open; the choices made here):
//  - whitening: M = D U diag(lambda)^-1/2 from the eigen-decomposition of
//    D G D, D = diag(G_kk^-1/2) (the parameters span ~24 decades in SI units);
//    M^T G M = 1, a rotation away from Eq. (mmatr);
//  - the Voronoi cell of a lattice from its relevant vectors (the unique
//    shortest pairs of the classes of the lattice modulo twice itself) and its
//    vertices (where four facet planes meet);
//  - nu, rule FSTAT_NU_DEEP_HOLES: the largest expansion across l that keeps
//    every vertex of the A4* Voronoi cell (its deep holes), shrunk by mu along
//    l, within R -- a covering of radius at most R, and the expansion factor of
//    the paper's worked two-dimensional example;
//    rule FSTAT_NU_COVERING: the paper's definition, the largest nu for which
//    the covering radius stays R, by bisection from the deep-hole value (the
//    covering radius grows with nu);
//  - l: among lattice vectors with |e0| <= |l| <= 4 max(|e0|, R), the largest
//    det S = mu nu^3 (the covering rule: over the three shortest admissible
//    lengths, one vector per symmetry class of A4*);
//  - f (Eq. opt2): the shortest lattice vector forming a primitive pair with l;
//    O3 turns its image, about e0, into M^-1 span(omega_0, omega_1);
//  - basis: l, f and the first completing pair with coefficients in [-2, 2],
//    then the sky projections of a2, a3 Lagrange-Gauss reduced, their omega_1
//    parts reduced modulo a1 and the omega_0 parts of a1..a3 modulo a0.
#include <algorithm>
#include <array>
#include <cmath>
#include <cstdint>
#include <numeric>
#include <vector>

#include "fstat.h"

#pragma clang fp contract(off)

namespace {

constexpr int D = 4;
constexpr double C_LIGHT = 299792458.0;  // m/s
constexpr double TWO_PI = 6.283185307179586476925286766559;
constexpr double THETA_A4STAR = 1.7655;  // thickness of A4*, Sec. IV

using Vec = std::array<double, D>;
using Mat = std::array<Vec, D>;  // Mat[i] is row i
using IVec = std::array<int64_t, D>;

double dot(const Vec& a, const Vec& b) {
  double s = 0.0;
  for (int i = 0; i < D; ++i) s += a[i] * b[i];
  return s;
}
double norm(const Vec& a) { return std::sqrt(dot(a, a)); }

Mat identity() {
  Mat m{};
  for (int i = 0; i < D; ++i) m[i][i] = 1.0;
  return m;
}

Mat mul(const Mat& A, const Mat& B) {
  Mat C{};
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      double s = 0.0;
      for (int k = 0; k < D; ++k) s += A[i][k] * B[k][j];
      C[i][j] = s;
    }
  return C;
}

Mat transpose(const Mat& A) {
  Mat T{};
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) T[i][j] = A[j][i];
  return T;
}

Vec combo(const IVec& z, const Mat& G) {  // sum_i z_i G[i]
  Vec v{};
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) v[j] += (double)z[i] * G[i][j];
  return v;
}

// Compensated sum (Neumaier).
struct Sum {
  double s = 0.0, c = 0.0;
  void add(double x) {
    const double t = s + x;
    c += std::fabs(s) >= std::fabs(x) ? (s - t) + x : (x - t) + s;
    s = t;
  }
  double value() const { return s + c; }
};

// Symmetric eigen-decomposition by cyclic Jacobi rotations: A = V diag(lam) V^T,
// the eigenvectors in the columns of V.
void jacobi_eigen(Mat A, Vec& lam, Mat& V) {
  V = identity();
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, diag = 0.0;
    for (int p = 0; p < D; ++p) {
      diag += A[p][p] * A[p][p];
      for (int q = p + 1; q < D; ++q) off += A[p][q] * A[p][q];
    }
    if (off <= 1e-32 * diag) break;
    for (int p = 0; p < D; ++p)
      for (int q = p + 1; q < D; ++q) {
        if (A[p][q] == 0.0) continue;
        const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < D; ++k) {
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < D; ++k) {
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < D; ++k) {
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  for (int i = 0; i < D; ++i) lam[i] = A[i][i];
}

// Solve A x = b (4x4) by Gaussian elimination with partial pivoting on the
// row-equilibrated system (rows of very different scale are common here: the
// whitening's rows span ~11 decades); false if A is numerically singular.
bool solve4(Mat A, Vec b, Vec& x) {
  for (int i = 0; i < D; ++i) {
    const double n = norm(A[i]);
    if (!(n > 0.0)) return false;
    for (auto& v : A[i]) v /= n;
    b[i] /= n;
  }
  for (int c = 0; c < D; ++c) {
    int piv = c;
    for (int r = c + 1; r < D; ++r)
      if (std::fabs(A[r][c]) > std::fabs(A[piv][c])) piv = r;
    if (std::fabs(A[piv][c]) < 1e-12) return false;
    std::swap(A[c], A[piv]);
    std::swap(b[c], b[piv]);
    for (int r = c + 1; r < D; ++r) {
      const double f = A[r][c] / A[c][c];
      for (int k = c; k < D; ++k) A[r][k] -= f * A[c][k];
      b[r] -= f * b[c];
    }
  }
  for (int r = D - 1; r >= 0; --r) {
    double s = b[r];
    for (int k = r + 1; k < D; ++k) s -= A[r][k] * x[k];
    x[r] = s / A[r][r];
  }
  return true;
}

double det4(const Mat& A) {
  Mat U = A;
  double det = 1.0;
  for (int c = 0; c < D; ++c) {
    int piv = c;
    for (int r = c + 1; r < D; ++r)
      if (std::fabs(U[r][c]) > std::fabs(U[piv][c])) piv = r;
    if (U[piv][c] == 0.0) return 0.0;
    if (piv != c) {
      std::swap(U[c], U[piv]);
      det = -det;
    }
    det *= U[c][c];
    for (int r = c + 1; r < D; ++r) {
      const double f = U[r][c] / U[c][c];
      for (int k = c; k < D; ++k) U[r][k] -= f * U[c][k];
    }
  }
  return det;
}

int64_t idet3(int64_t a, int64_t b, int64_t c, int64_t d, int64_t e, int64_t f, int64_t g, int64_t h, int64_t i) {
  return a * (e * i - f * h) - b * (d * i - f * g) + c * (d * h - e * g);
}

// Exact determinant of four integer rows (Laplace expansion along the last row).
int64_t idet4(const IVec& r0, const IVec& r1, const IVec& r2, const IVec& r3) {
  int64_t s = 0;
  for (int j = 0; j < D; ++j) {
    int c[3], n = 0;
    for (int k = 0; k < D; ++k)
      if (k != j) c[n++] = k;
    const int64_t minor = idet3(r0[c[0]], r0[c[1]], r0[c[2]], r1[c[0]], r1[c[1]], r1[c[2]], r2[c[0]], r2[c[1]],
                                r2[c[2]]);
    s += ((3 + j) % 2 ? -1 : 1) * r3[j] * minor;
  }
  return s;
}

// A4* with covering radius R, Eq. (gen); rows are basis vectors.
Mat a4star(double R) {
  const double s2 = std::sqrt(2.0), s3 = std::sqrt(3.0), s5 = std::sqrt(5.0), s6 = std::sqrt(6.0);
  Mat G{{{s2, 0, 0, 0},
         {1 / s2, std::sqrt(2.0 / 3.0) + 1 / s6, 0, 0},
         {1 / s2, 1 / s6, 1 / (2 * s3) + s3 / 2, 0},
         {-1 / (5 * s2) - 2 * s2 / 5, 1 / (5 * s6) - s6 / 5, -1 / (5 * s3) - s3 / 10, -1 / (2 * s5)}}};
  const double k = R * std::sqrt(2.5);
  for (auto& r : G)
    for (auto& x : r) x *= k;
  return G;
}

// Integer vectors z != 0 with |z G| <= rho, by enumeration over the upper
// triangular factor U of the Gram matrix (z^T G G^T z = |U z|^2).
struct ShortVectors {
  double U[D][D] = {};
  double lim;
  int64_t z[D] = {};
  std::vector<IVec> out;

  ShortVectors(const Mat& G, double rho) : lim(rho * rho * (1 + 1e-12)) {
    double Q[D][D], L[D][D] = {};
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) Q[i][j] = dot(G[i], G[j]);
    for (int j = 0; j < D; ++j) {
      double s = Q[j][j];
      for (int k = 0; k < j; ++k) s -= L[j][k] * L[j][k];
      L[j][j] = std::sqrt(s);
      for (int i = j + 1; i < D; ++i) {
        double t = Q[i][j];
        for (int k = 0; k < j; ++k) t -= L[i][k] * L[j][k];
        L[i][j] = t / L[j][j];
      }
    }
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j) U[i][j] = L[j][i];
    rec(D - 1, lim);
  }
  void rec(int i, double rem) {
    double c = 0.0;
    for (int j = i + 1; j < D; ++j) c += U[i][j] * (double)z[j];
    const double r = std::sqrt(std::max(rem, 0.0));
    const int64_t lo = (int64_t)std::ceil((-r - c) / U[i][i] - 1e-9);
    const int64_t hi = (int64_t)std::floor((r - c) / U[i][i] + 1e-9);
    for (int64_t zi = lo; zi <= hi; ++zi) {
      z[i] = zi;
      const double v = U[i][i] * (double)zi + c;
      if (i == 0) {
        bool nz = false;
        for (int k = 0; k < D; ++k) nz |= z[k] != 0;
        if (nz) out.push_back(IVec{z[0], z[1], z[2], z[3]});
      } else {
        rec(i - 1, rem - v * v);
      }
    }
    z[i] = 0;
  }
};

std::vector<IVec> short_vectors(const Mat& G, double rho) {
  ShortVectors sv(G, rho);
  std::vector<IVec> keep;
  for (const IVec& z : sv.out) {
    const Vec v = combo(z, G);
    if (dot(v, v) <= rho * rho * (1 + 1e-9)) keep.push_back(z);
  }
  return keep;
}

// Voronoi-relevant vectors: per nonzero class modulo 2, the shortest vectors
// when they are a single pair +-v.  Radius sqrt(sum |b*_i|^2): the
// nearest-plane bound on twice the covering radius.
std::vector<Vec> relevant_vectors(const Mat& G) {
  ShortVectors probe(G, 0.0);
  double rho2 = 0.0;
  for (int i = 0; i < D; ++i) rho2 += probe.U[i][i] * probe.U[i][i];
  const std::vector<IVec> Z = short_vectors(G, std::sqrt(rho2));
  std::vector<double> best(1 << D, INFINITY);
  std::vector<double> n2(Z.size());
  std::vector<int> cls(Z.size());
  for (size_t i = 0; i < Z.size(); ++i) {
    const Vec v = combo(Z[i], G);
    n2[i] = dot(v, v);
    int c = 0;
    for (int k = 0; k < D; ++k) c |= (int)(((Z[i][k] % 2) + 2) % 2) << k;
    cls[i] = c;
    best[c] = std::min(best[c], n2[i]);
  }
  std::vector<Vec> out;
  for (int c = 1; c < (1 << D); ++c) {
    std::vector<size_t> low;
    for (size_t i = 0; i < Z.size(); ++i)
      if (cls[i] == c && n2[i] <= best[c] * (1 + 1e-9)) low.push_back(i);
    if (low.size() == 2)
      for (size_t i : low) out.push_back(combo(Z[i], G));
  }
  return out;
}

// Vertices of the Voronoi cell of the origin.
std::vector<Vec> voronoi_vertices(const Mat& G) {
  const std::vector<Vec> rv = relevant_vectors(G);
  const int m = (int)rv.size();
  std::vector<double> b(m);
  double bmax = 0.0;
  for (int i = 0; i < m; ++i) {
    b[i] = 0.5 * dot(rv[i], rv[i]);
    bmax = std::max(bmax, b[i]);
  }
  std::vector<Vec> verts;
  for (int i0 = 0; i0 < m; ++i0)
    for (int i1 = i0 + 1; i1 < m; ++i1)
      for (int i2 = i1 + 1; i2 < m; ++i2)
        for (int i3 = i2 + 1; i3 < m; ++i3) {
          Vec x{};
          if (!solve4(Mat{rv[i0], rv[i1], rv[i2], rv[i3]}, Vec{b[i0], b[i1], b[i2], b[i3]}, x)) continue;
          bool ok = true;
          for (int k = 0; k < m && ok; ++k) ok = dot(rv[k], x) <= b[k] + 1e-9 * bmax;
          if (!ok) continue;
          bool dup = false;
          for (const Vec& y : verts) {
            Vec d{};
            for (int k = 0; k < D; ++k) d[k] = x[k] - y[k];
            dup |= norm(d) < 1e-9 * std::sqrt(bmax);
          }
          if (!dup) verts.push_back(x);
        }
  return verts;
}

// An orthogonal matrix (column convention) whose first column is the unit vector u:
// Gram-Schmidt on the coordinate axes, each time the axis farthest from the span so
// far (with m < 4 orthonormal columns some axis keeps a residual of at least 1/2).
Mat frame(const Vec& u) {
  std::vector<Vec> cols{u};
  while ((int)cols.size() < D) {
    Vec best{};
    double bn = -1.0;
    for (int e = 0; e < D; ++e) {
      Vec w{};
      w[e] = 1.0;
      for (const Vec& c : cols) {
        const double p = dot(w, c);
        for (int k = 0; k < D; ++k) w[k] -= p * c[k];
      }
      const double n = norm(w);
      if (n > bn) {
        bn = n;
        best = w;
      }
    }
    for (auto& x : best) x /= bn;
    cols.push_back(best);
  }
  Mat O{};
  for (int j = 0; j < D; ++j)
    for (int i = 0; i < D; ++i) O[i][j] = cols[j][i];
  if (det4(O) < 0)
    for (int i = 0; i < D; ++i) O[i][D - 1] = -O[i][D - 1];
  return O;
}

double covering_radius(const Mat& G) {
  double r = 0.0;
  for (const Vec& v : voronoi_vertices(G)) r = std::max(r, norm(v));
  return r;
}

// G0 O1 diag(mu, nu, nu, nu) O1^T: shrunk by mu along l, expanded by nu across it.
Mat scaled(const Mat& G0, const Vec& l, double mu, double nu) {
  Vec lh = l;
  const double n = norm(l);
  for (auto& x : lh) x /= n;
  const Mat O1 = frame(lh);
  Mat S{};
  S[0][0] = mu;
  for (int i = 1; i < D; ++i) S[i][i] = nu;
  return mul(mul(mul(G0, O1), S), transpose(O1));
}

double covering_nu(const Mat& G0, const Vec& l, double mu, double R, double lo) {
  double hi = lo * 1.25;
  while (covering_radius(scaled(G0, l, mu, hi)) <= R) {
    lo = hi;
    hi *= 1.25;
  }
  while (hi - lo > 1e-12 * lo) {
    const double mid = 0.5 * (lo + hi);
    if (covering_radius(scaled(G0, l, mu, mid)) <= R)
      lo = mid;
    else
      hi = mid;
  }
  return lo;
}

// Sorted |v . r| over the relevant vectors: shared by vectors a symmetry of the
// lattice maps onto each other (it permutes the relevant vectors).
std::vector<double> orbit_key(const Vec& v, const std::vector<Vec>& rv) {
  std::vector<double> k;
  for (const Vec& r : rv) k.push_back(std::fabs(dot(v, r)));
  std::sort(k.begin(), k.end());
  return k;
}

bool same_key(const std::vector<double>& a, const std::vector<double>& b) {
  if (a.size() != b.size()) return false;
  for (size_t i = 0; i < a.size(); ++i)
    if (std::fabs(a[i] - b[i]) > 1e-9 * (1.0 + std::fabs(a[i]))) return false;
  return true;
}

double expansion_nu(const std::vector<Vec>& verts, const Vec& l, double mu, double R) {
  Vec lh = l;
  const double ln = norm(l);
  for (auto& x : lh) x /= ln;
  double nu2 = INFINITY;
  for (const Vec& v : verts) {
    const double c = dot(v, lh);
    const double p2 = dot(v, v) - c * c;
    if (p2 > 1e-12 * R * R) nu2 = std::min(nu2, (R * R - mu * mu * c * c) / p2);
  }
  return std::sqrt(nu2);
}

bool primitive_pair(const IVec& a, const IVec& b) {
  int64_t g = 0;
  for (int i = 0; i < D; ++i)
    for (int j = i + 1; j < D; ++j) g = std::gcd(g, a[i] * b[j] - a[j] * b[i]);
  return g == 1;
}

bool finite_all(const double* x, int n) {
  for (int i = 0; i < n; ++i)
    if (!std::isfinite(x[i])) return false;
  return true;
}

}  // namespace

extern "C" {

fstat_status fstat_lattice_fisher(const fstat_segment* seg, const fstat_detector* det, const fstat_ephemeris* eph,
                                  double gamma[16]) {
  if (!seg || !det || !eph || !gamma) return FSTAT_EINVAL;
  if (seg->n < 2 || !(seg->dt > 0.0) || !std::isfinite(seg->dt) || !std::isfinite(seg->t0) ||
      !(eph->sidereal_day_s > 0.0))
    return FSTAT_EINVAL;
  const double ce = std::cos(eph->obliquity_rad), rc = det->radius_m * std::cos(det->lat_rad);
  auto m_at = [&](int64_t j, double m[D]) {
    const double t = (double)j * seg->dt, T = seg->t0 + t;
    const double ang = eph->orbit_omega * T + eph->orbit_phase0;
    const double th = eph->gmst0_rad + det->lon_rad + TWO_PI * T / eph->sidereal_day_s;
    const double xes = eph->orbit_radius_m * std::cos(ang), yes = eph->orbit_radius_m * std::sin(ang);
    m[0] = t;
    m[1] = 0.5 * t * t;
    m[2] = (yes + rc * std::sin(th) * ce) / C_LIGHT;  // mu_1
    m[3] = (xes + rc * std::cos(th)) / C_LIGHT;       // mu_2
  };
  Sum s1[D];
  int64_t kept = 0;
  double m[D];
  for (int64_t j = 0; j < seg->n; ++j) {
    if (seg->mask && !seg->mask[j]) continue;
    m_at(j, m);
    for (int k = 0; k < D; ++k) s1[k].add(m[k]);
    ++kept;
  }
  if (kept < 2) return FSTAT_EINVAL;
  double mean[D];
  for (int k = 0; k < D; ++k) mean[k] = s1[k].value() / (double)kept;
  Sum s2[D][D];
  for (int64_t j = 0; j < seg->n; ++j) {
    if (seg->mask && !seg->mask[j]) continue;
    m_at(j, m);
    for (int k = 0; k < D; ++k) m[k] -= mean[k];
    for (int k = 0; k < D; ++k)
      for (int l = k; l < D; ++l) s2[k][l].add(m[k] * m[l]);
  }
  for (int k = 0; k < D; ++k)
    for (int l = k; l < D; ++l) gamma[4 * k + l] = gamma[4 * l + k] = s2[k][l].value() / (double)kept;
  return FSTAT_OK;
}

fstat_status fstat_lattice_build(const double gamma[16], double dp0, double c0, int32_t rule, fstat_lattice* out) {
  if (!gamma || !out || !finite_all(gamma, 16) || !(dp0 > 0.0) || !std::isfinite(dp0) || !(c0 > 0.0) ||
      !(c0 < 1.0) || (rule != FSTAT_NU_DEEP_HOLES && rule != FSTAT_NU_COVERING))
    return FSTAT_EINVAL;
  Mat G{};
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      G[i][j] = gamma[4 * i + j];
      if (gamma[4 * i + j] != gamma[4 * j + i]) return FSTAT_EINVAL;
    }
  for (int i = 0; i < D; ++i)
    if (!(G[i][i] > 0.0)) return FSTAT_EINVAL;
  // whitening M: M^T G M = 1
  Vec dsc{};
  for (int i = 0; i < D; ++i) dsc[i] = 1.0 / std::sqrt(G[i][i]);
  Mat A{};
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) A[i][j] = dsc[i] * G[i][j] * dsc[j];
  Vec lam{};
  Mat V{};
  jacobi_eigen(A, lam, V);
  for (int i = 0; i < D; ++i)
    if (!(lam[i] > 1e-14)) return FSTAT_EINVAL;  // not (numerically) positive definite
  Mat M{};
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) M[i][j] = dsc[i] * V[i][j] / std::sqrt(lam[j]);
  // e0 = M^-1 a0
  Vec a0{dp0, 0, 0, 0}, e0{};
  if (!solve4(M, a0, e0)) return FSTAT_EINVAL;
  const double e0n = norm(e0);
  const double R = std::sqrt(1.0 - c0);
  const Mat G0 = a4star(R);
  const std::vector<Vec> verts = voronoi_vertices(G0);
  if (verts.size() != 120) return FSTAT_EINVAL;  // A4*: the 5! vertices of the permutohedron
  // l: the largest det S = mu nu^3
  std::vector<IVec> cand = short_vectors(G0, 4.0 * std::max(e0n, R));
  std::vector<double> len(cand.size());
  for (size_t i = 0; i < cand.size(); ++i) len[i] = norm(combo(cand[i], G0));
  std::vector<size_t> ord(cand.size());
  std::iota(ord.begin(), ord.end(), 0);
  std::stable_sort(ord.begin(), ord.end(), [&](size_t a, size_t b) { return len[a] < len[b]; });
  double best = -1.0, mu = 0.0, nu = 0.0;
  IVec zl{};
  std::vector<double> lengths;  // distinct admissible lengths, ascending
  for (size_t i : ord)
    if (len[i] >= e0n * (1 - 1e-12) && (lengths.empty() || len[i] > lengths.back() * (1 + 1e-9)))
      lengths.push_back(len[i]);
  const std::vector<Vec> rv = relevant_vectors(G0);
  std::vector<std::vector<double>> seen;
  for (size_t i : ord) {
    if (len[i] < e0n * (1 - 1e-12)) continue;
    const double m_ = e0n / len[i];
    double n_ = expansion_nu(verts, combo(cand[i], G0), m_, R);
    if (rule == FSTAT_NU_COVERING) {
      if (lengths.empty() || len[i] > lengths[std::min<size_t>(2, lengths.size() - 1)] * (1 + 1e-9)) continue;
      const std::vector<double> key = orbit_key(combo(cand[i], G0), rv);
      bool dup = false;
      for (const auto& k : seen) dup = dup || same_key(k, key);
      if (dup) continue;
      seen.push_back(key);
      n_ = covering_nu(G0, combo(cand[i], G0), m_, R, n_);
    }
    const double ds = m_ * n_ * n_ * n_;
    if (ds > best * (1 + 1e-12)) {
      best = ds;
      mu = m_;
      nu = n_;
      zl = cand[i];
    }
  }
  if (best <= 0.0) return FSTAT_EINVAL;
  Vec lh = combo(zl, G0), eh = e0;
  const double lnn = norm(lh);
  for (int k = 0; k < D; ++k) {
    lh[k] /= lnn;
    eh[k] /= e0n;
  }
  const Mat O1 = frame(lh), O2 = frame(eh);
  Mat S{};
  S[0][0] = mu;
  for (int i = 1; i < D; ++i) S[i][i] = nu;
  const Mat X = mul(mul(mul(G0, O1), S), transpose(O2));  // rows in whitened coordinates
  // f: shortest vector forming a primitive pair with l
  std::vector<IVec> fc = short_vectors(G0, 4.0 * R);
  std::vector<double> flen(fc.size());
  for (size_t i = 0; i < fc.size(); ++i) flen[i] = norm(combo(fc[i], G0));
  std::vector<size_t> ford(fc.size());
  std::iota(ford.begin(), ford.end(), 0);
  std::stable_sort(ford.begin(), ford.end(), [&](size_t a, size_t b) { return flen[a] < flen[b]; });
  IVec zf{};
  bool found = false;
  for (size_t i : ford)
    if (primitive_pair(zl, fc[i])) {
      zf = fc[i];
      found = true;
      break;
    }
  if (!found) return FSTAT_EINVAL;
  // O3 (Eq. opt2): about e0, take f's image into W = {x : (M x)_alpha = 0}
  Vec r2 = M[2], r3 = M[3];
  {
    const double n2 = norm(r2);
    for (auto& x : r2) x /= n2;
    const double p = dot(r3, r2);
    for (int k = 0; k < D; ++k) r3[k] -= p * r2[k];
    const double n3 = norm(r3);
    for (auto& x : r3) x /= n3;
  }
  Vec w{};
  double wbest = -1.0;
  for (int e = 0; e < D; ++e) {  // the unit vector of W orthogonal to e0
    Vec v{};
    v[e] = 1.0;
    for (const Vec* c : {&r2, &r3, &eh}) {
      const double p = dot(v, *c);
      for (int k = 0; k < D; ++k) v[k] -= p * (*c)[k];
    }
    const double n = norm(v);
    if (n > wbest) {
      wbest = n;
      w = v;
    }
  }
  for (auto& x : w) x /= wbest;
  Vec y = combo(zf, X), a{};
  const double ye = dot(y, eh);
  for (int k = 0; k < D; ++k) a[k] = y[k] - ye * eh[k];
  const double an = norm(a);
  if (!(an > 0.0)) return FSTAT_EINVAL;
  for (auto& x : a) x /= an;
  double c = dot(a, w);
  if (c < 0) {
    for (auto& x : w) x = -x;
    c = -c;
  }
  Mat O3 = identity();
  Vec bv{};
  for (int k = 0; k < D; ++k) bv[k] = w[k] - c * a[k];
  const double bn = norm(bv);
  if (bn > 1e-14) {
    for (auto& x : bv) x /= bn;
    const double s = std::sqrt(std::max(0.0, 1.0 - c * c));
    for (int i = 0; i < D; ++i)
      for (int j = 0; j < D; ++j)
        O3[i][j] += (c - 1.0) * (a[i] * a[j] + bv[i] * bv[j]) + s * (bv[i] * a[j] - a[i] * bv[j]);
  }
  const Mat Mopt = mul(mul(X, transpose(O3)), transpose(M));  // Eq. (opt2), rows in tau coordinates
  // basis completion: det[l; f; g; h] = h . cof(l, f, g) = +-1
  std::vector<IVec> box;
  for (int64_t i0 = -2; i0 <= 2; ++i0)
    for (int64_t i1 = -2; i1 <= 2; ++i1)
      for (int64_t i2 = -2; i2 <= 2; ++i2)
        for (int64_t i3 = -2; i3 <= 2; ++i3) box.push_back(IVec{i0, i1, i2, i3});
  std::vector<double> blen(box.size());
  for (size_t i = 0; i < box.size(); ++i) blen[i] = norm(combo(box[i], G0));
  std::vector<size_t> bord(box.size());
  std::iota(bord.begin(), bord.end(), 0);
  std::stable_sort(bord.begin(), bord.end(), [&](size_t p, size_t q) { return blen[p] < blen[q]; });
  IVec zg{}, zh{};
  found = false;
  for (size_t gi : bord) {
    const IVec& g = box[gi];
    IVec cof{};
    for (int e = 0; e < D; ++e) {
      IVec u{};
      u[e] = 1;
      cof[e] = idet4(zl, zf, g, u);
    }
    for (size_t hi : bord) {
      const IVec& h = box[hi];
      int64_t d = 0;
      for (int k = 0; k < D; ++k) d += h[k] * cof[k];
      if (d == 1 || d == -1) {
        zg = g;
        zh = h;
        found = true;
        break;
      }
    }
    if (found) break;
  }
  if (!found) return FSTAT_EINVAL;
  Mat B{combo(zl, Mopt), combo(zf, Mopt), combo(zg, Mopt), combo(zh, Mopt)};
  Vec scale{};
  for (int j = 0; j < D; ++j)
    for (int i = 0; i < D; ++i) scale[j] = std::max(scale[j], std::fabs(Mopt[i][j]));
  bool ok = std::fabs(B[0][0] / dp0 - 1.0) < 1e-9;
  for (int j = 1; j < D; ++j) ok = ok && std::fabs(B[0][j]) <= 1e-9 * scale[j];
  for (int j = 2; j < D; ++j) ok = ok && std::fabs(B[1][j]) <= 1e-9 * scale[j];
  if (!ok || B[1][1] == 0.0) return FSTAT_EINVAL;  // too ill-conditioned to meet the constraints
  B[0] = Vec{dp0, 0, 0, 0};
  B[1][2] = B[1][3] = 0.0;
  // reduction: sky projections of a2, a3 (Lagrange-Gauss), then modulo a1, a0
  Vec u = B[2], v = B[3];
  auto sky2 = [](const Vec& p, const Vec& q) { return p[2] * q[2] + p[3] * q[3]; };
  for (int it = 0; it < 100; ++it) {
    if (sky2(u, u) > sky2(v, v)) std::swap(u, v);
    const double q = std::nearbyint(sky2(u, v) / sky2(u, u));
    if (q == 0.0) break;
    for (int k = 0; k < D; ++k) v[k] -= q * u[k];
  }
  B[2] = u;
  B[3] = v;
  for (int i = 2; i < D; ++i) {
    const double q = std::nearbyint(B[i][1] / B[1][1]);
    for (int k = 0; k < D; ++k) B[i][k] -= q * B[1][k];
  }
  for (int i = 1; i < D; ++i) {
    const double q = std::nearbyint(B[i][0] / B[0][0]);
    for (int k = 0; k < D; ++k) B[i][k] -= q * B[0][k];
  }
  // shadows of the covering ellipsoid: G^-1 = M M^T
  const Mat Gi = mul(M, transpose(M));
  const double sa = Gi[2][2], sb = Gi[2][3], sd = Gi[3][3];
  const double lmax = 0.5 * (sa + sd) + std::sqrt(0.25 * (sa - sd) * (sa - sd) + sb * sb);
  for (int i = 0; i < D; ++i)
    for (int j = 0; j < D; ++j) {
      out->basis[4 * i + j] = B[i][j];
      out->gamma[4 * i + j] = G[i][j];
    }
  out->dp0 = dp0;
  out->c0 = c0;
  out->R = R;
  out->mu = mu;
  out->nu = nu;
  out->theta = THETA_A4STAR / best;
  out->margin_w1 = R * std::sqrt(Gi[1][1]);
  out->margin_sky = R * std::sqrt(lmax);
  out->rule = rule;
  out->reserved = 0;
  return FSTAT_OK;
}

fstat_status fstat_lattice_nodes(const fstat_lattice* lat, const fstat_lattice_region* reg,
                                 const fstat_ephemeris* eph, fstat_node* nodes, int32_t* coef, int64_t capacity,
                                 int64_t* count) {
  if (!lat || !reg || !eph || !count || capacity < 0 || (capacity > 0 && !nodes)) return FSTAT_EINVAL;
  if (!finite_all(lat->basis, 16) || !(lat->basis[0] > 0.0) || lat->basis[5] == 0.0 || !(reg->f_sky_hz > 0.0) ||
      !std::isfinite(reg->f_sky_hz) || !std::isfinite(reg->fdot_lo) || !std::isfinite(reg->fdot_hi) ||
      reg->fdot_lo > reg->fdot_hi || !std::isfinite(reg->sky_c1) || !std::isfinite(reg->sky_c2) ||
      !std::isfinite(reg->sky_radius) || reg->hemisphere < -1 || reg->hemisphere > 1 ||
      !std::isfinite(eph->obliquity_rad) || !(lat->margin_w1 >= 0.0) || !(lat->margin_sky >= 0.0))
    return FSTAT_EINVAL;
  const double* B = lat->basis;  // row-major [4][4]
  const double om = TWO_PI * reg->f_sky_hz, ma = lat->margin_sky, dp0 = B[0];
  const double s00 = B[10], s01 = B[11], s10 = B[14], s11 = B[15];  // sky projections of a2, a3
  const double det = s00 * s11 - s01 * s10;
  if (det == 0.0) return FSTAT_EINVAL;
  // S^-1 = [[s11, -s01], [-s10, s00]] / det; k = P S^-1
  const double i00 = s11 / det, i01 = -s01 / det, i10 = -s10 / det, i11 = s00 / det;
  const bool patch = reg->sky_radius > 0.0;
  const double c1 = patch ? reg->sky_c1 : 0.0, c2 = patch ? reg->sky_c2 : 0.0;
  const double rad = (patch ? reg->sky_radius : om) + ma;
  const double k0a = c1 * i00 + c2 * i10, k0b = c1 * i01 + c2 * i11;
  const double spa = rad * std::hypot(i00, i10), spb = rad * std::hypot(i01, i11);
  const double w_lo = TWO_PI * reg->fdot_lo - lat->margin_w1, w_hi = TWO_PI * reg->fdot_hi + lat->margin_w1;
  const double a10 = B[4], a11 = B[5];
  const double ce = std::cos(eph->obliquity_rad), se = std::sin(eph->obliquity_rad);
  int64_t n = 0;
  const int64_t k2lo = (int64_t)std::floor(k0a - spa), k2hi = (int64_t)std::ceil(k0a + spa);
  const int64_t k3lo = (int64_t)std::floor(k0b - spb), k3hi = (int64_t)std::ceil(k0b + spb);
  if ((double)(k2hi - k2lo) * (double)(k3hi - k3lo) > 1e10) return FSTAT_EINVAL;
  for (int64_t k2 = k2lo; k2 <= k2hi; ++k2)
    for (int64_t k3 = k3lo; k3 <= k3hi; ++k3) {
      const double p1 = (double)k2 * s00 + (double)k3 * s10, p2 = (double)k2 * s01 + (double)k3 * s11;
      if (std::hypot(p1, p2) > om + ma) continue;
      if (patch && std::hypot(p1 - c1, p2 - c2) > reg->sky_radius + ma) continue;
      const double w1 = (double)k2 * B[9] + (double)k3 * B[13];
      const double w0 = (double)k2 * B[8] + (double)k3 * B[12];
      double ka = (w_lo - w1) / a11, kb = (w_hi - w1) / a11;
      if (ka > kb) std::swap(ka, kb);
      // sky directions (alpha_1, alpha_2) = omega_s (n_y, n_x), ecliptic frame
      double nx = p2 / om, ny = p1 / om;
      const double r2 = nx * nx + ny * ny;
      double dirs[2][2];
      int nd = 0;
      auto put = [&](double x, double y, double z) {
        const double yq = y * ce - z * se, zq = y * se + z * ce;
        double al = std::atan2(yq, x);
        al = al - TWO_PI * std::floor(al / TWO_PI);
        if (al >= TWO_PI) al = 0.0;
        dirs[nd][0] = al;
        dirs[nd][1] = std::asin(std::max(-1.0, std::min(1.0, zq)));
        ++nd;
      };
      if (r2 >= 1.0) {
        const double r = std::sqrt(r2);
        put(nx / r, ny / r, 0.0);
      } else {
        const double nz = std::sqrt(1.0 - r2);
        if (reg->hemisphere >= 0) put(nx, ny, nz);
        if (reg->hemisphere <= 0) put(nx, ny, -nz);
      }
      for (int h = 0; h < nd; ++h)
        for (int64_t k1 = (int64_t)std::ceil(ka); k1 <= (int64_t)std::floor(kb); ++k1) {
          if (n < capacity) {
            const double om1 = (double)k1 * a11 + w1;
            const double om0 = (double)k1 * a10 + w0;
            const double x = om0 / dp0;
            double fr = x - std::floor(x);
            float off = (float)fr;
            if (off >= 1.0f) off = 0.0f;
            fstat_node& nd_ = nodes[n];
            nd_.alpha = dirs[h][0];
            nd_.delta = dirs[h][1];
            nd_.fdot = om1 / TWO_PI;
            nd_.seg = reg->seg;
            nd_.bin_offset = off;
            if (coef) {
              coef[3 * n] = (int32_t)k1;
              coef[3 * n + 1] = (int32_t)k2;
              coef[3 * n + 2] = (int32_t)k3;
            }
          }
          ++n;
        }
    }
  *count = n;
  return FSTAT_OK;
}

fstat_status fstat_lattice_segment(const fstat_segment* seg, const fstat_detector* det, const fstat_ephemeris* eph,
                                   double c0, int32_t rule, fstat_lattice* out) {
  if (!seg || !det || !eph || !out || seg->n < 2 || !(seg->dt > 0.0) || !std::isfinite(seg->dt)) return FSTAT_EINVAL;
  int64_t nfft = seg->nfft;
  if (nfft == 0) {
    nfft = 1;
    while (nfft < 2 * seg->n) nfft <<= 1;
  }
  if (nfft < seg->n || (nfft & (nfft - 1)) != 0) return FSTAT_EINVAL;
  double gamma[16];
  const fstat_status rc = fstat_lattice_fisher(seg, det, eph, gamma);
  if (rc != FSTAT_OK) return rc;
  // the angular frequency spacing of the segment's Fourier bins (Eq. DFT)
  return fstat_lattice_build(gamma, TWO_PI / ((double)nfft * seg->dt), c0, rule, out);
}

}  // extern "C"
