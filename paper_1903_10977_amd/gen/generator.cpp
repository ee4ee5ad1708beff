// Native generator of immersed multigrid problems (host C++ / OpenMP).
//
// Produces the inputs of the solver library's setup call: fine operator and
// load vector (eq:systemMulti with the scalar analogue of eq:operatorsMulti),
// two-scale restrictions (eq:coarsening), Galerkin coarse operators
// (Remark rem:gridParamCorr) and Schwarz blocks by encapsulating supports
// (smoothers subsection).  Cut-cell integration follows Figure 1's caption:
// bisection of cut cells to a maximum depth, triangulation of cut leaves,
// Gauss rules on the clipped simplices and on the approximate boundary.
//
// Readings shared with the CPU reference (written independently there):
//   * Omega = {psi > 0}; |psi| < 1e-13 counts as 0 (outside);
//   * geometry is sampled at the leaf-lattice vertices (spacing h / 2^depth):
//     an element is active when any leaf vertex in it is positive;
//   * cut leaf squares split along the (0,0)-(1,1) diagonal, cut leaf cubes
//     into the six Kuhn tetrahedra (permutations in lexicographic order);
//     the positive part of each simplex under the linear interpolant is
//     integrated with collapsed (Duffy) Gauss-Legendre rules, 2D polygons are
//     fanned from the first vertex met when walking the triangle's edges;
//   * a coarse element is active when a child is active; a function is
//     active when non-zero on an active element (minus box-Dirichlet ones);
//   * block(j) = {k active : active elements of supp phi_k are all in
//     supp phi_j}; Lagrange blocks only for vertex functions.
//
// This file is independent of the CPU reference: the B-spline values come
// from the triangular (de Boor) scheme, R from Boehm knot insertion, inside
// elements from tensor products of 1D element matrices, support containment
// from summed-area tables.

#include "../../include/imsmg_gen.h"

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>
#include <omp.h>

namespace {

thread_local std::string g_err;

struct GenError : std::runtime_error {
  int code;
  GenError(int c, const std::string &m) : std::runtime_error(m), code(c) {}
};

constexpr double kSnap = 1e-13;
constexpr double kPi = 3.14159265358979323846;

// ---------------------------------------------------------------- Gauss rules
struct Rule1D { std::vector<double> x, w; };  // on [0, 1]

Rule1D gauss_legendre01(int q) {
  Rule1D r;
  r.x.resize(q);
  r.w.resize(q);
  for (int i = 0; i < q; ++i) {
    // Newton iteration on P_q from the Chebyshev-like initial guess
    double z = std::cos(kPi * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      if (q == 1) { p1 = z; p0 = 1.0; }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= q; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    if (q == 1) { p1 = z; p0 = 1.0; }
    dp = q * (z * p1 - p0) / (z * z - 1.0);
    double wt = 2.0 / ((1.0 - z * z) * dp * dp);
    r.x[q - 1 - i] = 0.5 * (z + 1.0);
    r.w[q - 1 - i] = 0.5 * wt;
  }
  return r;
}

// ------------------------------------------------------------ 1D bases
struct Basis1D {
  int basis, n, p;
  double lo, hi, h;
  std::vector<double> knots;  // B-spline open knot vector
  Basis1D(int basis_, int n_, int p_, double lo_, double hi_)
      : basis(basis_), n(n_), p(p_), lo(lo_), hi(hi_), h((hi_ - lo_) / n_) {
    if (basis == IMSMG_GEN_BSPLINE) {
      knots.resize(n + 2 * p + 1);
      for (int i = 0; i < p; ++i) knots[i] = lo;
      for (int i = 0; i <= n; ++i) knots[p + i] = lo + (hi - lo) * double(i) / double(n);
      for (int i = 0; i < p; ++i) knots[p + n + 1 + i] = hi;
    }
  }
  int nfuncs() const { return basis == IMSMG_GEN_BSPLINE ? n + p : p * n + 1; }
  int first(int e) const { return basis == IMSMG_GEN_BSPLINE ? e : p * e; }
  // element range [lo_e, hi_e] of the support of function i
  void support(int i, int &a, int &b) const {
    if (basis == IMSMG_GEN_BSPLINE) {
      a = std::max(0, i - p);
      b = std::min(n - 1, i);
    } else if (i % p == 0) {
      a = std::max(0, i / p - 1);
      b = std::min(n - 1, i / p);
    } else {
      a = b = i / p;
    }
  }
  // values and derivatives of the p+1 functions non-zero on element e at x
  void eval(int e, double x, double *val, double *der) const {
    if (basis == IMSMG_GEN_BSPLINE) {
      bspline(e, x, val, der);
    } else {
      lagrange(e, x, val, der);
    }
  }
  // triangular scheme for the non-zero B-splines of degree d on span s
  void triangle(int s, int d, double x, double *N) const {
    double left[8], right[8];
    N[0] = 1.0;
    for (int j = 1; j <= d; ++j) {
      left[j] = x - knots[s + 1 - j];
      right[j] = knots[s + j] - x;
      double saved = 0.0;
      for (int r = 0; r < j; ++r) {
        double tmp = N[r] / (right[r + 1] + left[j - r]);
        N[r] = saved + right[r + 1] * tmp;
        saved = left[j - r] * tmp;
      }
      N[j] = saved;
    }
  }
  void bspline(int e, double x, double *val, double *der) const {
    const int s = e + p;
    triangle(s, p, x, val);
    if (p == 0) { der[0] = 0.0; return; }
    double Nm[8];
    triangle(s, p - 1, x, Nm);  // functions s-p+1 .. s of degree p-1
    for (int a = 0; a <= p; ++a) {
      const int i = s - p + a;
      double d = 0.0;
      if (a >= 1) {
        double den = knots[i + p] - knots[i];
        if (den > 0.0) d += p / den * Nm[a - 1];
      }
      if (a <= p - 1) {
        double den = knots[i + p + 1] - knots[i + 1];
        if (den > 0.0) d -= p / den * Nm[a];
      }
      der[a] = d;
    }
  }
  void lagrange(int e, double x, double *val, double *der) const {
    double xi[8];
    for (int k = 0; k <= p; ++k) xi[k] = lo + h * e + h * double(k) / double(p);
    for (int a = 0; a <= p; ++a) {
      double v = 1.0, d = 0.0;
      for (int b = 0; b <= p; ++b)
        if (b != a) v *= (x - xi[b]) / (xi[a] - xi[b]);
      for (int c = 0; c <= p; ++c) {
        if (c == a) continue;
        double t = 1.0 / (xi[a] - xi[c]);
        for (int b = 0; b <= p; ++b)
          if (b != a && b != c) t *= (x - xi[b]) / (xi[a] - xi[b]);
        d += t;
      }
      val[a] = v;
      der[a] = d;
    }
  }
};

// 1D two-scale matrix (coarse n_c -> fine 2 n_c), dense [nc_funcs][nf_funcs]
std::vector<double> two_scale(int basis, int nc, int p, double lo, double hi) {
  Basis1D cb(basis, nc, p, lo, hi), fb(basis, 2 * nc, p, lo, hi);
  const int mc = cb.nfuncs(), mf = fb.nfuncs();
  std::vector<double> R(size_t(mc) * mf, 0.0);
  if (basis == IMSMG_GEN_LAGRANGE) {
    // coarse functions sampled at fine nodes
    for (int k = 0; k < mf; ++k) {
      double x = lo + (hi - lo) * double(k) / double(p * 2 * nc);
      int e = std::min(nc - 1, int(std::floor((x - lo) / cb.h)));
      double v[8], d[8];
      cb.eval(e, x, v, d);
      for (int a = 0; a <= p; ++a) R[size_t(cb.first(e) + a) * mf + k] = v[a];
      // the coarse vertex function at an element boundary is shared with the neighbour
    }
    for (auto &x : R)
      if (std::fabs(x) < 1e-14) x = 0.0;
    return R;
  }
  // Boehm insertion of the coarse-span midpoints, applied to every coarse
  // function (rows of the identity in the coarse basis)
  std::vector<double> t = cb.knots;
  std::vector<std::vector<double>> C(mc, std::vector<double>(mc, 0.0));
  for (int i = 0; i < mc; ++i) C[i][i] = 1.0;
  for (int k = 0; k < nc; ++k) {
    double x = lo + (hi - lo) * double(2 * k + 1) / double(2 * nc);
    int m = int(C[0].size());
    int s = p;
    while (!(t[s] <= x && x < t[s + 1])) ++s;
    for (int i = 0; i < mc; ++i) {
      const std::vector<double> &P = C[i];
      std::vector<double> Q(m + 1, 0.0);
      for (int j = 0; j <= m; ++j) {
        if (j <= s - p) Q[j] = P[j];
        else if (j >= s + 1) Q[j] = P[j - 1];
        else {
          double alpha = (x - t[j]) / (t[j + p] - t[j]);
          Q[j] = alpha * P[j] + (1.0 - alpha) * P[j - 1];
        }
      }
      C[i].swap(Q);
    }
    t.insert(t.begin() + s + 1, x);
  }
  for (int i = 0; i < mc; ++i)
    for (int j = 0; j < mf; ++j) {
      double v = C[i][j];
      R[size_t(i) * mf + j] = std::fabs(v) < 1e-14 ? 0.0 : v;
    }
  return R;
}

// ------------------------------------------------------------- geometry
struct Geometry {
  int kind, dim;
  std::vector<double> discs;
  double phase[3], level, plane_x = 0.0;
  // the apple with a bite (box (-2,2)^3): apple body psi_1 and bite psi_2
  static void apple_parts(const double *x, double &p1, double &p2) {
    const double r = std::sqrt(x[0] * x[0] + x[1] * x[1]);
    const double zz = x[2] / 1.7, rr = r / (1.0 + x[2] / 17.0) - 0.7;
    p1 = 1.0 - zz * zz - rr * rr;
    p2 = (x[0] - 2.0) * (x[0] - 2.0) + x[1] * x[1] + x[2] * x[2] - 1.0;
  }
  double eval(const double *x) const {
    switch (kind) {
      case IMSMG_GEN_GEOM_NONE:
        return 1.0;
      case IMSMG_GEN_GEOM_DISCS: {
        double out = INFINITY;
        for (size_t k = 0; k + 2 < discs.size(); k += 3) {
          double dx = x[0] - discs[k], dy = x[1] - discs[k + 1];
          double d = std::sqrt(dx * dx + dy * dy) - discs[k + 2];
          out = std::min(out, d);
        }
        return out;
      }
      case IMSMG_GEN_GEOM_GYROID: {
        double X = 4.0 * kPi * x[0] + phase[0];
        double Y = 4.0 * kPi * x[1] + phase[1];
        double Z = 4.0 * kPi * x[2] + phase[2];
        double g = std::sin(X) * std::cos(Y) + std::sin(Y) * std::cos(Z) + std::sin(Z) * std::cos(X);
        return level - g;
      }
      case IMSMG_GEN_GEOM_STAR: {
        double th = std::atan2(x[1], x[0]);
        double r = std::sqrt(x[0] * x[0] + x[1] * x[1]);
        return 0.5 + 0.1 * std::sin(5.0 * th) - r;
      }
      case IMSMG_GEN_GEOM_APPLE: {
        double p1, p2;
        apple_parts(x, p1, p2);
        return std::min(p1, p2);
      }
      case IMSMG_GEN_GEOM_SLAB:
        return plane_x - x[0];
    }
    return 0.0;
  }
};

// ------------------------------------------------------------- CSR helpers
struct CSR {
  int32_t nrows = 0, ncols = 0;
  std::vector<int32_t> rowptr, col;
  std::vector<double> val;
  int64_t find(int32_t r, int32_t c) const {
    auto b = col.begin() + rowptr[r], e = col.begin() + rowptr[r + 1];
    auto it = std::lower_bound(b, e, c);
    if (it == e || *it != c) return -1;
    return it - col.begin();
  }
};

struct LevelData {
  int n = 0, depth = 0;
  int nf1 = 0;
  std::vector<uint8_t> active_el;     // n^d
  std::vector<double> eta;            // n^d volume fractions
  std::vector<int64_t> sat;           // summed-area table of active_el, (n+1)^d
  std::vector<int32_t> lat2c;         // lattice -> compact (-1 inactive)
  std::vector<int32_t> c2lat;         // compact -> lattice
  CSR A;
  std::vector<CSR> Ab;                // elasticity: component blocks (ci, cj) at ci * d + cj, values on A's pattern
  CSR R;                              // maps this level -> level-1
  std::vector<int32_t> bptr, bidx, bassoc;
  int n_cut = 0;
};

struct Problem {
  imsmg_gen_spec spec{};
  std::vector<double> discs;
  std::vector<LevelData> lv;
  std::vector<double> b, mass;
  double seconds = 0.0;
};

struct Ctx {
  const imsmg_gen_spec &s;
  int d, p;
  Geometry geo;
  int nleaf;
  std::vector<double> leaf;   // snapped psi on the leaf lattice, x fastest
  Rule1D gc, gs, gb;
  bool want_bnd = false;      // 3D: emit the approximate boundary's triangles
  Ctx(const imsmg_gen_spec &sp) : s(sp), d(sp.dim), p(sp.degree) {}
  size_t leaf_index(const int *L) const {
    size_t idx = 0;
    for (int a = d - 1; a >= 0; --a) idx = idx * size_t(nleaf + 1) + size_t(L[a]);
    return idx;
  }
};

int64_t sat_count(const LevelData &L, int d, const int *lo, const int *hi) {
  // active elements in the box [lo, hi] (inclusive), empty if any lo > hi
  for (int a = 0; a < d; ++a)
    if (lo[a] > hi[a]) return 0;
  const int N = L.n + 1;
  int64_t tot = 0;
  for (int corner = 0; corner < (1 << d); ++corner) {
    size_t idx = 0;
    int sign = 1;
    for (int a = d - 1; a >= 0; --a) {
      int c = (corner >> a) & 1 ? lo[a] : hi[a] + 1;
      if ((corner >> a) & 1) sign = -sign;
      idx = idx * N + c;
    }
    tot += sign * L.sat[idx];
  }
  return tot;
}

void build_sat(LevelData &L, int d) {
  const int n = L.n, N = n + 1;
  size_t tot = 1;
  for (int a = 0; a < d; ++a) tot *= N;
  L.sat.assign(tot, 0);
  if (d == 2) {
    for (int y = 1; y <= n; ++y)
      for (int x = 1; x <= n; ++x)
        L.sat[size_t(y) * N + x] = L.active_el[size_t(y - 1) * n + (x - 1)] + L.sat[size_t(y - 1) * N + x] +
                                   L.sat[size_t(y) * N + x - 1] - L.sat[size_t(y - 1) * N + x - 1];
  } else {
    auto S = [&](int x, int y, int z) -> int64_t & { return L.sat[(size_t(z) * N + y) * N + x]; };
    for (int z = 1; z <= n; ++z)
      for (int y = 1; y <= n; ++y)
        for (int x = 1; x <= n; ++x)
          S(x, y, z) = L.active_el[(size_t(z - 1) * n + (y - 1)) * n + (x - 1)] + S(x - 1, y, z) + S(x, y - 1, z) +
                       S(x, y, z - 1) - S(x - 1, y - 1, z) - S(x - 1, y, z - 1) - S(x, y - 1, z - 1) +
                       S(x - 1, y - 1, z - 1);
  }
}

// ------------------------------------------------------------ quadrature
struct QPoints {
  std::vector<double> x, w;          // volume points (d per point)
  std::vector<double> bx, bw, bn;    // boundary points, weights, normals
  void clear() { x.clear(); w.clear(); bx.clear(); bw.clear(); bn.clear(); }
};

void tensor_points(int d, const double *lo, const double *hi, const Rule1D &g, QPoints &Q) {
  const int q = int(g.x.size());
  double vol = 1.0;
  for (int a = 0; a < d; ++a) vol *= hi[a] - lo[a];
  int cnt = 1;
  for (int a = 0; a < d; ++a) cnt *= q;
  for (int t = 0; t < cnt; ++t) {
    int id[3] = {0, 0, 0}, r = t;
    for (int a = d - 1; a >= 0; --a) { id[a] = r % q; r /= q; }
    double wt = 1.0;
    for (int a = 0; a < d; ++a) {
      Q.x.push_back(lo[a] + (hi[a] - lo[a]) * g.x[id[a]]);
      wt *= g.w[id[a]];
    }
    Q.w.push_back(wt * vol);
  }
}

void tri_points(const double P[3][2], const Rule1D &g, QPoints &Q) {
  double e1[2] = {P[1][0] - P[0][0], P[1][1] - P[0][1]};
  double e2[2] = {P[2][0] - P[1][0], P[2][1] - P[1][1]};
  double J = std::fabs(e1[0] * e2[1] - e1[1] * e2[0]);
  const int q = int(g.x.size());
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) {
      double u = g.x[i], v = g.x[j];
      double xi = u, eta = u * v;
      Q.x.push_back(P[0][0] + xi * e1[0] + eta * e2[0]);
      Q.x.push_back(P[0][1] + xi * e1[1] + eta * e2[1]);
      Q.w.push_back(g.w[i] * g.w[j] * u * J);
    }
}

void tet_points(const double P[4][3], const Rule1D &g, QPoints &Q) {
  double e1[3], e2[3], e3[3];
  for (int a = 0; a < 3; ++a) {
    e1[a] = P[1][a] - P[0][a];
    e2[a] = P[2][a] - P[1][a];
    e3[a] = P[3][a] - P[2][a];
  }
  double det = e1[0] * (e2[1] * e3[2] - e2[2] * e3[1]) - e2[0] * (e1[1] * e3[2] - e1[2] * e3[1]) +
               e3[0] * (e1[1] * e2[2] - e1[2] * e2[1]);
  double J = std::fabs(det);
  const int q = int(g.x.size());
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j)
      for (int k = 0; k < q; ++k) {
        double u = g.x[i], v = g.x[j], s = g.x[k];
        double xi = u, eta = u * v, zeta = u * v * s;
        for (int a = 0; a < 3; ++a) Q.x.push_back(P[0][a] + xi * e1[a] + eta * e2[a] + zeta * e3[a]);
        Q.w.push_back(g.w[i] * g.w[j] * g.w[k] * u * u * v * J);
      }
}

inline void lerp_zero(const double *a, const double *b, double fa, double fb, int d, double *out) {
  double t = fa / (fa - fb);
  for (int k = 0; k < d; ++k) out[k] = a[k] + t * (b[k] - a[k]);
}

void clip_triangle(const double P[3][2], const double f[3], const Ctx &C, QPoints &Q) {
  double poly[4][2];
  int np = 0;
  for (int a = 0; a < 3; ++a) {
    int b = (a + 1) % 3;
    bool pa = f[a] > 0.0, pb = f[b] > 0.0;
    if (pa) { poly[np][0] = P[a][0]; poly[np][1] = P[a][1]; ++np; }
    if (pa != pb) { lerp_zero(P[a], P[b], f[a], f[b], 2, poly[np]); ++np; }
  }
  for (int k = 1; k + 1 < np; ++k) {
    double T[3][2] = {{poly[0][0], poly[0][1]}, {poly[k][0], poly[k][1]}, {poly[k + 1][0], poly[k + 1][1]}};
    tri_points(T, C.gs, Q);
  }
  int npos = (f[0] > 0.0) + (f[1] > 0.0) + (f[2] > 0.0);
  if (npos == 0 || npos == 3) return;
  double cuts[2][2];
  int nc = 0;
  for (int a = 0; a < 3 && nc < 2; ++a) {
    int b = (a + 1) % 3;
    if ((f[a] > 0.0) != (f[b] > 0.0)) { lerp_zero(P[a], P[b], f[a], f[b], 2, cuts[nc]); ++nc; }
  }
  // gradient of the linear interpolant: [P1-P0; P2-P0] g = [f1-f0; f2-f0]
  double m00 = P[1][0] - P[0][0], m01 = P[1][1] - P[0][1];
  double m10 = P[2][0] - P[0][0], m11 = P[2][1] - P[0][1];
  double r0 = f[1] - f[0], r1 = f[2] - f[0];
  double det = m00 * m11 - m01 * m10;
  double gx = (r0 * m11 - m01 * r1) / det;
  double gy = (m00 * r1 - r0 * m10) / det;
  double gn = std::sqrt(gx * gx + gy * gy);
  double nx = -gx / gn, ny = -gy / gn;
  double L = std::sqrt((cuts[1][0] - cuts[0][0]) * (cuts[1][0] - cuts[0][0]) +
                       (cuts[1][1] - cuts[0][1]) * (cuts[1][1] - cuts[0][1]));
  for (size_t i = 0; i < C.gb.x.size(); ++i) {
    double t = C.gb.x[i];
    Q.bx.push_back(cuts[0][0] + t * (cuts[1][0] - cuts[0][0]));
    Q.bx.push_back(cuts[0][1] + t * (cuts[1][1] - cuts[0][1]));
    Q.bw.push_back(C.gb.w[i] * L);
    Q.bn.push_back(nx);
    Q.bn.push_back(ny);
  }
}

void wedge_tets(const double *A, const double *B, const double *Cc, const double *A2, const double *B2,
                const double *C2, const Ctx &C, QPoints &Q) {
  const double *T[3][4] = {{A, B, Cc, A2}, {B, Cc, A2, B2}, {Cc, A2, B2, C2}};
  for (int t = 0; t < 3; ++t) {
    double P[4][3];
    for (int v = 0; v < 4; ++v)
      for (int a = 0; a < 3; ++a) P[v][a] = T[t][v][a];
    tet_points(P, C.gs, Q);
  }
}

// Gauss points of a triangle of the approximate boundary (3D): collapsed
// rule x = T0 + u (T1 - T0) + u v (T2 - T1), area measure, outward normal nn.
void surface_points(const double *T0, const double *T1, const double *T2, const double *nn, const Rule1D &g,
                    QPoints &Q) {
  double e1[3], e2[3];
  for (int a = 0; a < 3; ++a) {
    e1[a] = T1[a] - T0[a];
    e2[a] = T2[a] - T1[a];
  }
  const double cx = e1[1] * e2[2] - e1[2] * e2[1];
  const double cy = e1[2] * e2[0] - e1[0] * e2[2];
  const double cz = e1[0] * e2[1] - e1[1] * e2[0];
  const double J = std::sqrt(cx * cx + cy * cy + cz * cz);
  const int q = int(g.x.size());
  for (int i = 0; i < q; ++i)
    for (int j = 0; j < q; ++j) {
      const double u = g.x[i], uv = g.x[i] * g.x[j];
      for (int a = 0; a < 3; ++a) {
        Q.bx.push_back(T0[a] + u * e1[a] + uv * e2[a]);
        Q.bn.push_back(nn[a]);
      }
      Q.bw.push_back(g.w[i] * g.w[j] * u * J);
    }
}

void clip_tet(const double P[4][3], const double f[4], const Ctx &C, QPoints &Q) {
  int pos[4], neg[4], npos = 0, nneg = 0;
  for (int a = 0; a < 4; ++a) {
    if (f[a] > 0.0) pos[npos++] = a;
    else neg[nneg++] = a;
  }
  auto I = [&](int a, int b, double *out) { lerp_zero(P[a], P[b], f[a], f[b], 3, out); };
  if (npos == 0) return;
  if (npos == 4) { tet_points(P, C.gs, Q); return; }
  // outward normal of the zero set: -grad f / |grad f|, grad f from the
  // edges P_k - P_0 (Cramer's rule)
  double nn[3] = {0.0, 0.0, 0.0};
  if (C.want_bnd) {
    double M[3][3], r[3];
    for (int k = 0; k < 3; ++k) {
      for (int a = 0; a < 3; ++a) M[k][a] = P[k + 1][a] - P[0][a];
      r[k] = f[k + 1] - f[0];
    }
    auto det3 = [](const double A[3][3]) {
      return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1]) - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0]) +
             A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    };
    const double D = det3(M);
    double g[3];
    for (int a = 0; a < 3; ++a) {
      double Ma[3][3];
      for (int k = 0; k < 3; ++k)
        for (int b = 0; b < 3; ++b) Ma[k][b] = (b == a) ? r[k] : M[k][b];
      g[a] = det3(Ma) / D;
    }
    const double gn = std::sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
    for (int a = 0; a < 3; ++a) nn[a] = -g[a] / gn;
  }
  if (npos == 1) {
    int a = pos[0];
    double T[4][3];
    for (int k = 0; k < 3; ++k) T[0][k] = P[a][k];
    I(a, neg[0], T[1]);
    I(a, neg[1], T[2]);
    I(a, neg[2], T[3]);
    tet_points(T, C.gs, Q);
    if (C.want_bnd) surface_points(T[1], T[2], T[3], nn, C.gb, Q);
    return;
  }
  if (npos == 3) {
    int a = pos[0], b = pos[1], c = pos[2], dd = neg[0];
    double Ad[3], Bd[3], Cd[3];
    I(a, dd, Ad);
    I(b, dd, Bd);
    I(c, dd, Cd);
    wedge_tets(P[a], P[b], P[c], Ad, Bd, Cd, C, Q);
    if (C.want_bnd) surface_points(Ad, Bd, Cd, nn, C.gb, Q);
    return;
  }
  int a = pos[0], b = pos[1], c = neg[0], dd = neg[1];
  double Iac[3], Iad[3], Ibc[3], Ibd[3];
  I(a, c, Iac);
  I(a, dd, Iad);
  I(b, c, Ibc);
  I(b, dd, Ibd);
  wedge_tets(P[a], Iac, Iad, P[b], Ibc, Ibd, C, Q);
  // the quadrilateral zero set, split along Iac - Ibd
  if (C.want_bnd) {
    surface_points(Iac, Iad, Ibd, nn, C.gb, Q);
    surface_points(Iac, Ibd, Ibc, nn, C.gb, Q);
  }
}

// Quadrature of one element on a level of size h whose cells are bisected `depth` times.
void element_quadrature(const Ctx &C, const int *e, int depth, double h, QPoints &Q) {
  const int d = C.d;
  const int s = 1 << depth;
  const double hl = h / s;
  const double lo = C.s.box_lo;
  struct Frame { int o[3]; int size; };
  Frame root{{e[0] * s, e[1] * s, d == 3 ? e[2] * s : 0}, s};
  // depth-first; the child order only changes the summation order
  std::function<void(const Frame &)> rec;
  rec = [&](const Frame &F) {
    int cnt = 0, tot = 0;
    int hiN = F.size;
    if (d == 2) {
      for (int j = 0; j <= hiN; ++j)
        for (int i = 0; i <= hiN; ++i) {
          int L[3] = {F.o[0] + i, F.o[1] + j, 0};
          cnt += C.leaf[C.leaf_index(L)] > 0.0;
          ++tot;
        }
    } else {
      for (int k = 0; k <= hiN; ++k)
        for (int j = 0; j <= hiN; ++j)
          for (int i = 0; i <= hiN; ++i) {
            int L[3] = {F.o[0] + i, F.o[1] + j, F.o[2] + k};
            cnt += C.leaf[C.leaf_index(L)] > 0.0;
            ++tot;
          }
    }
    if (cnt == 0) return;
    if (cnt == tot) {
      double clo[3], chi[3];
      for (int a = 0; a < d; ++a) {
        clo[a] = lo + hl * F.o[a];
        chi[a] = lo + hl * (F.o[a] + F.size);
      }
      tensor_points(d, clo, chi, C.gc, Q);
      return;
    }
    if (F.size > 1) {
      int half = F.size / 2;
      for (int c = 0; c < (1 << d); ++c) {
        Frame ch;
        ch.size = half;
        ch.o[2] = 0;
        for (int a = 0; a < d; ++a) {
          int bit = (c >> (d - 1 - a)) & 1;  // first axis slowest
          ch.o[a] = F.o[a] + half * bit;
        }
        rec(ch);
      }
      return;
    }
    auto corner = [&](const int *L, double *x) {
      for (int a = 0; a < d; ++a) x[a] = lo + hl * L[a];
    };
    if (d == 2) {
      static const int tris[2][3][2] = {{{0, 0}, {1, 0}, {1, 1}}, {{0, 0}, {1, 1}, {0, 1}}};
      for (int t = 0; t < 2; ++t) {
        double P[3][2], f[3];
        for (int v = 0; v < 3; ++v) {
          int L[3] = {F.o[0] + tris[t][v][0], F.o[1] + tris[t][v][1], 0};
          corner(L, P[v]);
          f[v] = C.leaf[C.leaf_index(L)];
        }
        clip_triangle(P, f, C, Q);
      }
    } else {
      static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
      for (int t = 0; t < 6; ++t) {
        double P[4][3], f[4];
        int L[3] = {F.o[0], F.o[1], F.o[2]};
        corner(L, P[0]);
        f[0] = C.leaf[C.leaf_index(L)];
        for (int v = 0; v < 3; ++v) {
          L[perms[t][v]] += 1;
          corner(L, P[v + 1]);
          f[v + 1] = C.leaf[C.leaf_index(L)];
        }
        clip_tet(P, f, C, Q);
      }
    }
  };
  rec(root);
}


// --------------------------------------------------------------- stencils
struct Stencil {
  int d, p, K, W;  // K = (2p+1)^d slots, W = 2p+1
  explicit Stencil(int d_, int p_) : d(d_), p(p_) {
    W = 2 * p + 1;
    K = 1;
    for (int a = 0; a < d; ++a) K *= W;
  }
  // slot of lattice offset (dx, dy, dz), each in [-p, p]; x fastest
  int slot(const int *off) const {
    int s = 0;
    for (int a = d - 1; a >= 0; --a) s = s * W + (off[a] + p);
    return s;
  }
  void offset(int s, int *off) const {
    for (int a = 0; a < d; ++a) { off[a] = s % W - p; s /= W; }
  }
};

void lat_multi(int64_t L, int nf, int d, int *m) {
  for (int a = 0; a < d; ++a) { m[a] = int(L % nf); L /= nf; }
}
int64_t multi_lat(const int *m, int nf, int d) {
  int64_t L = 0;
  for (int a = d - 1; a >= 0; --a) L = L * nf + m[a];
  return L;
}

// Active functions of a level from its active elements (support boxes via SAT).
void activate_functions(LevelData &L, const Basis1D &B, int d, bool strong_box) {
  const int nf = B.nfuncs();
  L.nf1 = nf;
  int64_t tot = 1;
  for (int a = 0; a < d; ++a) tot *= nf;
  L.lat2c.assign(size_t(tot), -1);
  L.c2lat.clear();
  for (int64_t Lx = 0; Lx < tot; ++Lx) {
    int m[3] = {0, 0, 0}, lo[3], hi[3];
    lat_multi(Lx, nf, d, m);
    bool dir = false;
    for (int a = 0; a < d; ++a) {
      B.support(m[a], lo[a], hi[a]);
      if (m[a] == 0 || m[a] == nf - 1) dir = true;
    }
    if (strong_box && dir) continue;
    if (sat_count(L, d, lo, hi) > 0) {
      L.lat2c[size_t(Lx)] = int32_t(L.c2lat.size());
      L.c2lat.push_back(int32_t(Lx));
    }
  }
}

// Structural pattern: active i, j (lattice offset within +-p) sharing an active element.
void build_pattern(LevelData &L, const Basis1D &B, int d, const Stencil &st) {
  const int n = int(L.c2lat.size());
  const int nf = L.nf1;
  std::vector<std::vector<int32_t>> cols(n);
#pragma omp parallel for schedule(dynamic, 256)
  for (int i = 0; i < n; ++i) {
    int mi[3] = {0, 0, 0};
    lat_multi(L.c2lat[i], nf, d, mi);
    int ilo[3], ihi[3];
    for (int a = 0; a < d; ++a) B.support(mi[a], ilo[a], ihi[a]);
    for (int s = 0; s < st.K; ++s) {
      int off[3] = {0, 0, 0}, mj[3] = {0, 0, 0};
      st.offset(s, off);
      bool ok = true;
      for (int a = 0; a < d; ++a) {
        mj[a] = mi[a] + off[a];
        if (mj[a] < 0 || mj[a] >= nf) ok = false;
      }
      if (!ok) continue;
      int32_t j = L.lat2c[size_t(multi_lat(mj, nf, d))];
      if (j < 0) continue;
      int lo[3], hi[3];
      for (int a = 0; a < d; ++a) {
        int jlo, jhi;
        B.support(mj[a], jlo, jhi);
        lo[a] = std::max(ilo[a], jlo);
        hi[a] = std::min(ihi[a], jhi);
      }
      if (sat_count(L, d, lo, hi) > 0) cols[i].push_back(j);
    }
  }
  L.A.nrows = L.A.ncols = n;
  L.A.rowptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) L.A.rowptr[i + 1] = L.A.rowptr[i] + int32_t(cols[i].size());
  L.A.col.resize(L.A.rowptr[n]);
  for (int i = 0; i < n; ++i) std::copy(cols[i].begin(), cols[i].end(), L.A.col.begin() + L.A.rowptr[i]);
  L.A.val.assign(L.A.col.size(), 0.0);
}

struct Elem1D {
  // per element index: (p+1)x(p+1) stiffness, mass and first-derivative
  // matrices (D_ab = int phi_a' phi_b), (p+1) loads of 1 and sin(2 pi x)
  std::vector<double> S, M, D, F1, Fs;
};

Elem1D element_1d(const Basis1D &B, const Rule1D &g) {
  const int p = B.p, m = p + 1;
  Elem1D E;
  E.S.assign(size_t(B.n) * m * m, 0.0);
  E.M.assign(size_t(B.n) * m * m, 0.0);
  E.D.assign(size_t(B.n) * m * m, 0.0);
  E.F1.assign(size_t(B.n) * m, 0.0);
  E.Fs.assign(size_t(B.n) * m, 0.0);
  for (int e = 0; e < B.n; ++e) {
    double xl = B.lo + B.h * e, xr = B.lo + B.h * (e + 1);
    for (size_t q = 0; q < g.x.size(); ++q) {
      double x = xl + (xr - xl) * g.x[q];
      double w = g.w[q] * (xr - xl);
      double v[8], dv[8];
      B.eval(e, x, v, dv);
      double sn = std::sin(2.0 * kPi * x);
      for (int a = 0; a < m; ++a) {
        E.F1[size_t(e) * m + a] += w * v[a];
        E.Fs[size_t(e) * m + a] += w * sn * v[a];
        for (int b = 0; b < m; ++b) {
          E.S[(size_t(e) * m + a) * m + b] += w * dv[a] * dv[b];
          E.M[(size_t(e) * m + a) * m + b] += w * v[a] * v[b];
          E.D[(size_t(e) * m + a) * m + b] += w * dv[a] * v[b];
        }
      }
    }
  }
  return E;
}

// Fine-level assembly into the structural CSR of level L.
void assemble_fine(Ctx &C, Problem &P, LevelData &L, const Basis1D &B) {
  const int d = C.d, p = C.p, m = p + 1;
  int nloc = 1;
  for (int a = 0; a < d; ++a) nloc *= m;
  const int n = L.n;
  const double h = B.h;
  const bool penalty = C.s.bc == IMSMG_GEN_PENALTY;
  const double beta = penalty ? C.s.penalty_factor / h : 0.0;
  const int rhs = C.s.rhs;
  const bool neumann_data = rhs == IMSMG_GEN_RHS_MANUFACTURED && C.s.bc == IMSMG_GEN_BOX_DIRICHLET;
  const double fscale = d * (2.0 * kPi) * (2.0 * kPi);
  const Elem1D E = element_1d(B, C.gc);
  const int nrows = int(L.c2lat.size());
  P.b.assign(nrows, 0.0);
  if (C.s.with_mass) P.mass.assign(L.A.val.size(), 0.0);
  L.eta.assign(L.active_el.size(), 0.0);
  const int stride = B.basis == IMSMG_GEN_BSPLINE ? m : 2;  // elements this far apart share no function
  int ncolors = 1;
  for (int a = 0; a < d; ++a) ncolors *= stride;
  int ncut = 0;
  for (int color = 0; color < ncolors; ++color) {
    int cc[3] = {0, 0, 0}, r = color;
    for (int a = 0; a < d; ++a) { cc[a] = r % stride; r /= stride; }
    int cnt[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a) cnt[a] = (n - cc[a] + stride - 1) / stride;
    const int64_t total = int64_t(cnt[0]) * cnt[1] * cnt[2];
#pragma omp parallel reduction(+ : ncut)
    {
      std::vector<double> K(size_t(nloc) * nloc), Ml(size_t(nloc) * nloc), fb(nloc);
      std::vector<double> vals, ders;
      QPoints Q;
#pragma omp for schedule(dynamic, 64)
      for (int64_t t = 0; t < total; ++t) {
        int e[3] = {0, 0, 0};
        int64_t rr = t;
        for (int a = 0; a < d; ++a) { e[a] = cc[a] + stride * int(rr % cnt[a]); rr /= cnt[a]; }
        const size_t el = size_t(multi_lat(e, n, d));
        if (!L.active_el[el]) continue;
        // leaf-vertex count of this element decides inside / cut
        const int s = 1 << L.depth;
        int L0[3] = {e[0] * s, e[1] * s, d == 3 ? e[2] * s : 0};
        bool all_pos = true;
        for (int k = 0; k <= (d == 3 ? s : 0) && all_pos; ++k)
          for (int j = 0; j <= s && all_pos; ++j)
            for (int i = 0; i <= s; ++i) {
              int LL[3] = {L0[0] + i, L0[1] + j, L0[2] + k};
              if (!(C.leaf[C.leaf_index(LL)] > 0.0)) { all_pos = false; break; }
            }
        std::fill(K.begin(), K.end(), 0.0);
        std::fill(Ml.begin(), Ml.end(), 0.0);
        std::fill(fb.begin(), fb.end(), 0.0);
        if (all_pos) {
          // tensor products of 1D element matrices (same Gauss rule per axis)
          L.eta[el] = 1.0;
          for (int A = 0; A < nloc; ++A) {
            int oa[3] = {0, 0, 0}, ra = A;
            for (int a = 0; a < d; ++a) { oa[a] = ra % m; ra /= m; }
            double f1 = 1.0, fs = 1.0;
            for (int a = 0; a < d; ++a) {
              f1 *= E.F1[size_t(e[a]) * m + oa[a]];
              fs *= E.Fs[size_t(e[a]) * m + oa[a]];
            }
            if (rhs == IMSMG_GEN_RHS_ONE) fb[A] = f1;
            else if (rhs == IMSMG_GEN_RHS_MANUFACTURED) fb[A] = fscale * fs;
            for (int Bi = A; Bi < nloc; ++Bi) {
              int ob[3] = {0, 0, 0}, rb = Bi;
              for (int a = 0; a < d; ++a) { ob[a] = rb % m; rb /= m; }
              double kv = 0.0, mv = 1.0;
              for (int c = 0; c < d; ++c) {
                double t2 = 1.0;
                for (int a = 0; a < d; ++a) {
                  const std::vector<double> &T = (a == c) ? E.S : E.M;
                  t2 *= T[(size_t(e[a]) * m + oa[a]) * m + ob[a]];
                }
                kv += t2;
              }
              for (int a = 0; a < d; ++a) mv *= E.M[(size_t(e[a]) * m + oa[a]) * m + ob[a]];
              K[size_t(A) * nloc + Bi] = kv;
              Ml[size_t(A) * nloc + Bi] = mv;
            }
          }
        } else {
          ++ncut;
          Q.clear();
          element_quadrature(C, e, L.depth, h, Q);
          const size_t nq = Q.w.size();
          double vol = 0.0;
          vals.resize(size_t(d) * m);
          ders.resize(size_t(d) * m);
          std::vector<double> phi(nloc), grad(size_t(nloc) * d);
          for (size_t q = 0; q < nq; ++q) {
            const double *x = &Q.x[q * d];
            const double w = Q.w[q];
            vol += w;
            for (int a = 0; a < d; ++a) B.eval(e[a], x[a], &vals[size_t(a) * m], &ders[size_t(a) * m]);
            for (int A = 0; A < nloc; ++A) {
              int oa[3] = {0, 0, 0}, ra = A;
              for (int a = 0; a < d; ++a) { oa[a] = ra % m; ra /= m; }
              double v = 1.0;
              for (int a = 0; a < d; ++a) v *= vals[size_t(a) * m + oa[a]];
              phi[A] = v;
              for (int c = 0; c < d; ++c) {
                double g = 1.0;
                for (int a = 0; a < d; ++a) g *= (a == c) ? ders[size_t(a) * m + oa[a]] : vals[size_t(a) * m + oa[a]];
                grad[size_t(A) * d + c] = g;
              }
            }
            double f = 0.0;
            if (rhs == IMSMG_GEN_RHS_ONE) f = 1.0;
            else if (rhs == IMSMG_GEN_RHS_MANUFACTURED) {
              double u = 1.0;
              for (int a = 0; a < d; ++a) u *= std::sin(2.0 * kPi * x[a]);
              f = fscale * u;
            }
            for (int A = 0; A < nloc; ++A) {
              fb[A] += w * f * phi[A];
              for (int Bi = A; Bi < nloc; ++Bi) {
                double g = 0.0;
                for (int c = 0; c < d; ++c) g += grad[size_t(A) * d + c] * grad[size_t(Bi) * d + c];
                K[size_t(A) * nloc + Bi] += w * g;
                Ml[size_t(A) * nloc + Bi] += w * phi[A] * phi[Bi];
              }
            }
          }
          L.eta[el] = vol / std::pow(h, d);
          // boundary terms (2D approximate boundary)
          const size_t nb = Q.bw.size();
          for (size_t q = 0; q < nb; ++q) {
            const double *x = &Q.bx[q * d];
            const double *nn = &Q.bn[q * d];
            const double w = Q.bw[q];
            for (int a = 0; a < d; ++a) B.eval(e[a], x[a], &vals[size_t(a) * m], &ders[size_t(a) * m]);
            for (int A = 0; A < nloc; ++A) {
              int oa[3] = {0, 0, 0}, ra = A;
              for (int a = 0; a < d; ++a) { oa[a] = ra % m; ra /= m; }
              double v = 1.0;
              for (int a = 0; a < d; ++a) v *= vals[size_t(a) * m + oa[a]];
              phi[A] = v;
            }
            double g = 0.0;
            if (neumann_data) {
              for (int a = 0; a < d; ++a) {
                double t2 = 2.0 * kPi * std::cos(2.0 * kPi * x[a]);
                for (int b2 = 0; b2 < d; ++b2)
                  if (b2 != a) t2 *= std::sin(2.0 * kPi * x[b2]);
                g += t2 * nn[a];
              }
            }
            for (int A = 0; A < nloc; ++A) {
              fb[A] += w * g * phi[A];
              if (penalty)
                for (int Bi = A; Bi < nloc; ++Bi) K[size_t(A) * nloc + Bi] += beta * w * phi[A] * phi[Bi];
            }
          }
        }
        // scatter (upper triangle mirrored) into the structural CSR
        int32_t loc[64 * 8];
        for (int A = 0; A < nloc; ++A) {
          int oa[3] = {0, 0, 0}, ra = A, mf[3] = {0, 0, 0};
          for (int a = 0; a < d; ++a) { oa[a] = ra % m; ra /= m; mf[a] = B.first(e[a]) + oa[a]; }
          loc[A] = L.lat2c[size_t(multi_lat(mf, L.nf1, d))];
        }
        for (int A = 0; A < nloc; ++A) {
          if (loc[A] < 0) continue;
          P.b[loc[A]] += fb[A];
          for (int Bi = 0; Bi < nloc; ++Bi) {
            if (loc[Bi] < 0) continue;
            const int lo_ = std::min(A, Bi), hi_ = std::max(A, Bi);
            int64_t pos = L.A.find(loc[A], loc[Bi]);
            if (pos < 0) throw GenError(-1, "assembly entry outside the structural pattern");
            L.A.val[pos] += K[size_t(lo_) * nloc + hi_];
            if (C.s.with_mass) P.mass[pos] += Ml[size_t(lo_) * nloc + hi_];
          }
        }
      }
    }
  }
  L.n_cut = ncut;
}

// Fine-level assembly of linear elasticity (eq:operatorsMulti) into the
// component blocks L.Ab (values on the scalar structural pattern):
//   K[(a,c),(b,e)] = lambda d_c phi_a d_e phi_b
//                    + mu (delta_ce grad phi_a . grad phi_b + d_e phi_a d_c phi_b)
// plus, on boundary points of the Dirichlet part, lambda beta phi_a phi_b n_c n_e
// + 2 mu beta delta_ce phi_a phi_b (homogeneous data: no load from it), and
// the load f_c int phi_a.  Inside elements take tensor products of the 1D
// matrices S (d/dx on both), D (d/dx on the first function) and M.  Only the
// blocks c <= e are computed (c = e: a <= b) and mirrored, so the operator is
// exactly symmetric.
void assemble_fine_elasticity(Ctx &C, Problem &P, LevelData &L, const Basis1D &B) {
  const int d = C.d, p = C.p, m = p + 1;
  int nloc = 1;
  for (int a = 0; a < d; ++a) nloc *= m;
  const int n = L.n;
  const double h = B.h;
  const double lam = C.s.lame_lambda, mu = C.s.lame_mu;
  const bool penalty = C.s.bc == IMSMG_GEN_PENALTY;
  const double beta = penalty ? C.s.penalty_factor / h : 0.0;
  const bool bite = C.s.dirichlet_part == IMSMG_GEN_DIRICHLET_BITE;
  const Elem1D E = element_1d(B, C.gc);
  const int nrows = int(L.c2lat.size());
  const size_t nb = size_t(d) * d;
  L.Ab.assign(nb, CSR());
  for (size_t k = 0; k < nb; ++k) L.Ab[k].val.assign(L.A.col.size(), 0.0);
  P.b.assign(size_t(d) * nrows, 0.0);
  if (C.s.with_mass) P.mass.assign(L.A.val.size(), 0.0);
  L.eta.assign(L.active_el.size(), 0.0);
  const int stride = B.basis == IMSMG_GEN_BSPLINE ? m : 2;
  int ncolors = 1;
  for (int a = 0; a < d; ++a) ncolors *= stride;
  int ncut = 0;
  const size_t nl2 = size_t(nloc) * nloc;
  for (int color = 0; color < ncolors; ++color) {
    int cc[3] = {0, 0, 0}, r = color;
    for (int a = 0; a < d; ++a) { cc[a] = r % stride; r /= stride; }
    int cnt[3] = {1, 1, 1};
    for (int a = 0; a < d; ++a) cnt[a] = (n - cc[a] + stride - 1) / stride;
    const int64_t total = int64_t(cnt[0]) * cnt[1] * cnt[2];
#pragma omp parallel reduction(+ : ncut)
    {
      // T[c][e] = int d_c phi_a d_e phi_b (all a, b); K blocks; mass; loads
      std::vector<double> T(nb * nl2), K(nb * nl2), Ml(nl2), fb(size_t(d) * nloc), F1(nloc);
      std::vector<double> vals, ders, phi(nloc), grad(size_t(nloc) * d), gradT(size_t(nloc) * d);
      QPoints Q;
#pragma omp for schedule(dynamic, 64)
      for (int64_t t = 0; t < total; ++t) {
        int e[3] = {0, 0, 0};
        int64_t rr = t;
        for (int a = 0; a < d; ++a) { e[a] = cc[a] + stride * int(rr % cnt[a]); rr /= cnt[a]; }
        const size_t el = size_t(multi_lat(e, n, d));
        if (!L.active_el[el]) continue;
        const int sd = 1 << L.depth;
        int L0[3] = {e[0] * sd, e[1] * sd, d == 3 ? e[2] * sd : 0};
        bool all_pos = true;
        for (int k = 0; k <= (d == 3 ? sd : 0) && all_pos; ++k)
          for (int j = 0; j <= sd && all_pos; ++j)
            for (int i = 0; i <= sd; ++i) {
              int LL[3] = {L0[0] + i, L0[1] + j, L0[2] + k};
              if (!(C.leaf[C.leaf_index(LL)] > 0.0)) { all_pos = false; break; }
            }
        std::fill(T.begin(), T.end(), 0.0);
        std::fill(Ml.begin(), Ml.end(), 0.0);
        std::fill(F1.begin(), F1.end(), 0.0);
        std::fill(K.begin(), K.end(), 0.0);
        if (all_pos) {
          L.eta[el] = 1.0;
          for (int A = 0; A < nloc; ++A) {
            int oa[3] = {0, 0, 0}, ra = A;
            for (int a = 0; a < d; ++a) { oa[a] = ra % m; ra /= m; }
            double f1 = 1.0;
            for (int a = 0; a < d; ++a) f1 *= E.F1[size_t(e[a]) * m + oa[a]];
            F1[A] = f1;
            for (int Bi = 0; Bi < nloc; ++Bi) {
              int ob[3] = {0, 0, 0}, rb = Bi;
              for (int a = 0; a < d; ++a) { ob[a] = rb % m; rb /= m; }
              double mv = 1.0;
              for (int a = 0; a < d; ++a) mv *= E.M[(size_t(e[a]) * m + oa[a]) * m + ob[a]];
              Ml[size_t(A) * nloc + Bi] = mv;
              for (int c = 0; c < d; ++c)
                for (int ee = 0; ee < d; ++ee) {
                  double tv = 1.0;
                  for (int a = 0; a < d; ++a) {
                    const size_t eab = (size_t(e[a]) * m + oa[a]) * m + ob[a];
                    const size_t eba = (size_t(e[a]) * m + ob[a]) * m + oa[a];
                    if (a == c && a == ee) tv *= E.S[eab];
                    else if (a == c) tv *= E.D[eab];   // d/dx on phi_a
                    else if (a == ee) tv *= E.D[eba];  // d/dx on phi_b
                    else tv *= E.M[eab];
                  }
                  T[(size_t(c) * d + ee) * nl2 + size_t(A) * nloc + Bi] = tv;
                }
            }
          }
        } else {
          ++ncut;
          Q.clear();
          element_quadrature(C, e, L.depth, h, Q);
          const size_t nq = Q.w.size();
          double vol = 0.0;
          vals.resize(size_t(d) * m);
          ders.resize(size_t(d) * m);
          for (size_t q = 0; q < nq; ++q) {
            const double *x = &Q.x[q * d];
            const double w = Q.w[q];
            vol += w;
            for (int a = 0; a < d; ++a) B.eval(e[a], x[a], &vals[size_t(a) * m], &ders[size_t(a) * m]);
            for (int A = 0; A < nloc; ++A) {
              int oa[3] = {0, 0, 0}, ra = A;
              for (int a = 0; a < d; ++a) { oa[a] = ra % m; ra /= m; }
              double v = 1.0;
              for (int a = 0; a < d; ++a) v *= vals[size_t(a) * m + oa[a]];
              phi[A] = v;
              for (int c = 0; c < d; ++c) {
                double g = 1.0;
                for (int a = 0; a < d; ++a) g *= (a == c) ? ders[size_t(a) * m + oa[a]] : vals[size_t(a) * m + oa[a]];
                grad[size_t(A) * d + c] = g;
              }
            }
            // gradients component-major (contiguous over the local functions)
            for (int A = 0; A < nloc; ++A)
              for (int c = 0; c < d; ++c) gradT[size_t(c) * nloc + A] = grad[size_t(A) * d + c];
            for (int A = 0; A < nloc; ++A) {
              F1[A] += w * phi[A];
              if (C.s.with_mass) {
                const double wa = w * phi[A];
                double *row = &Ml[size_t(A) * nloc];
                for (int Bi = 0; Bi < nloc; ++Bi) row[Bi] += wa * phi[Bi];
              }
            }
            // T[c][e] for c <= e only (T[e][c]_ab = T[c][e]_ba)
            for (int c = 0; c < d; ++c)
              for (int ee = c; ee < d; ++ee) {
                const double *ge = &gradT[size_t(ee) * nloc];
                double *Tc = &T[(size_t(c) * d + ee) * nl2];
                for (int A = 0; A < nloc; ++A) {
                  const double wa = w * gradT[size_t(c) * nloc + A];
                  double *row = Tc + size_t(A) * nloc;
                  for (int Bi = 0; Bi < nloc; ++Bi) row[Bi] += wa * ge[Bi];
                }
              }
          }
          for (int c = 0; c < d; ++c)
            for (int ee = 0; ee < c; ++ee)
              for (int A = 0; A < nloc; ++A)
                for (int Bi = 0; Bi < nloc; ++Bi)
                  T[(size_t(c) * d + ee) * nl2 + size_t(A) * nloc + Bi] =
                      T[(size_t(ee) * d + c) * nl2 + size_t(Bi) * nloc + A];
          L.eta[el] = vol / std::pow(h, d);
          // penalty on the Dirichlet part of the approximate boundary
          const size_t nbq = Q.bw.size();
          if (penalty) {
            for (size_t q = 0; q < nbq; ++q) {
              const double *x = &Q.bx[q * d];
              const double *nn = &Q.bn[q * d];
              if (bite) {
                double p1, p2;
                Geometry::apple_parts(x, p1, p2);
                if (!(p2 <= p1)) continue;
              }
              const double w = Q.bw[q];
              for (int a = 0; a < d; ++a) B.eval(e[a], x[a], &vals[size_t(a) * m], &ders[size_t(a) * m]);
              for (int A = 0; A < nloc; ++A) {
                int oa[3] = {0, 0, 0}, ra = A;
                for (int a = 0; a < d; ++a) { oa[a] = ra % m; ra /= m; }
                double v = 1.0;
                for (int a = 0; a < d; ++a) v *= vals[size_t(a) * m + oa[a]];
                phi[A] = v;
              }
              for (int A = 0; A < nloc; ++A)
                for (int Bi = 0; Bi < nloc; ++Bi) {
                  const double pp = w * phi[A] * phi[Bi];
                  for (int c = 0; c < d; ++c)
                    for (int ee = 0; ee < d; ++ee) {
                      double kv = lam * beta * pp * nn[c] * nn[ee];
                      if (c == ee) kv += 2.0 * mu * beta * pp;
                      K[(size_t(c) * d + ee) * nl2 + size_t(A) * nloc + Bi] += kv;
                    }
                }
            }
          }
        }
        // K += lambda T[c][e] + mu T[e][c]^T-entry + mu delta_ce sum_g T[g][g]
        for (int c = 0; c < d; ++c)
          for (int ee = 0; ee < d; ++ee)
            for (int A = 0; A < nloc; ++A)
              for (int Bi = 0; Bi < nloc; ++Bi) {
                const size_t ab = size_t(A) * nloc + Bi;
                double kv = lam * T[(size_t(c) * d + ee) * nl2 + ab] + mu * T[(size_t(ee) * d + c) * nl2 + ab];
                if (c == ee) {
                  double lap = 0.0;
                  for (int g = 0; g < d; ++g) lap += T[(size_t(g) * d + g) * nl2 + ab];
                  kv += mu * lap;
                }
                K[(size_t(c) * d + ee) * nl2 + ab] += kv;
              }
        for (int c = 0; c < d; ++c)
          for (int A = 0; A < nloc; ++A) fb[size_t(c) * nloc + A] = C.s.force[c] * F1[A];
        // scatter the blocks c <= e (c = e: a <= b) and their mirror images
        int32_t loc[64 * 8];
        for (int A = 0; A < nloc; ++A) {
          int oa[3] = {0, 0, 0}, ra = A, mf[3] = {0, 0, 0};
          for (int a = 0; a < d; ++a) { oa[a] = ra % m; ra /= m; mf[a] = B.first(e[a]) + oa[a]; }
          loc[A] = L.lat2c[size_t(multi_lat(mf, L.nf1, d))];
        }
        for (int A = 0; A < nloc; ++A) {
          if (loc[A] < 0) continue;
          for (int c = 0; c < d; ++c) P.b[size_t(c) * nrows + loc[A]] += fb[size_t(c) * nloc + A];
          for (int Bi = 0; Bi < nloc; ++Bi) {
            if (loc[Bi] < 0) continue;
            const int64_t pos = L.A.find(loc[A], loc[Bi]);
            if (pos < 0) throw GenError(-1, "assembly entry outside the structural pattern");
            const int lo_ = std::min(A, Bi), hi_ = std::max(A, Bi);
            if (C.s.with_mass) P.mass[pos] += Ml[size_t(lo_) * nloc + hi_];
            for (int c = 0; c < d; ++c)
              for (int ee = 0; ee < d; ++ee) {
                // entry (A c, Bi ee) = canonical (c <= ee) block value
                double kv;
                if (c < ee) kv = K[(size_t(c) * d + ee) * nl2 + size_t(A) * nloc + Bi];
                else if (c > ee) kv = K[(size_t(ee) * d + c) * nl2 + size_t(Bi) * nloc + A];
                else kv = K[(size_t(c) * d + c) * nl2 + size_t(lo_) * nloc + hi_];
                L.Ab[size_t(c) * d + ee].val[pos] += kv;
              }
          }
        }
      }
    }
  }
  L.n_cut = ncut;
  L.A.val = L.Ab[0].val;
}

// Masked tensor two-scale restriction: rows = coarse active, cols = fine active.
void build_restriction(const LevelData &Lc, LevelData &Lf, int d, int basis, int p, double lo, double hi) {
  const int nc = Lc.n;
  std::vector<double> R1 = two_scale(basis, nc, p, lo, hi);
  const int mc = Lc.nf1, mf = Lf.nf1;
  // per coarse 1D index: list of (fine index, value)
  std::vector<std::vector<std::pair<int, double>>> rows(mc);
  for (int i = 0; i < mc; ++i)
    for (int k = 0; k < mf; ++k)
      if (R1[size_t(i) * mf + k] != 0.0) rows[i].push_back({k, R1[size_t(i) * mf + k]});
  const int n = int(Lc.c2lat.size());
  std::vector<std::vector<std::pair<int32_t, double>>> out(n);
#pragma omp parallel for schedule(dynamic, 256)
  for (int i = 0; i < n; ++i) {
    int mi[3] = {0, 0, 0};
    lat_multi(Lc.c2lat[i], mc, d, mi);
    const auto &rx = rows[mi[0]];
    const auto &ry = rows[mi[1]];
    static const std::vector<std::pair<int, double>> one{{0, 1.0}};
    const auto &rz = d == 3 ? rows[mi[2]] : one;
    for (const auto &z : rz)
      for (const auto &y : ry)
        for (const auto &x : rx) {
          int mfi[3] = {x.first, y.first, z.first};
          int32_t c = Lf.lat2c[size_t(multi_lat(mfi, mf, d))];
          if (c < 0) continue;
          double v = d == 3 ? z.second * (y.second * x.second) : y.second * x.second;
          out[i].push_back({c, v});
        }
  }
  CSR &R = Lf.R;
  R.nrows = n;
  R.ncols = int32_t(Lf.c2lat.size());
  R.rowptr.assign(n + 1, 0);
  for (int i = 0; i < n; ++i) R.rowptr[i + 1] = R.rowptr[i] + int32_t(out[i].size());
  R.col.resize(R.rowptr[n]);
  R.val.resize(R.rowptr[n]);
  for (int i = 0; i < n; ++i)
    for (size_t k = 0; k < out[i].size(); ++k) {
      R.col[R.rowptr[i] + k] = out[i][k].first;
      R.val[R.rowptr[i] + k] = out[i][k].second;
    }
}

// Galerkin A_c = R A R^T on the coarse structural pattern (T = A R^T first);
// Ac holds the pattern and receives the values.
void galerkin_csr(const CSR &R, const CSR &A, CSR &Ac) {
  const int nf = A.nrows, ncr = R.nrows;
  // R^T (fine row -> coarse entries)
  std::vector<int32_t> tptr(nf + 1, 0), tcol(R.col.size());
  std::vector<double> tval(R.col.size());
  for (size_t k = 0; k < R.col.size(); ++k) tptr[R.col[k] + 1]++;
  for (int i = 0; i < nf; ++i) tptr[i + 1] += tptr[i];
  {
    std::vector<int32_t> fill(tptr.begin(), tptr.end() - 1);
    for (int i = 0; i < ncr; ++i)
      for (int k = R.rowptr[i]; k < R.rowptr[i + 1]; ++k) {
        int32_t c = R.col[k];
        tcol[fill[c]] = i;
        tval[fill[c]] = R.val[k];
        fill[c]++;
      }
  }
  // T = A R^T, rows over fine, coarse columns sorted
  std::vector<std::vector<std::pair<int32_t, double>>> T(nf);
#pragma omp parallel
  {
    std::vector<double> acc(ncr, 0.0);
    std::vector<int32_t> touched;
#pragma omp for schedule(dynamic, 512)
    for (int k = 0; k < nf; ++k) {
      touched.clear();
      for (int a = A.rowptr[k]; a < A.rowptr[k + 1]; ++a) {
        const int32_t l = A.col[a];
        const double av = A.val[a];
        for (int t = tptr[l]; t < tptr[l + 1]; ++t) {
          const int32_t j = tcol[t];
          if (acc[j] == 0.0) {
            bool seen = false;
            for (int32_t u : touched) if (u == j) { seen = true; break; }
            if (!seen) touched.push_back(j);
          }
          acc[j] += av * tval[t];
        }
      }
      std::sort(touched.begin(), touched.end());
      T[k].reserve(touched.size());
      for (int32_t j : touched) { T[k].push_back({j, acc[j]}); acc[j] = 0.0; }
    }
  }
  bool outside = false;
#pragma omp parallel
  {
    std::vector<double> acc(ncr, 0.0);
    std::vector<uint8_t> hit(ncr, 0);
#pragma omp for schedule(dynamic, 256)
    for (int i = 0; i < ncr; ++i) {
      for (int a = R.rowptr[i]; a < R.rowptr[i + 1]; ++a) {
        const double rv = R.val[a];
        for (const auto &tj : T[R.col[a]]) {
          acc[tj.first] += rv * tj.second;
          hit[tj.first] = 1;
        }
      }
      for (int q = Ac.rowptr[i]; q < Ac.rowptr[i + 1]; ++q) {
        Ac.val[q] = acc[Ac.col[q]];
        acc[Ac.col[q]] = 0.0;
        hit[Ac.col[q]] = 0;
      }
      // anything left outside the structural pattern must be zero
      for (int a = R.rowptr[i]; a < R.rowptr[i + 1]; ++a)
        for (const auto &tj : T[R.col[a]]) {
          if (hit[tj.first]) {
            if (acc[tj.first] != 0.0) {
#pragma omp atomic write
              outside = true;
            }
            acc[tj.first] = 0.0;
            hit[tj.first] = 0;
          }
        }
    }
  }
  if (outside) throw GenError(-1, "Galerkin product has an entry outside the structural pattern");
}

// Galerkin coarse operator of level Lc from level Lf (per component block for
// elasticity: R = I (x) R_scalar keeps the blocks apart).
void galerkin(LevelData &Lc, const LevelData &Lf) {
  if (Lf.Ab.empty()) {
    galerkin_csr(Lf.R, Lf.A, Lc.A);
    return;
  }
  Lc.Ab.assign(Lf.Ab.size(), CSR());
  for (size_t k = 0; k < Lf.Ab.size(); ++k) {
    CSR Af = Lf.A;
    Af.val = Lf.Ab[k].val;
    CSR Ac = Lc.A;
    galerkin_csr(Lf.R, Af, Ac);
    Lc.Ab[k].val = std::move(Ac.val);
  }
  Lc.A.val = Lc.Ab[0].val;
}

// Blocks by encapsulating supports (vertex functions only for Lagrange).
void build_blocks(LevelData &L, const Basis1D &B, int d, const Stencil &st) {
  const int n = int(L.c2lat.size());
  const int nf = L.nf1;
  std::vector<std::vector<int32_t>> blk(n);
  std::vector<uint8_t> has(n, 0);
#pragma omp parallel for schedule(dynamic, 256)
  for (int j = 0; j < n; ++j) {
    int mj[3] = {0, 0, 0};
    lat_multi(L.c2lat[j], nf, d, mj);
    if (B.basis == IMSMG_GEN_LAGRANGE) {
      bool nodal = true;
      for (int a = 0; a < d; ++a) nodal = nodal && (mj[a] % B.p == 0);
      if (!nodal) continue;
    }
    has[j] = 1;
    int jlo[3], jhi[3];
    for (int a = 0; a < d; ++a) B.support(mj[a], jlo[a], jhi[a]);
    for (int s = 0; s < st.K; ++s) {
      int off[3] = {0, 0, 0}, mk[3] = {0, 0, 0};
      st.offset(s, off);
      bool ok = true;
      for (int a = 0; a < d; ++a) {
        mk[a] = mj[a] + off[a];
        if (mk[a] < 0 || mk[a] >= nf) ok = false;
      }
      if (!ok) continue;
      int32_t k = L.lat2c[size_t(multi_lat(mk, nf, d))];
      if (k < 0) continue;
      int klo[3], khi[3], ilo[3], ihi[3];
      for (int a = 0; a < d; ++a) {
        B.support(mk[a], klo[a], khi[a]);
        ilo[a] = std::max(klo[a], jlo[a]);
        ihi[a] = std::min(khi[a], jhi[a]);
      }
      const int64_t in_k = sat_count(L, d, klo, khi);
      const int64_t in_both = sat_count(L, d, ilo, ihi);
      if (in_k == in_both) blk[j].push_back(k);
    }
  }
  L.bptr.assign(1, 0);
  L.bidx.clear();
  L.bassoc.clear();
  for (int j = 0; j < n; ++j) {
    if (!has[j]) continue;
    L.bidx.insert(L.bidx.end(), blk[j].begin(), blk[j].end());
    L.bptr.push_back(int32_t(L.bidx.size()));
    L.bassoc.push_back(j);
  }
}

void build(Problem &P) {
  const imsmg_gen_spec &s = P.spec;
  Ctx C(s);
  const int d = s.dim, p = s.degree, nlev = s.levels;
  C.geo.kind = s.geometry;
  C.geo.dim = d;
  C.geo.discs = P.discs;
  for (int a = 0; a < 3; ++a) C.geo.phase[a] = s.phase[a];
  C.geo.level = s.gyroid_level;
  C.geo.plane_x = s.plane_x;
  const int qc = s.q_cell > 0 ? s.q_cell : p + 1;
  const int qs = s.q_simplex > 0 ? s.q_simplex : (d == 2 ? std::max(2 * p, 1) : 3 * p + 1);
  const int qb = s.q_bnd > 0 ? s.q_bnd : (d == 2 ? 2 * p + 1 : 3 * p + 1);
  C.gc = gauss_legendre01(qc);
  C.gs = gauss_legendre01(qs);
  C.gb = gauss_legendre01(qb);
  C.want_bnd = d == 3 && s.physics == IMSMG_GEN_ELASTICITY && s.bc == IMSMG_GEN_PENALTY;
  // leaf lattice
  C.nleaf = s.n << s.depth;
  const int N1 = C.nleaf + 1;
  size_t nl = 1;
  for (int a = 0; a < d; ++a) nl *= N1;
  C.leaf.resize(nl);
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < int64_t(nl); ++t) {
    int64_t r = t;
    double x[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) {
      int i = int(r % N1);
      r /= N1;
      x[a] = (s.box_hi - s.box_lo) * double(i) / double(C.nleaf) + s.box_lo;
    }
    double v = C.geo.eval(x);
    if (std::fabs(v) < kSnap) v = 0.0;
    C.leaf[t] = v;
  }
  P.lv.assign(nlev, LevelData());
  // finest level element activity from leaf vertices
  LevelData &F = P.lv[nlev - 1];
  F.n = s.n;
  F.depth = s.depth;
  size_t ne = 1;
  for (int a = 0; a < d; ++a) ne *= F.n;
  F.active_el.assign(ne, 0);
  const int sdep = 1 << s.depth;
#pragma omp parallel for schedule(static)
  for (int64_t t = 0; t < int64_t(ne); ++t) {
    int e[3] = {0, 0, 0};
    int64_t r = t;
    for (int a = 0; a < d; ++a) { e[a] = int(r % F.n); r /= F.n; }
    bool any = false;
    for (int k = 0; k <= (d == 3 ? sdep : 0) && !any; ++k)
      for (int j = 0; j <= sdep && !any; ++j)
        for (int i = 0; i <= sdep; ++i) {
          int LL[3] = {e[0] * sdep + i, e[1] * sdep + j, d == 3 ? e[2] * sdep + k : 0};
          if (C.leaf[C.leaf_index(LL)] > 0.0) { any = true; break; }
        }
    F.active_el[t] = any;
  }
  // coarser levels: active when a child is active
  for (int l = nlev - 2; l >= 0; --l) {
    LevelData &Lc = P.lv[l];
    const LevelData &Lf = P.lv[l + 1];
    if (Lf.n % 2) throw GenError(-1, "element count not divisible by 2^(levels-1)");
    Lc.n = Lf.n / 2;
    Lc.depth = Lf.depth + 1;
    size_t nec = 1;
    for (int a = 0; a < d; ++a) nec *= Lc.n;
    Lc.active_el.assign(nec, 0);
    for (size_t t = 0; t < nec; ++t) {
      int e[3] = {0, 0, 0};
      size_t r = t;
      for (int a = 0; a < d; ++a) { e[a] = int(r % Lc.n); r /= Lc.n; }
      bool any = false;
      for (int c = 0; c < (1 << d) && !any; ++c) {
        int ef[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) ef[a] = 2 * e[a] + ((c >> a) & 1);
        any = Lf.active_el[size_t(multi_lat(ef, Lf.n, d))];
      }
      Lc.active_el[t] = any;
    }
  }
  const bool strong = s.bc == IMSMG_GEN_BOX_DIRICHLET;
  const Stencil st(d, p);
  std::vector<Basis1D> bases;
  for (int l = 0; l < nlev; ++l) bases.emplace_back(s.basis, P.lv[l].n, p, s.box_lo, s.box_hi);
  for (int l = 0; l < nlev; ++l) {
    build_sat(P.lv[l], d);
    activate_functions(P.lv[l], bases[l], d, strong);
    build_pattern(P.lv[l], bases[l], d, st);
  }
  if (s.physics == IMSMG_GEN_ELASTICITY)
    assemble_fine_elasticity(C, P, F, bases[nlev - 1]);
  else
    assemble_fine(C, P, F, bases[nlev - 1]);
  // volume fractions of coarse elements: mean of the children
  for (int l = nlev - 2; l >= 0; --l) {
    LevelData &Lc = P.lv[l];
    const LevelData &Lf = P.lv[l + 1];
    Lc.eta.assign(Lc.active_el.size(), 0.0);
    for (size_t t = 0; t < Lc.active_el.size(); ++t) {
      int e[3] = {0, 0, 0};
      size_t r = t;
      for (int a = 0; a < d; ++a) { e[a] = int(r % Lc.n); r /= Lc.n; }
      double acc = 0.0;
      for (int c = 0; c < (1 << d); ++c) {
        int ef[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) ef[a] = 2 * e[a] + ((c >> a) & 1);
        acc += Lf.eta[size_t(multi_lat(ef, Lf.n, d))];
      }
      Lc.eta[t] = acc / (1 << d);
    }
  }
  for (int l = nlev - 1; l >= 1; --l) {
    build_restriction(P.lv[l - 1], P.lv[l], d, s.basis, p, s.box_lo, s.box_hi);
    galerkin(P.lv[l - 1], P.lv[l]);
  }
  for (int l = 1; l < nlev; ++l) build_blocks(P.lv[l], bases[l], d, st);
}

int fail(const GenError &e) {
  g_err = e.what();
  return e.code;
}

}  // namespace

struct imsmg_gen_problem {
  Problem P;
};

extern "C" {

const char *imsmg_gen_last_error(void) { return g_err.c_str(); }

int imsmg_gen_build(const imsmg_gen_spec *spec, imsmg_gen_problem **out) {
  g_err.clear();
  if (!spec || !out) { g_err = "null argument"; return -1; }
  *out = nullptr;
  const imsmg_gen_spec &s = *spec;
  if (s.dim < 2 || s.dim > 3 || s.degree < 1 || s.degree > 4 || s.n < 1 || s.levels < 1 || s.depth < 0 ||
      s.depth > 12 || (s.basis != IMSMG_GEN_BSPLINE && s.basis != IMSMG_GEN_LAGRANGE) || s.bc < 0 || s.bc > 2 ||
      s.rhs < 0 || s.rhs > 2 || s.geometry < 0 || s.geometry > 5 || !(s.box_hi > s.box_lo) ||
      (s.physics != IMSMG_GEN_POISSON && s.physics != IMSMG_GEN_ELASTICITY) ||
      (s.dirichlet_part != IMSMG_GEN_DIRICHLET_ALL && s.dirichlet_part != IMSMG_GEN_DIRICHLET_BITE)) {
    g_err = "invalid workload specification";
    return -1;
  }
  if (s.geometry == IMSMG_GEN_GEOM_DISCS && (s.ndiscs <= 0 || !s.discs)) { g_err = "discs missing"; return -1; }
  if ((s.geometry == IMSMG_GEN_GEOM_GYROID && s.dim != 3) || ((s.geometry == IMSMG_GEN_GEOM_DISCS || s.geometry == IMSMG_GEN_GEOM_STAR) && s.dim != 2)) {
    g_err = "geometry does not match the dimension";
    return -1;
  }
  if ((s.geometry == IMSMG_GEN_GEOM_APPLE || s.geometry == IMSMG_GEN_GEOM_SLAB) && s.dim != 3) {
    g_err = "the apple and the slab are 3D geometries";
    return -1;
  }
  if (s.n % (1 << (s.levels - 1))) { g_err = "n must be divisible by 2^(levels-1)"; return -1; }
  if (s.physics == IMSMG_GEN_ELASTICITY) {
    if (s.bc != IMSMG_GEN_PENALTY || s.basis != IMSMG_GEN_BSPLINE) {
      g_err = "elasticity: B-splines with penalty Dirichlet conditions";
      return -1;
    }
    if (s.dirichlet_part == IMSMG_GEN_DIRICHLET_BITE && s.geometry != IMSMG_GEN_GEOM_APPLE) {
      g_err = "the bite is a part of the apple's boundary";
      return -1;
    }
  } else if (s.dim == 3 && (s.bc == IMSMG_GEN_PENALTY || s.rhs == IMSMG_GEN_RHS_MANUFACTURED)) {
    g_err = "boundary integrals are implemented for 2D workloads only";
    return -1;
  }
  try {
    auto t0 = std::chrono::steady_clock::now();
    auto *p = new imsmg_gen_problem();
    p->P.spec = s;
    if (s.geometry == IMSMG_GEN_GEOM_DISCS) p->P.discs.assign(s.discs, s.discs + 3 * s.ndiscs);
    p->P.spec.discs = nullptr;
    int old = omp_get_max_threads();
    if (s.nthreads > 0) omp_set_num_threads(s.nthreads);
    try {
      build(p->P);
    } catch (...) {
      omp_set_num_threads(old);
      delete p;
      throw;
    }
    omp_set_num_threads(old);
    p->P.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    *out = p;
    return 0;
  } catch (const GenError &e) {
    return fail(e);
  } catch (const std::bad_alloc &) {
    g_err = "out of memory";
    return -2;
  } catch (const std::exception &e) {
    g_err = e.what();
    return -1;
  }
}

int imsmg_gen_level_info_get(const imsmg_gen_problem *p, int level, imsmg_gen_level_info *info) {
  if (!p || !info || level < 0 || level >= int(p->P.lv.size())) { g_err = "bad level"; return -1; }
  const LevelData &L = p->P.lv[level];
  const int d = p->P.spec.dim;
  info->n_active = int32_t(L.c2lat.size());
  info->nnz = int64_t(L.A.col.size());
  for (int a = 0; a < 3; ++a) info->lattice[a] = a < d ? L.nf1 : 1;
  info->n_elements = L.n;
  info->nblocks = int32_t(L.bassoc.size());
  info->block_nnz = int64_t(L.bidx.size());
  info->r_nnz = level > 0 ? int64_t(L.R.col.size()) : 0;
  info->n_cut = L.n_cut;
  {
    int32_t na = 0;
    int64_t nz = 0;
    const Basis1D B(p->P.spec.basis, L.n, p->P.spec.degree, p->P.spec.box_lo, p->P.spec.box_hi);
    for (size_t t = 0; t < L.active_el.size(); ++t) {
      if (!L.active_el[t]) continue;
      ++na;
      int e[3] = {0, 0, 0};
      size_t r = t;
      for (int a = 0; a < d; ++a) { e[a] = int(r % L.n); r /= L.n; }
      const int m = p->P.spec.degree + 1;
      int tot = 1;
      for (int a = 0; a < d; ++a) tot *= m;
      for (int A = 0; A < tot; ++A) {
        int mf[3] = {0, 0, 0}, ra = A;
        for (int a = 0; a < d; ++a) { mf[a] = B.first(e[a]) + ra % m; ra /= m; }
        if (L.lat2c[size_t(multi_lat(mf, L.nf1, d))] >= 0) ++nz;
      }
    }
    info->n_active_elements = na;
    info->elem_nnz = nz;
  }
  double em = 1.0;
  for (size_t t = 0; t < L.eta.size(); ++t)
    if (L.active_el[t]) em = std::min(em, L.eta[t]);
  info->eta_min = em;
  info->ncomp = L.Ab.empty() ? 1 : d;
  return 0;
}

int imsmg_gen_get_operator_block(const imsmg_gen_problem *p, int level, int ci, int cj, double *val) {
  if (!p || !val || level < 0 || level >= int(p->P.lv.size())) { g_err = "bad level"; return -1; }
  const LevelData &L = p->P.lv[level];
  const int nc = L.Ab.empty() ? 1 : p->P.spec.dim;
  if (ci < 0 || cj < 0 || ci >= nc || cj >= nc) { g_err = "bad component block"; return -1; }
  const std::vector<double> &v = L.Ab.empty() ? L.A.val : L.Ab[size_t(ci) * nc + cj].val;
  std::copy(v.begin(), v.end(), val);
  return 0;
}

int imsmg_gen_get_operator(const imsmg_gen_problem *p, int level, int32_t *d2l, int32_t *rowptr, int32_t *col,
                           double *val) {
  if (!p || level < 0 || level >= int(p->P.lv.size())) { g_err = "bad level"; return -1; }
  const LevelData &L = p->P.lv[level];
  if (d2l) std::copy(L.c2lat.begin(), L.c2lat.end(), d2l);
  if (rowptr) std::copy(L.A.rowptr.begin(), L.A.rowptr.end(), rowptr);
  if (col) std::copy(L.A.col.begin(), L.A.col.end(), col);
  if (val) std::copy(L.A.val.begin(), L.A.val.end(), val);
  return 0;
}

int imsmg_gen_get_restriction(const imsmg_gen_problem *p, int level, int32_t *rowptr, int32_t *col, double *val) {
  if (!p || level < 1 || level >= int(p->P.lv.size())) { g_err = "bad level"; return -1; }
  const CSR &R = p->P.lv[level].R;
  if (rowptr) std::copy(R.rowptr.begin(), R.rowptr.end(), rowptr);
  if (col) std::copy(R.col.begin(), R.col.end(), col);
  if (val) std::copy(R.val.begin(), R.val.end(), val);
  return 0;
}

int imsmg_gen_get_two_scale(const imsmg_gen_problem *p, int level, double *R1) {
  if (!p || !R1 || level < 1 || level >= int(p->P.lv.size())) { g_err = "bad level"; return -1; }
  const imsmg_gen_spec &s = p->P.spec;
  std::vector<double> R = two_scale(s.basis, p->P.lv[level - 1].n, s.degree, s.box_lo, s.box_hi);
  std::copy(R.begin(), R.end(), R1);
  return 0;
}

int imsmg_gen_get_blocks(const imsmg_gen_problem *p, int level, int32_t *ptr, int32_t *idx, int32_t *assoc) {
  if (!p || level < 0 || level >= int(p->P.lv.size())) { g_err = "bad level"; return -1; }
  const LevelData &L = p->P.lv[level];
  if (ptr) std::copy(L.bptr.begin(), L.bptr.end(), ptr);
  if (idx) std::copy(L.bidx.begin(), L.bidx.end(), idx);
  if (assoc) std::copy(L.bassoc.begin(), L.bassoc.end(), assoc);
  return 0;
}

// Colours for the multiplicative smoother from the lattice position m of a
// block's associated function: blocks of one colour share no element.
// B-splines and one-function blocks: sum_a (m_a mod (p+1)) (p+1)^a (function
// m is non-zero on elements m-p .. m per axis, so equal residues mod p+1 are
// at least p+1 apart); Lagrange vertex blocks (m_a = p v_a, elements
// v_a - 1 .. v_a): sum_a (v_a mod 2) 2^a.
int imsmg_gen_get_block_colours(const imsmg_gen_problem *p, int level, int kind, int32_t *colour) {
  if (!p || !colour || level < 0 || level >= int(p->P.lv.size()) || (kind != 0 && kind != 1)) {
    g_err = "bad block colour arguments";
    return -1;
  }
  const LevelData &L = p->P.lv[level];
  const imsmg_gen_spec &sp = p->P.spec;
  const int d = sp.dim, deg = sp.degree;
  const bool lagrange_blocks = kind == 0 && sp.basis == IMSMG_GEN_LAGRANGE;
  const int q = lagrange_blocks ? 2 : deg + 1;
  auto colour_of = [&](int32_t j) {
    int m[3] = {0, 0, 0};
    lat_multi(L.c2lat[size_t(j)], L.nf1, d, m);
    int c = 0;
    for (int a = d - 1; a >= 0; --a) c = c * q + (lagrange_blocks ? m[a] / deg : m[a]) % q;
    return int32_t(c);
  };
  if (kind == 0)
    for (size_t b = 0; b < L.bassoc.size(); ++b) colour[b] = colour_of(L.bassoc[b]);
  else
    for (size_t j = 0; j < L.c2lat.size(); ++j) colour[j] = colour_of(int32_t(j));
  return 0;
}

int imsmg_gen_lattice_colours(int n, const int32_t *dof_to_lattice, int nf1, int dim, int q, int stride,
                              int32_t *colour) {
  if (n < 0 || (n > 0 && (!dof_to_lattice || !colour)) || nf1 < 1 || dim < 1 || dim > 3 || q < 1 || stride < 1) {
    g_err = "bad lattice colour arguments";
    return -1;
  }
  for (int j = 0; j < n; ++j) {
    int m[3] = {0, 0, 0};
    lat_multi(dof_to_lattice[j], nf1, dim, m);
    int c = 0;
    for (int a = dim - 1; a >= 0; --a) c = c * q + (m[a] / stride) % q;
    colour[j] = c;
  }
  return 0;
}

int imsmg_gen_get_elements(const imsmg_gen_problem *p, int level, int32_t *eptr, int32_t *eidx, int32_t *elem) {
  if (!p || level < 0 || level >= int(p->P.lv.size())) { g_err = "bad level"; return -1; }
  const LevelData &L = p->P.lv[level];
  const int d = p->P.spec.dim;
  const Basis1D B(p->P.spec.basis, L.n, p->P.spec.degree, p->P.spec.box_lo, p->P.spec.box_hi);
  const int m = p->P.spec.degree + 1;
  int tot = 1;
  for (int a = 0; a < d; ++a) tot *= m;
  int32_t na = 0;
  int64_t nz = 0;
  if (eptr) eptr[0] = 0;
  for (size_t t = 0; t < L.active_el.size(); ++t) {
    if (!L.active_el[t]) continue;
    int e[3] = {0, 0, 0};
    size_t r = t;
    for (int a = 0; a < d; ++a) { e[a] = int(r % L.n); r /= L.n; }
    for (int A = 0; A < tot; ++A) {
      int mf[3] = {0, 0, 0}, ra = A;
      for (int a = 0; a < d; ++a) { mf[a] = B.first(e[a]) + ra % m; ra /= m; }
      const int32_t c = L.lat2c[size_t(multi_lat(mf, L.nf1, d))];
      if (c >= 0) {
        if (eidx) eidx[nz] = c;
        ++nz;
      }
    }
    if (elem) elem[na] = int32_t(t);
    ++na;
    if (eptr) eptr[na] = int32_t(nz);
  }
  return 0;
}

int imsmg_gen_get_rhs(const imsmg_gen_problem *p, double *b) {
  if (!p || !b) { g_err = "null argument"; return -1; }
  std::copy(p->P.b.begin(), p->P.b.end(), b);
  return 0;
}

int imsmg_gen_get_mass(const imsmg_gen_problem *p, double *val) {
  if (!p || !val) { g_err = "null argument"; return -1; }
  if (p->P.mass.empty()) { g_err = "mass matrix not assembled (with_mass = 0)"; return -1; }
  std::copy(p->P.mass.begin(), p->P.mass.end(), val);
  return 0;
}

int imsmg_gen_get_volume_fractions(const imsmg_gen_problem *p, int level, double *eta) {
  if (!p || !eta || level < 0 || level >= int(p->P.lv.size())) { g_err = "bad level"; return -1; }
  const LevelData &L = p->P.lv[level];
  std::copy(L.eta.begin(), L.eta.end(), eta);
  return 0;
}

double imsmg_gen_setup_seconds(const imsmg_gen_problem *p) { return p ? p->P.seconds : 0.0; }

void imsmg_gen_free(imsmg_gen_problem *p) { delete p; }

}  // extern "C"
