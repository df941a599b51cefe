// Host-side construction of the basis and quadrature tables (computed once at
// initialisation, Sec. 4.5 step 1).
//
//   Legendre polynomials and their scaling ...... App. A
//   Gauss-Legendre nodes (Newton, Lether start) . App. B
//   Gauss-Lobatto-Legendre nodes and weights .... App. C
//   total-degree product basis .................. Sec. 2.2, eq. set_basis_functions
//   positivity points (union of GLL x Gauss) .... Sec. 3.4, eq. union_quad_points
#include <cmath>
#include <stdexcept>

#include "dg_internal.h"

namespace dg {
namespace {

constexpr double kPi = 3.141592653589793238462643383279502884;

// Values P_0..P_n(x) and derivatives, filled by the Legendre recurrence
// n P_n = (2n-1) x P_{n-1} - (n-1) P_{n-2} and P_n' = n (P_{n-1} - x P_n)/(1-x^2)
// away from the end points; at +-1 the closed form P_n'(+-1) = (+-1)^(n+1) n(n+1)/2.
struct LegendreTable {
  double p[16], dp[16];
  LegendreTable(int n, double x) {
    p[0] = 1.0;
    dp[0] = 0.0;
    if (n >= 1) p[1] = x;
    for (int j = 2; j <= n; ++j) p[j] = ((2 * j - 1) * x * p[j - 1] - (j - 1) * p[j - 2]) / j;
    for (int j = 1; j <= n; ++j) {
      if (std::fabs(std::fabs(x) - 1.0) < 1e-300) {
        double s = (x > 0 || (j % 2 == 1)) ? 1.0 : -1.0;  // (+-1)^(j+1)
        dp[j] = s * 0.5 * j * (j + 1);
      } else {
        dp[j] = j * (p[j - 1] - x * p[j]) / (1.0 - x * x);
      }
    }
  }
};

// Second derivative of P_n from Legendre's equation (App. A, eq. legendre_dgl).
double legendre_d2(int n, double x) {
  LegendreTable t(n, x);
  return (2.0 * x * t.dp[n] - n * (n + 1.0) * t.p[n]) / (1.0 - x * x);
}

void gauss_legendre(int n, double *x, double *w) {
  // Roots of P_n by Newton-Raphson from the approximation quoted in App. B.
  for (int i = 0; i < n; ++i) {
    int q = n - i;  // q = n gives the smallest root
    double guess = (1.0 - 1.0 / (8.0 * n * n) + 1.0 / (8.0 * n * n * n)) *
                   std::cos(kPi * (4.0 * q - 1.0) / (4.0 * n + 2.0));
    double r = guess;
    for (int it = 0; it < 64; ++it) {
      LegendreTable t(n, r);
      double delta = t.p[n] / t.dp[n];
      r -= delta;
      if (std::fabs(delta) <= 1e-17) break;
    }
    LegendreTable t(n, r);
    x[i] = r;
    w[i] = 2.0 / ((1.0 - r * r) * t.dp[n] * t.dp[n]);
  }
}

void gauss_lobatto(int m, double *x, double *w) {
  // End points and the m-2 roots of P'_{m-1}; weights 2 / (m (m-1) P_{m-1}^2).
  int n = m - 1;
  x[0] = -1.0;
  x[m - 1] = 1.0;
  for (int i = 1; i < m - 1; ++i) {
    double r = -std::cos(kPi * i / n);
    for (int it = 0; it < 64; ++it) {
      LegendreTable t(n, r);
      double delta = t.dp[n] / legendre_d2(n, r);
      r -= delta;
      if (std::fabs(delta) <= 1e-17) break;
    }
    x[i] = r;
  }
  for (int i = 0; i < m; ++i) {
    LegendreTable t(n, x[i]);
    w[i] = 2.0 / (m * (m - 1.0) * t.p[n] * t.p[n]);
  }
}

// sqrt(2n+1) P_n(x) and its derivative.
double pt(int n, double x) { return std::sqrt(2.0 * n + 1.0) * LegendreTable(n, x).p[n]; }
double dpt(int n, double x) { return std::sqrt(2.0 * n + 1.0) * LegendreTable(n, x).dp[n]; }

}  // namespace

std::vector<int> mode_exponents(int d, int k) {
  std::vector<int> e;
  for (int total = 0; total <= k; ++total)
    for (int ex = total; ex >= 0; --ex)
      for (int ey = total - ex; ey >= 0; --ey) {
        int ez = total - ex - ey;
        if (d == 2 && ez > 0) continue;
        e.push_back(ex);
        e.push_back(ey);
        e.push_back(ez);
      }
  return e;
}

Shape make_shape(int d, int k) {
  Shape s;
  s.d = d;
  s.k = k;
  s.n1 = k + 1;
  s.nv = d + 2;
  s.N = (int)mode_exponents(d, k).size() / 3;
  s.Q = 1;
  for (int a = 0; a < d; ++a) s.Q *= s.n1;
  s.QF = s.Q / s.n1;
  s.M = (k + 4) / 2;
  if (s.M < 2) s.M = 2;
  s.NS = d * s.M * s.QF;
  return s;
}

Layout make_layout(const Shape &s) {
  Layout L;
  int o = 0;
  L.B = o;  o += s.Q * s.N;
  L.DW = o; o += s.d * s.Q * s.N;
  L.TF = o; o += s.d * 2 * s.QF * s.N;
  L.TW = o; o += s.d * 2 * s.QF * s.N;
  L.WQ = o; o += s.Q;
  L.PS = o; o += s.NS * s.N;
  L.XQ = o; o += 3 * s.Q;
  L.HG = o; o += s.d * 2 * 4 * s.QF * s.N;
  L.HW = o; o += s.d * 2 * 4 * s.QF * s.N;
  L.CM = o; o += 8 * s.N;
  L.total = o;
  return L;
}

std::vector<double> build_tables(const Shape &s, double *gll_w1) {
  if (s.n1 > 15 || s.M > 15) throw std::invalid_argument("degree too high");
  Layout L = make_layout(s);
  std::vector<double> t(L.total, 0.0);
  std::vector<int> e = mode_exponents(s.d, s.k);
  double gx[16], gw[16], lx[16], lw[16];
  gauss_legendre(s.n1, gx, gw);
  gauss_lobatto(s.M, lx, lw);
  *gll_w1 = lw[0];

  auto basis = [&](int l, const double *xi) {
    double v = 1.0;
    for (int a = 0; a < s.d; ++a) v *= pt(e[3 * l + a], xi[a]);
    return v;
  };
  auto dbasis = [&](int l, int a, const double *xi) {
    double v = 1.0;
    for (int b = 0; b < s.d; ++b) v *= (b == a) ? dpt(e[3 * l + b], xi[b]) : pt(e[3 * l + b], xi[b]);
    return v;
  };

  // volume nodes, x index fastest
  for (int q = 0; q < s.Q; ++q) {
    int idx[3] = {q % s.n1, (q / s.n1) % s.n1, q / (s.n1 * s.n1)};
    double xi[3] = {0.0, 0.0, 0.0};
    double wq = 1.0;
    for (int a = 0; a < s.d; ++a) {
      xi[a] = gx[idx[a]];
      wq *= gw[idx[a]];
    }
    t[L.WQ + q] = wq;
    for (int a = 0; a < 3; ++a) t[L.XQ + 3 * q + a] = xi[a];
    for (int l = 0; l < s.N; ++l) {
      t[L.B + q * s.N + l] = basis(l, xi);
      for (int a = 0; a < s.d; ++a) t[L.DW + (a * s.Q + q) * s.N + l] = dbasis(l, a, xi) * wq;
    }
  }
  // face nodes: tangential axes in increasing order, first tangential fastest
  for (int a = 0; a < s.d; ++a) {
    int tang[2], nt = 0;
    for (int b = 0; b < s.d; ++b)
      if (b != a) tang[nt++] = b;
    for (int side = 0; side < 2; ++side)
      for (int r = 0; r < s.QF; ++r) {
        int idx[2] = {r % s.n1, r / s.n1};
        double xi[3] = {0.0, 0.0, 0.0};
        xi[a] = side ? 1.0 : -1.0;
        double wr = 1.0;
        for (int j = 0; j < nt; ++j) {
          xi[tang[j]] = gx[idx[j]];
          wr *= gw[idx[j]];
        }
        for (int l = 0; l < s.N; ++l) {
          double v = basis(l, xi);
          t[L.TF + ((a * 2 + side) * s.QF + r) * s.N + l] = v;
          t[L.TW + ((a * 2 + side) * s.QF + r) * s.N + l] = v * wr;
        }
      }
  }
  // positivity points: for each axis a, GLL in a times Gauss in the others
  int p = 0;
  for (int a = 0; a < s.d; ++a) {
    int tang[2], nt = 0;
    for (int b = 0; b < s.d; ++b)
      if (b != a) tang[nt++] = b;
    for (int i = 0; i < s.M; ++i)
      for (int r = 0; r < s.QF; ++r) {
        int idx[2] = {r % s.n1, r / s.n1};
        double xi[3] = {0.0, 0.0, 0.0};
        xi[a] = lx[i];
        for (int j = 0; j < nt; ++j) xi[tang[j]] = gx[idx[j]];
        for (int l = 0; l < s.N; ++l) t[L.PS + p * s.N + l] = basis(l, xi);
        ++p;
      }
  }
  // hanging faces: coarse basis at (eta + sigma)/2 on each of the 2^(d-1)
  // fine faces (sub bit j = position along the j-th tangential axis)
  for (int a = 0; a < s.d; ++a) {
    int tang[2], nt = 0;
    for (int b = 0; b < s.d; ++b)
      if (b != a) tang[nt++] = b;
    for (int side = 0; side < 2; ++side)
      for (int sub = 0; sub < (1 << (s.d - 1)); ++sub)
        for (int r = 0; r < s.QF; ++r) {
          int idx[2] = {r % s.n1, r / s.n1};
          double xi[3] = {0.0, 0.0, 0.0};
          xi[a] = side ? 1.0 : -1.0;
          double wr = 1.0;
          for (int j = 0; j < nt; ++j) {
            xi[tang[j]] = 0.5 * (gx[idx[j]] + (((sub >> j) & 1) ? 1.0 : -1.0));
            wr *= gw[idx[j]];
          }
          for (int l = 0; l < s.N; ++l) {
            const long o2 = (((a * 2 + side) * 4 + sub) * s.QF + r) * s.N + l;
            const double v = basis(l, xi);
            t[L.HG + o2] = v;
            t[L.HW + o2] = v * wr / (double)(1 << (s.d - 1));
          }
        }
  }
  // child means: 2^-d sum_q w_q phi_l((xi_q + c)/2) (exact: degree <= k)
  for (int ch = 0; ch < (1 << s.d); ++ch)
    for (int l = 0; l < s.N; ++l) {
      double acc = 0.0;
      for (int q = 0; q < s.Q; ++q) {
        int idx[3] = {q % s.n1, (q / s.n1) % s.n1, q / (s.n1 * s.n1)};
        double xi[3] = {0.0, 0.0, 0.0}, wq = 1.0;
        for (int a = 0; a < s.d; ++a) {
          xi[a] = 0.5 * (gx[idx[a]] + (((ch >> a) & 1) ? 1.0 : -1.0));
          wq *= gw[idx[a]];
        }
        acc += basis(l, xi) * wq;
      }
      t[L.CM + ch * s.N + l] = acc / (double)(1 << s.d);
    }
  return t;
}

// Refinement matrices (eq. ref_pa_integral): P[c][j][l] is the coefficient of
// phi_j on child c of the coarse phi_l, i.e. 2^-d times the Gauss integral of
// phi_j(xi) phi_l((xi + s_c) / 2) over the reference cell, s_c the child's
// offset (+1 where bit a of c is set, else -1); exact at (k+1)^d nodes.
std::vector<double> refine_matrices(const Shape &s) {
  std::vector<int> e = mode_exponents(s.d, s.k);
  double gx[16], gw[16];
  gauss_legendre(s.n1, gx, gw);
  auto basis = [&](int l, const double *xi) {
    double v = 1.0;
    for (int a = 0; a < s.d; ++a) v *= pt(e[3 * l + a], xi[a]);
    return v;
  };
  const int nch = 1 << s.d;
  std::vector<double> P((size_t)nch * s.N * s.N, 0.0);
  for (int q = 0; q < s.Q; ++q) {
    int idx[3] = {q % s.n1, (q / s.n1) % s.n1, q / (s.n1 * s.n1)};
    double xi[3] = {0.0, 0.0, 0.0}, wq = 1.0;
    for (int a = 0; a < s.d; ++a) {
      xi[a] = gx[idx[a]];
      wq *= gw[idx[a]];
    }
    for (int ch = 0; ch < nch; ++ch) {
      double xm[3] = {0.0, 0.0, 0.0};
      for (int a = 0; a < s.d; ++a) xm[a] = 0.5 * (xi[a] + (((ch >> a) & 1) ? 1.0 : -1.0));
      for (int j = 0; j < s.N; ++j) {
        const double pj = basis(j, xi) * wq / (double)nch;
        for (int l = 0; l < s.N; ++l) P[((size_t)ch * s.N + j) * s.N + l] += pj * basis(l, xm);
      }
    }
  }
  return P;
}

// One-dimensional tables of the quadtree stage kernel (2D, sum-factorised
// along one axis): with n1 = k + 1 Gauss nodes g_i and weights w_i,
//   PG [n1][n1]  P~_e(g_i)          DG [n1][n1]  P~_e'(g_i)
//   GW [n1]      w_i                PB [2][n1]   P~_e(-1), P~_e(+1)
//   PH [2][n1][n1] P~_e((g_r + sigma)/2), sigma = -1 (lower half), +1 (upper)
std::vector<double> tables_1d(int k) {
  const int n1 = k + 1;
  std::vector<double> t((size_t)(4 * n1 * n1 + 3 * n1), 0.0);
  double g[8], gw[8];
  gauss_legendre(n1, g, gw);
  const int PG = 0, DG = n1 * n1, GW = 2 * n1 * n1, PB = GW + n1, PH = PB + 2 * n1;
  for (int i = 0; i < n1; ++i) {
    t[GW + i] = gw[i];
    for (int e = 0; e < n1; ++e) {
      t[PG + i * n1 + e] = pt(e, g[i]);
      t[DG + i * n1 + e] = dpt(e, g[i]);
    }
  }
  for (int e = 0; e < n1; ++e) {
    t[PB + e] = pt(e, -1.0);
    t[PB + n1 + e] = pt(e, 1.0);
  }
  for (int h = 0; h < 2; ++h)
    for (int r = 0; r < n1; ++r)
      for (int e = 0; e < n1; ++e) t[PH + (h * n1 + r) * n1 + e] = pt(e, 0.5 * (g[r] + (h ? 1.0 : -1.0)));
  return t;
}

}  // namespace dg
