/*
 * Plain single-threaded FP64 reference implementation of the modal DG scheme
 * for the compressible Euler equations of Schaal et al. (2015), "Astrophysical
 * hydrodynamics with a high order discontinuous Galerkin scheme and adaptive
 * mesh refinement".
 *
 * TEST INFRASTRUCTURE ONLY.  This is the oracle against which the GPU library
 * is checked.  Only the tests, the smoke check and the benchmark's CPU
 * baseline may load it.  It shares no code with the GPU library: its own
 * Legendre recurrence, Newton root finding, tables, flux, Riemann solver,
 * limiters and time integrator live here and nowhere else.
 *
 * Written for clarity, not speed: dense loops over cells, quadrature nodes and
 * basis functions, in the order the paper states the method.  Build with
 * -O2 -ffp-contract=off so no fused multiply-add changes the rounding.
 *
 * The same file compiles twice:
 *   - plain (real_t = double): the reference results;
 *   - with -DORC_CS (real_t = double complex): the complex-step derivative
 *     f'(x) v = Im f(x + i h v) / h, exact to rounding, used as the reference
 *     for the discrete adjoint.  Branches compare real parts only.
 *
 * Sources (sections and equations of the paper):
 *   Euler fluxes and EOS ............ Sec. 2.1, eqs. euler, flux_vectors, eos
 *   modal basis, orthonormality ..... Sec. 2.2, eqs. weights, set_basis_functions
 *   L2 projection of the ICs ........ Sec. 2.3
 *   weak form, volume/face terms .... Sec. 2.4, eqs. dg_projected, dg_term2, dg_term3
 *   time step ....................... Sec. 2.5 eq. time_step; Sec. 3.4 eq. time_step_pos
 *   component-wise TVB minmod ....... Sec. 3.1 eq. comp_limiter; Sec. 3.3
 *   characteristic TVB minmod ....... Sec. 3.2 eq. char_limiter; App. E
 *   positivity limiter .............. Sec. 3.4, eqs. union_quad_points, p_positivity
 *   AMR faces / limiting ............ Sec. 4 (hanging-face quadrature), Sec. 4.4
 *   refinement matrices ............. Sec. 4.2 eq. ref_pa_integral, App. F
 *   Legendre, Gauss, GLL ............ App. A, B, C
 *   SSP-RK3 ......................... App. D, table RK_3
 *   general explicit RK (tableau) ... App. D, table butcher, eqs. for w^{n+1}
 *                                     and rhs; tables RK_2, RK_4
 *   gravity source and time step .... Sec. 2.4 eq. gravity_term; Sec. 2.5
 *   refinement criterion ............ Sec. 4.1 eqs. cell_ref, node_ref
 *   2D quadtree of leaves (any depth, level jump <= 1 across faces) ... Sec. 4
 *   refine / derefine projections ... Sec. 4.2 eqs. ref_pa_integral,
 *                                     ref_weights; Sec. 4.3 eq. deref_weights
 * The HLLC Riemann solver is cited by the paper to Toro's textbook only; the
 * textbook HLLC with Einfeldt-Batten (Roe-averaged) wave-speed bounds is
 * used, with a Davis-bound option.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifndef M_PI
#define M_PI 3.14159265358979323846
#endif

#ifdef ORC_CS
#include <complex.h>
typedef double complex real_t;
#define RE(x) creal(x)
#define RSQRT(x) csqrt(x)
#define API(name) orc_cs_##name
#else
typedef double real_t;
#define RE(x) (x)
#define RSQRT(x) sqrt(x)
#define API(name) orc_##name
#endif

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENEGATIVE (-2)
#define ORC_ENOMEM (-3)

#define MAXK 4
#define MAXN 35  /* N_3(4) */
#define MAXQ 125 /* (k+1)^3 */
#define MAXQF 25 /* (k+1)^2 */
#define MAXV 5
#define MAXM 4   /* GLL points */
#define MAXS 300 /* d * m * (k+1)^(d-1) */

/* Run description.  Mirrored field by field by the Python wrapper. */
typedef struct {
  int dim, k;
  int n[3];
  double x0[3], len[3];
  double gamma, cfl;
  int bc[3];       /* 0 periodic, 1 transmissive (ghost trace = own trace)   */
  int flux;        /* 0 HLLC with Einfeldt-Batten speeds, 1 HLLC with Davis */
  int limiter;     /* 0 none, 1 component-wise minmod with TVB bound,
                      2 the same on the characteristic variables            */
  double beta, mtilde;
  int positivity;  /* 0/1 Zhang-Shu positivity limiter                      */
  double eps;
  int refine_lo[3], refine_hi[3]; /* static 2:1 box in base-cell indices      */
  const double *accel; /* external acceleration a = -grad Phi at the volume
                          nodes, [d][Q][ncell] (node order of
                          orc_node_coords), or NULL; uniform grids only      */
} orc_config;

/* ------------------------------------------------------------------------ */
/* Legendre polynomials (App. A) and quadrature rules (App. B, C)            */
/* ------------------------------------------------------------------------ */

/* P_n(x) and P_n'(x) by Bonnet's three-term recurrence,
 * (m+1) P_{m+1} = (2m+1) x P_m - m P_{m-1}, with P'_{m+1} = P'_{m-1} + (2m+1) P_m. */
static void legendre(int n, double x, double *P, double *dP) {
  double p0 = 1.0, p1 = x, d0 = 0.0, d1 = 1.0;
  if (n == 0) { *P = 1.0; *dP = 0.0; return; }
  for (int m = 1; m < n; ++m) {
    double p2 = ((2.0 * m + 1.0) * x * p1 - m * p0) / (m + 1.0);
    double d2 = d0 + (2.0 * m + 1.0) * p1;
    p0 = p1; p1 = p2; d0 = d1; d1 = d2;
  }
  *P = p1; *dP = d1;
}

/* Scaled Legendre polynomial sqrt(2n+1) P_n and its derivative (App. A). */
static double ptilde(int n, double x) { double P, dP; legendre(n, x, &P, &dP); return sqrt(2.0 * n + 1.0) * P; }
static double dptilde(int n, double x) { double P, dP; legendre(n, x, &P, &dP); return sqrt(2.0 * n + 1.0) * dP; }

/* n-point Gauss-Legendre rule (App. B): Newton on P_n from Lether's start
 * value, weights 2 / ((1 - x^2) P_n'(x)^2).  Returned in ascending order. */
static void gauss_rule(int n, double *x, double *w) {
  for (int q = 1; q <= n; ++q) {
    double nn = (double)n;
    double xi = (1.0 - 1.0 / (8.0 * nn * nn) + 1.0 / (8.0 * nn * nn * nn)) *
                cos(M_PI * (4.0 * q - 1.0) / (4.0 * nn + 2.0));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, xi, &P, &dP);
      double step = P / dP;
      xi -= step;
      if (fabs(step) < 1e-16) break;
    }
    double P, dP;
    legendre(n, xi, &P, &dP);
    x[n - q] = xi; /* q = 1 is the largest root */
    w[n - q] = 2.0 / ((1.0 - xi * xi) * dP * dP);
  }
}

/* m-point Gauss-Lobatto-Legendre rule (App. C): the end points and the roots
 * of P'_{m-1}; weights 2 / (m (m-1) P_{m-1}(x)^2).  Interior roots by Newton
 * on P'_{m-1}, whose derivative follows from Legendre's equation. */
static void gll_rule(int m, double *x, double *w) {
  int n = m - 1;
  x[0] = -1.0; x[m - 1] = 1.0;
  for (int j = 1; j < m - 1; ++j) {
    double xi = -cos(M_PI * j / (double)(m - 1));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, xi, &P, &dP);
      double d2P = (2.0 * xi * dP - n * (n + 1.0) * P) / (1.0 - xi * xi);
      double step = dP / d2P;
      xi -= step;
      if (fabs(step) < 1e-16) break;
    }
    x[j] = xi;
  }
  for (int j = 0; j < m; ++j) {
    double P, dP;
    legendre(n, x[j], &P, &dP);
    w[j] = 2.0 / (m * (m - 1.0) * P * P);
  }
}

/* ------------------------------------------------------------------------ */
/* Context: sizes and the tables of Sec. 2.2-2.4                             */
/* ------------------------------------------------------------------------ */

typedef struct {
  orc_config c;
  int d, k, n1, N, Q, Qf, nvar;
  long nx, ny, nz, ncell; /* one uniform block */
  double dx;
  double gx[MAXK + 1], gw[MAXK + 1];
  int e[MAXN][3];                        /* exponents of mode l            */
  double phiV[MAXQ][MAXN], dphiV[3][MAXQ][MAXN], wV[MAXQ];
  double phiF[3][2][MAXQF][MAXN], wF[MAXQF];
  int m; double lx[MAXM], lw[MAXM];      /* GLL rule for positivity       */
  int nS; double phiS[MAXS][MAXN];       /* union points S of Sec. 3.4     */
} ctx;

static double phi_at(const ctx *X, int l, const double *xi) {
  double v = 1.0;
  for (int a = 0; a < X->d; ++a) v *= ptilde(X->e[l][a], xi[a]);
  return v;
}

static double dphi_at(const ctx *X, int a, int l, const double *xi) {
  double v = 1.0;
  for (int b = 0; b < X->d; ++b) v *= (b == a) ? dptilde(X->e[l][b], xi[b]) : ptilde(X->e[l][b], xi[b]);
  return v;
}

/* Tangential axes of a face with normal axis a, in increasing order. */
static void tangential(int d, int a, int *t) {
  int j = 0;
  for (int b = 0; b < d; ++b) if (b != a) t[j++] = b;
}

static int ctx_init(const orc_config *c, ctx *X) {
  memset(X, 0, sizeof(*X));
  X->c = *c;
  if (c->dim < 2 || c->dim > 3 || c->k < 0 || c->k > MAXK) return ORC_EINVAL;
  if (c->limiter < 0 || c->limiter > 2) return ORC_EINVAL;
  X->d = c->dim; X->k = c->k; X->n1 = c->k + 1;
  X->nvar = c->dim + 2;
  X->nx = c->n[0]; X->ny = c->n[1]; X->nz = (c->dim == 3) ? c->n[2] : 1;
  if (X->nx < 1 || X->ny < 1 || X->nz < 1) return ORC_EINVAL;
  X->ncell = X->nx * X->ny * X->nz;
  X->dx = c->len[0] / c->n[0];
  for (int a = 1; a < X->d; ++a) /* the paper's cells are cubes */
    if (fabs(c->len[a] / c->n[a] - X->dx) > 1e-12 * X->dx) return ORC_EINVAL;

  /* Basis index set {u+v+w <= k} (eq. set_basis_functions), ordered by total
   * degree, then x-exponent descending, then y-exponent descending. */
  int l = 0;
  for (int deg = 0; deg <= X->k; ++deg)
    for (int ex = deg; ex >= 0; --ex)
      for (int ey = deg - ex; ey >= 0; --ey) {
        int ez = deg - ex - ey;
        if (X->d == 2 && ez != 0) continue;
        X->e[l][0] = ex; X->e[l][1] = ey; X->e[l][2] = ez;
        ++l;
      }
  X->N = l;

  gauss_rule(X->n1, X->gx, X->gw);
  X->Q = 1; for (int a = 0; a < X->d; ++a) X->Q *= X->n1;
  X->Qf = X->Q / X->n1;

  /* Volume nodes: tensor Gauss rule, x index fastest. */
  for (int q = 0; q < X->Q; ++q) {
    int iq[3] = {q % X->n1, (q / X->n1) % X->n1, q / (X->n1 * X->n1)};
    double xi[3] = {0, 0, 0}, w = 1.0;
    for (int a = 0; a < X->d; ++a) { xi[a] = X->gx[iq[a]]; w *= X->gw[iq[a]]; }
    X->wV[q] = w;
    for (int j = 0; j < X->N; ++j) {
      X->phiV[q][j] = phi_at(X, j, xi);
      for (int a = 0; a < X->d; ++a) X->dphiV[a][q][j] = dphi_at(X, a, j, xi);
    }
  }
  /* Face nodes: tensor Gauss rule on the d-1 tangential axes. */
  for (int r = 0; r < X->Qf; ++r) {
    int ir[2] = {r % X->n1, r / X->n1};
    double w = 1.0;
    for (int j = 0; j < X->d - 1; ++j) w *= X->gw[ir[j]];
    X->wF[r] = w;
  }
  for (int a = 0; a < X->d; ++a) {
    int t[2]; tangential(X->d, a, t);
    for (int s = 0; s < 2; ++s)
      for (int r = 0; r < X->Qf; ++r) {
        int ir[2] = {r % X->n1, r / X->n1};
        double xi[3] = {0, 0, 0};
        xi[a] = s ? 1.0 : -1.0;
        for (int j = 0; j < X->d - 1; ++j) xi[t[j]] = X->gx[ir[j]];
        for (int jb = 0; jb < X->N; ++jb) X->phiF[a][s][r][jb] = phi_at(X, jb, xi);
      }
  }
  /* Positivity points: smallest m >= (k+3)/2, S = union over a of
   * (GLL in axis a) x (Gauss in the others) (eq. union_quad_points). */
  X->m = (X->k + 4) / 2; /* ceil((k+3)/2) */
  if (X->m < 2) X->m = 2;
  gll_rule(X->m, X->lx, X->lw);
  X->nS = 0;
  for (int a = 0; a < X->d; ++a) {
    int t[2]; tangential(X->d, a, t);
    for (int r = 0; r < X->m; ++r)
      for (int q = 0; q < X->Qf; ++q) {
        int ir[2] = {q % X->n1, q / X->n1};
        double xi[3] = {0, 0, 0};
        xi[a] = X->lx[r];
        for (int j = 0; j < X->d - 1; ++j) xi[t[j]] = X->gx[ir[j]];
        for (int jb = 0; jb < X->N; ++jb) X->phiS[X->nS][jb] = phi_at(X, jb, xi);
        ++X->nS;
      }
  }
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Euler flux and HLLC (Sec. 2.1; Sec. 2.4 numerical flux)                   */
/* ------------------------------------------------------------------------ */

static inline real_t rabs(real_t x) { return RE(x) < 0 ? -x : x; }
static inline real_t rmin(real_t a, real_t b) { return RE(b) < RE(a) ? b : a; }
static inline real_t rmax(real_t a, real_t b) { return RE(b) > RE(a) ? b : a; }

static real_t pressure(const ctx *X, const real_t *U) {
  real_t ke = 0.0;
  for (int b = 0; b < X->d; ++b) ke += U[1 + b] * U[1 + b] / U[0];
  return (X->c.gamma - 1.0) * (U[X->d + 1] - 0.5 * ke);
}

/* Physical flux f_a(U) (eq. flux_vectors; in 2D without the third velocity). */
static void euler_flux(const ctx *X, const real_t *U, int a, real_t *F) {
  int d = X->d;
  real_t rho = U[0], E = U[d + 1];
  real_t p = pressure(X, U);
  real_t va = U[1 + a] / rho;
  F[0] = U[1 + a];
  for (int b = 0; b < d; ++b) F[1 + b] = U[1 + b] * va + (b == a ? p : 0.0);
  F[d + 1] = (E + p) * va;
}

/* HLLC flux in the +a direction between left state UL and right state UR. */
static void hllc(const ctx *X, const real_t *UL, const real_t *UR, int a, real_t *F) {
  int d = X->d, nv = X->nvar;
  double g = X->c.gamma;
  real_t rL = UL[0], rR = UR[0];
  real_t vL[3], vR[3];
  for (int b = 0; b < d; ++b) { vL[b] = UL[1 + b] / rL; vR[b] = UR[1 + b] / rR; }
  real_t pL = pressure(X, UL), pR = pressure(X, UR);
  real_t cL = RSQRT(g * pL / rL), cR = RSQRT(g * pR / rR);
  real_t uL = vL[a], uR = vR[a];
  real_t SL, SR;
  if (X->c.flux == 1) { /* Davis bounds */
    SL = rmin(uL - cL, uR - cR);
    SR = rmax(uL + cL, uR + cR);
  } else {              /* Einfeldt-Batten bounds with Roe averages */
    real_t sL = RSQRT(rL), sR = RSQRT(rR);
    real_t HL = (UL[d + 1] + pL) / rL, HR = (UR[d + 1] + pR) / rR;
    real_t q2 = 0.0, vt[3];
    for (int b = 0; b < d; ++b) { vt[b] = (sL * vL[b] + sR * vR[b]) / (sL + sR); q2 += vt[b] * vt[b]; }
    real_t Ht = (sL * HL + sR * HR) / (sL + sR);
    real_t ct2 = (g - 1.0) * (Ht - 0.5 * q2);
    real_t ct = RE(ct2) > 0 ? RSQRT(ct2) : 0.0;
    SL = rmin(uL - cL, vt[a] - ct);
    SR = rmax(uR + cR, vt[a] + ct);
  }
  real_t Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) /
              (rL * (SL - uL) - rR * (SR - uR));
  real_t FL[MAXV], FR[MAXV];
  if (0.0 <= RE(SL)) { euler_flux(X, UL, a, F); return; }
  if (0.0 <= RE(Ss)) {
    euler_flux(X, UL, a, FL);
    real_t fac = rL * (SL - uL) / (SL - Ss);
    real_t Us[MAXV];
    Us[0] = fac;
    for (int b = 0; b < d; ++b) Us[1 + b] = fac * (b == a ? Ss : vL[b]);
    Us[d + 1] = fac * (UL[d + 1] / rL + (Ss - uL) * (Ss + pL / (rL * (SL - uL))));
    for (int v = 0; v < nv; ++v) F[v] = FL[v] + SL * (Us[v] - UL[v]);
    return;
  }
  if (0.0 < RE(SR)) {
    euler_flux(X, UR, a, FR);
    real_t fac = rR * (SR - uR) / (SR - Ss);
    real_t Us[MAXV];
    Us[0] = fac;
    for (int b = 0; b < d; ++b) Us[1 + b] = fac * (b == a ? Ss : vR[b]);
    Us[d + 1] = fac * (UR[d + 1] / rR + (Ss - uR) * (Ss + pR / (rR * (SR - uR))));
    for (int v = 0; v < nv; ++v) F[v] = FR[v] + SR * (Us[v] - UR[v]);
    return;
  }
  euler_flux(X, UR, a, F);
}

/* ------------------------------------------------------------------------ */
/* Uniform-grid right-hand side (Sec. 2.4)                                   */
/* ------------------------------------------------------------------------ */

#define W(v, l, cell) w[((long)(v) * X->N + (l)) * X->ncell + (cell)]

/* Neighbour of `cell` along axis a in direction dir (+1/-1); -1 if the face
 * is a transmissive boundary. */
static long neighbour(const ctx *X, long cell, int a, int dir) {
  long i[3] = {cell % X->nx, (cell / X->nx) % X->ny, cell / (X->nx * X->ny)};
  long n[3] = {X->nx, X->ny, X->nz};
  i[a] += dir;
  if (i[a] < 0 || i[a] >= n[a]) {
    if (X->c.bc[a] == 1) return -1;
    i[a] = (i[a] + n[a]) % n[a];
  }
  return (i[2] * X->ny + i[1]) * X->nx + i[0];
}

/* Volume term V_j = sum_a sum_q f_a(U(xi_q)) dphi_j/dxi_a(xi_q) w_q (eq. dg_term2).
 * A, when not NULL, accumulates the absolute values of the summands (the
 * rounding-error scale of V_j, used by the tests' per-element bounds). */
static void volume_term(const ctx *X, const real_t *w, long cell, real_t V[MAXV][MAXN], double (*A)[MAXN]) {
  for (int v = 0; v < X->nvar; ++v) for (int j = 0; j < X->N; ++j) V[v][j] = 0.0;
  for (int q = 0; q < X->Q; ++q) {
    real_t U[MAXV], F[MAXV];
    for (int v = 0; v < X->nvar; ++v) {
      U[v] = 0.0;
      for (int l = 0; l < X->N; ++l) U[v] += W(v, l, cell) * X->phiV[q][l];
    }
    for (int a = 0; a < X->d; ++a) {
      euler_flux(X, U, a, F);
      for (int v = 0; v < X->nvar; ++v)
        for (int j = 0; j < X->N; ++j) {
          real_t t = F[v] * X->dphiV[a][q][j] * X->wV[q];
          V[v][j] += t;
          if (A) A[v][j] += fabs(RE(t));
        }
    }
  }
}

static void face_trace(const ctx *X, const real_t *w, long cell, int a, int s, int r, real_t *U) {
  for (int v = 0; v < X->nvar; ++v) {
    U[v] = 0.0;
    for (int l = 0; l < X->N; ++l) U[v] += W(v, l, cell) * X->phiF[a][s][r][l];
  }
}

/* Surface term S_j = sum over the 2d faces of the cell of
 * sum_r fbar . n phi_j(xi_r) w_r (eq. dg_term3); fbar is the HLLC flux of the
 * low-side and high-side traces, n the outward normal. */
static void surface_term(const ctx *X, const real_t *w, long cell, real_t S[MAXV][MAXN], double (*A)[MAXN]) {
  for (int v = 0; v < X->nvar; ++v) for (int j = 0; j < X->N; ++j) S[v][j] = 0.0;
  for (int a = 0; a < X->d; ++a)
    for (int s = 0; s < 2; ++s) {
      long nb = neighbour(X, cell, a, s ? +1 : -1);
      for (int r = 0; r < X->Qf; ++r) {
        real_t Uo[MAXV], Un[MAXV], F[MAXV];
        face_trace(X, w, cell, a, s, r, Uo);
        if (nb >= 0) face_trace(X, w, nb, a, 1 - s, r, Un);
        else for (int v = 0; v < X->nvar; ++v) Un[v] = Uo[v];
        if (s) hllc(X, Uo, Un, a, F); /* own cell is the low side  */
        else   hllc(X, Un, Uo, a, F); /* own cell is the high side */
        for (int v = 0; v < X->nvar; ++v)
          for (int j = 0; j < X->N; ++j) {
            real_t t = F[v] * X->phiF[a][s][r][j] * X->wF[r];
            if (s) S[v][j] += t; else S[v][j] -= t;
            if (A) A[v][j] += fabs(RE(t));
          }
      }
    }
}

/* Gravity source (eq. gravity_term): s = (0, rho a, rho v . a) with the
 * external acceleration a = -grad Phi given at the volume nodes, projected
 * onto phi_j with the volume rule: G_j = sum_q s(xi_q) phi_j(xi_q) w_q, the
 * integral over the cell being (|K| / 2^d) G_j. */
static void source_term(const ctx *X, const real_t *w, long cell, real_t G[MAXV][MAXN]) {
  for (int v = 0; v < X->nvar; ++v) for (int j = 0; j < X->N; ++j) G[v][j] = 0.0;
  for (int q = 0; q < X->Q; ++q) {
    real_t U[MAXV], s[MAXV];
    for (int v = 0; v < X->nvar; ++v) {
      U[v] = 0.0;
      for (int l = 0; l < X->N; ++l) U[v] += W(v, l, cell) * X->phiV[q][l];
    }
    s[0] = 0.0;
    real_t work = 0.0;
    for (int a = 0; a < X->d; ++a) {
      double acc = X->c.accel[((long)a * X->Q + q) * X->ncell + cell];
      s[1 + a] = U[0] * acc;   /* rho a     */
      work += U[1 + a] * acc;  /* m . a     */
    }
    s[X->d + 1] = work;
    for (int v = 0; v < X->nvar; ++v)
      for (int j = 0; j < X->N; ++j) G[v][j] += s[v] * X->phiV[q][j] * X->wV[q];
  }
}

/* dw_j/dt = -R = (|K|)^-1 (dx/2)^(d-1) (V_j - S_j) = (2/dx) 2^-d (V_j - S_j),
 * plus |K|^-1 (|K| / 2^d) G_j with a gravity source. */
static void rhs_cell(const ctx *X, const real_t *w, long cell, real_t Lc[MAXV][MAXN]) {
  real_t V[MAXV][MAXN], S[MAXV][MAXN];
  volume_term(X, w, cell, V, NULL);
  surface_term(X, w, cell, S, NULL);
  double fac = 2.0 / X->dx / (double)(1 << X->d);
  for (int v = 0; v < X->nvar; ++v)
    for (int j = 0; j < X->N; ++j) Lc[v][j] = fac * (V[v][j] - S[v][j]);
  if (X->c.accel) {
    real_t G[MAXV][MAXN];
    source_term(X, w, cell, G);
    for (int v = 0; v < X->nvar; ++v)
      for (int j = 0; j < X->N; ++j) Lc[v][j] += G[v][j] / (double)(1 << X->d);
  }
}

static void rhs_all(const ctx *X, const real_t *w, real_t *L) {
  for (long cell = 0; cell < X->ncell; ++cell) {
    real_t Lc[MAXV][MAXN];
    rhs_cell(X, w, cell, Lc);
    for (int v = 0; v < X->nvar; ++v)
      for (int j = 0; j < X->N; ++j) L[((long)v * X->N + j) * X->ncell + cell] = Lc[v][j];
  }
}

/* SSP-RK3 (table RK_3) in its convex-combination (Shu-Osher) form:
 * stage 1: w1 = w0 + dt L(w0); stage 2: w2 = 3/4 w0 + 1/4 (w1 + dt L(w1));
 * stage 3: w3 = 1/3 w0 + 2/3 (w2 + dt L(w2)). */
static const double RK3_A[3] = {0.0, 0.75, 1.0 / 3.0};
static const double RK3_B[3] = {1.0, 0.25, 2.0 / 3.0};

static void rk3_combine(int stage, real_t dt, const real_t *wn, const real_t *wp, const real_t *L,
                        real_t *out, long n) {
  double a = RK3_A[stage - 1], b = RK3_B[stage - 1];
  for (long i = 0; i < n; ++i)
    out[i] = (stage == 1) ? wp[i] + dt * L[i] : a * wn[i] + b * (wp[i] + dt * L[i]);
}

static long state_size(const ctx *X) { return (long)X->nvar * X->N * X->ncell; }

/* ------------------------------------------------------------------------ */
/* Exported functions                                                         */
/* ------------------------------------------------------------------------ */

#ifndef ORC_CS

int orc_sizes(const orc_config *c, long *out /* N, Q, Qf, nvar, ncell, m, nS */) {
  ctx *X = malloc(sizeof(ctx));
  if (!X) return ORC_ENOMEM;
  int st = ctx_init(c, X);
  if (st == ORC_OK) {
    out[0] = X->N; out[1] = X->Q; out[2] = X->Qf; out[3] = X->nvar; out[4] = X->ncell;
    out[5] = X->m; out[6] = X->nS;
  }
  free(X);
  return st;
}

int orc_gauss(int n, double *x, double *w) { if (n < 1 || n > 16) return ORC_EINVAL; gauss_rule(n, x, w); return ORC_OK; }
int orc_gll(int m, double *x, double *w) { if (m < 2 || m > 16) return ORC_EINVAL; gll_rule(m, x, w); return ORC_OK; }
void orc_legendre(int n, double x, double *P, double *dP) { legendre(n, x, P, dP); }

/* Basis exponents e[N][3] in mode order. */
int orc_exponents(const orc_config *c, int *e) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st == ORC_OK) for (int l = 0; l < X->N; ++l) for (int a = 0; a < 3; ++a) e[3 * l + a] = X->e[l][a];
  free(X);
  return st;
}

/* Basis values phi_l at arbitrary reference points xi[npts][3]: out[npts][N]. */
int orc_basis_at(const orc_config *c, long npts, const double *xi, double *out) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st == ORC_OK)
    for (long p = 0; p < npts; ++p)
      for (int l = 0; l < X->N; ++l) out[p * X->N + l] = phi_at(X, l, xi + 3 * p);
  free(X);
  return st;
}

/* Volume quadrature: nodes xi[Q][3], weights w[Q]. */
int orc_volume_rule(const orc_config *c, double *xi, double *wq) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st == ORC_OK)
    for (int q = 0; q < X->Q; ++q) {
      int iq[3] = {q % X->n1, (q / X->n1) % X->n1, q / (X->n1 * X->n1)};
      for (int a = 0; a < 3; ++a) xi[3 * q + a] = (a < X->d) ? X->gx[iq[a]] : 0.0;
      wq[q] = X->wV[q];
    }
  free(X);
  return st;
}

/* Physical coordinates of the projection nodes of every cell: x[ncell][Q][3]. */
int orc_node_coords(const orc_config *c, double *x) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st == ORC_OK)
    for (long cell = 0; cell < X->ncell; ++cell) {
      long i[3] = {cell % X->nx, (cell / X->nx) % X->ny, cell / (X->nx * X->ny)};
      for (int q = 0; q < X->Q; ++q) {
        int iq[3] = {q % X->n1, (q / X->n1) % X->n1, q / (X->n1 * X->n1)};
        for (int a = 0; a < 3; ++a) {
          double v = 0.0;
          if (a < X->d) v = c->x0[a] + (i[a] + 0.5) * X->dx + 0.5 * X->dx * X->gx[iq[a]];
          x[(cell * X->Q + q) * 3 + a] = v;
        }
      }
    }
  free(X);
  return st;
}

/* L2 projection of initial conditions (Sec. 2.3):
 * w_j = 2^-d sum_q u(xi_q) phi_j(xi_q) w_q, with u the conserved state built
 * from primitives prim[ncell][Q][5] = (rho, vx, vy, vz, p) at the nodes. */
int orc_project(const orc_config *c, const double *prim, double *w) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st != ORC_OK) { free(X); return st; }
  double scale = 1.0 / (double)(1 << X->d);
  for (long cell = 0; cell < X->ncell; ++cell) {
    double acc[MAXV][MAXN];
    memset(acc, 0, sizeof(acc));
    for (int q = 0; q < X->Q; ++q) {
      const double *pr = prim + (cell * X->Q + q) * 5;
      double U[MAXV], ke = 0.0;
      U[0] = pr[0];
      for (int b = 0; b < X->d; ++b) { U[1 + b] = pr[0] * pr[1 + b]; ke += pr[1 + b] * pr[1 + b]; }
      U[X->d + 1] = pr[4] / (c->gamma - 1.0) + 0.5 * pr[0] * ke;
      for (int v = 0; v < X->nvar; ++v)
        for (int j = 0; j < X->N; ++j) acc[v][j] += U[v] * X->phiV[q][j] * X->wV[q];
    }
    for (int v = 0; v < X->nvar; ++v)
      for (int j = 0; j < X->N; ++j) w[((long)v * X->N + j) * X->ncell + cell] = scale * acc[v][j];
  }
  free(X);
  return ORC_OK;
}

/* Conserved state at reference points xi[npts][3] of every cell:
 * out[ncell][npts][nvar]. */
int orc_eval_points(const orc_config *c, const double *w, long npts, const double *xi, double *out) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st != ORC_OK) { free(X); return st; }
  double *ph = malloc(sizeof(double) * npts * X->N);
  for (long p = 0; p < npts; ++p)
    for (int l = 0; l < X->N; ++l) ph[p * X->N + l] = phi_at(X, l, xi + 3 * p);
  for (long cell = 0; cell < X->ncell; ++cell)
    for (long p = 0; p < npts; ++p)
      for (int v = 0; v < X->nvar; ++v) {
        double s = 0.0;
        for (int l = 0; l < X->N; ++l) s += W(v, l, cell) * ph[p * X->N + l];
        out[(cell * npts + p) * X->nvar + v] = s;
      }
  free(ph); free(X);
  return ORC_OK;
}

/* Numerical flux at one point (for unit tests of the Riemann solver). */
int orc_hllc(const orc_config *c, const double *UL, const double *UR, int axis, double *F) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st == ORC_OK) hllc(X, UL, UR, axis, F);
  free(X);
  return st;
}

int orc_euler_flux(const orc_config *c, const double *U, int axis, double *F) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st == ORC_OK) euler_flux(X, U, axis, F);
  free(X);
  return st;
}

/* L = dw/dt for the whole grid. */
int orc_rhs(const orc_config *c, const double *w, double *L) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st == ORC_OK) rhs_all(X, w, L);
  free(X);
  return st;
}

/* L for a list of cells only: out[nvar][N][ncells]. */
int orc_rhs_cells(const orc_config *c, const double *w, long ncells, const long *cells, double *out) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st != ORC_OK) { free(X); return st; }
  for (long i = 0; i < ncells; ++i) {
    if (cells[i] < 0 || cells[i] >= X->ncell) { free(X); return ORC_EINVAL; }
    double Lc[MAXV][MAXN];
    rhs_cell(X, w, cells[i], Lc);
    for (int v = 0; v < X->nvar; ++v)
      for (int j = 0; j < X->N; ++j) out[((long)v * X->N + j) * ncells + i] = Lc[v][j];
  }
  free(X);
  return ORC_OK;
}

/* Volume and surface terms of a list of cells, scaled like L:
 * V_out = fac V, S_out = fac S, each [nvar][N][ncells], so that L = V_out - S_out.
 * Their magnitudes bound the rounding error of L (tests use them as the
 * conditioning scale of the right-hand side).  A_out (may be NULL) receives
 * fac times the sum of the absolute values of every summand of V and S: the
 * per-element rounding-error scale of L (a sum's rounding error is bounded by
 * a multiple of the unit roundoff times the sum of its terms' magnitudes). */
int orc_terms_cells(const orc_config *c, const double *w, long ncells, const long *cells, double *V_out,
                    double *S_out, double *A_out) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st != ORC_OK) { free(X); return st; }
  double fac = 2.0 / X->dx / (double)(1 << X->d);
  for (long i = 0; i < ncells; ++i) {
    if (cells[i] < 0 || cells[i] >= X->ncell) { free(X); return ORC_EINVAL; }
    double Vc[MAXV][MAXN], Sc[MAXV][MAXN], Ac[MAXV][MAXN];
    memset(Ac, 0, sizeof(Ac));
    volume_term(X, w, cells[i], Vc, Ac);
    surface_term(X, w, cells[i], Sc, Ac);
    for (int v = 0; v < X->nvar; ++v)
      for (int j = 0; j < X->N; ++j) {
        V_out[((long)v * X->N + j) * ncells + i] = fac * Vc[v][j];
        S_out[((long)v * X->N + j) * ncells + i] = fac * Sc[v][j];
        if (A_out) A_out[((long)v * X->N + j) * ncells + i] = fac * Ac[v][j];
      }
  }
  free(X);
  return ORC_OK;
}

/* Volume and surface terms separately for one cell (unit tests). */
int orc_terms_cell(const orc_config *c, const double *w, long cell, double *V, double *S) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st == ORC_OK) {
    double Vc[MAXV][MAXN], Sc[MAXV][MAXN];
    volume_term(X, w, cell, Vc, NULL);
    surface_term(X, w, cell, Sc, NULL);
    for (int v = 0; v < X->nvar; ++v)
      for (int j = 0; j < X->N; ++j) { V[v * X->N + j] = Vc[v][j]; S[v * X->N + j] = Sc[v][j]; }
  }
  free(X);
  return st;
}

/* Global time step (eq. time_step; eq. time_step_pos when the positivity
 * limiter is on): min over cells of CFL f_k / sum_a (|v_a| + c)/dx, from the
 * cell means. */
int orc_max_dt(const orc_config *c, const double *w, double *dt_out) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st != ORC_OK) { free(X); return st; }
  double fk = 1.0 / (2.0 * X->k + 1.0);
  if (c->positivity && X->lw[0] / 2.0 < fk) fk = X->lw[0] / 2.0;
  double dt = INFINITY;
  for (long cell = 0; cell < X->ncell; ++cell) {
    double U[MAXV];
    for (int v = 0; v < X->nvar; ++v) U[v] = W(v, 0, cell);
    double p = pressure(X, U);
    double cs = sqrt(c->gamma * p / U[0]);
    double rate = 0.0;
    for (int a = 0; a < X->d; ++a) rate += (fabs(U[1 + a] / U[0]) + cs) / X->dx;
    double dtc = c->cfl * fk / rate;
    if (dtc < dt) dt = dtc;
    if (c->accel) {
      /* gravity step (Sec. 2.5): dt <= c / (sqrt(2 gamma (gamma-1)) |grad Phi|),
       * |grad Phi| the largest over the cell's volume nodes */
      double amax = 0.0;
      for (int q = 0; q < X->Q; ++q) {
        double a2 = 0.0;
        for (int a = 0; a < X->d; ++a) {
          double g = c->accel[((long)a * X->Q + q) * X->ncell + cell];
          a2 += g * g;
        }
        if (sqrt(a2) > amax) amax = sqrt(a2);
      }
      if (amax > 0.0) {
        double dtg = cs / (sqrt(2.0 * c->gamma * (c->gamma - 1.0)) * amax);
        if (dtg < dt) dt = dtg;
      }
    }
  }
  *dt_out = dt;
  free(X);
  return ORC_OK;
}

/* Convex-combination step of SSP-RK3 alone (for the time-integrator pins). */
void orc_rk3_combine(int stage, double dt, const double *wn, const double *wp, const double *L,
                     double *out, long n) {
  rk3_combine(stage, dt, wn, wp, L, out, n);
}

/* One SSP-RK3 stage: w_out = a w_n + b (w_prev + dt L(w_prev)). */
int orc_rk3_stage(const orc_config *c, int stage, double dt, const double *wn, const double *wp,
                  double *out) {
  if (stage < 1 || stage > 3) return ORC_EINVAL;
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st != ORC_OK) { free(X); return st; }
  long n = state_size(X);
  double *L = malloc(sizeof(double) * n);
  rhs_all(X, wp, L);
  rk3_combine(stage, dt, wn, wp, L, out, n);
  free(L); free(X);
  return ORC_OK;
}

/* General explicit Runge-Kutta method given by its Butcher tableau (App. D:
 * w^{n+1} = w^n + dt sum_i b_i k_i, k_i = L(w^n + dt sum_{j<i} a_ij k_j) with
 * L = -R).  The main loop limits after every stage (Sec. 4.5); as for RK_3,
 * the values limited are the stage values of the tableau's Shu-Osher form
 * with a derivative term on the previous stage only:
 *   Y_0 = w^n,  Y_m = sum_{j<m} alpha_mj Y_j + beta_m dt L(Y_{m-1}),  m = 1..s,
 * and w^{n+1} = Y_s.  Writing every Y_j as w^n + dt sum_l Abar_jl k_l (Abar
 * is A with b appended as row s) and comparing the coefficients of k_l:
 *   beta_m = Abar_{m,m-1},
 *   Abar_{m,l} = sum_{j=l+1}^{m-1} alpha_mj Abar_{j,l}     (l = m-2 .. 0),
 * a triangular system for alpha_{m,1..m-1} with diagonal Abar_{l+1,l};
 * alpha_m0 = 1 - sum of the others (the coefficients of w^n agree).  The
 * form is unique when the subdiagonal of Abar is nonzero.  Without limiting
 * it is the tableau's method exactly; for table RK_3 it gives 3/4, 1/4 and
 * 1/3, 2/3, the form rk3_combine uses.  A is s x s row-major (only the strict
 * lower triangle may be nonzero), alpha is (s+1) x (s+1) row-major. */
#define MAXST 8
static int shu_osher(int s, const double *A, const double *b, double *alpha, double *beta) {
  if (s < 1 || s >= MAXST) return ORC_EINVAL;
  double Ab[MAXST][MAXST];
  for (int i = 0; i <= s; ++i)
    for (int j = 0; j < s; ++j) {
      Ab[i][j] = (i < s) ? A[i * s + j] : b[j];
      if (i < s && j >= i && Ab[i][j] != 0.0) return ORC_EINVAL; /* not explicit */
    }
  for (int l = 0; l < s; ++l)
    if (Ab[l + 1][l] == 0.0) return ORC_EINVAL;
  for (int i = 0; i < (s + 1) * (s + 1); ++i) alpha[i] = 0.0;
  beta[0] = 0.0;
  for (int m = 1; m <= s; ++m) {
    double *am = alpha + m * (s + 1);
    beta[m] = Ab[m][m - 1];
    for (int l = m - 2; l >= 0; --l) {
      double r = Ab[m][l];
      for (int j = l + 2; j <= m - 1; ++j) r -= am[j] * Ab[j][l];
      am[l + 1] = r / Ab[l + 1][l];
    }
    double rest = 0.0;
    for (int j = 1; j <= m - 1; ++j) rest += am[j];
    am[0] = 1.0 - rest;
  }
  return ORC_OK;
}

/* Y_m from Y_0..Y_{m-1} (contiguous, n values each) and L = L(Y_{m-1}). */
static void tableau_combine(int s, const double *alpha, const double *beta, int m, double dt, const double *Y,
                            const double *L, double *out, long n) {
  const double *am = alpha + m * (s + 1);
  for (long i = 0; i < n; ++i) {
    double acc = 0.0;
    for (int j = 0; j < m; ++j) acc += am[j] * Y[(long)j * n + i];
    out[i] = acc + beta[m] * dt * L[i];
  }
}

int orc_tableau_form(int s, const double *A, const double *b, double *alpha, double *beta) {
  return shu_osher(s, A, b, alpha, beta);
}

/* Stage value Y_m (1 <= m <= s) of the combination alone (time-integrator
 * pins with a scalar ODE). */
int orc_tableau_combine(int s, const double *A, const double *b, int m, double dt, const double *Y,
                        const double *L, double *out, long n) {
  double alpha[MAXST * MAXST], beta[MAXST];
  int st = shu_osher(s, A, b, alpha, beta);
  if (st != ORC_OK) return st;
  if (m < 1 || m > s) return ORC_EINVAL;
  tableau_combine(s, alpha, beta, m, dt, Y, L, out, n);
  return ORC_OK;
}

/* Stage value Y_m of the DG system: Y holds Y_0..Y_{m-1}, L is taken at Y_{m-1}. */
int orc_tableau_stage(const orc_config *c, int s, const double *A, const double *b, int m, double dt,
                      const double *Y, double *out) {
  double alpha[MAXST * MAXST], beta[MAXST];
  int st = shu_osher(s, A, b, alpha, beta);
  if (st != ORC_OK) return st;
  if (m < 1 || m > s) return ORC_EINVAL;
  ctx *X = malloc(sizeof(ctx));
  st = ctx_init(c, X);
  if (st != ORC_OK) { free(X); return st; }
  long n = state_size(X);
  double *L = malloc(sizeof(double) * n);
  rhs_all(X, Y + (long)(m - 1) * n, L);
  tableau_combine(s, alpha, beta, m, dt, Y, L, out, n);
  free(L); free(X);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Limiters (Sec. 3)                                                          */
/* ------------------------------------------------------------------------ */

/* minmod of Sec. 3.1 and its TVB-bounded form of Sec. 3.3: a is returned
 * unchanged when |a| <= M dx^2 = Mtilde dx. */
static double minmod3(double a, double b, double c) {
  if (a > 0 && b > 0 && c > 0) return fmin(a, fmin(b, c));
  if (a < 0 && b < 0 && c < 0) return -fmin(-a, fmin(-b, -c));
  return 0.0;
}

static double minmod_b(double a, double b, double c, double bound) {
  if (fabs(a) <= bound) return a;
  return minmod3(a, b, c);
}

/* Component-wise limiter (eq. comp_limiter, eq. comp_limiter_applied): for
 * every conserved component i the slopes sqrt(3) w_{1+a,i} are limited
 * against beta times the differences of the neighbouring means; if any slope
 * changes, the component keeps only its mean and the limited slopes.
 * `nbm` gives the neighbour means: nbm[(2a+s)*nvar*ncell + i*ncell + cell],
 * s = 0 the low (west/south/bottom) neighbour, s = 1 the high one. */
static void slope_limit(const ctx *X, double *w, const double *nbm, const double *dxc, const unsigned char *skip) {
  long nc = X->ncell;
  const double r3 = sqrt(3.0);
  for (long cell = 0; cell < nc; ++cell) {
    if (skip && skip[cell]) continue;
    double bound = X->c.mtilde * dxc[cell];
    for (int i = 0; i < X->nvar; ++i) {
      double mean = W(i, 0, cell);
      double mt[3];
      int limited = 0;
      for (int a = 0; a < X->d; ++a) {
        double mW = nbm[((long)(2 * a + 0) * X->nvar + i) * nc + cell];
        double mE = nbm[((long)(2 * a + 1) * X->nvar + i) * nc + cell];
        double A = r3 * W(i, 1 + a, cell);
        double m = minmod_b(A, X->c.beta * (mean - mW), X->c.beta * (mE - mean), bound);
        mt[a] = m;
        if (m != A) limited = 1;
      }
      if (limited) {
        for (int a = 0; a < X->d; ++a) W(i, 1 + a, cell) = mt[a] / r3;
        for (int l = X->d + 1; l < X->N; ++l) W(i, l, cell) = 0.0;
      }
    }
  }
}

/* Right eigenvectors (columns of R) and left eigenvectors (rows of L = R^-1)
 * of the flux Jacobian A_a = d f_a / d u at the state U, as App. E lists them
 * for a = x, y, z: eigenvalues v_a - c, v_a, v_a + c and two shear waves at
 * v_a; k = |v|^2 / 2 (the text prints v_3 cubed in k, a slip), the specific
 * stagnation enthalpy h = c^2 / (gamma - 1) + k, gamma_1 = gamma - 1,
 * phi = gamma_1 k and b = 1 / (2 c^2) (the text calls it beta).  In 2D the
 * matrices are those of 3D at v_3 = 0 without the row and column of m_z and
 * without the z shear wave, which decouple there.  R and L are nvar x nvar,
 * row-major.  Returns 0 if U has no positive density and pressure. */
static int eigvecs(const ctx *X, const double *U, int a, double *R, double *L) {
  int d = X->d, nv = X->nvar;
  double g = X->c.gamma, g1 = g - 1.0;
  double rho = U[0];
  double v[3] = {0.0, 0.0, 0.0};
  for (int b = 0; b < d; ++b) v[b] = U[1 + b] / rho;
  double k = 0.5 * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  double p = g1 * (U[d + 1] - rho * k);
  if (!(rho > 0.0) || !(p > 0.0)) return 0;
  double c = sqrt(g * p / rho);
  double h = c * c / g1 + k;
  double phi = g1 * k, b = 1.0 / (2.0 * c * c);
  double v1 = v[0], v2 = v[1], v3 = v[2];
  double R5[5][5], L5[5][5];
  if (a == 0) {
    double r[5][5] = {{1, 1, 1, 0, 0},
                      {v1 - c, v1, v1 + c, 0, 0},
                      {v2, v2, v2, -1, 0},
                      {v3, v3, v3, 0, 1},
                      {h - c * v1, k, h + c * v1, -v2, v3}};
    double l[5][5] = {{b * (phi + c * v1), -b * (g1 * v1 + c), -b * g1 * v2, -b * g1 * v3, b * g1},
                      {1 - 2 * b * phi, 2 * b * g1 * v1, 2 * b * g1 * v2, 2 * b * g1 * v3, -2 * b * g1},
                      {b * (phi - c * v1), -b * (g1 * v1 - c), -b * g1 * v2, -b * g1 * v3, b * g1},
                      {v2, 0, -1, 0, 0},
                      {-v3, 0, 0, 1, 0}};
    memcpy(R5, r, sizeof(r)); memcpy(L5, l, sizeof(l));
  } else if (a == 1) {
    double r[5][5] = {{1, 1, 1, 0, 0},
                      {v1, v1, v1, 1, 0},
                      {v2 - c, v2, v2 + c, 0, 0},
                      {v3, v3, v3, 0, -1},
                      {h - c * v2, k, h + c * v2, v1, -v3}};
    double l[5][5] = {{b * (phi + c * v2), -b * g1 * v1, -b * (g1 * v2 + c), -b * g1 * v3, b * g1},
                      {1 - 2 * b * phi, 2 * b * g1 * v1, 2 * b * g1 * v2, 2 * b * g1 * v3, -2 * b * g1},
                      {b * (phi - c * v2), -b * g1 * v1, -b * (g1 * v2 - c), -b * g1 * v3, b * g1},
                      {-v1, 1, 0, 0, 0},
                      {v3, 0, 0, -1, 0}};
    memcpy(R5, r, sizeof(r)); memcpy(L5, l, sizeof(l));
  } else {
    double r[5][5] = {{1, 1, 1, 0, 0},
                      {v1, v1, v1, -1, 0},
                      {v2, v2, v2, 0, 1},
                      {v3 - c, v3, v3 + c, 0, 0},
                      {h - c * v3, k, h + c * v3, -v1, v2}};
    double l[5][5] = {{b * (phi + c * v3), -b * g1 * v1, -b * g1 * v2, -b * (g1 * v3 + c), b * g1},
                      {1 - 2 * b * phi, 2 * b * g1 * v1, 2 * b * g1 * v2, 2 * b * g1 * v3, -2 * b * g1},
                      {b * (phi - c * v3), -b * g1 * v1, -b * g1 * v2, -b * (g1 * v3 - c), b * g1},
                      {v1, -1, 0, 0, 0},
                      {-v2, 0, 1, 0, 0}};
    memcpy(R5, r, sizeof(r)); memcpy(L5, l, sizeof(l));
  }
  /* conserved components and waves kept: all in 3D; in 2D rho, m_x, m_y, E
   * and the waves v-c, v, v+c and the in-plane shear wave */
  static const int cons2[4] = {0, 1, 2, 4}, wave2[4] = {0, 1, 2, 3};
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nv; ++j) {
      int ci = d == 3 ? i : cons2[i], wj = d == 3 ? j : wave2[j];
      int wi = d == 3 ? i : wave2[i], cj = d == 3 ? j : cons2[j];
      R[i * nv + j] = R5[ci][wj];
      L[i * nv + j] = L5[wi][cj];
    }
  return 1;
}

/* Characteristic limiter (Sec. 3.2, eq. char_limiter, with the bounded
 * minmod of Sec. 3.3): in each direction a the slopes w_{1+a} and the
 * differences of the neighbouring means go to characteristic variables with
 * L_a of the cell mean; sqrt(3) c_{1+a} is limited against beta L_a (w_1^K -
 * w_1^W) and beta L_a (w_1^E - w_1^K), field by field.  If any characteristic
 * slope changes, every component keeps its mean and the slopes R_a c~ (the
 * text writes R_x for the y and z directions as well; the inverses R_y, R_z
 * of L_y, L_z are meant), and the higher modes are dropped.  A cell whose mean
 * has no real sound speed is left as it is (the positivity limiter reports
 * it).  Same neighbour means as slope_limit. */
static void char_limit(const ctx *X, double *w, const double *nbm, const double *dxc, const unsigned char *skip) {
  long nc = X->ncell;
  int d = X->d, nv = X->nvar;
  const double r3 = sqrt(3.0);
  for (long cell = 0; cell < nc; ++cell) {
    if (skip && skip[cell]) continue;
    double bound = X->c.mtilde * dxc[cell];
    double U[MAXV];
    for (int i = 0; i < nv; ++i) U[i] = W(i, 0, cell);
    double R[3][MAXV * MAXV], L[MAXV * MAXV], ct[3][MAXV];
    int ok = 1, limited = 0;
    for (int a = 0; a < d && ok; ++a) {
      ok = eigvecs(X, U, a, R[a], L);
      if (!ok) break;
      double dW[MAXV], dE[MAXV];
      for (int i = 0; i < nv; ++i) {
        dW[i] = U[i] - nbm[((long)(2 * a + 0) * nv + i) * nc + cell];
        dE[i] = nbm[((long)(2 * a + 1) * nv + i) * nc + cell] - U[i];
      }
      for (int p = 0; p < nv; ++p) {
        double cs = 0.0, cw = 0.0, ce = 0.0;
        for (int i = 0; i < nv; ++i) {
          cs += L[p * nv + i] * W(i, 1 + a, cell);
          cw += L[p * nv + i] * dW[i];
          ce += L[p * nv + i] * dE[i];
        }
        double A = r3 * cs;
        double m = minmod_b(A, X->c.beta * cw, X->c.beta * ce, bound);
        ct[a][p] = m;
        if (m != A) limited = 1;
      }
    }
    if (!ok || !limited) continue;
    for (int a = 0; a < d; ++a)
      for (int i = 0; i < nv; ++i) {
        double s2 = 0.0;
        for (int p = 0; p < nv; ++p) s2 += R[a][i * nv + p] * (ct[a][p] / r3);
        W(i, 1 + a, cell) = s2;
      }
    for (int i = 0; i < nv; ++i)
      for (int l = d + 1; l < X->N; ++l) W(i, l, cell) = 0.0;
  }
}

/* App. E matrices at U for tests: R, L (nvar x nvar row-major).  Returns
 * ORC_EINVAL for a state without positive density and pressure. */
int orc_eigvecs(const orc_config *c, const double *U, int a, double *R, double *L) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st == ORC_OK && (a < 0 || a >= X->d || !eigvecs(X, U, a, R, L))) st = ORC_EINVAL;
  free(X);
  return st;
}

/* Root tau in [0,1] of p(ubar + tau (u - ubar)) = eps (eq. p_positivity, read
 * with the high-order part u - ubar scaled): (E - eps/(g-1)) rho - |m|^2/2 is
 * quadratic in tau.  Cancellation-free quadratic formula, then two Newton
 * steps; bisection if the discriminant comes out negative. */
static double tau_root(const ctx *X, const double *Ub, const double *Uq) {
  int d = X->d;
  double epsp = X->c.eps / (X->c.gamma - 1.0);
  double dr = Uq[0] - Ub[0], dE = Uq[d + 1] - Ub[d + 1];
  double dm2 = 0.0, mdm = 0.0, mb2 = 0.0;
  for (int b = 0; b < d; ++b) {
    double dm = Uq[1 + b] - Ub[1 + b];
    dm2 += dm * dm; mdm += Ub[1 + b] * dm; mb2 += Ub[1 + b] * Ub[1 + b];
  }
  double A = dE * dr - 0.5 * dm2;
  double B = dE * Ub[0] + (Ub[d + 1] - epsp) * dr - mdm;
  double C = (Ub[d + 1] - epsp) * Ub[0] - 0.5 * mb2;
  double t;
  double disc = B * B - 4.0 * A * C;
  if (A == 0.0) {
    t = -C / B;
  } else if (disc >= 0.0) {
    double qq = -0.5 * (B + copysign(sqrt(disc), B));
    double r1 = qq / A, r2 = (qq != 0.0) ? C / qq : r1;
    int ok1 = r1 >= 0.0 && r1 <= 1.0, ok2 = r2 >= 0.0 && r2 <= 1.0;
    t = (ok1 && ok2) ? fmin(r1, r2) : ok1 ? r1 : ok2 ? r2 : 0.0;
  } else {
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 60; ++it) {
      double mid = 0.5 * (lo + hi);
      if ((A * mid + B) * mid + C > 0.0) lo = mid; else hi = mid;
    }
    t = lo;
  }
  for (int it = 0; it < 2; ++it) {
    double gval = (A * t + B) * t + C, gd = 2.0 * A * t + B;
    if (gd != 0.0) t -= gval / gd;
  }
  if (t < 0.0) t = 0.0;
  if (t > 1.0) t = 1.0;
  return t;
}

/* Positivity limiter (Sec. 3.4) on every cell; extra check points of
 * individual cells are passed as (xcnt[cell], xphi) (the coarse side of
 * hanging faces, Sec. 4.4), nx_pts per cell with basis values xphi[cell][..][N].
 * Returns the number of cells whose mean density or mean pressure is <= eps. */
static long positivity_limit(const ctx *X, double *w, const int *xcnt, const double *xphi, int xmax,
                             const unsigned char *skip) {
  long bad = 0;
  int d = X->d, nv = X->nvar;
  double eps = X->c.eps;
  for (long cell = 0; cell < X->ncell; ++cell) {
    if (skip && skip[cell]) continue;
    double Ub[MAXV];
    for (int v = 0; v < nv; ++v) Ub[v] = W(v, 0, cell);
    double pb = pressure(X, Ub);
    if (!(Ub[0] > eps) || !(pb > eps)) { ++bad; continue; }
    int np = X->nS + (xcnt ? xcnt[cell] : 0);
    /* density */
    double rmin = INFINITY;
    for (int s = 0; s < np; ++s) {
      const double *ph = (s < X->nS) ? X->phiS[s] : xphi + ((long)cell * xmax + (s - X->nS)) * X->N;
      double r = 0.0;
      for (int l = 0; l < X->N; ++l) r += W(0, l, cell) * ph[l];
      if (r < rmin) rmin = r;
    }
    double th1 = (Ub[0] == rmin) ? 1.0 : fmin(fabs((Ub[0] - eps) / (Ub[0] - rmin)), 1.0);
    for (int l = 1; l < X->N; ++l) W(0, l, cell) *= th1;
    /* pressure */
    double th2 = 1.0;
    for (int s = 0; s < np; ++s) {
      const double *ph = (s < X->nS) ? X->phiS[s] : xphi + ((long)cell * xmax + (s - X->nS)) * X->N;
      double Uq[MAXV];
      for (int v = 0; v < nv; ++v) {
        Uq[v] = 0.0;
        for (int l = 0; l < X->N; ++l) Uq[v] += W(v, l, cell) * ph[l];
      }
      double ke = 0.0;
      for (int b = 0; b < d; ++b) ke += Uq[1 + b] * Uq[1 + b] / Uq[0];
      double pq = (X->c.gamma - 1.0) * (Uq[d + 1] - 0.5 * ke);
      if (pq < eps) {
        double t = tau_root(X, Ub, Uq);
        if (t < th2) th2 = t;
      }
    }
    for (int v = 0; v < nv; ++v)
      for (int l = 1; l < X->N; ++l) W(v, l, cell) *= th2;
  }
  return bad;
}

/* Neighbour means on the uniform grid (periodic or transmissive). */
static void uniform_neighbour_means(const ctx *X, const double *w, double *nbm) {
  long nc = X->ncell;
  for (int a = 0; a < X->d; ++a)
    for (int s = 0; s < 2; ++s)
      for (long cell = 0; cell < nc; ++cell) {
        long nb = neighbour(X, cell, a, s ? +1 : -1);
        if (nb < 0) nb = cell;
        for (int i = 0; i < X->nvar; ++i)
          nbm[((long)(2 * a + s) * X->nvar + i) * nc + cell] = W(i, 0, nb);
      }
}

/* Slope limiter, then positivity limiter, in place, on the cells that `skip`
 * does not mark (all cells if skip is NULL).  The neighbour means are read
 * before any cell is limited; the limiters never change a mean, so limiting a
 * subset of the cells gives those cells exactly what limiting all would. */
static int limit_masked(const orc_config *c, double *w, const unsigned char *skip) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st != ORC_OK) { free(X); return st; }
  long bad = 0;
  if (c->limiter) {
    double *nbm = malloc(sizeof(double) * 2 * X->d * X->nvar * X->ncell);
    double *dxc = malloc(sizeof(double) * X->ncell);
    for (long i = 0; i < X->ncell; ++i) dxc[i] = X->dx;
    uniform_neighbour_means(X, w, nbm);
    if (c->limiter == 2)
      char_limit(X, w, nbm, dxc, skip);
    else
      slope_limit(X, w, nbm, dxc, skip);
    free(nbm); free(dxc);
  }
  if (c->positivity) bad = positivity_limit(X, w, NULL, NULL, 0, skip);
  free(X);
  return bad ? ORC_ENEGATIVE : ORC_OK;
}

/* Slope limiter, then positivity limiter, in place (main loop, Sec. 4.5).
 * Returns ORC_ENEGATIVE if some cell mean is not positive. */
int orc_limit(const orc_config *c, double *w) { return limit_masked(c, w, NULL); }

/* The same on the listed cells only (flat indices); the other cells of w are
 * left as they are.  For sampled checks of large grids. */
int orc_limit_cells(const orc_config *c, double *w, long ncells, const long *cells) {
  long nc = 1;
  for (int a = 0; a < c->dim; ++a) nc *= c->n[a];
  unsigned char *skip = malloc(nc);
  if (!skip) return ORC_ENOMEM;
  memset(skip, 1, nc);
  for (long i = 0; i < ncells; ++i) {
    if (cells[i] < 0 || cells[i] >= nc) { free(skip); return ORC_EINVAL; }
    skip[cells[i]] = 0;
  }
  int st = limit_masked(c, w, skip);
  free(skip);
  return st;
}

/* Positivity check points S in reference coordinates: xi[nS][3]. */
int orc_positivity_points(const orc_config *c, double *xi) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st == ORC_OK) {
    int s = 0;
    for (int a = 0; a < X->d; ++a) {
      int t[2]; tangential(X->d, a, t);
      for (int r = 0; r < X->m; ++r)
        for (int q = 0; q < X->Qf; ++q) {
          int ir[2] = {q % X->n1, q / X->n1};
          double p[3] = {0, 0, 0};
          p[a] = X->lx[r];
          for (int j = 0; j < X->d - 1; ++j) p[t[j]] = X->gx[ir[j]];
          for (int b = 0; b < 3; ++b) xi[3 * s + b] = p[b];
          ++s;
        }
    }
  }
  free(X);
  return st;
}

/* ------------------------------------------------------------------------ */
/* Static 2:1 refined box (Sec. 4 hanging-face quadrature, Sec. 4.4)         */
/*                                                                            */
/* The base grid n[] is the coarse block; the base cells in [lo, hi) are a    */
/* hole covered by a fine block of 2(hi - lo) cells per axis with half the    */
/* edge length.  State layout: coarse block [nvar][N][ncoarse] (hole cells    */
/* present, ignored) followed by the fine block [nvar][N][nfine].            */
/* A coarse face next to the fine block is integrated with the quadrature     */
/* points of the 2^(d-1) fine faces covering it: the coarse trace is taken at */
/* the mapped coordinates (eta + sigma)/2 and the flux is lifted into the     */
/* coarse cell with weight w_r / 2^(d-1).                                     */
/* ------------------------------------------------------------------------ */

typedef struct {
  ctx Xc, Xf;            /* tables with the coarse / fine block geometry      */
  int lo[3], hi[3];
  long nf[3];
  long ncc, ncf;
  int nsub;              /* 2^(d-1) fine faces per coarse face               */
  double phiH[3][2][4][MAXQF][MAXN]; /* coarse basis at hanging-face nodes   */
  double cmean[8][MAXN]; /* mean of phi_l over child subcell c (first row of P_c) */
} amr;

static int amr_init(const orc_config *c, amr *M) {
  if (c->accel) return ORC_EINVAL; /* gravity on uniform grids only */
  int st = ctx_init(c, &M->Xc);
  if (st != ORC_OK) return st;
  int d = M->Xc.d;
  for (int a = 0; a < 3; ++a) { M->lo[a] = c->refine_lo[a]; M->hi[a] = c->refine_hi[a]; M->nf[a] = 1; }
  long nb[3] = {M->Xc.nx, M->Xc.ny, M->Xc.nz};
  for (int a = 0; a < d; ++a) {
    if (M->lo[a] < 1 || M->hi[a] > nb[a] - 1 || M->hi[a] <= M->lo[a]) return ORC_EINVAL;
    M->nf[a] = 2L * (M->hi[a] - M->lo[a]);
  }
  M->Xf = M->Xc;
  M->Xf.nx = M->nf[0]; M->Xf.ny = M->nf[1]; M->Xf.nz = (d == 3) ? M->nf[2] : 1;
  M->Xf.ncell = M->Xf.nx * M->Xf.ny * M->Xf.nz;
  M->Xf.dx = 0.5 * M->Xc.dx;
  for (int a = 0; a < 3; ++a) M->Xf.c.bc[a] = 0;
  M->ncc = M->Xc.ncell; M->ncf = M->Xf.ncell;
  M->nsub = 1 << (d - 1);
  const ctx *X = &M->Xc;
  for (int a = 0; a < d; ++a) {
    int t[2]; tangential(d, a, t);
    for (int s = 0; s < 2; ++s)
      for (int sub = 0; sub < M->nsub; ++sub)
        for (int r = 0; r < X->Qf; ++r) {
          int ir[2] = {r % X->n1, r / X->n1};
          double xi[3] = {0, 0, 0};
          xi[a] = s ? 1.0 : -1.0;
          for (int j = 0; j < d - 1; ++j) {
            double sig = ((sub >> j) & 1) ? 1.0 : -1.0;
            xi[t[j]] = 0.5 * (X->gx[ir[j]] + sig);
          }
          for (int l = 0; l < X->N; ++l) M->phiH[a][s][sub][r][l] = phi_at(X, l, xi);
        }
  }
  /* child means: 2^-d int phi_l((xi + c)/2) dxi with (k+1)^d Gauss points */
  for (int ch = 0; ch < (1 << d); ++ch)
    for (int l = 0; l < X->N; ++l) {
      double acc = 0.0;
      for (int q = 0; q < X->Q; ++q) {
        int iq[3] = {q % X->n1, (q / X->n1) % X->n1, q / (X->n1 * X->n1)};
        double xi[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) xi[a] = 0.5 * (X->gx[iq[a]] + (((ch >> a) & 1) ? 1.0 : -1.0));
        acc += phi_at(X, l, xi) * X->wV[q];
      }
      M->cmean[ch][l] = acc / (double)(1 << d);
    }
  return ORC_OK;
}

static void unflat(const ctx *X, long cell, long *i) {
  i[0] = cell % X->nx; i[1] = (cell / X->nx) % X->ny; i[2] = cell / (X->nx * X->ny);
}
static long flat(const ctx *X, const long *i) { return (i[2] * X->ny + i[1]) * X->nx + i[0]; }

static int amr_in_hole(const amr *M, const long *i) {
  for (int a = 0; a < M->Xc.d; ++a)
    if (i[a] < M->lo[a] || i[a] >= M->hi[a]) return 0;
  return 1;
}

/* coarse base-cell neighbour index along a (periodic), or -1 at a transmissive wall */
static int amr_coarse_nb(const amr *M, const long *i, int a, int dir, long *j) {
  long n[3] = {M->Xc.nx, M->Xc.ny, M->Xc.nz};
  for (int b = 0; b < 3; ++b) j[b] = i[b];
  j[a] += dir;
  if (j[a] < 0 || j[a] >= n[a]) {
    if (M->Xc.c.bc[a] == 1) return -1;
    j[a] = (j[a] + n[a]) % n[a];
  }
  return 0;
}

static void amr_state(const ctx *X, const double *wb, long cell, const double *ph, double *U) {
  for (int v = 0; v < X->nvar; ++v) {
    double s = 0.0;
    for (int l = 0; l < X->N; ++l) s += wb[((long)v * X->N + l) * X->ncell + cell] * ph[l];
    U[v] = s;
  }
}

/* Surface term of a coarse cell, hanging faces included. */
static void amr_surface_coarse(const amr *M, const double *wc, const double *wf, long cell, double S[MAXV][MAXN],
                               double (*A)[MAXN]) {
  const ctx *X = &M->Xc, *Y = &M->Xf;
  int d = X->d;
  for (int v = 0; v < X->nvar; ++v) for (int j = 0; j < X->N; ++j) S[v][j] = 0.0;
  long i[3]; unflat(X, cell, i);
  for (int a = 0; a < d; ++a) {
    int t[2]; tangential(d, a, t);
    for (int s = 0; s < 2; ++s) {
      long j[3];
      int wall = amr_coarse_nb(M, i, a, s ? 1 : -1, j);
      if (wall == 0 && amr_in_hole(M, j)) {
        for (int sub = 0; sub < M->nsub; ++sub) {
          long fi[3] = {0, 0, 0};
          fi[a] = 2 * (j[a] - M->lo[a]) + (s ? 0 : 1);
          for (int q = 0; q < d - 1; ++q) fi[t[q]] = 2 * (j[t[q]] - M->lo[t[q]]) + ((sub >> q) & 1);
          long fcell = flat(Y, fi);
          for (int r = 0; r < X->Qf; ++r) {
            double Uc[MAXV], Uf[MAXV], F[MAXV];
            amr_state(X, wc, cell, M->phiH[a][s][sub][r], Uc);
            amr_state(Y, wf, fcell, Y->phiF[a][1 - s][r], Uf);
            if (s) hllc(X, Uc, Uf, a, F); else hllc(X, Uf, Uc, a, F);
            for (int v = 0; v < X->nvar; ++v)
              for (int l = 0; l < X->N; ++l) {
                double tt = F[v] * M->phiH[a][s][sub][r][l] * X->wF[r] / (double)M->nsub;
                if (s) S[v][l] += tt; else S[v][l] -= tt;
                if (A) A[v][l] += fabs(tt);
              }
          }
        }
      } else {
        long nb = wall ? -1 : flat(X, j);
        for (int r = 0; r < X->Qf; ++r) {
          double Uo[MAXV], Un[MAXV], F[MAXV];
          amr_state(X, wc, cell, X->phiF[a][s][r], Uo);
          if (nb >= 0) amr_state(X, wc, nb, X->phiF[a][1 - s][r], Un);
          else for (int v = 0; v < X->nvar; ++v) Un[v] = Uo[v];
          if (s) hllc(X, Uo, Un, a, F); else hllc(X, Un, Uo, a, F);
          for (int v = 0; v < X->nvar; ++v)
            for (int l = 0; l < X->N; ++l) {
              double tt = F[v] * X->phiF[a][s][r][l] * X->wF[r];
              if (s) S[v][l] += tt; else S[v][l] -= tt;
              if (A) A[v][l] += fabs(tt);
            }
        }
      }
    }
  }
}

/* Surface term of a fine cell: neighbours outside the fine block are coarse. */
static void amr_surface_fine(const amr *M, const double *wc, const double *wf, long cell, double S[MAXV][MAXN],
                             double (*A)[MAXN]) {
  const ctx *X = &M->Xc, *Y = &M->Xf;
  int d = Y->d;
  for (int v = 0; v < Y->nvar; ++v) for (int j = 0; j < Y->N; ++j) S[v][j] = 0.0;
  long f[3]; unflat(Y, cell, f);
  for (int a = 0; a < d; ++a) {
    int t[2]; tangential(d, a, t);
    for (int s = 0; s < 2; ++s) {
      long g2[3] = {f[0], f[1], f[2]};
      g2[a] += s ? 1 : -1;
      int inside = g2[a] >= 0 && g2[a] < M->nf[a];
      for (int r = 0; r < Y->Qf; ++r) {
        double Uo[MAXV], Un[MAXV], F[MAXV];
        amr_state(Y, wf, cell, Y->phiF[a][s][r], Uo);
        if (inside) {
          amr_state(Y, wf, flat(Y, g2), Y->phiF[a][1 - s][r], Un);
        } else {
          long base[3] = {0, 0, 0}, j[3];
          for (int b = 0; b < d; ++b) base[b] = M->lo[b] + f[b] / 2;
          amr_coarse_nb(M, base, a, s ? 1 : -1, j);
          int sub = 0;
          for (int q = 0; q < d - 1; ++q) sub |= (int)(f[t[q]] % 2) << q;
          amr_state(X, wc, flat(X, j), M->phiH[a][1 - s][sub][r], Un);
        }
        if (s) hllc(Y, Uo, Un, a, F); else hllc(Y, Un, Uo, a, F);
        for (int v = 0; v < Y->nvar; ++v)
          for (int l = 0; l < Y->N; ++l) {
            double tt = F[v] * Y->phiF[a][s][r][l] * Y->wF[r];
            if (s) S[v][l] += tt; else S[v][l] -= tt;
            if (A) A[v][l] += fabs(tt);
          }
      }
    }
  }
}

/* dw/dt of one cell in the combined numbering (coarse cells 0..ncc-1, then
 * fine cells), each block with its own dx in the factor of eq.
 * spatial_discretisation; zero for a hole cell. */
static void amr_rhs_cell(const amr *M, const double *w, long cell, double Lc[MAXV][MAXN]) {
  const double *wc = w, *wf = w + (long)M->Xc.nvar * M->Xc.N * M->ncc;
  int nv = M->Xc.nvar, N = M->Xc.N, d = M->Xc.d;
  double V[MAXV][MAXN], S[MAXV][MAXN];
  double fac;
  if (cell < M->ncc) {
    long i[3]; unflat(&M->Xc, cell, i);
    if (amr_in_hole(M, i)) {
      for (int v = 0; v < nv; ++v) for (int j = 0; j < N; ++j) Lc[v][j] = 0.0;
      return;
    }
    fac = 2.0 / M->Xc.dx / (double)(1 << d);
    volume_term(&M->Xc, wc, cell, V, NULL);
    amr_surface_coarse(M, wc, wf, cell, S, NULL);
  } else {
    fac = 2.0 / M->Xf.dx / (double)(1 << d);
    volume_term(&M->Xf, wf, cell - M->ncc, V, NULL);
    amr_surface_fine(M, wc, wf, cell - M->ncc, S, NULL);
  }
  for (int v = 0; v < nv; ++v)
    for (int j = 0; j < N; ++j) Lc[v][j] = fac * (V[v][j] - S[v][j]);
}

static void amr_rhs_all(const amr *M, const double *w, double *L) {
  double *Lc = L, *Lf = L + (long)M->Xc.nvar * M->Xc.N * M->ncc;
  int nv = M->Xc.nvar, N = M->Xc.N;
  for (long cell = 0; cell < M->ncc + M->ncf; ++cell) {
    double Lk[MAXV][MAXN];
    amr_rhs_cell(M, w, cell, Lk);
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < N; ++j) {
        if (cell < M->ncc) Lc[((long)v * N + j) * M->ncc + cell] = Lk[v][j];
        else Lf[((long)v * N + j) * M->ncf + (cell - M->ncc)] = Lk[v][j];
      }
  }
}

/* fac V and fac S of every cell of both blocks (hole cells zero), so that
 * L = V - S; their magnitudes are the conditioning scale of the RHS.  Ao (may
 * be NULL): fac times the summed magnitudes of every summand, as in
 * orc_terms_cells. */
int orc_amr_terms(const orc_config *c, const double *w, double *Vo, double *So, double *Ao) {
  amr *M = malloc(sizeof(amr));
  int st = amr_init(c, M);
  if (st != ORC_OK) { free(M); return st; }
  const double *wc = w, *wf = w + (long)M->Xc.nvar * M->Xc.N * M->ncc;
  int nv = M->Xc.nvar, N = M->Xc.N, d = M->Xc.d;
  long off = (long)nv * N * M->ncc;
  double facc = 2.0 / M->Xc.dx / (double)(1 << d), facf = 2.0 / M->Xf.dx / (double)(1 << d);
  for (long cell = 0; cell < M->ncc; ++cell) {
    long i[3]; unflat(&M->Xc, cell, i);
    double V[MAXV][MAXN], S[MAXV][MAXN], A[MAXV][MAXN];
    memset(A, 0, sizeof(A));
    int hole = amr_in_hole(M, i);
    if (!hole) { volume_term(&M->Xc, wc, cell, V, A); amr_surface_coarse(M, wc, wf, cell, S, A); }
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < N; ++j) {
        Vo[((long)v * N + j) * M->ncc + cell] = hole ? 0.0 : facc * V[v][j];
        So[((long)v * N + j) * M->ncc + cell] = hole ? 0.0 : facc * S[v][j];
        if (Ao) Ao[((long)v * N + j) * M->ncc + cell] = hole ? 0.0 : facc * A[v][j];
      }
  }
  for (long cell = 0; cell < M->ncf; ++cell) {
    double V[MAXV][MAXN], S[MAXV][MAXN], A[MAXV][MAXN];
    memset(A, 0, sizeof(A));
    volume_term(&M->Xf, wf, cell, V, A);
    amr_surface_fine(M, wc, wf, cell, S, A);
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < N; ++j) {
        Vo[off + ((long)v * N + j) * M->ncf + cell] = facf * V[v][j];
        So[off + ((long)v * N + j) * M->ncf + cell] = facf * S[v][j];
        if (Ao) Ao[off + ((long)v * N + j) * M->ncf + cell] = facf * A[v][j];
      }
  }
  free(M);
  return ORC_OK;
}

/* fac V, fac S and fac times the summed magnitudes of their summands for a
 * list of cells in the combined numbering (coarse cells, then fine cells),
 * each output [nvar][N][ncells]; hole cells give zeros.  L = V - S. */
int orc_amr_terms_cells(const orc_config *c, const double *w, long ncells, const long *cells, double *Vo,
                        double *So, double *Ao) {
  amr *M = malloc(sizeof(amr));
  int st = amr_init(c, M);
  if (st != ORC_OK) { free(M); return st; }
  const double *wc = w, *wf = w + (long)M->Xc.nvar * M->Xc.N * M->ncc;
  int nv = M->Xc.nvar, N = M->Xc.N, d = M->Xc.d;
  double facc = 2.0 / M->Xc.dx / (double)(1 << d), facf = 2.0 / M->Xf.dx / (double)(1 << d);
  for (long n = 0; n < ncells; ++n) {
    long cell = cells[n];
    if (cell < 0 || cell >= M->ncc + M->ncf) { free(M); return ORC_EINVAL; }
    double V[MAXV][MAXN], S[MAXV][MAXN], A[MAXV][MAXN];
    memset(V, 0, sizeof(V)); memset(S, 0, sizeof(S)); memset(A, 0, sizeof(A));
    double fac;
    if (cell < M->ncc) {
      long i[3]; unflat(&M->Xc, cell, i);
      fac = facc;
      if (!amr_in_hole(M, i)) { volume_term(&M->Xc, wc, cell, V, A); amr_surface_coarse(M, wc, wf, cell, S, A); }
    } else {
      fac = facf;
      volume_term(&M->Xf, wf, cell - M->ncc, V, A);
      amr_surface_fine(M, wc, wf, cell - M->ncc, S, A);
    }
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < N; ++j) {
        Vo[((long)v * N + j) * ncells + n] = fac * V[v][j];
        So[((long)v * N + j) * ncells + n] = fac * S[v][j];
        Ao[((long)v * N + j) * ncells + n] = fac * A[v][j];
      }
  }
  free(M);
  return ORC_OK;
}

static long amr_state_size(const amr *M) { return (long)M->Xc.nvar * M->Xc.N * (M->ncc + M->ncf); }

int orc_amr_sizes(const orc_config *c, long *out /* ncoarse, nfine, nf[3] */) {
  amr *M = malloc(sizeof(amr));
  if (!M) return ORC_ENOMEM;
  int st = amr_init(c, M);
  if (st == ORC_OK) { out[0] = M->ncc; out[1] = M->ncf; out[2] = M->nf[0]; out[3] = M->nf[1]; out[4] = M->nf[2]; }
  free(M);
  return st;
}

/* Projection nodes of both blocks: x[ncoarse + nfine][Q][3]. */
int orc_amr_node_coords(const orc_config *c, double *x) {
  amr *M = malloc(sizeof(amr));
  int st = amr_init(c, M);
  if (st != ORC_OK) { free(M); return st; }
  const ctx *B[2] = {&M->Xc, &M->Xf};
  double x0f[3];
  for (int a = 0; a < 3; ++a) x0f[a] = c->x0[a] + M->lo[a] * M->Xc.dx;
  long off = 0;
  for (int b = 0; b < 2; ++b) {
    const ctx *X = B[b];
    for (long cell = 0; cell < X->ncell; ++cell) {
      long i[3]; unflat(X, cell, i);
      for (int q = 0; q < X->Q; ++q) {
        int iq[3] = {q % X->n1, (q / X->n1) % X->n1, q / (X->n1 * X->n1)};
        for (int a = 0; a < 3; ++a) {
          double v = 0.0;
          if (a < X->d) v = (b ? x0f[a] : c->x0[a]) + (i[a] + 0.5) * X->dx + 0.5 * X->dx * X->gx[iq[a]];
          x[((off + cell) * X->Q + q) * 3 + a] = v;
        }
      }
    }
    off += X->ncell;
  }
  free(M);
  return ORC_OK;
}

/* L2 projection on both blocks (prim[ncoarse + nfine][Q][5]). */
int orc_amr_project(const orc_config *c, const double *prim, double *w) {
  amr *M = malloc(sizeof(amr));
  int st = amr_init(c, M);
  if (st != ORC_OK) { free(M); return st; }
  const ctx *B[2] = {&M->Xc, &M->Xf};
  long off = 0;
  double *wb = w;
  for (int b = 0; b < 2; ++b) {
    const ctx *X = B[b];
    double scale = 1.0 / (double)(1 << X->d);
    for (long cell = 0; cell < X->ncell; ++cell) {
      double acc[MAXV][MAXN];
      memset(acc, 0, sizeof(acc));
      for (int q = 0; q < X->Q; ++q) {
        const double *pr = prim + ((off + cell) * X->Q + q) * 5;
        double U[MAXV], ke = 0.0;
        U[0] = pr[0];
        for (int bb = 0; bb < X->d; ++bb) { U[1 + bb] = pr[0] * pr[1 + bb]; ke += pr[1 + bb] * pr[1 + bb]; }
        U[X->d + 1] = pr[4] / (c->gamma - 1.0) + 0.5 * pr[0] * ke;
        for (int v = 0; v < X->nvar; ++v)
          for (int j = 0; j < X->N; ++j) acc[v][j] += U[v] * X->phiV[q][j] * X->wV[q];
      }
      for (int v = 0; v < X->nvar; ++v)
        for (int j = 0; j < X->N; ++j) wb[((long)v * X->N + j) * X->ncell + cell] = scale * acc[v][j];
    }
    off += X->ncell;
    wb += (long)X->nvar * X->N * X->ncell;
  }
  free(M);
  return ORC_OK;
}

int orc_amr_rhs(const orc_config *c, const double *w, double *L) {
  amr *M = malloc(sizeof(amr));
  int st = amr_init(c, M);
  if (st == ORC_OK) amr_rhs_all(M, w, L);
  free(M);
  return st;
}

/* dw/dt of the listed cells (combined numbering): out[nvar][N][ncells]. */
int orc_amr_rhs_cells(const orc_config *c, const double *w, long ncells, const long *cells, double *out) {
  amr *M = malloc(sizeof(amr));
  int st = amr_init(c, M);
  if (st != ORC_OK) { free(M); return st; }
  int nv = M->Xc.nvar, N = M->Xc.N;
  for (long n = 0; n < ncells; ++n) {
    if (cells[n] < 0 || cells[n] >= M->ncc + M->ncf) { free(M); return ORC_EINVAL; }
    double Lk[MAXV][MAXN];
    amr_rhs_cell(M, w, cells[n], Lk);
    for (int v = 0; v < nv; ++v)
      for (int j = 0; j < N; ++j) out[((long)v * N + j) * ncells + n] = Lk[v][j];
  }
  free(M);
  return ORC_OK;
}

int orc_amr_rk3_stage(const orc_config *c, int stage, double dt, const double *wn, const double *wp, double *out) {
  if (stage < 1 || stage > 3) return ORC_EINVAL;
  amr *M = malloc(sizeof(amr));
  int st = amr_init(c, M);
  if (st != ORC_OK) { free(M); return st; }
  long n = amr_state_size(M);
  double *L = malloc(sizeof(double) * n);
  amr_rhs_all(M, wp, L);
  rk3_combine(stage, dt, wn, wp, L, out, n);
  free(L); free(M);
  return ORC_OK;
}

/* Stage value Y_m of a general tableau on the refined mesh (see
 * orc_tableau_stage). */
int orc_amr_tableau_stage(const orc_config *c, int s, const double *A, const double *b, int m, double dt,
                          const double *Y, double *out) {
  double alpha[MAXST * MAXST], beta[MAXST];
  int st = shu_osher(s, A, b, alpha, beta);
  if (st != ORC_OK) return st;
  if (m < 1 || m > s) return ORC_EINVAL;
  amr *M = malloc(sizeof(amr));
  st = amr_init(c, M);
  if (st != ORC_OK) { free(M); return st; }
  long n = amr_state_size(M);
  double *L = malloc(sizeof(double) * n);
  amr_rhs_all(M, Y + (long)(m - 1) * n, L);
  tableau_combine(s, alpha, beta, m, dt, Y, L, out, n);
  free(L); free(M);
  return ORC_OK;
}

/* Time step over both blocks, each cell with its own edge length. */
int orc_amr_max_dt(const orc_config *c, const double *w, double *dt_out) {
  amr *M = malloc(sizeof(amr));
  int st = amr_init(c, M);
  if (st != ORC_OK) { free(M); return st; }
  double fk = 1.0 / (2.0 * M->Xc.k + 1.0);
  if (c->positivity && M->Xc.lw[0] / 2.0 < fk) fk = M->Xc.lw[0] / 2.0;
  double dt = INFINITY;
  const ctx *B[2] = {&M->Xc, &M->Xf};
  const double *wb = w;
  for (int b = 0; b < 2; ++b) {
    const ctx *X = B[b];
    for (long cell = 0; cell < X->ncell; ++cell) {
      long i[3]; unflat(X, cell, i);
      if (b == 0 && amr_in_hole(M, i)) continue;
      double U[MAXV];
      for (int v = 0; v < X->nvar; ++v) U[v] = wb[((long)v * X->N) * X->ncell + cell];
      double p = pressure(X, U);
      double cs = sqrt(c->gamma * p / U[0]);
      double rate = 0.0;
      for (int a = 0; a < X->d; ++a) rate += (fabs(U[1 + a] / U[0]) + cs) / X->dx;
      double dtc = c->cfl * fk / rate;
      if (dtc < dt) dt = dtc;
    }
    wb += (long)X->nvar * X->N * X->ncell;
  }
  *dt_out = dt;
  free(M);
  return ORC_OK;
}

/* Limiters on the refined mesh (Sec. 4.4): a coarse cell sees, across a
 * refined face, the mean of the 2^d fine cells of that base cell; a fine cell
 * sees, across the block boundary, the mean of the coarse polynomial over the
 * child subcell next to it.  Coarse cells with hanging faces also check
 * positivity at the hanging-face quadrature points. */
/* sel (may be NULL: every cell) marks, in the combined numbering (coarse
 * cells, then fine cells), the cells to limit. */
static int amr_limit_masked(const orc_config *c, double *w, const unsigned char *sel) {
  amr *M = malloc(sizeof(amr));
  int st = amr_init(c, M);
  if (st != ORC_OK) { free(M); return st; }
  const ctx *X = &M->Xc, *Y = &M->Xf;
  int d = X->d, nv = X->nvar, N = X->N;
  double *wc = w, *wf = w + (long)nv * N * M->ncc;
  long bad = 0;
  /* hole[] marks the coarse cells that are not limited: the hole cells, and
   * with a selection every unselected one; fskip[] the same for fine cells */
  unsigned char *hole = malloc(M->ncc);
  unsigned char *fskip = NULL;
  for (long cell = 0; cell < M->ncc; ++cell) {
    long i[3]; unflat(X, cell, i);
    hole[cell] = (unsigned char)(amr_in_hole(M, i) || (sel && !sel[cell]));
  }
  if (sel) {
    fskip = malloc(M->ncf);
    for (long cell = 0; cell < M->ncf; ++cell) fskip[cell] = (unsigned char)!sel[M->ncc + cell];
  }
  if (c->limiter) {
    double *nbc = malloc(sizeof(double) * 2 * d * nv * M->ncc);
    double *nbf = malloc(sizeof(double) * 2 * d * nv * M->ncf);
    double *dxc = malloc(sizeof(double) * M->ncc), *dxf = malloc(sizeof(double) * M->ncf);
    for (long i = 0; i < M->ncc; ++i) dxc[i] = X->dx;
    for (long i = 0; i < M->ncf; ++i) dxf[i] = Y->dx;
    for (long cell = 0; cell < M->ncc; ++cell) {
      long i[3]; unflat(X, cell, i);
      for (int a = 0; a < d; ++a)
        for (int s = 0; s < 2; ++s) {
          long j[3];
          int wall = amr_coarse_nb(M, i, a, s ? 1 : -1, j);
          for (int v = 0; v < nv; ++v) {
            double m;
            if (wall) m = wc[((long)v * N) * M->ncc + cell];
            else if (amr_in_hole(M, j)) {
              m = 0.0;
              for (int ch = 0; ch < (1 << d); ++ch) {
                long fi[3] = {0, 0, 0};
                for (int b = 0; b < d; ++b) fi[b] = 2 * (j[b] - M->lo[b]) + ((ch >> b) & 1);
                m += wf[((long)v * N) * M->ncf + flat(Y, fi)];
              }
              m /= (double)(1 << d);
            } else m = wc[((long)v * N) * M->ncc + flat(X, j)];
            nbc[((long)(2 * a + s) * nv + v) * M->ncc + cell] = m;
          }
        }
    }
    for (long cell = 0; cell < M->ncf; ++cell) {
      long f[3]; unflat(Y, cell, f);
      for (int a = 0; a < d; ++a)
        for (int s = 0; s < 2; ++s) {
          long g2[3] = {f[0], f[1], f[2]};
          g2[a] += s ? 1 : -1;
          for (int v = 0; v < nv; ++v) {
            double m;
            if (g2[a] >= 0 && g2[a] < M->nf[a]) {
              m = wf[((long)v * N) * M->ncf + flat(Y, g2)];
            } else {
              long base[3] = {0, 0, 0}, j[3];
              for (int b = 0; b < d; ++b) base[b] = M->lo[b] + f[b] / 2;
              amr_coarse_nb(M, base, a, s ? 1 : -1, j);
              int ch = 0;
              for (int b = 0; b < d; ++b) {
                int bit = (b == a) ? (s ? 0 : 1) : (int)(f[b] % 2);
                ch |= bit << b;
              }
              m = 0.0;
              for (int l = 0; l < N; ++l) m += wc[((long)v * N + l) * M->ncc + flat(X, j)] * M->cmean[ch][l];
            }
            nbf[((long)(2 * a + s) * nv + v) * M->ncf + cell] = m;
          }
        }
    }
    if (c->limiter == 2) {
      char_limit(X, wc, nbc, dxc, hole);
      char_limit(Y, wf, nbf, dxf, fskip);
    } else {
      slope_limit(X, wc, nbc, dxc, hole);
      slope_limit(Y, wf, nbf, dxf, fskip);
    }
    free(nbc); free(nbf); free(dxc); free(dxf);
  }
  if (c->positivity) {
    /* extra points: coarse trace at the hanging-face nodes */
    int xmax = 2 * d * M->nsub * X->Qf;
    int *xcnt = calloc(M->ncc, sizeof(int));
    double *xphi = malloc(sizeof(double) * M->ncc * xmax * N);
    for (long cell = 0; cell < M->ncc; ++cell) {
      if (hole[cell]) continue;
      long i[3]; unflat(X, cell, i);
      for (int a = 0; a < d; ++a)
        for (int s = 0; s < 2; ++s) {
          long j[3];
          if (amr_coarse_nb(M, i, a, s ? 1 : -1, j) == 0 && amr_in_hole(M, j))
            for (int sub = 0; sub < M->nsub; ++sub)
              for (int r = 0; r < X->Qf; ++r) {
                memcpy(xphi + ((long)cell * xmax + xcnt[cell]) * N, M->phiH[a][s][sub][r], sizeof(double) * N);
                ++xcnt[cell];
              }
        }
    }
    bad += positivity_limit(X, wc, xcnt, xphi, xmax, hole);
    bad += positivity_limit(Y, wf, NULL, NULL, 0, fskip);
    free(xcnt); free(xphi);
  }
  free(hole);
  free(fskip);
  free(M);
  return bad ? ORC_ENEGATIVE : ORC_OK;
}

int orc_amr_limit(const orc_config *c, double *w) { return amr_limit_masked(c, w, NULL); }

/* The limiters on the listed cells only, in the combined numbering (coarse
 * cells 0..ncoarse-1, then fine cells); other cells are left as they are. */
int orc_amr_limit_cells(const orc_config *c, double *w, long ncells, const long *cells) {
  amr *M = malloc(sizeof(amr));
  int st = amr_init(c, M);
  long nt = M->ncc + M->ncf;
  free(M);
  if (st != ORC_OK) return st;
  unsigned char *sel = calloc(nt, 1);
  if (!sel) return ORC_ENOMEM;
  for (long i = 0; i < ncells; ++i) {
    if (cells[i] < 0 || cells[i] >= nt) { free(sel); return ORC_EINVAL; }
    sel[cells[i]] = 1;
  }
  st = amr_limit_masked(c, w, sel);
  free(sel);
  return st;
}

/* (P_c)_{j,l} = 2^-d int phi_l((xi + c)/2) phi_j(xi) dxi: the L2 projection of
 * a coarse polynomial onto child c (eq. ref_pa_integral and App. F, with the
 * coarse basis at the mapped point).  Out: P[N][N] row-major. */
/* Refinement matrix of child c (eq. ref_pa_integral): (P_c)_jl = 2^-d
 * int over the reference cell of phi_j(xi) phi_l(child map of xi), with the
 * (k+1)^d Gauss rule (exact: degree 2k per axis).  Child c has bit a set if
 * it is the upper half along axis a. */
static void refine_matrix(const ctx *X, int child, double *P) {
  int d = X->d;
  for (int j = 0; j < X->N; ++j)
    for (int l = 0; l < X->N; ++l) {
      double acc = 0.0;
      for (int q = 0; q < X->Q; ++q) {
        int iq[3] = {q % X->n1, (q / X->n1) % X->n1, q / (X->n1 * X->n1)};
        double xi[3] = {0, 0, 0}, xm[3] = {0, 0, 0};
        for (int a = 0; a < d; ++a) {
          xi[a] = X->gx[iq[a]];
          xm[a] = 0.5 * (xi[a] + (((child >> a) & 1) ? 1.0 : -1.0));
        }
        acc += phi_at(X, l, xm) * phi_at(X, j, xi) * X->wV[q];
      }
      P[j * X->N + l] = acc / (double)(1 << d);
    }
}

int orc_refine_matrix(const orc_config *c, int child, double *P) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st != ORC_OK) { free(X); return st; }
  if (child < 0 || child >= (1 << X->d)) { free(X); return ORC_EINVAL; }
  refine_matrix(X, child, P);
  free(X);
  return ORC_OK;
}

/* A configuration with or without a refined box: the base grid (the coarse
 * block) and, if the box is non-empty, the box [lo, hi) and its fine block. */
typedef struct {
  ctx X;
  int box, lo[3], hi[3];
  long nf[3], ncf;
} grid2;

static int grid2_init(const orc_config *c, grid2 *G) {
  int st = ctx_init(c, &G->X);
  if (st != ORC_OK) return st;
  G->box = 0;
  G->ncf = 0;
  for (int a = 0; a < 3; ++a) { G->lo[a] = c->refine_lo[a]; G->hi[a] = c->refine_hi[a]; G->nf[a] = 1; }
  for (int a = 0; a < G->X.d; ++a)
    if (G->lo[a] != G->hi[a]) G->box = 1;
  if (G->box) {
    amr *M = malloc(sizeof(amr));
    st = amr_init(c, M); /* validates the box */
    free(M);
    if (st != ORC_OK) return st;
    G->ncf = 1;
    for (int a = 0; a < G->X.d; ++a) { G->nf[a] = 2L * (G->hi[a] - G->lo[a]); G->ncf *= G->nf[a]; }
  }
  return ORC_OK;
}

static int grid2_in_box(const grid2 *G, const long *i) {
  if (!G->box) return 0;
  for (int a = 0; a < G->X.d; ++a)
    if (i[a] < G->lo[a] || i[a] >= G->hi[a]) return 0;
  return 1;
}

static void cell_ijk(const ctx *X, long cell, long *i) {
  i[0] = cell % X->nx; i[1] = (cell / X->nx) % X->ny; i[2] = cell / ((long)X->nx * X->ny);
}

/* flat index in the fine block of child c of base cell i */
static long grid2_fine(const grid2 *G, const long *i, int c) {
  long f[3] = {0, 0, 0};
  for (int a = 0; a < G->X.d; ++a) f[a] = 2 * (i[a] - G->lo[a]) + ((c >> a) & 1);
  return (f[2] * G->nf[1] + f[1]) * G->nf[0] + f[0];
}

/* coefficient (v, l) of a state of grid G: coarse cell or fine cell */
#define WC(G, w, v, l, cell) (w)[((long)(v) * (G)->X.N + (l)) * (G)->X.ncell + (cell)]
#define WF(G, w, v, l, f) (w)[(long)(G)->X.nvar * (G)->X.N * (G)->X.ncell + ((long)(v) * (G)->X.N + (l)) * (G)->ncf + (f)]

/* Refinement flags per base cell (Sec. 4.1): a cell of the base grid is
 * flagged if max_a |w_rho,1+a| > alpha w_t (eq. cell_ref; the density slope
 * coefficients are the changes across the half-cell divided by sqrt(3)); a
 * base cell that is refined now stays flagged if the same holds for its node
 * weights, the derefined projection of its 2^d children (eq. deref_weights),
 * against w_t / alpha (eq. node_ref). */
int orc_amr_flags(const orc_config *c, const double *w, double wt, double alpha, int *flags) {
  grid2 *G = malloc(sizeof(grid2));
  int st = grid2_init(c, G);
  if (st != ORC_OK) { free(G); return st; }
  const ctx *X = &G->X;
  int d = X->d, nc = 1 << d;
  double *P = malloc(sizeof(double) * 8 * MAXN * MAXN);
  for (int ch = 0; ch < nc; ++ch) refine_matrix(X, ch, P + (long)ch * MAXN * MAXN);
  for (long cell = 0; cell < X->ncell; ++cell) {
    long i[3];
    cell_ijk(X, cell, i);
    double m = 0.0, bound;
    if (grid2_in_box(G, i)) {
      for (int a = 0; a < d; ++a) {
        double node = 0.0; /* node weight of mode 1+a of the density */
        for (int ch = 0; ch < nc; ++ch) {
          long f = grid2_fine(G, i, ch);
          for (int l = 0; l < X->N; ++l) node += P[(long)ch * MAXN * MAXN + l * X->N + (1 + a)] * WF(G, w, 0, l, f);
        }
        node /= (double)nc;
        if (fabs(node) > m) m = fabs(node);
      }
      bound = wt / alpha;
    } else {
      for (int a = 0; a < d; ++a)
        if (fabs(WC(G, w, 0, 1 + a, cell)) > m) m = fabs(WC(G, w, 0, 1 + a, cell));
      bound = alpha * wt;
    }
    flags[cell] = m > bound;
  }
  free(P); free(G);
  return ORC_OK;
}

/* New state on the grid of c_new from a state on the grid of c_old (same base
 * grid, either with or without a box): a base cell that stays unrefined is
 * copied; one that leaves the box takes the derefinement of its children
 * (eq. deref_weights: w^K = 2^-d sum_c P_c^T w^c); a fine cell of a base cell
 * already refined is copied, one of a newly refined base cell is the
 * refinement of the coarse polynomial (eq. ref_weights: w^c = P_c w^K).
 * Base cells inside the new box (the hole) are set to zero. */
int orc_amr_regrid(const orc_config *c_old, const double *w_old, const orc_config *c_new, double *w_new) {
  grid2 *A = malloc(sizeof(grid2)), *B = malloc(sizeof(grid2));
  int st = grid2_init(c_old, A);
  if (st == ORC_OK) st = grid2_init(c_new, B);
  if (st == ORC_OK && (A->X.d != B->X.d || A->X.k != B->X.k || A->X.ncell != B->X.ncell)) st = ORC_EINVAL;
  if (st != ORC_OK) { free(A); free(B); return st; }
  const ctx *X = &A->X;
  int d = X->d, nc = 1 << d, N = X->N, nv = X->nvar;
  double *P = malloc(sizeof(double) * 8 * MAXN * MAXN);
  for (int ch = 0; ch < nc; ++ch) refine_matrix(X, ch, P + (long)ch * MAXN * MAXN);
  for (long cell = 0; cell < X->ncell; ++cell) {
    long i[3];
    cell_ijk(X, cell, i);
    int in_old = grid2_in_box(A, i), in_new = grid2_in_box(B, i);
    for (int v = 0; v < nv; ++v) {
      if (in_new) {
        for (int l = 0; l < N; ++l) WC(B, w_new, v, l, cell) = 0.0;
        for (int ch = 0; ch < nc; ++ch) {
          long fn = grid2_fine(B, i, ch);
          if (in_old) {
            long fo = grid2_fine(A, i, ch);
            for (int l = 0; l < N; ++l) WF(B, w_new, v, l, fn) = WF(A, w_old, v, l, fo);
          } else {
            for (int j = 0; j < N; ++j) {
              double acc = 0.0;
              for (int l = 0; l < N; ++l) acc += P[(long)ch * MAXN * MAXN + j * N + l] * WC(A, w_old, v, l, cell);
              WF(B, w_new, v, j, fn) = acc;
            }
          }
        }
      } else if (in_old) {
        for (int j = 0; j < N; ++j) {
          double acc = 0.0;
          for (int ch = 0; ch < nc; ++ch) {
            long fo = grid2_fine(A, i, ch);
            for (int l = 0; l < N; ++l) acc += P[(long)ch * MAXN * MAXN + l * N + j] * WF(A, w_old, v, l, fo);
          }
          WC(B, w_new, v, j, cell) = acc / (double)nc;
        }
      } else {
        for (int l = 0; l < N; ++l) WC(B, w_new, v, l, cell) = WC(A, w_old, v, l, cell);
      }
    }
  }
  free(P); free(A); free(B);
  return ORC_OK;
}


/* ------------------------------------------------------------------------ */
/* Quadtree of leaf cells in 2D (Sec. 4: cells split into 2^d children at any */
/* level, the level jump across a face at most one)                          */
/*                                                                            */
/* Leaf i has level lev[i] >= 0 and integer position (ix[i], iy[i]) on its     */
/* level: level 0 is the base grid n[], a level-l cell has edge dx / 2^l and  */
/* covers [x0 + ix h, x0 + (ix + 1) h) x [y0 + iy h, y0 + (iy + 1) h).  The     */
/* state is [nvar][N][nleaf] in leaf order.  Written from the geometry alone: */
/* every face of a leaf is cut into the overlaps with the leaves across it    */
/* (found by brute force), each overlap integrated with the (k+1)-point Gauss */
/* rule mapped onto it, both traces evaluated at the physical node through    */
/* each cell's own reference coordinates, and the lifted flux weighted by the */
/* overlap's share of the leaf's face.  With 2:1 balance this is the          */
/* hanging-face quadrature of Sec. 4 (coarse trace at (eta + sigma)/2, weight */
/* w_r / 2 on the coarse side).                                               */
/* ------------------------------------------------------------------------ */

typedef struct {
  ctx X;          /* tables; X.ncell = nleaf, X.dx = base edge              */
  long nleaf;
  int lmax;
  long NX, NY;    /* domain in units of the finest level                   */
  long *bx0, *bx1, *by0, *by1; /* leaf boxes in those units                */
} tree;

static void tree_free(tree *T) { free(T->bx0); free(T->bx1); free(T->by0); free(T->by1); }

static int tree_init(const orc_config *c, long nleaf, const int *lev, const long *ix, const long *iy, tree *T) {
  memset(T, 0, sizeof(*T));
  if (c->dim != 2 || c->accel || nleaf < 1) return ORC_EINVAL;
  int st = ctx_init(c, &T->X);
  if (st != ORC_OK) return st;
  T->nleaf = nleaf;
  T->X.ncell = nleaf;
  T->lmax = 0;
  for (long i = 0; i < nleaf; ++i) {
    if (lev[i] < 0 || lev[i] > 20) return ORC_EINVAL;
    if (lev[i] > T->lmax) T->lmax = lev[i];
  }
  T->NX = (long)c->n[0] << T->lmax;
  T->NY = (long)c->n[1] << T->lmax;
  T->bx0 = malloc(sizeof(long) * nleaf); T->bx1 = malloc(sizeof(long) * nleaf);
  T->by0 = malloc(sizeof(long) * nleaf); T->by1 = malloc(sizeof(long) * nleaf);
  long area = 0;
  for (long i = 0; i < nleaf; ++i) {
    long s = 1L << (T->lmax - lev[i]);
    if (ix[i] < 0 || iy[i] < 0 || ix[i] >= ((long)c->n[0] << lev[i]) || iy[i] >= ((long)c->n[1] << lev[i])) {
      tree_free(T);
      return ORC_EINVAL;
    }
    T->bx0[i] = ix[i] * s; T->bx1[i] = (ix[i] + 1) * s;
    T->by0[i] = iy[i] * s; T->by1[i] = (iy[i] + 1) * s;
    area += s * s;
  }
  /* a tiling: no two leaves overlap and together they cover the domain */
  for (long i = 0; i < nleaf; ++i)
    for (long j = i + 1; j < nleaf; ++j)
      if (T->bx0[i] < T->bx1[j] && T->bx0[j] < T->bx1[i] && T->by0[i] < T->by1[j] && T->by0[j] < T->by1[i]) {
        tree_free(T);
        return ORC_EINVAL;
      }
  if (area != T->NX * T->NY) { tree_free(T); return ORC_EINVAL; }
  return ORC_OK;
}

/* The leaves across face (a, s) of leaf i and their overlaps [o0, o1) with it
 * along the tangential axis, sorted by o0; returns the count (0 at a
 * transmissive wall).  Periodic axes wrap. */
static int tree_across(const tree *T, long i, int a, int s, long *nb, long *o0, long *o1) {
  const long *n0 = a == 0 ? T->bx0 : T->by0, *n1 = a == 0 ? T->bx1 : T->by1;
  const long *t0 = a == 0 ? T->by0 : T->bx0, *t1 = a == 0 ? T->by1 : T->bx1;
  long L = a == 0 ? T->NX : T->NY;
  long f = s ? n1[i] : n0[i];
  if ((f == 0 || f == L) && T->X.c.bc[a] == 1) return 0;
  f = ((f % L) + L) % L;
  int m = 0;
  for (long j = 0; j < T->nleaf; ++j) {
    long g = s ? n0[j] : n1[j] % L;
    if (g != f) continue;
    long lo = t0[i] > t0[j] ? t0[i] : t0[j], hi = t1[i] < t1[j] ? t1[i] : t1[j];
    if (hi <= lo) continue;
    if (m == 4) return -1;
    nb[m] = j; o0[m] = lo; o1[m] = hi; ++m;
  }
  for (int p = 1; p < m; ++p)
    for (int q = p; q > 0 && o0[q] < o0[q - 1]; --q) {
      long t;
      t = nb[q]; nb[q] = nb[q - 1]; nb[q - 1] = t;
      t = o0[q]; o0[q] = o0[q - 1]; o0[q - 1] = t;
      t = o1[q]; o1[q] = o1[q - 1]; o1[q - 1] = t;
    }
  return m;
}

/* value of leaf i's polynomial (all variables) at reference point xi */
static void tree_eval(const tree *T, const double *w, long i, const double *xi, double *U) {
  const ctx *X = &T->X;
  for (int v = 0; v < X->nvar; ++v) {
    double s = 0.0;
    for (int l = 0; l < X->N; ++l) s += W(v, l, i) * phi_at(X, l, xi);
    U[v] = s;
  }
}

/* Surface term of leaf i (eq. dg_term3 over the overlaps of its faces). */
static int tree_surface(const tree *T, const double *w, long i, double S[MAXV][MAXN], double (*A)[MAXN]) {
  const ctx *X = &T->X;
  for (int v = 0; v < X->nvar; ++v) for (int j = 0; j < X->N; ++j) S[v][j] = 0.0;
  for (int a = 0; a < 2; ++a) {
    int b = 1 - a; /* tangential axis */
    const long *t0 = b == 0 ? T->bx0 : T->by0, *t1 = b == 0 ? T->bx1 : T->by1;
    for (int s = 0; s < 2; ++s) {
      long nb[4], o0[4], o1[4];
      int m = tree_across(T, i, a, s, nb, o0, o1);
      if (m < 0) return ORC_EINVAL;
      int wall = (m == 0);
      if (wall) { nb[0] = i; o0[0] = t0[i]; o1[0] = t1[i]; m = 1; }
      for (int p = 0; p < m; ++p) {
        long j = nb[p];
        double ratio = (double)(o1[p] - o0[p]) / (double)(t1[i] - t0[i]);
        for (int r = 0; r < X->n1; ++r) {
          /* reference coordinates of the node in leaf i and in leaf j */
          double xi[3] = {0, 0, 0}, xj[3] = {0, 0, 0};
          xi[a] = s ? 1.0 : -1.0;
          xj[a] = s ? -1.0 : 1.0;
          xi[b] = ((double)(o0[p] + o1[p] - t0[i] - t1[i]) + (double)(o1[p] - o0[p]) * X->gx[r]) /
                  (double)(t1[i] - t0[i]);
          xj[b] = ((double)(o0[p] + o1[p] - t0[j] - t1[j]) + (double)(o1[p] - o0[p]) * X->gx[r]) /
                  (double)(t1[j] - t0[j]);
          double Uo[MAXV], Un[MAXV], F[MAXV];
          tree_eval(T, w, i, xi, Uo);
          if (wall) for (int v = 0; v < X->nvar; ++v) Un[v] = Uo[v];
          else tree_eval(T, w, j, xj, Un);
          if (s) hllc(X, Uo, Un, a, F); else hllc(X, Un, Uo, a, F);
          for (int v = 0; v < X->nvar; ++v)
            for (int l = 0; l < X->N; ++l) {
              double tt = F[v] * phi_at(X, l, xi) * (X->gw[r] * ratio);
              if (s) S[v][l] += tt; else S[v][l] -= tt;
              if (A) A[v][l] += fabs(tt);
            }
        }
      }
    }
  }
  return ORC_OK;
}

/* fac V and fac S (L = V - S), fac = (2/dx_i) 2^-d with the leaf's own
 * edge, of the listed leaves (cells[0..ncells), all leaves if cells is NULL),
 * out[nvar][N][ncells]; Ao (may be NULL): fac times the summed magnitudes of
 * every summand of V and S (the rounding scale of each element). */
static int tree_terms(const orc_config *c, long nleaf, const int *lev, const long *ix, const long *iy,
                      const double *w, long ncells, const long *cells, double *Vo, double *So, double *Ao) {
  tree *T = malloc(sizeof(tree));
  int st = tree_init(c, nleaf, lev, ix, iy, T);
  if (st != ORC_OK) { free(T); return st; }
  const ctx *X = &T->X;
  for (long k = 0; k < ncells && st == ORC_OK; ++k) {
    long i = cells ? cells[k] : k;
    if (i < 0 || i >= nleaf) { st = ORC_EINVAL; break; }
    double V[MAXV][MAXN], S[MAXV][MAXN], A[MAXV][MAXN];
    memset(A, 0, sizeof(A));
    volume_term(X, w, i, V, A);
    st = tree_surface(T, w, i, S, A);
    double dxi = X->dx / (double)(1L << lev[i]);
    double fac = 2.0 / dxi / 4.0;
    for (int v = 0; v < X->nvar; ++v)
      for (int j = 0; j < X->N; ++j) {
        long e = ((long)v * X->N + j) * ncells + k;
        Vo[e] = fac * V[v][j];
        So[e] = fac * S[v][j];
        if (Ao) Ao[e] = fac * A[v][j];
      }
  }
  tree_free(T); free(T);
  return st;
}

int orc_tree_terms(const orc_config *c, long nleaf, const int *lev, const long *ix, const long *iy,
                   const double *w, double *Vo, double *So, double *Ao) {
  return tree_terms(c, nleaf, lev, ix, iy, w, nleaf, NULL, Vo, So, Ao);
}

/* The same for the listed leaves only (sampled checks of large meshes). */
int orc_tree_terms_cells(const orc_config *c, long nleaf, const int *lev, const long *ix, const long *iy,
                         const double *w, long ncells, const long *cells, double *Vo, double *So, double *Ao) {
  return tree_terms(c, nleaf, lev, ix, iy, w, ncells, cells, Vo, So, Ao);
}

/* L = dw/dt on every leaf: (2/dx_i) 2^-d (V - S) with the leaf's own edge. */
int orc_tree_rhs(const orc_config *c, long nleaf, const int *lev, const long *ix, const long *iy,
                 const double *w, double *L) {
  tree *T = malloc(sizeof(tree));
  int st = tree_init(c, nleaf, lev, ix, iy, T);
  if (st != ORC_OK) { free(T); return st; }
  const ctx *X = &T->X;
  for (long i = 0; i < nleaf && st == ORC_OK; ++i) {
    double V[MAXV][MAXN], S[MAXV][MAXN];
    volume_term(X, w, i, V, NULL);
    st = tree_surface(T, w, i, S, NULL);
    double dxi = X->dx / (double)(1L << lev[i]);
    double fac = 2.0 / dxi / 4.0;
    for (int v = 0; v < X->nvar; ++v)
      for (int j = 0; j < X->N; ++j) L[((long)v * X->N + j) * nleaf + i] = fac * (V[v][j] - S[v][j]);
  }
  tree_free(T); free(T);
  return st;
}

/* dt = CFL f_k / max over leaves of sum_a (|v_a| + c)/dx_i of the leaf mean. */
int orc_tree_max_dt(const orc_config *c, long nleaf, const int *lev, const long *ix, const long *iy,
                    const double *w, double *dt_out) {
  tree *T = malloc(sizeof(tree));
  int st = tree_init(c, nleaf, lev, ix, iy, T);
  if (st != ORC_OK) { free(T); return st; }
  const ctx *X = &T->X;
  double fk = 1.0 / (2.0 * X->k + 1.0);
  if (c->positivity && X->lw[0] / 2.0 < fk) fk = X->lw[0] / 2.0;
  double dt = INFINITY;
  for (long i = 0; i < nleaf; ++i) {
    double U[MAXV];
    for (int v = 0; v < X->nvar; ++v) U[v] = W(v, 0, i);
    double p = pressure(X, U);
    double cs = sqrt(c->gamma * p / U[0]);
    double dxi = X->dx / (double)(1L << lev[i]);
    double rate = 0.0;
    for (int a = 0; a < X->d; ++a) rate += (fabs(U[1 + a] / U[0]) + cs) / dxi;
    double dtc = c->cfl * fk / rate;
    if (dtc < dt) dt = dtc;
  }
  *dt_out = dt;
  tree_free(T); free(T);
  return ORC_OK;
}


/* Mean over the level-l cell (X, Y) of the piecewise polynomial solution
 * (the neighbour value of the limiters at refinement boundaries, Sec. 4.4):
 * a leaf of the same level gives its mean; a coarser leaf the mean of its
 * polynomial over that cell (its projection onto the smaller volume, here by
 * the (k+1)^2-point Gauss rule on the sub-box, exact for the degree); finer
 * leaves inside the cell their area-weighted means (the node weights). */
static void tree_region_mean(const tree *T, const double *w, const int *lev, int l, long X0, long Y0, double *m) {
  const ctx *X = &T->X;
  long s = 1L << (T->lmax - l);
  long r0 = X0 * s, r1 = r0 + s, q0 = Y0 * s, q1 = q0 + s;
  for (int v = 0; v < X->nvar; ++v) m[v] = 0.0;
  for (long j = 0; j < T->nleaf; ++j) {
    if (!(T->bx0[j] < r1 && r0 < T->bx1[j] && T->by0[j] < q1 && q0 < T->by1[j])) continue;
    if (lev[j] == l) {
      for (int v = 0; v < X->nvar; ++v) m[v] = W(v, 0, j);
      return;
    }
    if (lev[j] < l) {
      double js = (double)(T->bx1[j] - T->bx0[j]);
      double lo[2] = {(2.0 * (r0 - T->bx0[j])) / js - 1.0, (2.0 * (q0 - T->by0[j])) / js - 1.0};
      double hs = (double)s / js; /* half-width of the sub-box in j's reference coordinates */
      for (int q = 0; q < X->Q; ++q) {
        double xi[3] = {lo[0] + hs * (1.0 + X->gx[q % X->n1]), lo[1] + hs * (1.0 + X->gx[q / X->n1]), 0.0};
        for (int v = 0; v < X->nvar; ++v) {
          double u = 0.0;
          for (int ll = 0; ll < X->N; ++ll) u += W(v, ll, j) * phi_at(X, ll, xi);
          m[v] += u * X->wV[q] / 4.0;
        }
      }
      return;
    }
    double frac = 1.0 / (double)(1L << (2 * (lev[j] - l)));
    for (int v = 0; v < X->nvar; ++v) m[v] += W(v, 0, j) * frac;
  }
}

/* Slope limiter (Sec. 3.1-3.3) and positivity limiter (Sec. 3.4) on a
 * quadtree, in place, with the AMR rules of Sec. 4.4: the neighbour value on
 * each side is the mean of the solution over the cell of the leaf's own size
 * there (tree_region_mean, from the state before any limiting), the TVB
 * bound uses the leaf's own edge, and a leaf with finer neighbours also
 * checks positivity at its trace points on the faces to them. */
static int tree_limit(const orc_config *c, long nleaf, const int *lev, const long *ix, const long *iy, double *w,
                      const unsigned char *skip) {
  tree *T = malloc(sizeof(tree));
  int st = tree_init(c, nleaf, lev, ix, iy, T);
  if (st != ORC_OK) { free(T); return st; }
  const ctx *X = &T->X;
  int nv = X->nvar, N = X->N;
  long bad = 0;
  if (c->limiter) {
    double *nbm = calloc((size_t)4 * nv * nleaf, sizeof(double));
    double *dxc = malloc(sizeof(double) * nleaf);
    for (long i = 0; i < nleaf; ++i) {
      dxc[i] = X->dx / (double)(1L << lev[i]);
      if (skip && skip[i]) continue;
      for (int a = 0; a < 2; ++a)
        for (int s = 0; s < 2; ++s) {
          long Xn = ix[i] + (a == 0 ? (s ? 1 : -1) : 0), Yn = iy[i] + (a == 1 ? (s ? 1 : -1) : 0);
          long nxl = (long)c->n[0] << lev[i], nyl = (long)c->n[1] << lev[i];
          int wall = 0;
          if (Xn < 0 || Xn >= nxl) { if (c->bc[0] == 1) wall = 1; else Xn = (Xn + nxl) % nxl; }
          if (Yn < 0 || Yn >= nyl) { if (c->bc[1] == 1) wall = 1; else Yn = (Yn + nyl) % nyl; }
          double m[MAXV];
          if (wall) for (int v = 0; v < nv; ++v) m[v] = W(v, 0, i);
          else tree_region_mean(T, w, lev, lev[i], Xn, Yn, m);
          for (int v = 0; v < nv; ++v) nbm[((long)(2 * a + s) * nv + v) * nleaf + i] = m[v];
        }
    }
    if (c->limiter == 2) char_limit(X, w, nbm, dxc, skip);
    else slope_limit(X, w, nbm, dxc, skip);
    free(nbm); free(dxc);
  }
  if (c->positivity) {
    int xmax = 4 * 4 * X->n1;
    int *xcnt = calloc(nleaf, sizeof(int));
    double *xphi = malloc(sizeof(double) * nleaf * xmax * N);
    for (long i = 0; i < nleaf; ++i)
      for (int a = 0; a < 2 && !(skip && skip[i]); ++a) {
        int b = 1 - a;
        const long *t0 = b == 0 ? T->bx0 : T->by0, *t1 = b == 0 ? T->bx1 : T->by1;
        for (int s = 0; s < 2; ++s) {
          long nb[4], o0[4], o1[4];
          int m = tree_across(T, i, a, s, nb, o0, o1);
          for (int p = 0; p < m; ++p) {
            if (o1[p] - o0[p] == t1[i] - t0[i]) continue; /* not a smaller neighbour */
            for (int r = 0; r < X->n1; ++r) {
              double xi[3] = {0, 0, 0};
              xi[a] = s ? 1.0 : -1.0;
              xi[b] = ((double)(o0[p] + o1[p] - t0[i] - t1[i]) + (double)(o1[p] - o0[p]) * X->gx[r]) /
                      (double)(t1[i] - t0[i]);
              for (int l = 0; l < N; ++l) xphi[((long)i * xmax + xcnt[i]) * N + l] = phi_at(X, l, xi);
              ++xcnt[i];
            }
          }
        }
      }
    bad = positivity_limit(X, w, xcnt, xphi, xmax, skip);
    free(xcnt); free(xphi);
  }
  tree_free(T); free(T);
  return bad ? ORC_ENEGATIVE : ORC_OK;
}

int orc_tree_limit(const orc_config *c, long nleaf, const int *lev, const long *ix, const long *iy, double *w) {
  return tree_limit(c, nleaf, lev, ix, iy, w, NULL);
}

/* The limiters on the listed leaves only (neighbour values from the state as
 * given; the other leaves are left as they are). */
int orc_tree_limit_cells(const orc_config *c, long nleaf, const int *lev, const long *ix, const long *iy, double *w,
                         long ncells, const long *cells) {
  unsigned char *skip = malloc(nleaf);
  if (!skip) return ORC_ENOMEM;
  memset(skip, 1, nleaf);
  for (long k = 0; k < ncells; ++k) {
    if (cells[k] < 0 || cells[k] >= nleaf) { free(skip); return ORC_EINVAL; }
    skip[cells[k]] = 0;
  }
  int st = tree_limit(c, nleaf, lev, ix, iy, w, skip);
  free(skip);
  return st;
}

/* Physical coordinates of every leaf's volume nodes, x[2][Q][nleaf]. */
int orc_tree_node_coords(const orc_config *c, long nleaf, const int *lev, const long *ix, const long *iy,
                         double *x) {
  tree *T = malloc(sizeof(tree));
  int st = tree_init(c, nleaf, lev, ix, iy, T);
  if (st != ORC_OK) { free(T); return st; }
  const ctx *X = &T->X;
  for (long i = 0; i < nleaf; ++i) {
    double h = X->dx / (double)(1L << lev[i]);
    for (int q = 0; q < X->Q; ++q) {
      int iq[2] = {q % X->n1, q / X->n1};
      x[((long)0 * X->Q + q) * nleaf + i] = c->x0[0] + h * (ix[i] + 0.5 * (1.0 + X->gx[iq[0]]));
      x[((long)1 * X->Q + q) * nleaf + i] = c->x0[1] + h * (iy[i] + 0.5 * (1.0 + X->gx[iq[1]]));
    }
  }
  tree_free(T); free(T);
  return ORC_OK;
}

/* L2 projection (Sec. 2.3) of primitives prim[nleaf][Q][5] = (rho, vx, vy, vz,
 * p) at each leaf's volume nodes: the same per-cell projection as on a
 * uniform grid, the leaf edge does not enter. */
int orc_tree_project(const orc_config *c, long nleaf, const int *lev, const long *ix, const long *iy,
                     const double *prim, double *w) {
  tree *T = malloc(sizeof(tree));
  int st = tree_init(c, nleaf, lev, ix, iy, T);
  if (st != ORC_OK) { free(T); return st; }
  const ctx *X = &T->X;
  for (long i = 0; i < nleaf; ++i) {
    double acc[MAXV][MAXN];
    memset(acc, 0, sizeof(acc));
    for (int q = 0; q < X->Q; ++q) {
      const double *pr = prim + (i * X->Q + q) * 5;
      double U[MAXV], ke = 0.0;
      U[0] = pr[0];
      for (int b = 0; b < 2; ++b) { U[1 + b] = pr[0] * pr[1 + b]; ke += pr[1 + b] * pr[1 + b]; }
      U[3] = pr[4] / (c->gamma - 1.0) + 0.5 * pr[0] * ke;
      for (int v = 0; v < X->nvar; ++v)
        for (int j = 0; j < X->N; ++j) acc[v][j] += U[v] * X->phiV[q][j] * X->wV[q];
    }
    for (int v = 0; v < X->nvar; ++v)
      for (int j = 0; j < X->N; ++j) W(v, j, i) = 0.25 * acc[v][j];
  }
  tree_free(T); free(T);
  return ORC_OK;
}

#else /* ORC_CS: complex-step directional derivatives */

/* Directional derivative of the RHS: dL = Im L(w + i h v) / h (and L = Re). */
int orc_cs_rhs(const orc_config *c, const double *w, const double *v, double h, double *L, double *dL) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st != ORC_OK) { free(X); return st; }
  long n = state_size(X);
  real_t *wc = malloc(sizeof(real_t) * n), *Lc = malloc(sizeof(real_t) * n);
  for (long i = 0; i < n; ++i) wc[i] = w[i] + I * h * v[i];
  rhs_all(X, wc, Lc);
  for (long i = 0; i < n; ++i) { L[i] = creal(Lc[i]); dL[i] = cimag(Lc[i]) / h; }
  free(wc); free(Lc); free(X);
  return ORC_OK;
}

/* Directional derivative of nsteps SSP-RK3 steps at fixed dt, unlimited. */
int orc_cs_traj(const orc_config *c, const double *w0, const double *v, double h, int nsteps, double dt,
                double *wT, double *dwT) {
  ctx *X = malloc(sizeof(ctx));
  int st = ctx_init(c, X);
  if (st != ORC_OK) { free(X); return st; }
  long n = state_size(X);
  real_t *u0 = malloc(sizeof(real_t) * n), *u1 = malloc(sizeof(real_t) * n),
         *u2 = malloc(sizeof(real_t) * n), *L = malloc(sizeof(real_t) * n);
  for (long i = 0; i < n; ++i) u0[i] = w0[i] + I * h * v[i];
  for (int s = 0; s < nsteps; ++s) {
    rhs_all(X, u0, L); rk3_combine(1, dt, u0, u0, L, u1, n);
    rhs_all(X, u1, L); rk3_combine(2, dt, u0, u1, L, u2, n);
    rhs_all(X, u2, L); rk3_combine(3, dt, u0, u2, L, u1, n);
    real_t *t = u0; u0 = u1; u1 = t;
  }
  for (long i = 0; i < n; ++i) { wT[i] = creal(u0[i]); dwT[i] = cimag(u0[i]) / h; }
  free(u0); free(u1); free(u2); free(L); free(X);
  return ORC_OK;
}

#endif
