// HIP kernels of libdg for CDNA4 (gfx950) and the C ABI declared in dg.h.
//
// Work decomposition: one thread per cell.  A thread
//   1. reads the cell's modal weights (coalesced: x-fastest SoA layout),
//   2. evaluates the volume integral of eq. dg_term2: the state at each
//      (k+1)^d Gauss node, the Euler flux there, and the projection onto
//      the basis gradients,
//   3. evaluates the face integral of eq. dg_term3 on its 2d faces: the own
//      trace from registers, the neighbour trace from the neighbour's
//      weights (cache resident), the HLLC flux, and the lift onto the basis,
//   4. forms L = (2/dx) 2^-d (V - S) and, fused, the SSP-RK3 stage update.
// Each interior face is evaluated by both of its cells with the same code and
// the same inputs, so the two contributions are bitwise opposite: the cell
// means are updated conservatively without atomics or a second pass.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <mutex>
#include <cstring>
#include <cstdlib>
#include <new>
#include <type_traits>
#include <algorithm>
#include <unordered_map>
#include <utility>
#include <vector>

#include "dg_internal.h"

namespace dg {

template <int D, int K>
struct Cfg {
  static constexpr int NV = D + 2;
  static constexpr int N1 = K + 1;
  static constexpr int N = D == 2 ? (K + 1) * (K + 2) / 2 : (K + 1) * (K + 2) * (K + 3) / 6;
  static constexpr int Q = D == 2 ? N1 * N1 : N1 * N1 * N1;
  static constexpr int QF = Q / N1;
  static constexpr int M = (K + 4) / 2 < 2 ? 2 : (K + 4) / 2;
  static constexpr int NS = D * M * QF;
  static constexpr int B = 0;
  static constexpr int DW = B + Q * N;
  static constexpr int TF = DW + D * Q * N;
  static constexpr int TW = TF + D * 2 * QF * N;
  static constexpr int WQ = TW + D * 2 * QF * N;
  static constexpr int PS = WQ + Q;
  static constexpr int XQ = PS + NS * N;
  static constexpr int HG = XQ + 3 * Q;
  static constexpr int HW = HG + D * 2 * 4 * QF * N;
  static constexpr int CM = HW + D * 2 * 4 * QF * N;
  static constexpr int TOTAL = CM + 8 * N;
};

struct Grid {
  int nx, ny, nz;
  long ncell;
  int bc[3];
  double fac;    // (2/dx) 2^-d
  double gamma;
  // block order of the 3D MFMA stage kernel (block_order): strips of xg
  // blocks, xzc planes per XCD, xp blocks per plane; xg = 0: launch order
  int xg, xzc, xp;
};

// The launch's blocks go to the eight XCDs in turn (block b to XCD b mod 8),
// each XCD with its own L2.  For a 3D grid of whole 64-cell blocks per plane
// (xp of them) and a multiple of eight planes, XCD x takes the planes
// [x xzc, (x + 1) xzc), and its j-th block is strip lo of plane zz of
// strip row hi, strips (xg blocks, one x-row when the row is whole blocks)
// fastest, then the planes, then the strip rows: a block's z neighbours ran
// xg blocks earlier on the same XCD and its y neighbours xg xzc blocks
// earlier, so both are mostly still in that XCD's L2 (in launch order the
// y neighbours sit on another XCD).  A permutation of the blocks whatever
// the dispatch does.
__device__ inline long block_order(const Grid &g, long b) {
  if (g.xg == 0) return b;
  const long x = b & 7, j = b >> 3;
  const long lo = j % g.xg, r = j / g.xg;
  const long zz = r % g.xzc, hi = r / g.xzc;
  return (x * g.xzc + zz) * g.xp + hi * g.xg + lo;
}

enum : int { FLAG_NEGATIVE = 1, FLAG_NAN = 2 };

// Flat index of the neighbour of (ix,iy,iz) along axis a in direction dir,
// or -1 at a transmissive boundary.
__device__ inline long neighbour(const Grid &g, int ix, int iy, int iz, int a, int dir) {
  int i[3] = {ix, iy, iz};
  int n[3] = {g.nx, g.ny, g.nz};
  i[a] += dir;
  if (i[a] < 0 || i[a] >= n[a]) {
    if (g.bc[a] == DG_BC_TRANSMISSIVE) return -1;
    i[a] = i[a] < 0 ? i[a] + n[a] : i[a] - n[a];
  }
  return ((long)i[2] * g.ny + i[1]) * g.nx + i[0];
}

// Reciprocal and reciprocal square root from the hardware estimates plus
// Newton steps (within an ulp or two; the IEEE-rounded division and square
// root expand into much longer dependent sequences).  Used by the Riemann
// solver and the volume flux.
__device__ inline double vrcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ inline double vrsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  // y <- y (3 - x y^2) / 2, twice
  double h = 0.5 * x;
  double t = fma(-h, y * y, 0.5);
  y = fma(y, t, y);
  t = fma(-h, y * y, 0.5);
  return fma(y, t, y);
}
__device__ inline float vrcp(float x) {
  float r = __builtin_amdgcn_rcpf(x);
  return fmaf(r, fmaf(-x, r, 1.0f), r);
}
__device__ inline float vrsq(float x) {
  float y = __builtin_amdgcn_rsqf(x);
  return fmaf(y, fmaf(-0.5f * x, y * y, 0.5f), y);
}

// Signal rate sum_a (|v_a| + c)/dx of a cell mean U (eq. time_step); `bad`
// records a non-positive density or pressure.  Shared by every kernel that
// forms the time step, so that all of them obtain bitwise the same rate.
template <int D>
__device__ inline double cell_rate(const double *U, double gamma, double dx, bool &bad, double gk = 0.0,
                                   double amax = 0.0) {
  double ke = 0.0;
#pragma unroll
  for (int b = 0; b < D; ++b) ke += U[1 + b] * U[1 + b] / U[0];
  const double p = (gamma - 1.0) * (U[D + 1] - 0.5 * ke);
  bad |= !(U[0] > 0.0) || !(p > 0.0);
  const double c = sqrt(gamma * p / U[0]);
  double rate = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) rate += (fabs(U[1 + a] / U[0]) + c) / dx;
  // gravity step (Sec. 2.5) dt <= c / (sqrt(2 gamma (gamma-1)) |grad Phi|) as a
  // rate against the same CFL f_k: gk = CFL f_k sqrt(2 gamma (gamma-1))
  if (amax > 0.0) rate = fmax(rate, gk * amax / c);
  return rate;
}

// maximum over the 64 lanes of a wave (all lanes active)
__device__ inline double wave_max(double x) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
  return x;
}

// The maximum signal rate is reduced into RATE_SLOTS 64-bit words, one per
// 128-byte line, each holding the bit pattern of a non-negative double (such
// doubles order like their bits, so atomicMax on the pattern is a max); the
// rate is the largest slot.  Workgroup b folds into slot b mod 8, i.e. one
// slot per XCD: a single word taking every workgroup's atomic serialises
// them.
constexpr int RATE_SLOTS = 8, RATE_STRIDE = 16;
static_assert(RATE_SLOTS * RATE_STRIDE == DG_RATE_STATE, "layout of the carried rate state");
__device__ inline unsigned long long *rate_slot(unsigned long long *w, int b) {
  return w + RATE_STRIDE * (b % RATE_SLOTS);
}

// Time-step work that the fused SSP-RK3 step hands to the stage kernels
// (see k_rhs_tile2d); `word` is the carried rate state (RATE_SLOTS slots).
enum : int { RATE_NONE = 0, RATE_DT = 1, RATE_CLEAR = 2, RATE_FOLD = 3 };
struct RateOp {
  unsigned long long *word;
  double *dt_out;
  double cfl_fk;  // CFL times the order factor of the time step
  double dx;
  int op;
  const double *gmax = nullptr;  // per cell the largest |grad Phi| at its nodes (gravity), or null
  double gk = 0.0;               // CFL f_k sqrt(2 gamma (gamma-1))
};

// Euler flux f_a(U) (eq. flux_vectors; 2D drops the third velocity).
template <int D, class R>
__device__ inline void euler_flux(const R *U, int a, R gm1, R *F) {
  const R ir = vrcp(U[0]);
  R ke = R(0);
#pragma unroll
  for (int b = 0; b < D; ++b) ke = fma(U[1 + b], U[1 + b] * ir, ke);
  const R p = gm1 * (U[D + 1] - R(0.5) * ke);
  const R va = U[1 + a] * ir;
  F[0] = U[1 + a];
#pragma unroll
  for (int b = 0; b < D; ++b) F[1 + b] = fma(U[1 + b], va, b == a ? p : R(0));
  F[D + 1] = (U[D + 1] + p) * va;
}

// Scalar helpers so that the Riemann solver runs on doubles and on floats
// with the same sequence of operations.
__device__ inline double vfma(double a, double b, double c) { return fma(a, b, c); }
__device__ inline double vsqrt(double a) { return sqrt(a); }
__device__ inline double vmin(double a, double b) { return b < a ? b : a; }
__device__ inline double vmax(double a, double b) { return b > a ? b : a; }
__device__ inline double val(double a) { return a; }
__device__ inline float vfma(float a, float b, float c) { return fmaf(a, b, c); }
__device__ inline float vsqrt(float a) { return sqrtf(a); }
__device__ inline float vmin(float a, float b) { return b < a ? b : a; }
__device__ inline float vmax(float a, float b) { return b > a ? b : a; }
__device__ inline double val(float a) { return a; }


template <class T>
__device__ inline T cst(double x);
template <>
__device__ inline double cst<double>(double x) { return x; }
template <>
__device__ inline float cst<float>(double x) { return (float)x; }

// HLLC numerical flux in +a between traces UL (low side) and UR (high side),
// in the compact form F = F_K + S_K^(-/+) (U*_K - U_K) with K = L if S* >= 0
// (S_L^- = min(S_L, 0)) and K = R otherwise (S_R^+ = max(S_R, 0)); this
// equals the four-region selection of the textbook solver.  Wave-speed
// bounds: Einfeldt-Batten (Roe-averaged, FX = 0) or Davis (FX = 1).
//
// The choice is a template parameter, not a run-time flag: with a uniform
// flag branched on inside loops that run under different exec masks (the
// hanging sub-faces of the refined box), the compiler built the flag's lane
// mask under one exec mask and reused it under another, so lanes that had
// been inactive took the other branch.
template <class T, int D, int FX, bool SEL = false>
__device__ inline void hllc(const T *UL, const T *UR, int a, double g, T *F) {
  // The normal axis a may be a run-time value: components are picked with
  // unrolled compares (no dynamic register indexing).  One reciprocal square
  // root per side gives sqrt(rho) and 1/rho.  SEL: every arm of a
  // conditional is evaluated and the result selected, so the solver contains
  // no branch (a conditional with a costly arm otherwise becomes a divergent
  // branch, which splits the caller's code into separately scheduled blocks;
  // the one-thread-per-cell kernels run faster with the branches).  The
  // results are the same bit for bit.
  const T gm1 = cst<T>(g - 1.0), gg = cst<T>(g), half = cst<T>(0.5);
  const T zero = cst<T>(0.0);
  const T rsL = vrsq(UL[0]), rsR = vrsq(UR[0]);
  const T irL = rsL * rsL, irR = rsR * rsR;
  T vL[D], vR[D], keL = zero, keR = zero, uL = zero, uR = zero, mL = zero, mR = zero;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    vL[b] = UL[1 + b] * irL;
    vR[b] = UR[1 + b] * irR;
    keL = vfma(UL[1 + b], vL[b], keL);
    keR = vfma(UR[1 + b], vR[b], keR);
    if (b == a) {
      uL = vL[b];
      uR = vR[b];
      mL = UL[1 + b];
      mR = UR[1 + b];
    }
  }
  const T pL = gm1 * (UL[D + 1] - half * keL);
  const T pR = gm1 * (UR[D + 1] - half * keR);
  // c = sqrt(g p / rho) = g p rsq(g p rho)
  const T gpL = gg * pL, gpR = gg * pR;
  const T cL = gpL * vrsq(gpL * UL[0]), cR = gpR * vrsq(gpR * UR[0]);
  T SL, SR;
  if constexpr (FX == DG_HLLC_DAVIS) {
    SL = vmin(uL - cL, uR - cR);
    SR = vmax(uL + cL, uR + cR);
  } else {
    const T sL = UL[0] * rsL, sR = UR[0] * rsR;
    const T is = vrcp(sL + sR);
    T q2 = zero, ut = zero;
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const T vt = (sL * vL[b] + sR * vR[b]) * is;
      q2 = vfma(vt, vt, q2);
      if (b == a) ut = vt;
    }
    const T HL = (UL[D + 1] + pL) * irL, HR = (UR[D + 1] + pR) * irR;
    const T Ht = (sL * HL + sR * HR) * is;
    const T ct2 = gm1 * (Ht - half * q2);
    T ct;
    if constexpr (SEL) {
      const T rq = vrsq(ct2);
      ct = val(ct2) > 0.0 ? ct2 * rq : zero;
    } else {
      ct = val(ct2) > 0.0 ? ct2 * vrsq(ct2) : zero;
    }
    SL = vmin(uL - cL, ut - ct);
    SR = vmax(uR + cR, ut + ct);
  }
  const T dL = SL - uL, dR = SR - uR;
  const T Ss = (pR - pL + mL * dL - mR * dR) * vrcp(UL[0] * dL - UR[0] * dR);
  const bool left = val(Ss) >= 0.0;
  T U[D + 2];
#pragma unroll
  for (int v = 0; v < D + 2; ++v) U[v] = left ? UL[v] : UR[v];
  const T SK = left ? SL : SR;
  T SKc;
  if constexpr (SEL) {
    const T SLc = vmin(SL, zero), SRc = vmax(SR, zero);
    SKc = left ? SLc : SRc;
  } else {
    SKc = left ? vmin(SL, zero) : vmax(SR, zero);
  }
  const T irK = left ? irL : irR, pK = left ? pL : pR;
  const T uK = left ? uL : uR, dK = left ? dL : dR, mK = left ? mL : mR;
  T FK[D + 2];
  // physical flux of the selected side
  FK[0] = mK;
#pragma unroll
  for (int b = 0; b < D; ++b) FK[1 + b] = vfma(U[1 + b], uK, b == a ? pK : zero);
  FK[D + 1] = (U[D + 1] + pK) * uK;
  // star state rho_K (S_K - u_K)/(S_K - S*) (1, S* n + v_t, E_K/rho_K + (S* - u_K)(S* + p_K/(rho_K (S_K - u_K))))
  // with r = rho_K (S_K - u_K) and f = r / (S_K - S*): f p_K / r = p_K / (S_K - S*)
  const T ivS = vrcp(SK - Ss);
  const T fac = (U[0] * dK) * ivS;
  T Us[D + 2];
  Us[0] = fac;
#pragma unroll
  for (int b = 0; b < D; ++b) Us[1 + b] = fac * (b == a ? Ss : U[1 + b] * irK);
  Us[D + 1] = vfma(fac, vfma(Ss - uK, Ss, U[D + 1] * irK), (Ss - uK) * pK * ivS);
#pragma unroll
  for (int v = 0; v < D + 2; ++v) F[v] = vfma(SKc, Us[v] - U[v], FK[v]);
}

// Reverse-mode derivative of hllc<double, D, FX>: for the cotangent gF of the
// flux, gUL = (dF/dUL)^T gF and gUR = (dF/dUR)^T gF.  The forward values are
// recomputed with the same expressions as hllc, so every branch (the
// wave-speed bounds, S* >= 0, the min/max against 0) is taken as there; one
// forward and one reverse sweep give both sides' rows at once.
template <int D, int FX>
__device__ inline void hllc_vjp(const double *UL, const double *UR, int a, double g, const double *gF,
                                double *gUL, double *gUR) {
  constexpr int NV = D + 2;
  const double gm1 = g - 1.0;
  // ---- forward
  const double rsL = vrsq(UL[0]), rsR = vrsq(UR[0]);
  const double irL = rsL * rsL, irR = rsR * rsR;
  double vL[D], vR[D], keL = 0.0, keR = 0.0, uL = 0.0, uR = 0.0, mL = 0.0, mR = 0.0;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    vL[b] = UL[1 + b] * irL;
    vR[b] = UR[1 + b] * irR;
    keL = fma(UL[1 + b], vL[b], keL);
    keR = fma(UR[1 + b], vR[b], keR);
    if (b == a) {
      uL = vL[b];
      uR = vR[b];
      mL = UL[1 + b];
      mR = UR[1 + b];
    }
  }
  const double pL = gm1 * (UL[D + 1] - 0.5 * keL);
  const double pR = gm1 * (UR[D + 1] - 0.5 * keR);
  const double kpL = g * pL, kpR = g * pR;  // gamma p
  const double yL = vrsq(kpL * UL[0]), yR = vrsq(kpR * UR[0]);
  const double cL = kpL * yL, cR = kpR * yR;
  double SL, SR;
  bool sl2, sr2;  // the min/max took its second operand
  double sL = 0.0, sR = 0.0, is = 0.0, vt[D], q2 = 0.0, ut = 0.0, HL = 0.0, HR = 0.0, ct2 = 0.0, ct = 0.0;
#pragma unroll
  for (int b = 0; b < D; ++b) vt[b] = 0.0;
  if constexpr (FX == DG_HLLC_DAVIS) {
    const double x1 = uL - cL, y1 = uR - cR, x2 = uL + cL, y2 = uR + cR;
    sl2 = y1 < x1;
    sr2 = y2 > x2;
    SL = sl2 ? y1 : x1;
    SR = sr2 ? y2 : x2;
  } else {
    sL = UL[0] * rsL;
    sR = UR[0] * rsR;
    is = vrcp(sL + sR);
#pragma unroll
    for (int b = 0; b < D; ++b) {
      vt[b] = (sL * vL[b] + sR * vR[b]) * is;
      q2 = fma(vt[b], vt[b], q2);
      if (b == a) ut = vt[b];
    }
    HL = (UL[D + 1] + pL) * irL;
    HR = (UR[D + 1] + pR) * irR;
    const double Ht = (sL * HL + sR * HR) * is;
    ct2 = gm1 * (Ht - 0.5 * q2);
    ct = ct2 > 0.0 ? ct2 * vrsq(ct2) : 0.0;
    const double x1 = uL - cL, y1 = ut - ct, x2 = uR + cR, y2 = ut + ct;
    sl2 = y1 < x1;
    sr2 = y2 > x2;
    SL = sl2 ? y1 : x1;
    SR = sr2 ? y2 : x2;
  }
  const double dL = SL - uL, dR = SR - uR;
  const double iden = vrcp(UL[0] * dL - UR[0] * dR);
  const double Ss = (pR - pL + mL * dL - mR * dR) * iden;
  const bool left = Ss >= 0.0;
  double UK[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) UK[v] = left ? UL[v] : UR[v];
  const double SK = left ? SL : SR;
  const bool pass = left ? !(0.0 < SL) : !(0.0 > SR);  // S_K^-/+ equals S_K (else 0)
  const double SKc = pass ? SK : 0.0;
  const double irK = left ? irL : irR, pK = left ? pL : pR, uK = left ? uL : uR, dK = left ? dL : dR;
  const double ivS = vrcp(SK - Ss);
  const double fac = (UK[0] * dK) * ivS;
  const double A = fma(Ss - uK, Ss, UK[D + 1] * irK);
  double Us[NV];
  Us[0] = fac;
#pragma unroll
  for (int b = 0; b < D; ++b) Us[1 + b] = fac * (b == a ? Ss : UK[1 + b] * irK);
  Us[D + 1] = fma(fac, A, (Ss - uK) * pK * ivS);

  // ---- reverse: F = F_K + SKc (Us - U_K)
  double gUK[NV], gSKc = 0.0;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    gSKc = fma(gF[v], Us[v] - UK[v], gSKc);
    gUK[v] = -SKc * gF[v];
  }
  double gfac = SKc * gF[0], gSs = 0.0, guK = 0.0, girK = 0.0, gpK = 0.0, givS = 0.0;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    const double gu = SKc * gF[1 + b];
    if (b == a) {
      gfac = fma(gu, Ss, gfac);
      gSs = fma(gu, fac, gSs);
    } else {
      gfac = fma(gu, UK[1 + b] * irK, gfac);
      gUK[1 + b] = fma(gu, fac * irK, gUK[1 + b]);
      girK = fma(gu, fac * UK[1 + b], girK);
    }
  }
  {
    const double ge = SKc * gF[D + 1];
    gfac = fma(ge, A, gfac);
    const double gA = ge * fac;
    gSs = fma(gA, 2.0 * Ss - uK, gSs);
    guK = fma(-gA, Ss, guK);
    gUK[D + 1] = fma(gA, irK, gUK[D + 1]);
    girK = fma(gA, UK[D + 1], girK);
    const double t = Ss - uK, gt = ge * pK * ivS;
    gpK = fma(ge, t * ivS, gpK);
    givS = fma(ge, t * pK, givS);
    gSs += gt;
    guK -= gt;
  }
  // fac = rho_K d_K ivS, ivS = 1/(S_K - S*)
  gUK[0] = fma(gfac, dK * ivS, gUK[0]);
  double gdK = gfac * UK[0] * ivS;
  givS = fma(gfac, UK[0] * dK, givS);
  double gSK = -givS * ivS * ivS;
  gSs = fma(givS, ivS * ivS, gSs);
  // F_K
  gUK[1 + a] += gF[0];
#pragma unroll
  for (int b = 0; b < D; ++b) {
    gUK[1 + b] = fma(gF[1 + b], uK, gUK[1 + b]);
    guK = fma(gF[1 + b], UK[1 + b], guK);
  }
  gpK += gF[1 + a];
  gUK[D + 1] = fma(gF[D + 1], uK, gUK[D + 1]);
  gpK = fma(gF[D + 1], uK, gpK);
  guK = fma(gF[D + 1], UK[D + 1] + pK, guK);
  if (pass) gSK += gSKc;
  // d_K = S_K - u_K
  gSK += gdK;
  guK -= gdK;
  // the K side back to L or R
  double gSL = left ? gSK : 0.0, gSR = left ? 0.0 : gSK;
  double gpL = left ? gpK : 0.0, gpR = left ? 0.0 : gpK;
  double guL = left ? guK : 0.0, guR = left ? 0.0 : guK;
  double girL = left ? girK : 0.0, girR = left ? 0.0 : girK;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    gUL[v] = left ? gUK[v] : 0.0;
    gUR[v] = left ? 0.0 : gUK[v];
  }
  // S* = num / den
  const double gnum = gSs * iden, gden = -gSs * Ss * iden;
  gpR += gnum;
  gpL -= gnum;
  gUL[1 + a] = fma(gnum, dL, gUL[1 + a]);
  gUR[1 + a] = fma(-gnum, dR, gUR[1 + a]);
  double gdL = fma(gnum, mL, gden * UL[0]);
  double gdR = fma(-gnum, mR, -gden * UR[0]);
  gUL[0] = fma(gden, dL, gUL[0]);
  gUR[0] = fma(-gden, dR, gUR[0]);
  gSL += gdL;
  guL -= gdL;
  gSR += gdR;
  guR -= gdR;
  // wave-speed bounds
  double gcL = 0.0, gcR = 0.0;
  if constexpr (FX == DG_HLLC_DAVIS) {
    if (sl2) { guR += gSL; gcR -= gSL; } else { guL += gSL; gcL -= gSL; }
    if (sr2) { guR += gSR; gcR += gSR; } else { guL += gSR; gcL += gSR; }
  } else {
    double gut = 0.0, gct = 0.0;
    if (sl2) { gut += gSL; gct -= gSL; } else { guL += gSL; gcL -= gSL; }
    if (sr2) { gut += gSR; gct += gSR; } else { guR += gSR; gcR += gSR; }
    const double gct2 = ct2 > 0.0 ? 0.5 * gct * vrsq(ct2) : 0.0;
    const double gHt = gct2 * gm1, gq2 = -0.5 * gm1 * gct2;
    double gsL = gHt * HL * is, gsR = gHt * HR * is, gis = gHt * (sL * HL + sR * HR);
    const double gHL = gHt * sL * is, gHR = gHt * sR * is;
#pragma unroll
    for (int b = 0; b < D; ++b) {
      const double gv = fma(2.0 * vt[b], gq2, b == a ? gut : 0.0);
      gsL = fma(gv, vL[b] * is, gsL);
      gsR = fma(gv, vR[b] * is, gsR);
      gis = fma(gv, sL * vL[b] + sR * vR[b], gis);
      // vt depends on vL, vR: folded into the velocity gradients below
      gUL[1 + b] = fma(gv * sL * is, irL, gUL[1 + b]);
      girL = fma(gv * sL * is, UL[1 + b], girL);
      gUR[1 + b] = fma(gv * sR * is, irR, gUR[1 + b]);
      girR = fma(gv * sR * is, UR[1 + b], girR);
    }
    gsL = fma(-gis, is * is, gsL);
    gsR = fma(-gis, is * is, gsR);
    // H = (E + p) / rho
    gUL[D + 1] = fma(gHL, irL, gUL[D + 1]);
    gpL = fma(gHL, irL, gpL);
    girL = fma(gHL, UL[D + 1] + pL, girL);
    gUR[D + 1] = fma(gHR, irR, gUR[D + 1]);
    gpR = fma(gHR, irR, gpR);
    girR = fma(gHR, UR[D + 1] + pR, girR);
    // s = sqrt(rho)
    gUL[0] = fma(gsL, 0.5 * rsL, gUL[0]);
    gUR[0] = fma(gsR, 0.5 * rsR, gUR[0]);
  }
  // c = sqrt(g p / rho): dc/dp = g y / 2, dc/drho = -c / (2 rho)
  gpL = fma(gcL, 0.5 * g * yL, gpL);
  gUL[0] = fma(-gcL, 0.5 * cL * irL, gUL[0]);
  gpR = fma(gcR, 0.5 * g * yR, gpR);
  gUR[0] = fma(-gcR, 0.5 * cR * irR, gUR[0]);
  // u = m_a / rho (as v_a); p = gm1 (E - ke/2), ke = sum m_b v_b, v_b = m_b / rho
  const double gkeL = -0.5 * gm1 * gpL, gkeR = -0.5 * gm1 * gpR;
  gUL[D + 1] = fma(gm1, gpL, gUL[D + 1]);
  gUR[D + 1] = fma(gm1, gpR, gUR[D + 1]);
#pragma unroll
  for (int b = 0; b < D; ++b) {
    const double gvL = fma(gkeL, UL[1 + b], b == a ? guL : 0.0);
    const double gvR = fma(gkeR, UR[1 + b], b == a ? guR : 0.0);
    gUL[1 + b] = fma(gkeL, vL[b], fma(gvL, irL, gUL[1 + b]));
    gUR[1 + b] = fma(gkeR, vR[b], fma(gvR, irR, gUR[1 + b]));
    girL = fma(gvL, UL[1 + b], girL);
    girR = fma(gvR, UR[1 + b], girR);
  }
  // ir = 1 / rho
  gUL[0] = fma(-girL, irL * irL, gUL[0]);
  gUR[0] = fma(-girR, irR * irR, gUR[0]);
}

// ---------------------------------------------------------------------------
// One stage of the time integrator in Shu-Osher form (App. D): with u the
// stage input, out = cu u + cl dt L(u) + sum_k a_k y_k over earlier stage
// values y_k (the stage values of an explicit Runge-Kutta tableau; SSP-RK3 is
// cu = cl = 1, then 1/4, 1/4 with 3/4 w^n, then 2/3, 2/3 with 1/3 w^n).
// ---------------------------------------------------------------------------
constexpr int MIX_MAX = 4;
struct Mix {
  const double *y[MIX_MAX];
  double a[MIX_MAX];
  double cu, cl;
  int n;
};

// the terms k >= k0 of the sum, added to o
__device__ inline double mix_tail(const Mix &m, double o, long i, int k0) {
#pragma unroll
  for (int k = 0; k < MIX_MAX; ++k)
    if (k >= k0 && k < m.n) o = fma(m.a[k], m.y[k][i], o);
  return o;
}

__device__ inline double mix_out(const Mix &m, double u, double L, double cldt, long i) {
  return mix_tail(m, fma(cldt, L, m.cu * u), i, 0);
}

// ---------------------------------------------------------------------------
// Right-hand side and fused stage.
// mode 0: out = L;  mode 1: out = the stage combination mx (above).
// ---------------------------------------------------------------------------
// GRAV: add the gravity source (eq. gravity_term) from grav, the external
// acceleration at the volume nodes times (dx/2) w_q, [D][Q][ncell] (FP64 only).
template <int D, int K, class R, int FX, bool GRAV = false>
__global__ __launch_bounds__(256) void k_rhs_stage(const double *__restrict__ tab, const R *__restrict__ tabr,
                                                   const double *__restrict__ w, double *__restrict__ out,
                                                   const double *__restrict__ dtp, const float *__restrict__ vext,
                                                   Grid g, int mode, Mix mx, int *__restrict__ flag,
                                                   const double *__restrict__ grav) {
  // R is the type of the contractions and fluxes (double, or float for the
  // mixed-precision path); the lift of the cell mean and the stage update are
  // always FP64.
  using C = Cfg<D, K>;
  const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  const long nc = g.ncell;
  const int ix = (int)(cell % g.nx);
  const int iy = (int)((cell / g.nx) % g.ny);
  const int iz = (int)(cell / ((long)g.nx * g.ny));
  const R gm1 = (R)(g.gamma - 1.0);

  R wc[C::NV][C::N];
#pragma unroll
  for (int v = 0; v < C::NV; ++v)
#pragma unroll
    for (int l = 0; l < C::N; ++l) wc[v][l] = (R)w[(long)(v * C::N + l) * nc + cell];

  R acc[C::NV][C::N];  // modes l >= 1
  double acc0[C::NV];  // mode 0 (the cell mean), FP64
#pragma unroll
  for (int v = 0; v < C::NV; ++v) {
    acc0[v] = 0.0;
#pragma unroll
    for (int l = 0; l < C::N; ++l) acc[v][l] = R(0);
  }

  // volume integral (eq. dg_term2); dphi_1 = 0, so it never touches mode 0.
  // With vext the volume term comes precomputed (BF16 MFMA path).
  if (vext) {
#pragma unroll
    for (int v = 0; v < C::NV; ++v)
#pragma unroll
      for (int l = 1; l < C::N; ++l) acc[v][l] = (R)vext[(long)(v * C::N + l) * nc + cell];
  }
#pragma unroll 1
  for (int q = 0; q < (vext ? 0 : C::Q); ++q) {
    R U[C::NV];
    const R *bq = tabr + C::B + q * C::N;
#pragma unroll
    for (int v = 0; v < C::NV; ++v) {
      R s = R(0);
#pragma unroll
      for (int l = 0; l < C::N; ++l) s = fma(wc[v][l], bq[l], s);
      U[v] = s;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      R F[C::NV];
      euler_flux<D, R>(U, a, gm1, F);
      const R *dw = tabr + C::DW + (a * C::Q + q) * C::N;
#pragma unroll
      for (int v = 0; v < C::NV; ++v)
#pragma unroll
        for (int l = 1; l < C::N; ++l) acc[v][l] = fma(F[v], dw[l], acc[v][l]);
    }
    if constexpr (GRAV) {
      // s = (0, rho a, m . a) at the node, projected onto every mode
      static_assert(sizeof(R) == sizeof(double), "the gravity source is FP64");
      double sv[C::NV];
      double work = 0.0;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double ga = grav[(long)(a * C::Q + q) * nc + cell];
        sv[1 + a] = U[0] * ga;
        work = fma(U[1 + a], ga, work);
      }
      sv[D + 1] = work;
#pragma unroll
      for (int v = 1; v < C::NV; ++v) {
        acc0[v] = fma(sv[v], bq[0], acc0[v]);
#pragma unroll
        for (int l = 1; l < C::N; ++l) acc[v][l] = fma(sv[v], bq[l], acc[v][l]);
      }
    }
  }

  // face integral (eq. dg_term3) over the 2d faces.  One call site of the
  // Riemann solver: the low and high cell of a face feed it the same
  // (U_low, U_high) and obtain the same flux bit for bit.
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      const long nb = neighbour(g, ix, iy, iz, a, s ? 1 : -1);
      const long src = nb >= 0 ? nb : cell;
      R wb[C::NV][C::N];
#pragma unroll
      for (int v = 0; v < C::NV; ++v)
#pragma unroll
        for (int l = 0; l < C::N; ++l) wb[v][l] = (R)w[(long)(v * C::N + l) * nc + src];
      const R *to = tabr + C::TF + (a * 2 + s) * C::QF * C::N;
      const R *tn = tabr + C::TF + (a * 2 + (1 - s)) * C::QF * C::N;
      const R *tw = tabr + C::TW + (a * 2 + s) * C::QF * C::N;
      const double *tw0 = tab + C::TW + (a * 2 + s) * C::QF * C::N;
#pragma unroll 1
      for (int r = 0; r < C::QF; ++r) {
        R Uo[C::NV], Un[C::NV], UL[C::NV], UR[C::NV], F[C::NV];
#pragma unroll
        for (int v = 0; v < C::NV; ++v) {
          R so = R(0), sn = R(0);
#pragma unroll
          for (int l = 0; l < C::N; ++l) {
            so = fma(wc[v][l], to[r * C::N + l], so);
            sn = fma(wb[v][l], tn[r * C::N + l], sn);
          }
          Uo[v] = so;
          Un[v] = nb >= 0 ? sn : so;  // transmissive: ghost trace = own trace
          UL[v] = s ? Uo[v] : Un[v];
          UR[v] = s ? Un[v] : Uo[v];
        }
        hllc<R, D, FX>(UL, UR, a, g.gamma, F);
#pragma unroll
        for (int v = 0; v < C::NV; ++v) {
          const R f = s ? -F[v] : F[v];
          acc0[v] = fma((double)f, tw0[r * C::N], acc0[v]);
#pragma unroll
          for (int l = 1; l < C::N; ++l) acc[v][l] = fma(f, tw[r * C::N + l], acc[v][l]);
        }
      }
    }
  }

  bool bad = false;
  const double cldt = (mode == 0) ? 0.0 : mx.cl * *dtp;
#pragma unroll
  for (int v = 0; v < C::NV; ++v)
#pragma unroll
    for (int l = 0; l < C::N; ++l) {
      const long i = (long)(v * C::N + l) * nc + cell;
      const double L = g.fac * (l == 0 ? acc0[v] : (double)acc[v][l]);
      bad |= (L != L);
      // FP64: the coefficient loaded at the start, not read again
      const double u = sizeof(R) == sizeof(double) ? (double)wc[v][l] : w[i];
      out[i] = (mode == 0) ? L : mix_out(mx, u, L, cldt, i);
    }
  if (bad) atomicOr(flag, FLAG_NAN);
}

// ---------------------------------------------------------------------------
// 2D right-hand side + SSP-RK3 stage on LDS tiles, four lanes per cell.
//
// In 2D there are four conserved variables and a workgroup owns a TX x TY
// tile of cells with four adjacent lanes per cell (lane = 4 cell + sub), so a
// 256^2 grid still gives four waves per SIMD to hide the latency of the
// FP64 divisions and square roots of the flux evaluations.
//   P0  weights of the tile and its one-cell halo (no corners) into LDS with
//       coalesced row loads, all in flight together;
//   P1  every face of the tile once: the (face, node) tasks are spread over
//       the whole workgroup; each forms both traces from LDS, calls the HLLC
//       solver and stores the flux in LDS;
//   P2  the volume integral: the (k+1)^2 nodes of a cell are split over its
//       four lanes, and a reduce-scatter across the four lanes (DPP quad
//       permutations, no LDS) leaves lane `sub` with variable `sub`;
//   P3  after a barrier each lane lifts the four face fluxes of its
//       variable and applies the stage update to it.
// A face on a tile boundary is evaluated by both tiles with identical code
// and inputs, so the two cells receive bitwise-opposite contributions.
// ---------------------------------------------------------------------------
// TS = 1: 8x8 tiles (256 threads).  Four such work-groups fit a CU at k = 2
// (LDS 35 KB, 124 VGPRs each), and once they drift apart the load, compute and
// store phases of different tiles overlap, which one 1024-thread work-group
// per CU cannot do; a small grid also spreads over more CUs.
// TS = 0: 16x16 or 16x8 tiles (see tile2d_small for which runs when).
template <int K, int TS = 0>
struct Tile2D {
  static constexpr int TX = 8, TY = 8;
};
#ifndef DG_TILE2D_TY2
#define DG_TILE2D_TY2 16
#endif
#ifndef DG_TILE2D_TY3
#define DG_TILE2D_TY3 8
#endif
template <>
struct Tile2D<1, 0> { static constexpr int TX = 16, TY = 16; };
template <>
struct Tile2D<2, 0> { static constexpr int TX = 16, TY = DG_TILE2D_TY2; };
template <>
struct Tile2D<3, 0> { static constexpr int TX = 16, TY = DG_TILE2D_TY3; };
template <>
struct Tile2D<4, 0> { static constexpr int TX = 16, TY = 8; };

// Whether a stage runs on 8x8 tiles: always for k <= 3 (faster at every grid
// size measured, 256^2 to 1024^2); at k = 4 an 8x8 work-group needs 85 KB of
// LDS and more than 256 registers per lane, so a CU runs one wave per SIMD
// and the 16x8 tiles (two per SIMD) run unless the grid has fewer of them
// than the GPU has CUs.  force = 0 or 1 overrides the choice.
constexpr long kCusPerGpu = 256;
inline bool tile2d_small(int k, long large_tiles, int force) {
  if (force >= 0) return force == 1;
  return k <= 3 || large_tiles < kCusPerGpu;
}

// Exchange of a value with the lane `sub ^ 1` or `sub ^ 2` of the same quad
// (DPP quad permutation, no LDS traffic).
template <int CTRL>
__device__ inline double quad_swap(double x) {
  const int lo = __double2loint(x), hi = __double2hiint(x);
  const int lo2 = __builtin_amdgcn_mov_dpp(lo, CTRL, 0xF, 0xF, false);
  const int hi2 = __builtin_amdgcn_mov_dpp(hi, CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi2, lo2);
}
template <int CTRL>
__device__ inline float quad_swap(float x) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(x), CTRL, 0xF, 0xF, false));
}
constexpr int kQuadXor1 = 0xB1;  // quad_perm [1,0,3,2]
constexpr int kQuadXor2 = 0x4E;  // quad_perm [2,3,0,1]
// value of lane J of the quad
template <int J>
__device__ inline double quad_from(double x) {
  return quad_swap<J | (J << 2) | (J << 4) | (J << 6)>(x);
}

template <int K, class R, int FX, bool GRAV = false, int TS = 0>
__global__ __launch_bounds__((4 * Tile2D<K, TS>::TX * Tile2D<K, TS>::TY)) void k_rhs_tile2d(
    const double *__restrict__ tab, const R *__restrict__ tabr, const double *__restrict__ w,
    double *__restrict__ out, const double *__restrict__ dtp, const float *__restrict__ vext, Grid g, int mode,
    Mix mx, int *__restrict__ flag, RateOp ro, const double *__restrict__ grav) {
  // GRAV: gravity source from grav as in k_rhs_stage (FP64 only).
  // R: type of the contractions and fluxes (double, or float in the mixed
  // path); the lift of the cell mean and the stage update are FP64.
  // ro (fused step): RATE_DT takes dt = CFL f_k / max rate from the slots of
  // ro.word instead of *dtp and block 0 stores it to ro.dt_out; RATE_CLEAR
  // zeroes the slots; RATE_FOLD folds the signal rate of the new cell means
  // into them.
  using C = Cfg<2, K>;
  constexpr int TX = Tile2D<K, TS>::TX, TY = Tile2D<K, TS>::TY, NCELL = TX * TY, NT = 4 * NCELL;
  constexpr int NV = C::NV, N = C::N, QF = C::QF, Q = C::Q, NW = NV * N;
  static_assert(NV == 4, "four lanes per cell carry the four 2D variables");
  constexpr int HX = TX + 2, HY = TY + 2, HC = HX * HY;
  constexpr int NFX = TY * (TX + 1), NFY = (TY + 1) * TX;  // x- and y-faces of the tile
  constexpr int NTASK = (NFX + NFY) * QF;
  __shared__ R sw[NW * HC];
  __shared__ R sf[(NFX + NFY) * QF * NV];  // [face][node][var]
  __shared__ unsigned long long smax;       // block maximum of the signal rate
  __shared__ double sdt;                    // the stage's dt
  __shared__ R stab[C::WQ];                 // basis, derivative-weight, trace and lifting tables

  const int tid = threadIdx.x;
  const int cidx = tid >> 2, sub = tid & 3;
  // the stage's dt (or the carried rate) and the small tables are loaded
  // before the halo and stored after it, so that no load waits on another
  // (a relaxed atomic read keeps it a vector load: a scalar load would be
  // waited for together with the kernel arguments, before the halo loads)
  unsigned long long dbits = 0ull;  // dt, or one slot of the carried rate
  if (mode != 0 && tid < (ro.op == RATE_DT ? RATE_SLOTS : 1)) {
    const unsigned long long *src =
        ro.op == RATE_DT ? ro.word + RATE_STRIDE * tid : reinterpret_cast<const unsigned long long *>(dtp);
    dbits = __hip_atomic_load(src, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  constexpr int TPT = (C::WQ + NT - 1) / NT;
  R tv[TPT];
#pragma unroll
  for (int j = 0; j < TPT; ++j) tv[j] = tid + j * NT < C::WQ ? tabr[tid + j * NT] : R(0);
  if (tid == 0) smax = 0ull;
  if (blockIdx.x == 0 && ro.op == RATE_CLEAR && tid < RATE_SLOTS) ro.word[RATE_STRIDE * tid] = 0ull;
  const int tx = cidx % TX, ty = cidx / TX;
  // Workgroups are dispatched round-robin over the 8 XCDs (block b runs on
  // XCD b mod 8).  Give each XCD a contiguous band of tiles so that the halo
  // rows it re-reads stay in its own L2: a bijection for any tile count.
  const int ntx = (g.nx + TX - 1) / TX;
  const int ntiles = gridDim.x;
  const int xcd = blockIdx.x % 8, j = blockIdx.x / 8;
  const int q8 = ntiles / 8, r8 = ntiles % 8;
  const int tile = xcd * q8 + min(xcd, r8) + j;
  const int bx0 = (tile % ntx) * TX, by0 = (tile / ntx) * TY;
  const long nc = g.ncell;
  const int nxt = min(TX, g.nx - bx0), nyt = min(TY, g.ny - by0);

  // P0: tile and halo weights into LDS (periodic wrap; transmissive ghosts are
  // resolved at the faces).  Thread t owns halo position h = t mod HC for the
  // weights vl = t / HC, t / HC + R0, ...: the cell index is formed once and
  // the NW / R0 loads of a thread are all in flight together.
  {
    constexpr int R0 = NT / HC;
    static_assert(R0 >= 1 && NW % R0 == 0, "whole rows of halo positions");
    const int h = tid % HC, v0 = tid / HC;
    const int lx = h % HX - 1, ly = h / HX - 1;
    const bool corner = (lx < 0 || lx >= TX) && (ly < 0 || ly >= TY);
    if (v0 < R0 && !corner) {
      // periodic wrap of the halo; positions past the first halo column/row
      // of a partial tile are never read and are only kept inside the grid
      int gx = bx0 + lx, gy = by0 + ly;
      gx = gx < 0 ? gx + g.nx : (gx >= g.nx ? gx - g.nx : gx);
      gy = gy < 0 ? gy + g.ny : (gy >= g.ny ? gy - g.ny : gy);
      gx = min(gx, g.nx - 1);
      gy = min(gy, g.ny - 1);
      const double *src = w + (long)v0 * nc + (long)gy * g.nx + gx;
      R *dst = sw + v0 * HC + h;
      double vals[NW / R0];
#pragma unroll
      for (int j = 0; j < NW / R0; ++j) vals[j] = src[(long)j * R0 * nc];
#pragma unroll
      for (int j = 0; j < NW / R0; ++j) dst[j * R0 * HC] = (R)vals[j];
    }
  }
#pragma unroll
  for (int j = 0; j < TPT; ++j)
    if (tid + j * NT < C::WQ) stab[tid + j * NT] = tv[j];
  if (tid < 64) {  // wave 0: the largest slot (lanes past the slots hold 0)
    if (ro.op == RATE_DT) {
#pragma unroll
      for (int off = RATE_SLOTS / 2; off > 0; off >>= 1) {
        const unsigned long long o =
            (unsigned long long)__double_as_longlong(__shfl_xor(__longlong_as_double((long long)dbits), off));
        dbits = o > dbits ? o : dbits;
      }
    }
    if (tid == 0) {
      const double dv = __longlong_as_double((long long)dbits);
      const double dt = ro.op == RATE_DT ? ro.cfl_fk / dv : dv;
      sdt = dt;
      if (blockIdx.x == 0 && ro.op == RATE_DT) ro.dt_out[0] = dt;
    }
  }
  __syncthreads();

  // P1: face-node tasks.  x-face (fx, fy) lies between halo cells
  // (fx, fy+1) and (fx+1, fy+1); y-face (fx, fy) between (fx+1, fy) and
  // (fx+1, fy+1).
  const bool tr_x = g.bc[0] == DG_BC_TRANSMISSIVE, tr_y = g.bc[1] == DG_BC_TRANSMISSIVE;
  for (int t = tid; t < NTASK; t += NT) {
    const int f = t / QF, r = t % QF;
    int a, pl, ph;
    bool ghost_lo, ghost_hi;
    if (f < NFX) {
      const int fy = f / (TX + 1), fx = f % (TX + 1);
      a = 0;
      pl = (fy + 1) * HX + fx;
      ph = pl + 1;
      const int gxl = bx0 + fx - 1;  // global x of the low cell
      ghost_lo = tr_x && gxl < 0;
      ghost_hi = tr_x && gxl >= g.nx - 1;
    } else {
      const int f2 = f - NFX;
      const int fy = f2 / TX, fx = f2 % TX;
      a = 1;
      pl = fy * HX + fx + 1;
      ph = pl + HX;
      const int gyl = by0 + fy - 1;
      ghost_lo = tr_y && gyl < 0;
      ghost_hi = tr_y && gyl >= g.ny - 1;
    }
    const R *tlo = stab + C::TF + ((a * 2 + 1) * QF + r) * N;  // low cell at xi_a = +1
    const R *thi = stab + C::TF + ((a * 2 + 0) * QF + r) * N;  // high cell at xi_a = -1
    R UL[NV], UR[NV], F[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      R sl = R(0), sh = R(0);
#pragma unroll
      for (int l = 0; l < N; ++l) {
        sl = fma(sw[(v * N + l) * HC + pl], tlo[l], sl);
        sh = fma(sw[(v * N + l) * HC + ph], thi[l], sh);
      }
      UL[v] = ghost_lo ? sh : sl;
      UR[v] = ghost_hi ? sl : sh;
    }
    hllc<R, 2, FX>(UL, UR, a, g.gamma, F);
#pragma unroll
    for (int v = 0; v < NV; ++v) sf[t * NV + v] = F[v];
  }

  // P2: volume integral (eq. dg_term2) over the nodes q = sub, sub+4, ...;
  // dphi_1 = 0, so mode 0 receives nothing (except from a gravity source)
  const int own = (ty + 1) * HX + (tx + 1);
  const bool real = tx < nxt && ty < nyt;
  const long cellg = (long)(by0 + min(ty, nyt - 1)) * g.nx + (bx0 + min(tx, nxt - 1));
  R acc[NV][N];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int l = 0; l < N; ++l) acc[v][l] = R(0);
  {
    R wc[NV][N];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int l = 0; l < N; ++l) wc[v][l] = sw[(v * N + l) * HC + own];
    const R gm1 = (R)(g.gamma - 1.0);
#pragma unroll 1
    for (int q = sub; q < (vext ? 0 : Q); q += 4) {
      const R *bq = stab + C::B + q * N;
      R U[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        R s = R(0);
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(wc[v][l], bq[l], s);
        U[v] = s;
      }
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        R F[NV];
        euler_flux<2, R>(U, a, gm1, F);
        const R *dw = stab + C::DW + (a * Q + q) * N;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int l = 1; l < N; ++l) acc[v][l] = fma(F[v], dw[l], acc[v][l]);
      }
      if constexpr (GRAV) {
        // s = (0, rho a, m . a) at the node, projected onto every mode (mode
        // 0 included: acc[v][0] is only used by the source)
        static_assert(sizeof(R) == sizeof(double), "the gravity source is FP64");
        const double gx = grav[(long)q * nc + cellg], gy = grav[(long)(Q + q) * nc + cellg];
        const double sv[NV] = {0.0, U[0] * gx, U[0] * gy, fma(U[1], gx, U[2] * gy)};
#pragma unroll
        for (int v = 1; v < NV; ++v)
#pragma unroll
          for (int l = 0; l < N; ++l) acc[v][l] = fma(sv[v], bq[l], acc[v][l]);
      }
    }
  }
  // reduce-scatter over the quad: lane sub keeps variable sub
  R part[2][N];
  {
    const bool hi2 = sub & 2;
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int l = GRAV ? 0 : 1; l < N; ++l) {
        const R keep = hi2 ? acc[2 + j][l] : acc[j][l];
        const R send = hi2 ? acc[j][l] : acc[2 + j][l];
        part[j][l] = keep + quad_swap<kQuadXor2>(send);
      }
  }
  R accv[N];
  accv[0] = R(0);
  {
    const bool hi1 = sub & 1;
#pragma unroll
    for (int l = GRAV ? 0 : 1; l < N; ++l) {
      const R keep = hi1 ? part[1][l] : part[0][l];
      const R send = hi1 ? part[0][l] : part[1][l];
      accv[l] = keep + quad_swap<kQuadXor1>(send);
    }
  }
  if (vext && real) {
    const long c2 = (long)(by0 + ty) * g.nx + (bx0 + tx);
#pragma unroll
    for (int l = 1; l < N; ++l) accv[l] = (R)vext[(long)(sub * N + l) * nc + c2];
  }
  // the stage update's operands (variable sub of the own cell), loaded before
  // the barrier so that their latency overlaps it and the lift
  double wo[N], wno[N];
  const long cell = (long)(by0 + min(ty, nyt - 1)) * g.nx + (bx0 + min(tx, nxt - 1));
#pragma unroll
  for (int l = 0; l < N; ++l) {
    const long i = (long)(sub * N + l) * nc + cell;
    wo[l] = (mode != 0) ? w[i] : 0.0;
    wno[l] = (mode != 0 && mx.n > 0) ? mx.y[0][i] : 0.0;
  }
  __syncthreads();

  // P3: lift the four face fluxes of variable `sub` (eq. dg_term3) and update;
  // the mean is lifted in FP64
  double mean = 0.0;  // new mean of variable sub
  if (real) {
    const int v = sub;
    double acc0 = GRAV ? (double)accv[0] : 0.0;  // the mean's volume term is the source's alone
    // one face per iteration keeps its lifting weights (uniform) in scalar
    // registers without spilling the other faces' weights
#pragma unroll 1
    for (int f = 0; f < 4; ++f) {
      const int a = f >> 1, side = f & 1;  // side 0: low face (xi_a = -1), 1: high face
      const int fi = a == 0 ? ty * (TX + 1) + tx + side : NFX + (ty + side) * TX + tx;
#pragma unroll
      for (int r = 0; r < QF; ++r) {
        const R *tw = stab + C::TW + ((a * 2 + side) * QF + r) * N;
        const R F = sf[(fi * QF + r) * NV + v];
        const R fv = side ? -F : F;
        double t0;
        if constexpr (sizeof(R) == sizeof(double))
          t0 = tw[0];
        else
          t0 = tab[C::TW + ((a * 2 + side) * QF + r) * N];
        acc0 = fma((double)fv, t0, acc0);
#pragma unroll
        for (int l = 1; l < N; ++l) accv[l] = fma(fv, tw[l], accv[l]);
      }
    }
    bool bad = false;
    const double cldt = mx.cl * sdt;
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const long i = (long)(v * N + l) * nc + cell;
      const double L = g.fac * (l == 0 ? acc0 : (double)accv[l]);
      bad |= (L != L);
      double o = L;
      if (mode != 0) {
        o = fma(cldt, L, mx.cu * wo[l]);
        if (mx.n > 0) o = fma(mx.a[0], wno[l], o);
        o = mix_tail(mx, o, i, 1);
      }
      out[i] = o;
      if (l == 0) mean = o;
    }
    if (bad) atomicOr(flag, FLAG_NAN);
  }
  if (ro.op == RATE_FOLD) {
    // rate of the new cell mean (the limiters leave means unchanged, so it is
    // the rate of the limited state too): a wave max, one LDS max per wave,
    // one global max per block
    double r = 0.0;
    if (real) {
      const double U[4] = {quad_from<0>(mean), quad_from<1>(mean), quad_from<2>(mean), quad_from<3>(mean)};
      bool neg = false;
      r = cell_rate<2>(U, g.gamma, ro.dx, neg, ro.gk, ro.gmax ? ro.gmax[cell] : 0.0);
      if (neg && sub == 0) atomicOr(flag, FLAG_NEGATIVE);
    }
    r = wave_max(r);
    if ((tid & 63) == 0) atomicMax(&smax, (unsigned long long)__double_as_longlong(r));
    __syncthreads();
    if (tid == 0) atomicMax(rate_slot(ro.word, blockIdx.x), smax);
  }
}

// ---------------------------------------------------------------------------
// 3D right-hand side + stage with the contractions on MFMA (FP64; FP32 and
// BF16 forms below).
//
// Every contraction of eqs. dg_term2 and dg_term3 is a small GEMM batched
// over cells, run with v_mfma_f64_16x16x4f64 (D[16x16] += A[16x4] B[4x16]):
// a wave owns 16 consecutive cells (the GEMM columns), lane l = 16 g + c
// holds B[g][c] and A[c][g] and receives D[4r + g][c] in its register r,
// r = 0..3 (the operand layouts, checked on the device).
//   evaluation  U_v[p][c] = sum_l E[p][l] w_v[l][c]        (A = table E,
//               rows p = volume nodes or the nine points of one face side;
//               B = the cells' modal weights, K = modes in steps of 4);
//   projection  acc_v[j][c] += sum_p T[j][p] F_v[p][c]     (A = table T,
//               rows j = modes; B = fluxes at the points).
// The evaluation leaves in lane (g, c) the state of cell c at points
// 4r + g, r = 0..3, all five variables, so the Euler flux and the HLLC flux
// are computed in-lane (VALU, overlapping the matrix pipe), and register r of
// that result is directly the B operand of the projection over the points
// {4r + k : k = 0..3}: the tables' K order follows it, so no data moves
// between lanes.  Tables (the A operands, laid out per lane) sit in LDS.
// Point and mode indices 4r + g make whole registers r padding (points or
// modes past the end), which are skipped at compile time.
// As in k_rhs_stage, each face is evaluated by both of its cells from the
// same weights, tables and operation order, so both obtain the same flux.
// ---------------------------------------------------------------------------
// The refined box's geometry (see k_rhs_amr below).
struct AmrGrid {
  int n[3];    // base (coarse) grid
  int lo[3], hi[3];
  int nf[3];   // fine block
  long ncc, ncf;
  int bc[3];
  double facc, facf, dxc, dxf;
  double gamma;
};

template <int D>
__device__ inline bool amr_in_hole(const AmrGrid &g, const int *i) {
#pragma unroll
  for (int a = 0; a < D; ++a)
    if (i[a] < g.lo[a] || i[a] >= g.hi[a]) return false;
  return true;
}

// base-grid neighbour along a (periodic); false at a transmissive wall
template <int D>
__device__ inline bool amr_coarse_nb(const AmrGrid &g, const int *i, int a, int dir, int *j) {
#pragma unroll
  for (int b = 0; b < 3; ++b) j[b] = i[b];
  j[a] += dir;
  if (j[a] < 0 || j[a] >= g.n[a]) {
    if (g.bc[a] == DG_BC_TRANSMISSIVE) return false;
    j[a] = j[a] < 0 ? j[a] + g.n[a] : j[a] - g.n[a];
  }
  return true;
}

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// D += A B on the 16x16x4 MFMA of the contraction type.  The FP32 form's
// result rows lie transposed within each group of four: register r of lane
// (g, c) holds D[4 g + r][c] (FP64: D[4 r + g][c]), which the FP32 tables
// undo by storing row 4 g + r at operand row 4 r + g (mf3_tables_f32), so
// the kernel's register and lane bookkeeping is that of the FP64 form.
template <class R>
struct Mv4;
template <>
struct Mv4<double> {
  using T = d4;
  static __device__ inline T mma(double a, double b, T c) { return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0); }
};
template <>
struct Mv4<float> {
  using T = f4;
  static __device__ inline T mma(float a, float b, T c) { return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0); }
};

template <int K, class R = double>
struct Mf3 {
  using C = Cfg<3, K>;
  static constexpr int N = C::N, Q = C::Q, QF = C::QF, NV = C::NV;
  static constexpr int NKS = (N + 3) / 4;    // K steps of the evaluation (modes)
  static constexpr int NQT = (Q + 15) / 16;  // volume-node tiles
  static constexpr int NFT = (QF + 15) / 16; // face-point tiles per side
  static constexpr int NMT = (N + 15) / 16;  // mode tiles of the result
  // operand blocks of 64 doubles (one per lane): the volume phase's, then
  // the face phase's
  static constexpr int EV = 0;                              // [NQT][NKS]
  static constexpr int PV = EV + NQT * NKS;                 // [3][NQT][4][NMT]
  static constexpr int EF = PV + 3 * NQT * 4 * NMT;         // [3][2][NFT][NKS]
  static constexpr int LF = EF + 6 * NFT * NKS;             // [3][2][NFT][4][NMT]
  static constexpr int OPS = LF + 6 * NFT * 4 * NMT;
  // refined box only (read from global memory): the coarse trace at the
  // points of each of a side's four sub-faces, and the sub-face lift
  static constexpr int HGA = OPS;                            // [3][2][4][NFT][NKS]
  static constexpr int HWA = HGA + 24 * NFT * NKS;           // [3][2][4][NFT][4][NMT]
  static constexpr int AOPS = HWA + 24 * NFT * 4 * NMT;
  // when all of them exceed 64 KB (k = 3, FP64: 97 KB), LDS holds one
  // phase's blocks at a time (58 KB), the face phase's loaded after the volume
  static constexpr bool SPLIT = OPS * 64 * (int)sizeof(R) > 65536;
  // FP32 path: the FP64 lift weights of mode 0, per lane group g, [6][NFT][4][4]
  // (regular faces), then [6][4][NFT][4][4] (refined box: sub-faces)
  static constexpr int LW = 6 * NFT * 16, LWH = LW, LWTOT = LW + 24 * NFT * 16;
  // BF16 path: the volume's A operands as BF16 pairs, blocks of 64 lanes x 8
  // values, hi then lo: evaluation [NQT][2], projection [3][NQC][NMT][2]
  // (NQC chunks of two node tiles, the 32 K values of v_mfma_f32_16x16x32_bf16)
  static constexpr int NQC = (NQT + 1) / 2;
  static constexpr int BEV = 0, BPV = BEV + NQT * 2, BOPS = BPV + 3 * NQC * NMT * 2;
  static constexpr int VOPS = EF, FOPS = OPS - EF;
  static constexpr int LDSOPS = !SPLIT ? OPS : (VOPS > FOPS ? VOPS : FOPS);
  static constexpr int FBASE = SPLIT ? EF : 0;  // LDS block of face-phase operand o: o - FBASE
};

// Two waves per SIMD (<= 256 registers per lane) wherever they do not spill
// heavily: at one wave the matrix pipe idled while the wave waited on its
// own MFMA results and loads (128^3, k = 2: 5.3 ms against 3.2 ms per
// launch; refined blast, k = 2: 1.50 against 0.99 ms).  Uniform grids at
// k = 3 spill 12 to 90 registers at two waves and still gain (96^3, FP64
// 4.06 -> 3.52 ms, FP32 3.09 -> 2.35 ms, BF16 3.26 -> 2.26 ms); only FP64 on
// the refined box at k = 3 keeps one wave (two would spill ~460 registers).
// Three FP32 waves at k = 2 were slower (2.56 against 2.39 ms).
//
// AMR: the refined box of Sec. 4 (static 2:1 box; state = coarse block, then
// fine block).  Blocks of the grid cover the coarse block's cells, then the
// fine block's, so a wave holds 16 cells of one block.  Faces are classified
// per column as in k_rhs_amr_quad: regular, wall, hanging (a coarse cell
// facing the fine block: four sub-faces, the coarse trace at the sub-face's
// points (eq. ref_pa_integral's mapped points, table HG) against the fine
// cell's own trace, lifted with the sub-face weights w_r / 2^(d-1), table HW)
// and coarse-neighbour (a fine cell on the block boundary: its own trace
// against the coarse trace at its sub-face's points).  Each kind's traces
// come from their own MFMA chain started at zero and are selected per
// column, so both cells of a hanging face form each trace from the same
// table, the same weights and the same chain: the same flux bit for bit.
// The hanging and coarse-neighbour chains run only in waves that hold such
// a column, with their tables read from global memory.
//
// R = float (the FP32 path): contractions, fluxes and Riemann solves in FP32
// on v_mfma_f32_16x16x4f32; the lift of mode 0 (the cell mean) is summed in
// FP64 from the FP32 face fluxes (tlw: its FP64 weights per lane group), and
// the stage update is FP64, as in k_rhs_stage.
// VB (the BF16 path, R = float): the volume integral's two contractions on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation, every operand a BF16 pair
// x = hi + lo and every product the three MFMAs lo hi + hi lo + hi hi (as in
// k_volume_bf16), straight into the FP32 accumulators that the faces then
// continue: evaluation D[p][c] = sum_m E[p][m] w[m][c] over the modes padded
// to 32 (lane (g, c) holds modes 8 g + e of cell c as B), projection
// D[j][c] = sum_q T[j][q] F[q][c] over two node tiles at a time (K index
// 8 g + e = node 16 (2 tp + e / 4) + 4 (e % 4) + g, which is register e % 4
// of tile 2 tp + e / 4 in lane (g, c): the FP32 evaluation result is the B
// operand without moving data between lanes).
// PER (uniform grid): every axis periodic, so no wall faces (their selects
// compiled out).
template <int K, int FX, bool AMR, class R = double, bool VB = false, bool PER = false>
__global__ __launch_bounds__(256, (sizeof(R) == 4 || K == 2 || !AMR) ? 2 : 1) void k_rhs_mfma3d(
    const R *__restrict__ tmf, const double *__restrict__ tlw, const bf16x8 *__restrict__ tvb,
    const double *__restrict__ w, double *__restrict__ out, const double *__restrict__ dtp, Grid g, AmrGrid ag,
    int mode, Mix mx, int *__restrict__ flag) {
  using M = Mf3<K, R>;
  using V4 = typename Mv4<R>::T;
  constexpr int N = M::N, NV = M::NV, NKS = M::NKS, NMT = M::NMT, QF = M::QF, Q = M::Q, NW = NV * N;
  constexpr bool LO64 = sizeof(R) == sizeof(float);  // mode 0 lifted in FP64
  // REUSE (FP64): the stage update takes the cell's own coefficient from the
  // B operand wb (mode 4 ks + gq in register ks, the same double) instead of
  // reading it again after the face phase, when it has mostly left the
  // caches (128^3, k=2: 2.84 -> 2.67 ms; refined blast, k=3: 2.68 -> 2.59
  // ms).  Not where keeping wb live to the end spills (uniform grids at
  // k = 3: 90 -> 146 registers).  PREY (refined box, one block per CU): the
  // first extra state of the stage combination (the step's initial state in
  // SSP-RK3 stages 2 and 3) is loaded with the cell's own and parked in LDS
  // (ysl) for the update (2.59 -> 2.44 ms; at k = 2 on uniform grids, two
  // blocks per CU, the 31 KB more LDS per block cost more than it saved:
  // 2.66 -> 2.99 ms).
  constexpr bool REUSE = sizeof(R) == sizeof(double) && (AMR ? K == 3 : K == 2);
  constexpr bool PREY = REUSE && AMR;
  static_assert(!VB || (LO64 && N <= 32), "BF16 volume: FP32 kernel, at most 32 modes");
  // VB: LDS holds the face phase's FP32 operands and the BF16 volume operands
  constexpr int FB = VB ? M::EF : M::FBASE;  // LDS block of face-phase operand o: o - FB
  __shared__ R tl[(VB ? M::FOPS : M::LDSOPS) * 64];
  __shared__ double lws[LO64 ? M::LW : 1];
  __shared__ bf16x8 tvl[VB ? M::BOPS * 64 : 1];
  __shared__ double ysl[PREY ? 4 * NV * NKS * 64 : 1];  // per wave, variable, K step, lane
  if constexpr (VB) {
    for (int i = threadIdx.x; i < M::FOPS * 64; i += blockDim.x) tl[i] = tmf[M::EF * 64 + i];
    for (int i = threadIdx.x; i < M::BOPS * 64; i += blockDim.x) tvl[i] = tvb[i];
  } else {
    for (int i = threadIdx.x; i < (M::SPLIT ? M::VOPS : M::OPS) * 64; i += blockDim.x) tl[i] = tmf[i];
  }
  if constexpr (LO64)
    for (int i = threadIdx.x; i < M::LW; i += blockDim.x) lws[i] = tlw[i];
  __syncthreads();

  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int gq = lane >> 4, col = lane & 15;
  // the block of cells this wave works on: the uniform grid, or (AMR) the
  // coarse or the fine block, at offset boff in the state
  long nc, blk = blockIdx.x, boff = 0;
  bool fine = false;
  int bn[3];
  double fac, gam;
  if constexpr (AMR) {
    const long nbc = (ag.ncc + 63) / 64;
    fine = blk >= nbc;
    if (fine) blk -= nbc;
    nc = fine ? ag.ncf : ag.ncc;
    boff = fine ? (long)NW * ag.ncc : 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) bn[a] = fine ? ag.nf[a] : ag.n[a];
    fac = fine ? ag.facf : ag.facc;
    gam = ag.gamma;
  } else {
    blk = block_order(g, blk);
    nc = g.ncell;
    bn[0] = g.nx;
    bn[1] = g.ny;
    bn[2] = g.nz;
    fac = g.fac;
    gam = g.gamma;
  }
  const double *wbk = w + boff;  // this block's state
  const long cell = (blk * 4 + wv) * 16 + col;
  const bool valid = cell < nc;
  const long cs = valid ? cell : nc - 1;  // a valid address for the padding columns
  // 32-bit index arithmetic (dg_init admits blocks of at most 2^31 cells)
  const unsigned cu = (unsigned)cs, pl = (unsigned)bn[0] * (unsigned)bn[1];
  int ci[3] = {(int)(cu % (unsigned)bn[0]), (int)((cu / (unsigned)bn[0]) % (unsigned)bn[1]), (int)(cu / pl)};
  bool hole = false;
  if constexpr (AMR) hole = !fine && amr_in_hole<3>(ag, ci);
  const R gm1 = (R)(gam - 1.0);
  auto op = [&](int o) { return tl[o * 64 + lane]; };               // volume-phase operand
  auto opf = [&](int o) { return tl[(o - FB) * 64 + lane]; };      // face-phase operand
  auto opg = [&](int o) { return tmf[(long)o * 64 + lane]; };        // hanging-face operand (global)

  // the cell's weights as B operands: wb[v][ks] = w_v[mode 4 ks + gq].  Loads
  // of padding (modes past N, columns past the grid) read a valid address
  // and are zeroed by a select: no branches, so the scheduler can overlap
  // loads, matrix and vector work across the whole kernel
  // (addresses: a per-lane offset per K step plus the variable's uniform
  // offset, which keeps the 64-bit index arithmetic out of the vector ALU)
  auto lane_offsets = [&](long stride, long cellidx, long (&o)[NKS]) {
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) {
      const int m = 4 * ks + gq;
      o[ks] = (long)(m < N ? m : N - 1) * stride + cellidx;
    }
  };
  R wb[NV][NKS];
  {
    long o[NKS];
    lane_offsets(nc, cs, o);
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) {
        const double x = wbk[(long)(v * N) * nc + o[ks]];
        wb[v][ks] = (4 * ks + gq < N && valid) ? (R)x : R(0);
      }
  }
  const bool pre = PREY && mode != 0 && mx.n > 0;
  if (pre) {
    long o[NKS];
    lane_offsets(nc, cs, o);
    const double *y0 = mx.y[0] + boff;
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) ysl[((wv * NV + v) * NKS + ks) * 64 + lane] = y0[(long)(v * N) * nc + o[ks]];
  }

  V4 acc[NV][NMT];
  double acc0[NV];  // FP32 path: this lane's share of the mode-0 lift, FP64
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    acc0[v] = 0.0;
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt) acc[v][mt] = V4{R(0), R(0), R(0), R(0)};
  }

  // volume integral (eq. dg_term2)
  if constexpr (VB) {
    // B operands of the evaluation: modes 8 gq + e of this column's cell
    bf16x8 wh[NV], wl[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int m = 8 * gq + e, mc = m < N ? m : N - 1;
        const double xd = wbk[(long)(v * N + mc) * nc + cs];
        const float x = (m < N && valid) ? (float)xd : 0.0f;
        const __bf16 hi = (__bf16)x;
        wh[v][e] = hi;
        wl[v][e] = (__bf16)(x - (float)hi);
      }
#pragma unroll
    for (int tp = 0; tp < M::NQC; ++tp) {
      f4 U[NV][2];
#pragma unroll
      for (int dt = 0; dt < 2; ++dt) {
        const int t = 2 * tp + dt;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          f4 z = {0.0f, 0.0f, 0.0f, 0.0f};
          if (t < M::NQT) {
            const bf16x8 eh = tvl[(M::BEV + 2 * t) * 64 + lane], el = tvl[(M::BEV + 2 * t + 1) * 64 + lane];
            z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(el, wh[v], z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(eh, wl[v], z, 0, 0, 0);
            z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(eh, wh[v], z, 0, 0, 0);
          }
          U[v][dt] = z;
        }
      }
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        bf16x8 fh[NV], fl[NV];
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const int dt = e >> 2, i = e & 3, p0 = 16 * (2 * tp + dt) + 4 * i;
          if (p0 >= Q) {  // a whole register of padding nodes
#pragma unroll
            for (int v = 0; v < NV; ++v) fh[v][e] = fl[v][e] = (__bf16)0.0f;
            continue;
          }
          const bool ok = p0 + gq < Q;
          R Ur[NV], F[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) Ur[v] = ok ? U[v][dt][i] : (v == 0 ? R(1) : (v == NV - 1 ? R(1) : R(0)));
          euler_flux<3, R>(Ur, a, gm1, F);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const float f = ok ? F[v] : 0.0f;
            const __bf16 hi = (__bf16)f;
            fh[v][e] = hi;
            fl[v][e] = (__bf16)(f - (float)hi);
          }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int mt = 0; mt < NMT; ++mt) {
            const int o = M::BPV + ((a * M::NQC + tp) * NMT + mt) * 2;
            const bf16x8 th = tvl[o * 64 + lane], tlo = tvl[(o + 1) * 64 + lane];
            acc[v][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(tlo, fh[v], acc[v][mt], 0, 0, 0);
            acc[v][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th, fl[v], acc[v][mt], 0, 0, 0);
            acc[v][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(th, fh[v], acc[v][mt], 0, 0, 0);
          }
      }
    }
  } else
#pragma unroll
  for (int t = 0; t < M::NQT; ++t) {
    V4 U[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      V4 z = {R(0), R(0), R(0), R(0)};
#pragma unroll
      for (int ks = 0; ks < NKS; ++ks) z = Mv4<R>::mma(op(M::EV + t * NKS + ks), wb[v][ks], z);
      U[v] = z;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (16 * t + 4 * r >= Q) continue;
      const bool ok = 16 * t + 4 * r + gq < Q;
      R Ur[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) Ur[v] = ok ? U[v][r] : (v == 0 ? R(1) : (v == NV - 1 ? R(1) : R(0)));
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        R F[NV];
        euler_flux<3, R>(Ur, a, gm1, F);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const R f = ok ? F[v] : R(0);
#pragma unroll
          for (int mt = 0; mt < NMT; ++mt)
            acc[v][mt] = Mv4<R>::mma(op(M::PV + ((a * M::NQT + t) * 4 + r) * NMT + mt), f, acc[v][mt]);
        }
      }
    }
  }

  if constexpr (M::SPLIT && !VB) {
    __syncthreads();  // every wave is done with the volume-phase operands
    for (int i = threadIdx.x; i < M::FOPS * 64; i += blockDim.x) tl[i] = tmf[M::EF * 64 + i];
    __syncthreads();
  }

  // one MFMA chain over the K steps: D = sum_ks A(o0 + ks) B[ks]
  auto chain = [&](auto &&A, int o0, const R (&B)[NKS]) {
    V4 z = {R(0), R(0), R(0), R(0)};
#pragma unroll
    for (int ks = 0; ks < NKS; ++ks) z = Mv4<R>::mma(A(o0 + ks), B[ks], z);
    return z;
  };
  // Riemann solves at this lane's points of one face tile and their lift
  // (table op L0 + r NMT + mt; FP32 path: mode 0 in FP64 with the weights
  // lw[4 r + gq]), the flux zeroed in the columns `drop`
  auto solve_lift = [&](auto &&A, int L0, const double *lw, int a, int s, int ft, const V4 (&To)[NV],
                        const V4 (&Tn)[NV], bool drop) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      if (16 * ft + 4 * r >= QF) continue;
      // every lane solves (points past QF: zero traces, the result discarded
      // by the select below), so that no branch splits the kernel
      const bool pt = 16 * ft + 4 * r + gq < QF;
      R Fh[NV], UL[NV], UR[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        UL[v] = s ? To[v][r] : Tn[v][r];
        UR[v] = s ? Tn[v][r] : To[v][r];
      }
      hllc<R, 3, FX, true>(UL, UR, a, gam, Fh);
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const R f = (drop || !pt) ? R(0) : Fh[v];
        if constexpr (LO64) acc0[v] = fma((double)f, lw[4 * r + gq], acc0[v]);
#pragma unroll
        for (int mt = 0; mt < NMT; ++mt) acc[v][mt] = Mv4<R>::mma(A(L0 + r * NMT + mt), f, acc[v][mt]);
      }
    }
  };

  // face integral (eq. dg_term3), each of the 2d sides from this cell's side
  // (unrolled: the next side's neighbour loads and table reads are issued
  // while the current side's Riemann solves run)
#pragma unroll
  for (int fs = 0; fs < 6; ++fs) {
    const int a = fs >> 1, s = fs & 1;
    const int dir = s ? 1 : -1;
    // kind 0 regular, 1 wall (ghost = own trace), 2 hanging, 3 coarse neighbour
    int kind = 0, hsub = 0, j[3] = {0, 0, 0};
    long src = cs;
    const double *nsrc = wbk;
    long nn = nc;
    if constexpr (AMR) {
      if (!valid || hole) {
        kind = 1;
      } else if (!fine) {
        if (!amr_coarse_nb<3>(ag, ci, a, dir, j)) kind = 1;
        else if (amr_in_hole<3>(ag, j)) kind = 2;
        else src = ((long)j[2] * ag.n[1] + j[1]) * ag.n[0] + j[0];
      } else {
        int f2[3] = {ci[0], ci[1], ci[2]};
        f2[a] += dir;
        if (f2[a] >= 0 && f2[a] < ag.nf[a]) {
          src = ((long)f2[2] * ag.nf[1] + f2[1]) * ag.nf[0] + f2[0];
        } else {
          const int t0 = (a == 0) ? 1 : 0, t1 = (a == 2) ? 1 : 2;
          int base[3];
#pragma unroll
          for (int b = 0; b < 3; ++b) base[b] = ag.lo[b] + ci[b] / 2;
          amr_coarse_nb<3>(ag, base, a, dir, j);
          kind = 3;
          src = ((long)j[2] * ag.n[1] + j[1]) * ag.n[0] + j[0];
          nsrc = w;
          nn = ag.ncc;
          hsub = (ci[t0] & 1) | ((ci[t1] & 1) << 1);
        }
      }
    } else {
      // periodic wrap or (transmissive) the cell itself, as selects
      int j2[3] = {ci[0], ci[1], ci[2]};
      const int n = bn[a], i2 = j2[a] + dir;
      const bool outside = (i2 < 0) | (i2 >= n);
      j2[a] = i2 < 0 ? i2 + n : (i2 >= n ? i2 - n : i2);
      kind = (!PER && (outside & (g.bc[a] == DG_BC_TRANSMISSIVE))) ? 1 : 0;
      const long nb = ((long)j2[2] * bn[1] + j2[1]) * bn[0] + j2[0];
      src = kind ? cs : nb;
    }
    R nbw[NV][NKS];
    {
      long o[NKS];
      lane_offsets(nn, src, o);
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int ks = 0; ks < NKS; ++ks) {
          const double x = nsrc[(long)(v * N) * nn + o[ks]];
          nbw[v][ks] = 4 * ks + gq < N ? (R)x : R(0);
        }
    }
#pragma unroll
    for (int ft = 0; ft < M::NFT; ++ft) {
      V4 To[NV], Tn[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        To[v] = chain(opf, M::EF + ((a * 2 + s) * M::NFT + ft) * NKS, wb[v]);
        const V4 zn = chain(opf, M::EF + ((a * 2 + (1 - s)) * M::NFT + ft) * NKS, nbw[v]);
        Tn[v] = kind == 0 ? zn : To[v];  // wall: ghost trace = own trace
      }
      if constexpr (AMR) {
        // a fine cell facing the coarse block: the coarse neighbour's trace
        // at this cell's sub-face points
#pragma unroll 1
        for (int hs = 0; hs < 4; ++hs) {
          if (!__any(kind == 3 && hsub == hs)) continue;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const V4 zh = chain(opg, M::HGA + (((a * 2 + (1 - s)) * 4 + hs) * M::NFT + ft) * NKS, nbw[v]);
            Tn[v] = (kind == 3 && hsub == hs) ? zh : Tn[v];
          }
        }
      }
      solve_lift(opf, M::LF + (((a * 2 + s) * M::NFT + ft) * 4) * NMT,
                 LO64 ? lws + ((a * 2 + s) * M::NFT + ft) * 16 : nullptr, a, s, ft, To, Tn, kind == 2);
    }
    if constexpr (AMR) {
      // a coarse cell facing the fine block: its 2^(d-1) sub-faces
      if (__any(kind == 2)) {
        const int t0 = (a == 0) ? 1 : 0, t1 = (a == 2) ? 1 : 2;
#pragma unroll 1
        for (int sb = 0; sb < 4; ++sb) {
          long fcell = 0;
          if (kind == 2) {
            int fi[3] = {0, 0, 0};
            fi[a] = 2 * (j[a] - ag.lo[a]) + (s ? 0 : 1);
            fi[t0] = 2 * (j[t0] - ag.lo[t0]) + (sb & 1);
            fi[t1] = 2 * (j[t1] - ag.lo[t1]) + ((sb >> 1) & 1);
            fcell = ((long)fi[2] * ag.nf[1] + fi[1]) * ag.nf[0] + fi[0];
          }
          const double *wf = w + (long)NW * ag.ncc;
          R fw[NV][NKS];
          long o[NKS];
          lane_offsets(ag.ncf, fcell, o);
#pragma unroll
          for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int ks = 0; ks < NKS; ++ks) {
              const double x = wf[(long)(v * N) * ag.ncf + o[ks]];
              fw[v][ks] = 4 * ks + gq < N ? (R)x : R(0);
            }
#pragma unroll
          for (int ft = 0; ft < M::NFT; ++ft) {
            V4 To[NV], Tn[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              To[v] = chain(opg, M::HGA + (((a * 2 + s) * 4 + sb) * M::NFT + ft) * NKS, wb[v]);
              Tn[v] = chain(opf, M::EF + ((a * 2 + (1 - s)) * M::NFT + ft) * NKS, fw[v]);
            }
            solve_lift(opg, M::HWA + ((((a * 2 + s) * 4 + sb) * M::NFT + ft) * 4) * NMT,
                       LO64 ? tlw + M::LWH + (((a * 2 + s) * 4 + sb) * M::NFT + ft) * 16 : nullptr, a, s, ft, To,
                       Tn, kind != 2);
          }
        }
      }
    }
  }

  // FP32 path: the four lane groups' shares of the mode-0 lift, summed in
  // the same order in every lane
  if constexpr (LO64) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double t = acc0[v];
      t += __shfl_xor(t, 16);
      t += __shfl_xor(t, 32);
      acc0[v] = t;
    }
  }

  // assembly (L = (2/dx) 2^-d (V - S)) and the fused stage update; a hole
  // cell of the coarse block gets L = 0
  bool bad = false;
  const double cldt = (mode == 0) ? 0.0 : mx.cl * *dtp;
  const long ol = boff + (long)gq * nc + cs;  // this lane's part of the output index
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int mt = 0; mt < NMT; ++mt)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int jm = 16 * mt + 4 * r + gq;
        if (jm < N && valid) {
          const long i = (long)(v * N + 16 * mt + 4 * r) * nc + ol;
          const double Lv = (LO64 && jm == 0) ? acc0[v] : (double)acc[v][mt][r];
          const double L = hole ? 0.0 : fac * Lv;
          bad |= (L != L);
          // mode 4 ks + gq of the cell in K step ks = 4 mt + r (< NKS for jm < N)
          const int ks = 4 * mt + r < NKS ? 4 * mt + r : NKS - 1;
          const double u = REUSE ? (double)wb[v][ks] : w[i];
          double o = L;
          if (mode != 0) {  // mix_out, with the first extra term from LDS when parked
            o = fma(hole ? 0.0 : cldt, L, mx.cu * u);
            if (pre) o = fma(mx.a[0], ysl[((wv * NV + v) * NKS + ks) * 64 + lane], o);
            o = mix_tail(mx, o, i, pre ? 1 : 0);
          }
          out[i] = o;
        }
      }
  if (bad) atomicOr(flag, FLAG_NAN);
}

// ---------------------------------------------------------------------------
// Discrete adjoint of the right-hand side and of the SSP-RK3 stages.
//
// mu = (dL/dw)^T lam for L = fac (V - S):
//   volume: mu_K[u][l] += sum_q B[q][l] sum_a (J_a(U_q)^T Lam_a,q)[u] with
//           Lam_a,q[v] = sum_j lam_K[v][j] DW[a][q][j] and J_a = d f_a / dU
//           (analytic transposed Euler Jacobian);
//   faces:  for a face with low cell A and high cell B the flux enters
//           L_A with -TW(+1) and L_B with +TW(-1); its cotangent is
//           g = -lam_A . TW(+1) + lam_B . TW(-1), and the own cell receives
//           (dF/dU_own)^T g lifted with TF, from one reverse sweep through
//           the Riemann solver (hllc_vjp, same branches as the forward pass).
// mode 0: out = mu;  mode 3: out = cb (lam + dt mu), acc_out = ca lam;
// mode 2: out = cb (lam + dt mu), acc_out = acc + ca lam;
// mode 1: out = acc + lam + dt mu.
// ---------------------------------------------------------------------------
template <int D>
__device__ inline void euler_flux_vjp(const double *U, int a, double g, const double *Lam, double *G) {
  const double gm1 = g - 1.0;
  const double ir = 1.0 / U[0];
  double v[D], q2 = 0.0, lv = 0.0;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    v[b] = U[1 + b] * ir;
    q2 = fma(v[b], v[b], q2);
    lv = fma(Lam[1 + b], v[b], lv);
  }
  const double p = gm1 * (U[D + 1] - 0.5 * U[0] * q2);
  const double H = (U[D + 1] + p) * ir;
  const double va = v[a], la = Lam[1 + a], lE = Lam[D + 1];
  const double hk = 0.5 * gm1 * q2;
  G[0] += -va * lv + la * hk + lE * va * (hk - H);
#pragma unroll
  for (int c = 0; c < D; ++c)
    G[1 + c] += (c == a ? Lam[0] + lv + lE * H : 0.0) + Lam[1 + c] * va - gm1 * v[c] * (la + lE * va);
  G[D + 1] += la * gm1 + lE * g * va;
}

template <int D, int K, int FX>
__global__ __launch_bounds__(256) void k_adjoint(const double *__restrict__ tab, const double *__restrict__ w,
                                                 const double *__restrict__ lam, const double *acc_in,
                                                 double *__restrict__ out, double *acc_out,
                                                 const double *__restrict__ dtp, Grid g, int mode, double ca,
                                                 double cb, int *__restrict__ flag) {
  using C = Cfg<D, K>;
  const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.ncell) return;
  const long nc = g.ncell;
  const int ix = (int)(cell % g.nx);
  const int iy = (int)((cell / g.nx) % g.ny);
  const int iz = (int)(cell / ((long)g.nx * g.ny));

  double wc[C::NV][C::N], lc[C::NV][C::N], mu[C::NV][C::N];
#pragma unroll
  for (int v = 0; v < C::NV; ++v)
#pragma unroll
    for (int l = 0; l < C::N; ++l) {
      const long i = (long)(v * C::N + l) * nc + cell;
      wc[v][l] = w[i];
      lc[v][l] = lam[i];
      mu[v][l] = 0.0;
    }

  // volume term
#pragma unroll 1
  for (int q = 0; q < C::Q; ++q) {
    const double *bq = tab + C::B + q * C::N;
    double U[C::NV], G[C::NV];
#pragma unroll
    for (int v = 0; v < C::NV; ++v) {
      double s = 0.0;
#pragma unroll
      for (int l = 0; l < C::N; ++l) s = fma(wc[v][l], bq[l], s);
      U[v] = s;
      G[v] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const double *dw = tab + C::DW + (a * C::Q + q) * C::N;
      double Lam[C::NV];
#pragma unroll
      for (int v = 0; v < C::NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < C::N; ++l) s = fma(lc[v][l], dw[l], s);
        Lam[v] = s;
      }
      euler_flux_vjp<D>(U, a, g.gamma, Lam, G);
    }
#pragma unroll
    for (int u = 0; u < C::NV; ++u)
#pragma unroll
      for (int l = 0; l < C::N; ++l) mu[u][l] = fma(G[u], bq[l], mu[u][l]);
  }

  // face terms
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      const long nb = neighbour(g, ix, iy, iz, a, s ? 1 : -1);
      const long src = nb >= 0 ? nb : cell;
      // own side: trace with TF(s), lambda against TW(s); neighbour side with
      // TF(1-s), TW(1-s) (the low cell's lambda meets TW(+1), the high cell's
      // TW(-1)); the neighbour's weights are streamed from L1/L2 per node
      const double *to = tab + C::TF + (a * 2 + s) * C::QF * C::N;
      const double *tn = tab + C::TF + (a * 2 + (1 - s)) * C::QF * C::N;
      const double *two = tab + C::TW + (a * 2 + s) * C::QF * C::N;
      const double *twn = tab + C::TW + (a * 2 + (1 - s)) * C::QF * C::N;
#pragma unroll 1
      for (int r = 0; r < C::QF; ++r) {
        double Uo[C::NV], Un[C::NV], gv[C::NV];
#pragma unroll
        for (int v = 0; v < C::NV; ++v) {
          double so = 0.0, sn = 0.0, lo = 0.0, ln = 0.0;
#pragma unroll
          for (int l = 0; l < C::N; ++l) {
            const long i = (long)(v * C::N + l) * nc + src;
            so = fma(wc[v][l], to[r * C::N + l], so);
            sn = fma(w[i], tn[r * C::N + l], sn);
            lo = fma(lc[v][l], two[r * C::N + l], lo);
            ln = fma(lam[i], twn[r * C::N + l], ln);
          }
          if (nb < 0) ln = 0.0;  // the ghost cell of a transmissive boundary has no equation
          Uo[v] = so;
          Un[v] = nb >= 0 ? sn : so;
          gv[v] = s ? ln - lo : lo - ln;  // lam_high . TW(-1) - lam_low . TW(+1)
        }
        // (dF/dU_own)^T g by one reverse sweep through the Riemann solver; a
        // transmissive ghost copies the own trace, so both sides count
        double UL[C::NV], UR[C::NV], gL[C::NV], gR[C::NV];
#pragma unroll
        for (int v = 0; v < C::NV; ++v) {
          UL[v] = s ? Uo[v] : Un[v];
          UR[v] = s ? Un[v] : Uo[v];
        }
        hllc_vjp<D, FX>(UL, UR, a, g.gamma, gv, gL, gR);
#pragma unroll
        for (int u = 0; u < C::NV; ++u) {
          const double h = (s ? gL[u] : gR[u]) + (nb >= 0 ? 0.0 : (s ? gR[u] : gL[u]));
#pragma unroll
          for (int l = 0; l < C::N; ++l) mu[u][l] = fma(h, to[r * C::N + l], mu[u][l]);
        }
      }
    }
  }

  const double dt = (mode == 0) ? 0.0 : *dtp;
  bool bad = false;
#pragma unroll
  for (int v = 0; v < C::NV; ++v)
#pragma unroll
    for (int l = 0; l < C::N; ++l) {
      const long i = (long)(v * C::N + l) * nc + cell;
      const double m = g.fac * mu[v][l];
      bad |= (m != m);
      if (mode == 0) {
        out[i] = m;
      } else if (mode == 1) {
        out[i] = acc_in[i] + (lc[v][l] + dt * m);
      } else {
        out[i] = cb * (lc[v][l] + dt * m);
        acc_out[i] = (mode == 3) ? ca * lc[v][l] : acc_in[i] + ca * lc[v][l];
      }
    }
  if (bad) atomicOr(flag, FLAG_NAN);
}

// ---------------------------------------------------------------------------
// L2 projection of nodal primitive data (Sec. 2.3).
// ---------------------------------------------------------------------------
template <int D, int K>
__global__ __launch_bounds__(256) void k_project(const double *__restrict__ tab, const double *__restrict__ prim,
                                                 long pstride, long poff, double *__restrict__ w, long nc,
                                                 double gamma) {
  // prim[c][q][pstride] holds the block's cells at offset poff; w is one block
  using C = Cfg<D, K>;
  const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= nc) return;
  double acc[C::NV][C::N];
#pragma unroll
  for (int v = 0; v < C::NV; ++v)
#pragma unroll
    for (int l = 0; l < C::N; ++l) acc[v][l] = 0.0;
  for (int q = 0; q < C::Q; ++q) {
    double pr[5];
#pragma unroll
    for (int c = 0; c < 5; ++c) pr[c] = prim[((long)c * C::Q + q) * pstride + poff + cell];
    double U[C::NV];
    double ke = 0.0;
    U[0] = pr[0];
#pragma unroll
    for (int b = 0; b < D; ++b) {
      U[1 + b] = pr[0] * pr[1 + b];
      ke += pr[1 + b] * pr[1 + b];
    }
    U[D + 1] = pr[4] / (gamma - 1.0) + 0.5 * pr[0] * ke;
    const double wq = tab[C::WQ + q];
#pragma unroll
    for (int v = 0; v < C::NV; ++v)
#pragma unroll
      for (int l = 0; l < C::N; ++l) acc[v][l] = fma(U[v] * wq, tab[C::B + q * C::N + l], acc[v][l]);
  }
  const double scale = 1.0 / (double)(1 << D);
#pragma unroll
  for (int v = 0; v < C::NV; ++v)
#pragma unroll
    for (int l = 0; l < C::N; ++l) w[(long)(v * C::N + l) * nc + cell] = scale * acc[v][l];
}

// ---------------------------------------------------------------------------
// Time step (eq. time_step / time_step_pos): max over cells of the signal
// rate sum_a (|v_a| + c)/dx of the cell mean; dt = CFL f_k / max rate.
// ---------------------------------------------------------------------------

__device__ inline double block_max(double x) {
  __shared__ double red[16];
  x = wave_max(x);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = x;
  __syncthreads();
  const int nw = (blockDim.x + 63) >> 6;
  x = (threadIdx.x < nw) ? red[threadIdx.x] : 0.0;
  if (wid == 0) x = wave_max(x);
  return x;
}

// max over cells of sum_a (|v_a| + c)/dx of the cell mean: every block folds
// its maximum into its rate slot with an atomic max; k_dt_final then writes
// dt = CFL f_k / (largest slot) and clears the slots for the next call.  The
// kernel boundary orders the two, so no device-scope fence is needed.
template <int D>
__global__ __launch_bounds__(256) void k_rate(const double *__restrict__ w, long nc, int N, double gamma, double dx,
                                              unsigned long long *ratemax, int *__restrict__ flag,
                                              const double *__restrict__ gmax, double gk) {
  double m = 0.0;
  bool bad = false;
  for (long cell = (long)blockIdx.x * blockDim.x + threadIdx.x; cell < nc; cell += (long)gridDim.x * blockDim.x) {
    double U[D + 2];
#pragma unroll
    for (int v = 0; v < D + 2; ++v) U[v] = w[(long)v * N * nc + cell];
    m = fmax(m, cell_rate<D>(U, gamma, dx, bad, gk, gmax ? gmax[cell] : 0.0));
  }
  if (bad) atomicOr(flag, FLAG_NEGATIVE);
  m = block_max(m);
  if (threadIdx.x == 0) atomicMax(rate_slot(ratemax, blockIdx.x), (unsigned long long)__double_as_longlong(m));
}

__global__ void k_dt_final(unsigned long long *ratemax, double cfl_fk, double *__restrict__ dt) {
  if (threadIdx.x == 0) {
    unsigned long long m = 0ull;
    for (int k = 0; k < RATE_SLOTS; ++k) {
      const unsigned long long v = ratemax[RATE_STRIDE * k];
      m = v > m ? v : m;
      ratemax[RATE_STRIDE * k] = 0ull;
    }
    dt[0] = cfl_fk / __longlong_as_double((long long)m);
  }
}

// Gravity set-up: from the external acceleration a at the volume nodes
// ([D][Q][ncell]) the source kernels' operand (dx/2) w_q a and, per cell, the
// largest |a| over its nodes for the time step.
template <int D, int K>
__global__ __launch_bounds__(256) void k_grav_setup(const double *__restrict__ tab, const double *__restrict__ accel,
                                                    long nc, double hdx, double *__restrict__ grav,
                                                    double *__restrict__ gmax) {
  using C = Cfg<D, K>;
  const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= nc) return;
  double amax = 0.0;
  for (int q = 0; q < C::Q; ++q) {
    const double wq = hdx * tab[C::WQ + q];
    double a2 = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const long i = (long)(a * C::Q + q) * nc + cell;
      const double ga = accel[i];
      a2 = fma(ga, ga, a2);
      grav[i] = wq * ga;
    }
    amax = fmax(amax, sqrt(a2));
  }
  gmax[cell] = amax;
}

// Clears the rate slots (a kernel rather than a memset, so that the call can
// be captured into a graph).
__global__ void k_rate_zero(unsigned long long *word) {
  if (threadIdx.x < RATE_SLOTS) word[RATE_STRIDE * threadIdx.x] = 0ull;
}

// ---------------------------------------------------------------------------
// Limiters (Sec. 3.1, 3.3, 3.4), one thread per cell, in place.  Cell means
// are read from the neighbours and never written, so the pass is race free.
// ---------------------------------------------------------------------------
__device__ inline double minmod3(double a, double b, double c) {
  if (a > 0.0 && b > 0.0 && c > 0.0) return fmin(a, fmin(b, c));
  if (a < 0.0 && b < 0.0 && c < 0.0) return -fmin(-a, fmin(-b, -c));
  return 0.0;
}

// Eigen-structure of the Euler flux Jacobian in direction a at a cell mean
// (App. E), applied in factored form instead of as dense matrices.  With
// k = |v|^2/2, h = c^2/(gamma-1) + k, b = 1/(2c^2), the pressure perturbation
// P(x) = (gamma-1)(k x_rho - v.x_m + x_E) and U_a(x) = v_a x_rho - x_{m_a},
// the characteristic variables of a conserved vector x are
//   acoustic (v_a - c):  b (P + c U_a)
//   entropy  (v_a):      x_rho - 2 b P
//   acoustic (v_a + c):  b (P - c U_a)
//   shear    (v_a):      x_{m_t} - v_t x_rho   for each direction t != a,
// and to_cons is the inverse map.  The shear waves are oriented with a plus
// sign throughout (App. E flips some of them): negating an eigenvector and its
// left counterpart leaves R c~ unchanged, and minmod is odd, so the limited
// slopes do not depend on the orientation.
template <int D>
struct CharBasis {
  double v[D], k, c, h, g1, b;

  // false if the mean has no positive density and pressure
  __device__ bool init(const double *U, double gamma) {
    const double ir = 1.0 / U[0];
    k = 0.0;
#pragma unroll
    for (int t = 0; t < D; ++t) {
      v[t] = U[1 + t] * ir;
      k = fma(v[t], v[t], k);
    }
    k *= 0.5;
    g1 = gamma - 1.0;
    const double p = g1 * (U[D + 1] - U[0] * k);
    if (!(U[0] > 0.0) || !(p > 0.0)) return false;
    const double c2 = gamma * p * ir;
    c = sqrt(c2);
    h = c2 / g1 + k;
    b = 0.5 / c2;
    return true;
  }

  template <int A>
  __device__ void to_char(const double *x, double *ch) const {
    double vm = 0.0;
#pragma unroll
    for (int t = 0; t < D; ++t) vm = fma(v[t], x[1 + t], vm);
    const double P = g1 * (k * x[0] - vm + x[D + 1]);
    const double Ua = v[A] * x[0] - x[1 + A];
    ch[0] = b * (P + c * Ua);
    ch[1] = x[0] - 2.0 * b * P;
    ch[2] = b * (P - c * Ua);
    int j = 3;
#pragma unroll
    for (int t = 0; t < D; ++t)
      if (t != A) ch[j++] = x[1 + t] - v[t] * x[0];
  }

  template <int A>
  __device__ void to_cons(const double *ch, double *x) const {
    const double S = ch[0] + ch[1] + ch[2], Dc = ch[2] - ch[0];
    x[0] = S;
    x[1 + A] = v[A] * S + c * Dc;
    double E = h * (ch[0] + ch[2]) + k * ch[1] + c * v[A] * Dc;
    int j = 3;
#pragma unroll
    for (int t = 0; t < D; ++t)
      if (t != A) {
        x[1 + t] = v[t] * S + ch[j];
        E = fma(v[t], ch[j], E);
        ++j;
      }
    x[D + 1] = E;
  }
};

// Characteristic TVB limiter of one cell (eq. char_limiter with the bound of
// Sec. 3.3): in each direction the slope sqrt(3) w_{1+a} and the neighbour
// mean differences go to characteristic variables at the cell mean and are
// limited field by field; if any field changes, all slopes are rebuilt from
// the limited characteristic slopes and the higher modes are dropped.  The
// means are kept.  nbmean(a, s, m) writes the mean of the neighbour on side
// s (0 low, 1 high) in direction a.  A mean without a real sound speed is
// left alone (the positivity pass flags it).
template <int D, int N, class NbMean>
__device__ inline bool char_limit_cell(double (&wc)[D + 2][N], NbMean &&nbmean, double gamma, double beta,
                                       double bound) {
  constexpr int NV = D + 2;
  double U[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) U[v] = wc[v][0];
  CharBasis<D> e;
  if (!e.init(U, gamma)) return false;
  const double r3 = sqrt(3.0);
  double ct[D][NV];
  bool limited = false;
  auto dir = [&](auto A_) {
    constexpr int A = decltype(A_)::value;
    double x[NV], lo[NV], hi[NV], cs[NV], cw[NV], ce[NV];
    nbmean(A, 0, lo);
    nbmean(A, 1, hi);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      x[v] = wc[v][1 + A];
      lo[v] = U[v] - lo[v];
      hi[v] = hi[v] - U[v];
    }
    e.template to_char<A>(x, cs);
    e.template to_char<A>(lo, cw);
    e.template to_char<A>(hi, ce);
#pragma unroll
    for (int q = 0; q < NV; ++q) {
      const double Aq = r3 * cs[q];
      const double m = (fabs(Aq) <= bound) ? Aq : minmod3(Aq, beta * cw[q], beta * ce[q]);
      ct[A][q] = m / r3;
      limited |= (m != Aq);
    }
  };
  dir(std::integral_constant<int, 0>{});
  dir(std::integral_constant<int, 1>{});
  if constexpr (D == 3) dir(std::integral_constant<int, 2>{});
  if (!limited) return false;
  auto back = [&](auto A_) {
    constexpr int A = decltype(A_)::value;
    double x[NV];
    e.template to_cons<A>(ct[A], x);
#pragma unroll
    for (int v = 0; v < NV; ++v) wc[v][1 + A] = x[v];
  };
  back(std::integral_constant<int, 0>{});
  back(std::integral_constant<int, 1>{});
  if constexpr (D == 3) back(std::integral_constant<int, 2>{});
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int l = D + 1; l < N; ++l) wc[v][l] = 0.0;
  return true;
}

// Root in [0,1] of (E(t) - eps/(g-1)) rho(t) - |m(t)|^2/2 = 0 along
// U(t) = Ub + t (Uq - Ub): quadratic formula without cancellation, then two
// Newton steps; bisection when rounding makes the discriminant negative.
template <int D>
__device__ inline double tau_root(const double *Ub, const double *Uq, double gamma, double eps) {
  const double e1 = eps / (gamma - 1.0);
  const double dr = Uq[0] - Ub[0], dE = Uq[D + 1] - Ub[D + 1];
  double dm2 = 0.0, mdm = 0.0, mb2 = 0.0;
#pragma unroll
  for (int b = 0; b < D; ++b) {
    const double dm = Uq[1 + b] - Ub[1 + b];
    dm2 += dm * dm;
    mdm += Ub[1 + b] * dm;
    mb2 += Ub[1 + b] * Ub[1 + b];
  }
  const double A = dE * dr - 0.5 * dm2;
  const double Bq = dE * Ub[0] + (Ub[D + 1] - e1) * dr - mdm;
  const double Cq = (Ub[D + 1] - e1) * Ub[0] - 0.5 * mb2;
  double t;
  const double disc = Bq * Bq - 4.0 * A * Cq;
  if (A == 0.0) {
    t = -Cq / Bq;
  } else if (disc >= 0.0) {
    const double qq = -0.5 * (Bq + copysign(sqrt(disc), Bq));
    const double r1 = qq / A, r2 = (qq != 0.0) ? Cq / qq : r1;
    const bool ok1 = r1 >= 0.0 && r1 <= 1.0, ok2 = r2 >= 0.0 && r2 <= 1.0;
    t = (ok1 && ok2) ? fmin(r1, r2) : ok1 ? r1 : ok2 ? r2 : 0.0;
  } else {
    double lo = 0.0, hi = 1.0;
    for (int it = 0; it < 60; ++it) {
      const double mid = 0.5 * (lo + hi);
      if ((A * mid + Bq) * mid + Cq > 0.0) lo = mid; else hi = mid;
    }
    t = lo;
  }
  for (int it = 0; it < 2; ++it) {
    const double gv = (A * t + Bq) * t + Cq, gd = 2.0 * A * t + Bq;
    if (gd != 0.0) t -= gv / gd;
  }
  return fmin(fmax(t, 0.0), 1.0);
}

// Smallest x over the 64 lanes of the wave (every lane active).
__device__ inline double wave_min(double x) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) x = fmin(x, __shfl_xor(x, o));
  return x;
}

// Appends the cells of this wave with need set to the list plist (plist[0]
// counts, plist[1 + i] holds the i-th cell id): one atomic per wave.  Every
// lane of the wave must call.
__device__ inline void wave_append(bool need, int id, int *plist) {
  const unsigned long long m = __ballot(need);
  if (!m) return;
  const int lane = threadIdx.x & 63, leader = __ffsll(m) - 1;
  int base = 0;
  if (lane == leader) base = atomicAdd(plist, __popcll(m));
  base = __shfl(base, leader);
  if (need) plist[1 + base + __popcll(m & ((1ull << lane) - 1))] = id;
}

// The point loop of the positivity pass (Sec. 3.4) for one cell, its
// points shared by the 64 lanes of a wave (every lane calls with the same
// cell): the cell's coefficient (v, l) is c[(v N + l) st]; h is its
// hanging-side mask (0 on uniform grids), passed to pts.count(h) and
// pts.row(h, i), the number of its points and the basis row of point i.
// Every lane evaluates its share of the points, theta_1 and theta_2 come
// from minima over the wave, and lane 0 stores the scaled modes l >= 1.
// Point values, theta_1 and theta_2 are formed with the same operations in
// the same order as a single-lane loop, so the result is the same bit for
// bit.
template <int D, int N, class Pts>
__device__ inline void positivity_cell(double *c, long st, int h, const Pts &pts, double gamma, double eps) {
  constexpr int NV = D + 2;
  const int lane = threadIdx.x & 63;
  const int np = pts.count(h);
  double cf[NV][N];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int l = 0; l < N; ++l) cf[v][l] = c[(long)(v * N + l) * st];
  double rmin = INFINITY;
  for (int i = lane; i < np; i += 64) {
    const double *ph = pts.row(h, i);
    double r = 0.0;
#pragma unroll
    for (int l = 0; l < N; ++l) r = fma(cf[0][l], ph[l], r);
    rmin = fmin(rmin, r);
  }
  rmin = wave_min(rmin);
  double Ub[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) Ub[v] = cf[v][0];
  const double th1 = (Ub[0] == rmin) ? 1.0 : fmin(fabs((Ub[0] - eps) / (Ub[0] - rmin)), 1.0);
#pragma unroll
  for (int l = 1; l < N; ++l) cf[0][l] *= th1;
  double th2 = 1.0;
  for (int i = lane; i < np; i += 64) {
    const double *ph = pts.row(h, i);
    double Uq[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      double u = 0.0;
#pragma unroll
      for (int l = 0; l < N; ++l) u = fma(cf[v][l], ph[l], u);
      Uq[v] = u;
    }
    double ke = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) ke = fma(Uq[1 + b], Uq[1 + b], ke);
    ke *= vrcp(Uq[0]);  // |m|^2 / rho with one reciprocal per point
    const double pq = (gamma - 1.0) * (Uq[D + 1] - 0.5 * ke);
    if (pq < eps) th2 = fmin(th2, tau_root<D>(Ub, Uq, gamma, eps));
  }
  th2 = wave_min(th2);
  if (lane == 0) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int l = 1; l < N; ++l) c[(long)(v * N + l) * st] = cf[v][l] * th2;
  }
}

// CHAR selects the characteristic limiter (eq. char_limiter) for the slope
// pass, else the component-wise one (eq. comp_limiter).
// Exponent of axis a in mode l (modes ordered by total degree, then
// x-exponent descending, then y-exponent descending).
template <int D>
__host__ __device__ constexpr int mode_exp(int l, int a) {
  int n = 0;
  for (int t = 0; t <= 8; ++t)
    for (int ex = t; ex >= 0; --ex)
      for (int ey = t - ex; ey >= 0; --ey) {
        const int ez = t - ex - ey;
        if (D == 2 && ez > 0) continue;
        if (n == l) return a == 0 ? ex : a == 1 ? ey : ez;
        ++n;
      }
  return 0;
}

static_assert(mode_exp<3>(1, 0) == 1 && mode_exp<3>(2, 1) == 1 && mode_exp<3>(3, 2) == 1 && mode_exp<3>(4, 0) == 2 &&
                  mode_exp<3>(5, 1) == 1 && mode_exp<3>(6, 2) == 1 && mode_exp<3>(9, 2) == 2 && mode_exp<2>(3, 0) == 2 &&
                  mode_exp<2>(5, 1) == 2 && mode_exp<3>(10, 0) == 3,
              "mode order: total degree, then x-exponent descending, then y-exponent descending");

// max over the reference cell of |phi_l| = prod_a sqrt(2 e_a + 1), from
// |P_n| <= 1 on [-1, 1]
template <int D>
__host__ __device__ constexpr double basis_bound(int l) {
  constexpr double r[9] = {1.0, 1.7320508075688772, 2.2360679774997898, 2.6457513110645907, 3.0,
                           3.3166247903554, 3.6055512754639891, 3.872983346207417, 4.1231056256176606};
  double b = 1.0;
  for (int a = 0; a < D; ++a) b *= r[mode_exp<D>(l, a)];
  return b;
}

// basis_bound of modes 0..N-1, evaluated by the compiler (a call left to run
// time would index the table with a computed exponent and put it in scratch
// memory)
template <int D, int N>
struct BasisBounds {
  double b[N];
  __host__ __device__ constexpr BasisBounds() : b() {
    for (int l = 0; l < N; ++l) b[l] = basis_bound<D>(l);
  }
};

// True when the cell's polynomial has, at every point of the reference cell,
// a density and a pressure above eps by a margin (1e-10 of the quantities'
// scale) far above the rounding of the point evaluations: then the
// positivity pass of Sec. 3.4 finds every point value >= eps, so theta_1 =
// theta_2 = 1 exactly and it would leave the cell unchanged; the point loop
// is skipped.  Bounds: |u(xi) - u_mean| <= sum_{l>=1} |w_l| max|phi_l| per
// variable, and p = (gamma-1)(E - |m|^2 / (2 rho)) >= (gamma-1)(E_lo -
// |m|_hi^2 / (2 rho_lo)).
// sum_{l>=1} |w_l| max|phi_l| of one variable's coefficients c
template <int D, int N>
__device__ inline double basis_excursion(const double *c) {
  constexpr BasisBounds<D, N> bb;
  double r = 0.0;
#pragma unroll
  for (int l = 1; l < N; ++l) r = fma(fabs(c[l]), bb.b[l], r);
  return r;
}

// the test above from the means and excursions R of the D + 2 variables
template <int D>
__device__ inline bool positivity_certain_mr(const double *mean, const double *R, double gamma, double eps) {
  const double rlo = mean[0] - R[0];
  if (!(rlo > eps + 1e-10 * (fabs(mean[0]) + R[0]))) return false;
  double m2 = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const double m = fabs(mean[1 + a]) + R[1 + a];
    m2 = fma(m, m, m2);
  }
  const double ke = 0.5 * m2 / rlo;
  const double plo = (gamma - 1.0) * ((mean[D + 1] - R[D + 1]) - ke);
  const double scale = (gamma - 1.0) * (fabs(mean[D + 1]) + R[D + 1] + ke);
  return plo > eps + 1e-10 * scale;
}

template <int D, int N>
__device__ inline bool positivity_certain(const double (&wc)[D + 2][N], double gamma, double eps) {
  double mean[D + 2], R[D + 2];
#pragma unroll
  for (int v = 0; v < D + 2; ++v) {
    mean[v] = wc[v][0];
    R[v] = basis_excursion<D, N>(wc[v]);
  }
  return positivity_certain_mr<D>(mean, R, gamma, eps);
}

template <int D, int K, bool CHAR>
__global__ __launch_bounds__(256) void k_limit(const double *__restrict__ tab, double *__restrict__ w, Grid g,
                                               int slope, double beta, double bound, int posit, double eps,
                                               int *__restrict__ flag, int *__restrict__ plist) {
  using C = Cfg<D, K>;
  // lanes past the grid stay in the wave (the list of troubled cells is
  // appended per wave) on a copy of the last cell, and store nothing
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = tid < g.ncell;
  const long cell = act ? tid : g.ncell - 1;
  const long nc = g.ncell;
  const int ix = (int)(cell % g.nx);
  const int iy = (int)((cell / g.nx) % g.ny);
  const int iz = (int)(cell / ((long)g.nx * g.ny));
  // the slope pass needs the means and slopes only: the higher modes are
  // loaded after it (and not at all where it dropped them), which keeps the
  // two register sets from being live together
  constexpr int NL = D + 1 < C::N ? D + 1 : C::N;
  double wc[C::NV][C::N];
  bool dropped[C::NV];
#pragma unroll
  for (int v = 0; v < C::NV; ++v) {
    dropped[v] = false;
#pragma unroll
    for (int l = 0; l < NL; ++l) wc[v][l] = w[(long)(v * C::N + l) * nc + cell];
  }

  if (slope && K >= 1) {
    const double r3 = sqrt(3.0);
    long nbl[D], nbh[D];
#pragma unroll
    for (int a = 0; a < D; ++a) {
      nbl[a] = neighbour(g, ix, iy, iz, a, -1);
      nbh[a] = neighbour(g, ix, iy, iz, a, 1);
      if (nbl[a] < 0) nbl[a] = cell;
      if (nbh[a] < 0) nbh[a] = cell;
    }
    if constexpr (CHAR) {
      auto nbmean = [&](int a, int s, double *m) {
        const long nb = s ? nbh[a] : nbl[a];
#pragma unroll
        for (int v = 0; v < C::NV; ++v) m[v] = w[(long)(v * C::N) * nc + nb];
      };
      const bool lim = char_limit_cell<D, C::N>(wc, nbmean, g.gamma, beta, bound);
#pragma unroll
      for (int v = 0; v < C::NV; ++v) dropped[v] = lim;
    } else
#pragma unroll
    for (int i = 0; i < C::NV; ++i) {
      const double mean = wc[i][0];
      double mt[D];
      bool limited = false;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double mlo = w[(long)(i * C::N) * nc + nbl[a]];
        const double mhi = w[(long)(i * C::N) * nc + nbh[a]];
        const double A = r3 * wc[i][1 + a];
        const double m = (fabs(A) <= bound) ? A : minmod3(A, beta * (mean - mlo), beta * (mhi - mean));
        mt[a] = m;
        limited |= (m != A);
      }
      if (limited) {
#pragma unroll
        for (int a = 0; a < D; ++a) wc[i][1 + a] = mt[a] / r3;
      }
      dropped[i] = limited;
    }
  }
  // the higher modes: zero where the slope pass dropped them
#pragma unroll
  for (int v = 0; v < C::NV; ++v)
#pragma unroll
    for (int l = NL; l < C::N; ++l) wc[v][l] = dropped[v] ? 0.0 : w[(long)(v * C::N + l) * nc + cell];

  if (posit) {
    double Ub[C::NV];
#pragma unroll
    for (int v = 0; v < C::NV; ++v) Ub[v] = wc[v][0];
    double keb = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) keb = fma(Ub[1 + b], Ub[1 + b], keb);
    keb *= vrcp(Ub[0]);
    const double pb = (g.gamma - 1.0) * (Ub[D + 1] - 0.5 * keb);
    const bool bad = !(Ub[0] > eps) || !(pb > eps);
    if (bad && act) atomicOr(flag, FLAG_NEGATIVE);
    // a cell whose bounds leave positivity open goes to k_positivity's list
    wave_append(act && !bad && !positivity_certain<D, C::N>(wc, g.gamma, eps), (int)cell, plist);
  }
  // write back the modes j >= 1 of the variables the slope pass changed
  // (the means are never changed; an unlimited variable's coefficients are
  // the ones in memory, so most cells of a smooth flow store nothing)
  if (act) {
#pragma unroll
    for (int v = 0; v < C::NV; ++v)
      if (dropped[v])
#pragma unroll
        for (int l = 1; l < C::N; ++l) w[(long)(v * C::N + l) * nc + cell] = wc[v][l];
  }
}

// ---------------------------------------------------------------------------
// Volume integral (eq. dg_term2) with BF16 inputs on MFMA, FP32 accumulation.
//
// Both contractions of the volume term are small GEMMs batched over cells:
//   A  U[cell, q] = sum_m w[cell, m] phi_m(xi_q)            (per variable)
//   B  V[cell, j] = sum_a sum_q F_a[cell, q] dphi_j/dxi_a(xi_q) w_q
// One wave handles 16 cells with v_mfma_f32_16x16x32_bf16 (A: 16x32, B: 32x16,
// C: 16x16 FP32).  Modes are padded to 32 and nodes to a multiple of 32 with
// zero table entries.  The stage-A result leaves, for every variable, four
// cells at one node in each lane, so the Euler flux is evaluated in-lane in
// FP32; the fluxes go through LDS as BF16 to the A-operand layout of stage B.
// V (FP32) is written to a scratch state that the stage kernel consumes.
// Mode 0 of V is exactly zero (dphi_1 = 0).
// Every operand x (weights, fluxes, tables) is carried as a BF16 pair
// x = hi + lo, hi = bf16(x), lo = bf16(x - hi), and each product as the three
// MFMAs lo*hi + hi*lo + hi*hi (the lo*lo term is below FP32 rounding of the
// sum): about 16 significant bits per operand instead of 8, so the rounding
// of a large flux (the pressure in a momentum flux) no longer swamps a small
// field's volume term.
// ---------------------------------------------------------------------------
template <int D, int K>
struct Mfma {
  static constexpr int NP = 32;                                  // padded modes
  static constexpr int QP = ((Cfg<D, K>::Q + 31) / 32) * 32;     // padded nodes
  static constexpr int NQT = QP / 16;                            // node tiles (stage A)
  static constexpr int NQC = QP / 32;                            // node chunks (stage B)
  static constexpr int PB = 0;                                   // phi [QP][NP]
  static constexpr int DB = PB + QP * NP;                        // dphi w, transposed [D][NP][QP]
  static constexpr int LO = DB + D * NP * QP;                    // the same tables' low parts
  static constexpr int TOTAL = 2 * LO;
};

template <int D, int K>
__global__ __launch_bounds__(256) void k_volume_bf16(const __bf16 *__restrict__ tb, const double *__restrict__ w,
                                                     long nc, float *__restrict__ vout, double gamma) {
  using C = Cfg<D, K>;
  using M = Mfma<D, K>;
  constexpr int NV = C::NV, N = C::N, QP = M::QP, NP = M::NP;
  __shared__ __bf16 fs[2][4][NV][16][QP];  // one flux direction at a time, per wave (hi, lo)
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int row = lane & 15, grp = lane >> 4;
  const long c0 = ((long)blockIdx.x * 4 + wv) * 16;
  const float gm1 = (float)(gamma - 1.0);

  // stage A: nodal values
  f32x4 U[NV][M::NQT];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    bf16x8 A, Al;
    const long cell = c0 + row;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int m = 8 * grp + e;
      const float x = (m < N && cell < nc) ? (float)w[(long)(v * N + m) * nc + cell] : 0.0f;
      A[e] = (__bf16)x;
      Al[e] = (__bf16)(x - (float)A[e]);
    }
#pragma unroll
    for (int t = 0; t < M::NQT; ++t) {
      const bf16x8 B = *reinterpret_cast<const bf16x8 *>(tb + M::PB + (16 * t + row) * NP + 8 * grp);
      const bf16x8 Bl = *reinterpret_cast<const bf16x8 *>(tb + M::LO + M::PB + (16 * t + row) * NP + 8 * grp);
      f32x4 z = {0.0f, 0.0f, 0.0f, 0.0f};
      z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, B, z, 0, 0, 0);
      z = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bl, z, 0, 0, 0);
      U[v][t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, z, 0, 0, 0);
    }
  }
  // stages A' and B per direction: the Euler flux f_a at (cell 4 grp + i,
  // node 16 t + row) into LDS as BF16, then its projection onto the gradient
  // table of direction a, accumulated over a in FP32
  constexpr int MT = (N + 15) / 16;  // only the tiles that hold modes
  f32x4 acc[NV][MT];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) acc[v][mt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int a = 0; a < D; ++a) {
#pragma unroll
    for (int t = 0; t < M::NQT; ++t)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int q = 16 * t + row;
        const int cl = 4 * grp + i;
        const bool ok = q < C::Q && c0 + cl < nc;
        float Uq[NV], F[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) Uq[v] = U[v][t][i];
        if (ok) {
          euler_flux<D, float>(Uq, a, gm1, F);
        } else {
#pragma unroll
          for (int v = 0; v < NV; ++v) F[v] = 0.0f;
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const __bf16 hi = (__bf16)F[v];
          fs[0][wv][v][cl][q] = hi;
          fs[1][wv][v][cl][q] = (__bf16)(F[v] - (float)hi);
        }
      }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int ch = 0; ch < M::NQC; ++ch) {
          const bf16x8 A = *reinterpret_cast<const bf16x8 *>(&fs[0][wv][v][row][ch * 32 + 8 * grp]);
          const bf16x8 Al = *reinterpret_cast<const bf16x8 *>(&fs[1][wv][v][row][ch * 32 + 8 * grp]);
          const long tbo = M::DB + (a * NP + mt * 16 + row) * QP + ch * 32 + 8 * grp;
          const bf16x8 B = *reinterpret_cast<const bf16x8 *>(tb + tbo);
          const bf16x8 Bl = *reinterpret_cast<const bf16x8 *>(tb + M::LO + tbo);
          acc[v][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(Al, B, acc[v][mt], 0, 0, 0);
          acc[v][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, Bl, acc[v][mt], 0, 0, 0);
          acc[v][mt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(A, B, acc[v][mt], 0, 0, 0);
        }
    __syncthreads();  // the next direction overwrites fs
  }
  // lane (row, grp) holds mode j of the four consecutive cells c0 + 4 grp + i:
  // one 16-byte store when they are all in range and the address is aligned
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
      const int j = mt * 16 + row;
      const long cb = c0 + 4 * grp;
      if (j < N) {
        float *dst = vout + (long)(v * N + j) * nc + cb;
        if (cb + 3 < nc && (reinterpret_cast<uintptr_t>(dst) & 15) == 0) {
          *reinterpret_cast<f32x4 *>(dst) = acc[v][mt];
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (cb + i < nc) dst[i] = acc[v][mt][i];
        }
      }
    }
}

// ---------------------------------------------------------------------------
// Static 2:1 refined box (hanging-face quadrature of Sec. 4, limiting at the
// refinement boundary of Sec. 4.4).  State: coarse block [nvar][N][ncc]
// (base grid; the base cells in [lo, hi) form a hole, ignored) followed by
// the fine block [nvar][N][ncf] (2(hi - lo) cells per axis, half the edge).
// A coarse face next to the hole is integrated at the Gauss points of the
// 2^(d-1) fine faces covering it: the coarse trace at (eta + sigma)/2 (table
// HG), lifted into the coarse cell with weight w_r / 2^(d-1) (table HW).
// Both sides evaluate the flux of a hanging node from the same traces with
// the same code, so the contributions cancel exactly in the sum of the means.
// One thread per cell over both blocks.
// ---------------------------------------------------------------------------
template <int D, int K, class R, int FX>
__global__ __launch_bounds__(256) void k_rhs_amr(const double *__restrict__ tab, const R *__restrict__ tabr,
                                                 const double *__restrict__ w, double *__restrict__ out,
                                                 const double *__restrict__ dtp, const float *__restrict__ vext,
                                                 AmrGrid g, int mode, Mix mx, int *__restrict__ flag) {
  using C = Cfg<D, K>;
  constexpr int NV = C::NV, N = C::N, QF = C::QF, NW = NV * N, NSUB = 1 << (D - 1);
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= g.ncc + g.ncf) return;
  const bool fine = tid >= g.ncc;
  const long cell = fine ? tid - g.ncc : tid;
  const long ncb = fine ? g.ncf : g.ncc;
  const double *wcb = w, *wfb = w + (long)NW * g.ncc;
  const double *wb = fine ? wfb : wcb;
  const long boff = fine ? (long)NW * g.ncc : 0;
  const int bn0 = fine ? g.nf[0] : g.n[0], bn1 = fine ? g.nf[1] : g.n[1];
  int i[3] = {(int)(cell % bn0), (int)((cell / bn0) % bn1), (int)(cell / ((long)bn0 * bn1))};
  const double cldt = (mode == 0) ? 0.0 : mx.cl * *dtp;
  if (!fine && amr_in_hole<D>(g, i)) {
    // hole cells carry no solution: L = 0
#pragma unroll 1
    for (int vl = 0; vl < NW; ++vl) {
      const long ii = boff + (long)vl * ncb + cell;
      out[ii] = (mode == 0) ? 0.0 : mix_out(mx, w[ii], 0.0, 0.0, ii);
    }
    return;
  }
  const R gm1 = (R)(g.gamma - 1.0);
  R wc[NV][N];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int l = 0; l < N; ++l) wc[v][l] = (R)wb[(long)(v * N + l) * ncb + cell];
  R acc[NV][N];
  double acc0[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    acc0[v] = 0.0;
#pragma unroll
    for (int l = 0; l < N; ++l) acc[v][l] = R(0);
  }
  // volume integral (precomputed in vext on the BF16 MFMA path)
  if (vext) {
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int l = 1; l < N; ++l) acc[v][l] = (R)vext[boff + (long)(v * N + l) * ncb + cell];
  }
#pragma unroll 1
  for (int q = 0; q < (vext ? 0 : C::Q); ++q) {
    R U[NV];
    const R *bq = tabr + C::B + q * N;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      R s = R(0);
#pragma unroll
      for (int l = 0; l < N; ++l) s = fma(wc[v][l], bq[l], s);
      U[v] = s;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) {
      R F[NV];
      euler_flux<D, R>(U, a, gm1, F);
      const R *dw = tabr + C::DW + (a * C::Q + q) * N;
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int l = 1; l < N; ++l) acc[v][l] = fma(F[v], dw[l], acc[v][l]);
    }
  }
  // faces
#pragma unroll
  for (int a = 0; a < D; ++a) {
    int t0 = 0, t1 = 0;  // tangential axes
    {
      int m = 0, tt[2] = {0, 0};
#pragma unroll
      for (int b = 0; b < D; ++b)
        if (b != a) tt[m++] = b;
      t0 = tt[0];
      t1 = tt[1];
    }
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      // classify the neighbour: 0 regular (same block), 1 wall, 2 hanging
      // (coarse cell facing the fine block), 3 coarse neighbour of a fine cell
      int kind = 0;
      long nbcell = cell;
      const double *nbb = wb;
      long nbn = ncb;
      int j[3], sub = 0;
      if (!fine) {
        if (!amr_coarse_nb<D>(g, i, a, s ? 1 : -1, j)) {
          kind = 1;
        } else if (amr_in_hole<D>(g, j)) {
          kind = 2;
        } else {
          nbcell = ((long)j[2] * g.n[1] + j[1]) * g.n[0] + j[0];
        }
      } else {
        int f2[3] = {i[0], i[1], i[2]};
        f2[a] += s ? 1 : -1;
        if (f2[a] >= 0 && f2[a] < g.nf[a]) {
          nbcell = ((long)f2[2] * g.nf[1] + f2[1]) * g.nf[0] + f2[0];
        } else {
          kind = 3;
          int base[3] = {0, 0, 0};
#pragma unroll
          for (int b = 0; b < D; ++b) base[b] = g.lo[b] + i[b] / 2;
          amr_coarse_nb<D>(g, base, a, s ? 1 : -1, j);
          nbcell = ((long)j[2] * g.n[1] + j[1]) * g.n[0] + j[0];
          nbb = wcb;
          nbn = g.ncc;
          sub = (i[t0] & 1) | (D == 3 ? ((i[t1] & 1) << 1) : 0);
        }
      }
      const int nsub = (kind == 2) ? NSUB : 1;
#pragma unroll 1
      for (int sb = 0; sb < nsub; ++sb) {
        if (kind == 2) {
          // the fine cell of sub-face sb behind this coarse face
          int fi[3] = {0, 0, 0};
          fi[a] = 2 * (j[a] - g.lo[a]) + (s ? 0 : 1);
          fi[t0] = 2 * (j[t0] - g.lo[t0]) + (sb & 1);
          if (D == 3) fi[t1] = 2 * (j[t1] - g.lo[t1]) + ((sb >> 1) & 1);
          nbcell = ((long)fi[2] * g.nf[1] + fi[1]) * g.nf[0] + fi[0];
          nbb = wfb;
          nbn = g.ncf;
          sub = sb;
        }
        R wnb[NV][N];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int l = 0; l < N; ++l) wnb[v][l] = (R)nbb[(long)(v * N + l) * nbn + nbcell];
        // own and neighbour evaluation tables, and the lift table
        const R *to = (kind == 2) ? tabr + C::HG + ((a * 2 + s) * 4 + sub) * QF * N
                                  : tabr + C::TF + (a * 2 + s) * QF * N;
        const R *tn = (kind == 3) ? tabr + C::HG + ((a * 2 + (1 - s)) * 4 + sub) * QF * N
                                  : tabr + C::TF + (a * 2 + (1 - s)) * QF * N;
        const R *tw = (kind == 2) ? tabr + C::HW + ((a * 2 + s) * 4 + sub) * QF * N
                                  : tabr + C::TW + (a * 2 + s) * QF * N;
        const double *tw0 = (kind == 2) ? tab + C::HW + ((a * 2 + s) * 4 + sub) * QF * N
                                        : tab + C::TW + (a * 2 + s) * QF * N;
#pragma unroll 1
        for (int r = 0; r < QF; ++r) {
          R Uo[NV], Un[NV], UL[NV], UR[NV], F[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            R so = R(0), sn = R(0);
#pragma unroll
            for (int l = 0; l < N; ++l) {
              so = fma(wc[v][l], to[r * N + l], so);
              sn = fma(wnb[v][l], tn[r * N + l], sn);
            }
            Uo[v] = so;
            Un[v] = (kind == 1) ? so : sn;
            UL[v] = s ? Uo[v] : Un[v];
            UR[v] = s ? Un[v] : Uo[v];
          }
          hllc<R, D, FX>(UL, UR, a, g.gamma, F);
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const R f = s ? -F[v] : F[v];
            acc0[v] = fma((double)f, tw0[r * N], acc0[v]);
#pragma unroll
            for (int l = 1; l < N; ++l) acc[v][l] = fma(f, tw[r * N + l], acc[v][l]);
          }
        }
      }
    }
  }
  const double fac = fine ? g.facf : g.facc;
  bool bad = false;
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const long ii = boff + (long)(v * N + l) * ncb + cell;
      const double L = fac * (l == 0 ? acc0[v] : (double)acc[v][l]);
      bad |= (L != L);
      out[ii] = (mode == 0) ? L : mix_out(mx, w[ii], L, cldt, ii);
    }
  if (bad) atomicOr(flag, FLAG_NAN);
}

// ---------------------------------------------------------------------------
// Refined-box RHS + stage at d = 3 with four lanes per cell (a quad), for the
// FP64 path at k = 3, where one thread per cell needs more registers than a
// lane has.  Lane s owns variable s and the energy modes [s M4, (s+1) M4):
// its weights, its accumulators, and per face the same slice of the
// neighbour's weights.  Nodes are taken four at a time: every lane forms its
// owned part of the traces (or nodal values) at the four nodes, a quad
// transpose hands lane t the full state at node t (energy partials summed in
// a fixed order), lane t evaluates the flux there, and a transpose back (plus
// a broadcast of the energy flux) returns to lane s the fluxes of its own
// variable at the four nodes for the projection or the lift.  Both cells of a
// face form each trace from the same weights, tables and summation order, so
// they still obtain the identical flux.
// ---------------------------------------------------------------------------
// lane s holds row s of a 4x4 block; afterwards it holds column s
__device__ inline void quad_transpose(double (&x)[4], int sub) {
  const bool b1 = sub & 2, b0 = sub & 1;
  double r0 = quad_swap<kQuadXor2>(b1 ? x[0] : x[2]);
  double r1 = quad_swap<kQuadXor2>(b1 ? x[1] : x[3]);
  const double y0 = b1 ? r0 : x[0], y1 = b1 ? r1 : x[1], y2 = b1 ? x[2] : r0, y3 = b1 ? x[3] : r1;
  r0 = quad_swap<kQuadXor1>(b0 ? y0 : y1);
  r1 = quad_swap<kQuadXor1>(b0 ? y2 : y3);
  x[0] = b0 ? r0 : y0;
  x[1] = b0 ? y1 : r0;
  x[2] = b0 ? r1 : y2;
  x[3] = b0 ? y3 : r1;
}

template <int K, int FX, bool UNI>
__global__ __launch_bounds__(256) void k_rhs_amr_quad(const double *__restrict__ tab, const double *__restrict__ w,
                                                      double *__restrict__ out, const double *__restrict__ dtp,
                                                      AmrGrid g, int mode, Mix mx, int *__restrict__ flag) {
  // UNI: a uniform grid (no fine block, an empty hole), so every face is a
  // regular or a wall face and the face tables are the same for all lanes
  constexpr int D = 3;
  using C = Cfg<D, K>;
  constexpr int NV = C::NV, N = C::N, QF = C::QF, Q = C::Q, NW = NV * N, NSUB = 4;
  constexpr int M4 = (N + 3) / 4;
  // nodes go in rounds of four; in a last, partial round the lanes past the
  // end take the last node again and their contributions are dropped
  const long tid = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 2;
  const int sub = threadIdx.x & 3;
  if (tid >= g.ncc + g.ncf) return;  // the four lanes of a cell leave together
  const bool fine = tid >= g.ncc;
  const long cell = fine ? tid - g.ncc : tid;
  const long ncb = fine ? g.ncf : g.ncc;
  const double *wcb = w, *wfb = w + (long)NW * g.ncc;
  const double *wb = fine ? wfb : wcb;
  const long boff = fine ? (long)NW * g.ncc : 0;
  const int bn0 = fine ? g.nf[0] : g.n[0], bn1 = fine ? g.nf[1] : g.n[1];
  int i[3] = {(int)(cell % bn0), (int)((cell / bn0) % bn1), (int)(cell / ((long)bn0 * bn1))};
  const double cldt = (mode == 0) ? 0.0 : mx.cl * *dtp;
  if (!fine && amr_in_hole<D>(g, i)) {
#pragma unroll 1
    for (int vl = sub; vl < NW; vl += 4) {
      const long ii = boff + (long)vl * ncb + cell;
      out[ii] = (mode == 0) ? 0.0 : mix_out(mx, w[ii], 0.0, 0.0, ii);
    }
    return;
  }
  const double gm1 = g.gamma - 1.0;
  double wo[N], we[M4], acc[N], acce[M4];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    wo[l] = wb[(long)(sub * N + l) * ncb + cell];
    acc[l] = 0.0;
  }
#pragma unroll
  for (int m = 0; m < M4; ++m) {
    const int j = sub * M4 + m;
    we[m] = (j < N) ? wb[(long)(4 * N + j) * ncb + cell] : 0.0;
    acce[m] = 0.0;
  }

  // volume integral (eq. dg_term2), nodes q0 .. q0+3 per round
#pragma unroll 1
  for (int q0 = 0; q0 < Q; q0 += 4) {
    double u[4], e[4];
#pragma unroll 1
    for (int t = 0; t < 4; ++t) {
      const double *bq = tab + C::B + min(q0 + t, Q - 1) * N;
      double su = 0.0, se = 0.0;
#pragma unroll
      for (int l = 0; l < N; ++l) su = fma(wo[l], bq[l], su);
#pragma unroll
      for (int m = 0; m < M4; ++m) {
        const int j = sub * M4 + m;
        se = fma(we[m], bq[j < N ? j : 0], se);
      }
#pragma unroll
      for (int tt = 0; tt < 4; ++tt) {
        u[tt] = (tt == t) ? su : u[tt];
        e[tt] = (tt == t) ? se : e[tt];
      }
    }
    quad_transpose(u, sub);
    quad_transpose(e, sub);
    double U[NV] = {u[0], u[1], u[2], u[3], (e[0] + e[1]) + (e[2] + e[3])};
    const double ir = vrcp(U[0]);
    double vel[D], ke = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) {
      vel[b] = U[1 + b] * ir;
      ke = fma(U[1 + b], vel[b], ke);
    }
    const double p = gm1 * (U[4] - 0.5 * ke);
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double fv[4] = {U[1 + a], 0.0, 0.0, 0.0};
#pragma unroll
      for (int b = 0; b < D; ++b) fv[1 + b] = fma(U[1 + b], vel[a], b == a ? p : 0.0);
      const double fe_own = (U[4] + p) * vel[a];
      quad_transpose(fv, sub);  // fv[t]: flux of variable sub at node q0 + t
      const double fe[4] = {quad_from<0>(fe_own), quad_from<1>(fe_own), quad_from<2>(fe_own), quad_from<3>(fe_own)};
#pragma unroll 1
      for (int t = 0; t < (Q % 4 == 0 ? 4 : min(4, Q - q0)); ++t) {
        const double *dw = tab + C::DW + (a * Q + q0 + t) * N;
        double ft = fv[0], f4t = fe[0];
#pragma unroll
        for (int tt = 1; tt < 4; ++tt) {
          ft = (tt == t) ? fv[tt] : ft;
          f4t = (tt == t) ? fe[tt] : f4t;
        }
#pragma unroll
        for (int l = 1; l < N; ++l) acc[l] = fma(ft, dw[l], acc[l]);
#pragma unroll
        for (int m = 0; m < M4; ++m) {
          const int j = sub * M4 + m;
          if (j >= 1 && j < N) acce[m] = fma(f4t, dw[j], acce[m]);
        }
      }
    }
  }

  // faces (eq. dg_term3), hanging faces as in k_rhs_amr
#pragma unroll 1
  for (int a = 0; a < D; ++a) {
    const int t0 = (a == 0) ? 1 : 0, t1 = (a == 2) ? 1 : 2;
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      int kind = 0;
      long nbcell = cell;
      const double *nbb = wb;
      long nbn = ncb;
      int j[3] = {0, 0, 0}, hsub = 0;
      if constexpr (UNI) {
        if (!amr_coarse_nb<D>(g, i, a, s ? 1 : -1, j))
          kind = 1;
        else
          nbcell = ((long)j[2] * g.n[1] + j[1]) * g.n[0] + j[0];
      } else if (!fine) {
        if (!amr_coarse_nb<D>(g, i, a, s ? 1 : -1, j)) {
          kind = 1;
        } else if (amr_in_hole<D>(g, j)) {
          kind = 2;
        } else {
          nbcell = ((long)j[2] * g.n[1] + j[1]) * g.n[0] + j[0];
        }
      } else {
        int f2[3] = {i[0], i[1], i[2]};
        f2[a] += s ? 1 : -1;
        if (f2[a] >= 0 && f2[a] < g.nf[a]) {
          nbcell = ((long)f2[2] * g.nf[1] + f2[1]) * g.nf[0] + f2[0];
        } else {
          kind = 3;
          int base[3] = {0, 0, 0};
#pragma unroll
          for (int b = 0; b < D; ++b) base[b] = g.lo[b] + i[b] / 2;
          amr_coarse_nb<D>(g, base, a, s ? 1 : -1, j);
          nbcell = ((long)j[2] * g.n[1] + j[1]) * g.n[0] + j[0];
          nbb = wcb;
          nbn = g.ncc;
          hsub = (i[t0] & 1) | ((i[t1] & 1) << 1);
        }
      }
      const int nsub = (!UNI && kind == 2) ? NSUB : 1;
#pragma unroll 1
      for (int sb = 0; sb < nsub; ++sb) {
        if (!UNI && kind == 2) {
          int fi[3] = {0, 0, 0};
          fi[a] = 2 * (j[a] - g.lo[a]) + (s ? 0 : 1);
          fi[t0] = 2 * (j[t0] - g.lo[t0]) + (sb & 1);
          fi[t1] = 2 * (j[t1] - g.lo[t1]) + ((sb >> 1) & 1);
          nbcell = ((long)fi[2] * g.nf[1] + fi[1]) * g.nf[0] + fi[0];
          nbb = wfb;
          nbn = g.ncf;
          hsub = sb;
        }
        // the neighbour's slice of weights owned by this lane
        double no[N], ne[M4];
        {
          const double *pn = nbb + (long)(sub * N) * nbn + nbcell;
#pragma unroll
          for (int l = 0; l < N; ++l, pn += nbn) no[l] = *pn;
          const double *pe = nbb + (long)(4 * N + sub * M4) * nbn + nbcell;
#pragma unroll
          for (int m = 0; m < M4; ++m, pe += nbn) ne[m] = (sub * M4 + m < N) ? *pe : 0.0;
        }
        const double *to = (!UNI && kind == 2) ? tab + C::HG + ((a * 2 + s) * 4 + hsub) * QF * N
                                               : tab + C::TF + (a * 2 + s) * QF * N;
        const double *tn = (!UNI && kind == 3) ? tab + C::HG + ((a * 2 + (1 - s)) * 4 + hsub) * QF * N
                                               : tab + C::TF + (a * 2 + (1 - s)) * QF * N;
        const double *tw = (!UNI && kind == 2) ? tab + C::HW + ((a * 2 + s) * 4 + hsub) * QF * N
                                               : tab + C::TW + (a * 2 + s) * QF * N;
#pragma unroll 1
        for (int r0 = 0; r0 < QF; r0 += 4) {
          // one node at a time (the tables of a hanging face differ between
          // cells, so they are vector loads; this bounds how many are live)
          double uo[4], eo[4], un[4], en[4];
#pragma unroll 1
          for (int t = 0; t < 4; ++t) {
            const int rt = min(r0 + t, QF - 1);
            const double *ro = to + rt * N, *rn = tn + rt * N;
            double so = 0.0, sn = 0.0, xo = 0.0, xn = 0.0;
#pragma unroll
            for (int l = 0; l < N; ++l) {
              so = fma(wo[l], ro[l], so);
              sn = fma(no[l], rn[l], sn);
            }
#pragma unroll
            for (int m = 0; m < M4; ++m) {
              const int jj = sub * M4 + m;
              xo = fma(we[m], ro[jj < N ? jj : 0], xo);
              xn = fma(ne[m], rn[jj < N ? jj : 0], xn);
            }
#pragma unroll
            for (int tt = 0; tt < 4; ++tt) {
              uo[tt] = (tt == t) ? so : uo[tt];
              un[tt] = (tt == t) ? sn : un[tt];
              eo[tt] = (tt == t) ? xo : eo[tt];
              en[tt] = (tt == t) ? xn : en[tt];
            }
          }
          quad_transpose(uo, sub);
          quad_transpose(eo, sub);
          quad_transpose(un, sub);
          quad_transpose(en, sub);
          double Uo[NV] = {uo[0], uo[1], uo[2], uo[3], (eo[0] + eo[1]) + (eo[2] + eo[3])};
          double Un[NV] = {un[0], un[1], un[2], un[3], (en[0] + en[1]) + (en[2] + en[3])};
          double UL[NV], UR[NV], F[NV];
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            const double nv = (kind == 1) ? Uo[v] : Un[v];  // wall: ghost trace = own trace
            UL[v] = s ? Uo[v] : nv;
            UR[v] = s ? nv : Uo[v];
          }
          hllc<double, D, FX>(UL, UR, a, g.gamma, F);
          double fv[4] = {F[0], F[1], F[2], F[3]};
          quad_transpose(fv, sub);  // fv[t]: flux of variable sub at node r0 + t
          const double fe[4] = {quad_from<0>(F[4]), quad_from<1>(F[4]), quad_from<2>(F[4]), quad_from<3>(F[4])};
#pragma unroll 1
          for (int t = 0; t < (QF % 4 == 0 ? 4 : min(4, QF - r0)); ++t) {
            const double *rw = tw + (r0 + t) * N;
            double ft = fv[0], f4t = fe[0];
#pragma unroll
            for (int tt = 1; tt < 4; ++tt) {
              ft = (tt == t) ? fv[tt] : ft;
              f4t = (tt == t) ? fe[tt] : f4t;
            }
            const double f = s ? -ft : ft, f4 = s ? -f4t : f4t;
#pragma unroll
            for (int l = 0; l < N; ++l) acc[l] = fma(f, rw[l], acc[l]);
#pragma unroll
            for (int m = 0; m < M4; ++m) {
              const int jj = sub * M4 + m;
              if (jj < N) acce[m] = fma(f4, rw[jj], acce[m]);
            }
          }
        }
      }
    }
  }

  const double fac = fine ? g.facf : g.facc;
  bool bad = false;
  auto emit = [&](int vl, double L) {
    const long ii = boff + (long)vl * ncb + cell;
    bad |= (L != L);
    out[ii] = (mode == 0) ? L : mix_out(mx, w[ii], L, cldt, ii);
  };
#pragma unroll
  for (int l = 0; l < N; ++l) emit(sub * N + l, fac * acc[l]);
#pragma unroll
  for (int m = 0; m < M4; ++m) {
    const int jj = sub * M4 + m;
    if (jj < N) emit(4 * N + jj, fac * acce[m]);
  }
  if (bad) atomicOr(flag, FLAG_NAN);
}

// ---------------------------------------------------------------------------
// 2D adjoint with four lanes per cell: lane s owns variable s (its weights,
// its lambda and its mu).  Nodes go in rounds of four (a last, partial round
// repeats the last node and drops its contributions): each lane forms its
// variable's part at the four nodes, a quad transpose hands lane t all four
// variables at node t for the transposed Euler flux or the reverse sweep
// through the Riemann solver, and a transpose back returns to lane s its
// variable's cotangents.  The arithmetic and its order are those of
// k_adjoint; one thread per cell holds three state-sized register sets there
// and spills at k = 3.
// ---------------------------------------------------------------------------
template <int K, int FX>
__global__ __launch_bounds__(256) void k_adjoint_quad2d(const double *__restrict__ tab, const double *__restrict__ w,
                                                        const double *__restrict__ lam, const double *acc_in,
                                                        double *__restrict__ out, double *acc_out,
                                                        const double *__restrict__ dtp, Grid g, int mode, double ca,
                                                        double cb, int *__restrict__ flag) {
  constexpr int D = 2;
  using C = Cfg<D, K>;
  constexpr int NV = C::NV, N = C::N, Q = C::Q, QF = C::QF;
  static_assert(NV == 4, "one lane per variable");
  const long cell = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 2;
  const int sub = threadIdx.x & 3;
  if (cell >= g.ncell) return;  // the four lanes of a cell leave together
  const long nc = g.ncell;
  const int ix = (int)(cell % g.nx), iy = (int)((cell / g.nx) % g.ny);

  double wv[N], lv[N], mu[N];
#pragma unroll
  for (int l = 0; l < N; ++l) {
    const long i = (long)(sub * N + l) * nc + cell;
    wv[l] = w[i];
    lv[l] = lam[i];
    mu[l] = 0.0;
  }

  // volume term
#pragma unroll 1
  for (int q0 = 0; q0 < Q; q0 += 4) {
    double u[4], lx[4], ly[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int qt = min(q0 + t, Q - 1);
      const double *bq = tab + C::B + qt * N;
      const double *d0 = tab + C::DW + qt * N, *d1 = tab + C::DW + (Q + qt) * N;
      double su = 0.0, s0 = 0.0, s1 = 0.0;
#pragma unroll
      for (int l = 0; l < N; ++l) {
        su = fma(wv[l], bq[l], su);
        s0 = fma(lv[l], d0[l], s0);
        s1 = fma(lv[l], d1[l], s1);
      }
      u[t] = su;
      lx[t] = s0;
      ly[t] = s1;
    }
    quad_transpose(u, sub);  // lane t: the four variables at node q0 + t
    quad_transpose(lx, sub);
    quad_transpose(ly, sub);
    double G[NV] = {0.0, 0.0, 0.0, 0.0};
    euler_flux_vjp<D>(u, 0, g.gamma, lx, G);
    euler_flux_vjp<D>(u, 1, g.gamma, ly, G);
    quad_transpose(G, sub);  // G[t]: component sub at node q0 + t
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      if (Q % 4 == 0 || q0 + t < Q) {
        const double *bq = tab + C::B + (q0 + t) * N;
#pragma unroll
        for (int l = 0; l < N; ++l) mu[l] = fma(G[t], bq[l], mu[l]);
      }
    }
  }

  // face terms: own side with TF(s), TW(s); neighbour side with TF(1-s),
  // TW(1-s) (see k_adjoint)
#pragma unroll 1
  for (int a = 0; a < D; ++a) {
#pragma unroll 1
    for (int s = 0; s < 2; ++s) {
      const long nb = neighbour(g, ix, iy, 0, a, s ? 1 : -1);
      const long src = nb >= 0 ? nb : cell;
      double wnb[N], lnb[N];
#pragma unroll
      for (int l = 0; l < N; ++l) {
        const long i = (long)(sub * N + l) * nc + src;
        wnb[l] = w[i];
        lnb[l] = lam[i];
      }
      const double *to = tab + C::TF + (a * 2 + s) * QF * N;
      const double *tn = tab + C::TF + (a * 2 + (1 - s)) * QF * N;
      const double *two = tab + C::TW + (a * 2 + s) * QF * N;
      const double *twn = tab + C::TW + (a * 2 + (1 - s)) * QF * N;
#pragma unroll 1
      for (int r0 = 0; r0 < QF; r0 += 4) {
        double uo[4], un[4], lo[4], ln[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int rt = min(r0 + t, QF - 1);
          double so = 0.0, sn = 0.0, xo = 0.0, xn = 0.0;
#pragma unroll
          for (int l = 0; l < N; ++l) {
            so = fma(wv[l], to[rt * N + l], so);
            sn = fma(wnb[l], tn[rt * N + l], sn);
            xo = fma(lv[l], two[rt * N + l], xo);
            xn = fma(lnb[l], twn[rt * N + l], xn);
          }
          uo[t] = so;
          un[t] = sn;
          lo[t] = xo;
          ln[t] = xn;
        }
        quad_transpose(uo, sub);  // lane t: the four variables at node r0 + t
        quad_transpose(un, sub);
        quad_transpose(lo, sub);
        quad_transpose(ln, sub);
        double UL[NV], UR[NV], gv[NV], gL[NV], gR[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          if (nb < 0) ln[v] = 0.0;  // the ghost cell of a transmissive boundary has no equation
          const double nv = nb >= 0 ? un[v] : uo[v];
          gv[v] = s ? ln[v] - lo[v] : lo[v] - ln[v];  // lam_high . TW(-1) - lam_low . TW(+1)
          UL[v] = s ? uo[v] : nv;
          UR[v] = s ? nv : uo[v];
        }
        hllc_vjp<D, FX>(UL, UR, a, g.gamma, gv, gL, gR);
        double h[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) h[v] = (s ? gL[v] : gR[v]) + (nb >= 0 ? 0.0 : (s ? gR[v] : gL[v]));
        quad_transpose(h, sub);  // h[t]: component sub at node r0 + t
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          if (QF % 4 == 0 || r0 + t < QF) {
#pragma unroll
            for (int l = 0; l < N; ++l) mu[l] = fma(h[t], to[(r0 + t) * N + l], mu[l]);
          }
        }
      }
    }
  }

  const double dt = (mode == 0) ? 0.0 : *dtp;
  bool bad = false;
#pragma unroll
  for (int l = 0; l < N; ++l) {
    const long i = (long)(sub * N + l) * nc + cell;
    const double m = g.fac * mu[l];
    bad |= (m != m);
    if (mode == 0) {
      out[i] = m;
    } else if (mode == 1) {
      out[i] = acc_in[i] + (lv[l] + dt * m);
    } else {
      out[i] = cb * (lv[l] + dt * m);
      acc_out[i] = (mode == 3) ? ca * lv[l] : acc_in[i] + ca * lv[l];
    }
  }
  if (bad) atomicOr(flag, FLAG_NAN);
}

// Time step over both blocks (each cell with its own edge length); same
// two-kernel reduction as k_rate / k_dt_final.
template <int D>
__global__ __launch_bounds__(256) void k_rate_amr(const double *__restrict__ w, AmrGrid g, int N,
                                                  unsigned long long *ratemax, int *__restrict__ flag) {
  double m = 0.0;
  bool bad = false;
  const long ntot = g.ncc + g.ncf;
  for (long t = (long)blockIdx.x * blockDim.x + threadIdx.x; t < ntot; t += (long)gridDim.x * blockDim.x) {
    const bool fine = t >= g.ncc;
    const long cell = fine ? t - g.ncc : t;
    if (!fine) {
      int i[3] = {(int)(cell % g.n[0]), (int)((cell / g.n[0]) % g.n[1]), (int)(cell / ((long)g.n[0] * g.n[1]))};
      if (amr_in_hole<D>(g, i)) continue;
    }
    const double *wb = fine ? w + (long)(D + 2) * N * g.ncc : w;
    const long ncb = fine ? g.ncf : g.ncc;
    const double dx = fine ? g.dxf : g.dxc;
    double U[D + 2];
#pragma unroll
    for (int v = 0; v < D + 2; ++v) U[v] = wb[(long)v * N * ncb + cell];
    m = fmax(m, cell_rate<D>(U, g.gamma, dx, bad));
  }
  if (bad) atomicOr(flag, FLAG_NEGATIVE);
  m = block_max(m);
  if (threadIdx.x == 0) atomicMax(rate_slot(ratemax, blockIdx.x), (unsigned long long)__double_as_longlong(m));
}

// ---------------------------------------------------------------------------
// Adaptive refinement of the one-box mesh (Sec. 4.1-4.3).  A mesh is a base
// grid plus, optionally, one box [lo, hi) of base cells split 2^d ways; a
// state holds the base block, then the fine block.
// ---------------------------------------------------------------------------
struct BoxGrid {
  int n[3], lo[3], hi[3], nf[3];
  long ncc, ncf;
  int box;  // 0: no refined box
};

template <int D>
__device__ inline bool bg_in_box(const BoxGrid &g, const int *i) {
  if (!g.box) return false;
#pragma unroll
  for (int a = 0; a < D; ++a)
    if (i[a] < g.lo[a] || i[a] >= g.hi[a]) return false;
  return true;
}

// fine-block index of child ch (bit a: upper half along a) of base cell i
template <int D>
__device__ inline long bg_fine(const BoxGrid &g, const int *i, int ch) {
  int f[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < D; ++a) f[a] = 2 * (i[a] - g.lo[a]) + ((ch >> a) & 1);
  return ((long)f[2] * g.nf[1] + f[1]) * g.nf[0] + f[0];
}

// Refinement flags (eqs. cell_ref, node_ref): per base cell, the largest
// density slope coefficient |w_rho,1+a| against thr_cell = alpha w_t, or for a
// refined base cell that of its node weights (the derefined projection of
// its children, eq. deref_weights) against thr_node = w_t / alpha.  Flagged
// cells also widen box = (min i, max i) by atomics.
template <int D, int K>
__global__ __launch_bounds__(256) void k_amr_flags(const double *__restrict__ w, const double *__restrict__ P,
                                                   BoxGrid g, double thr_cell, double thr_node, int *__restrict__ flags,
                                                   int *__restrict__ box) {
  constexpr int N = Cfg<D, K>::N, NCH = 1 << D;
  const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.ncc) return;
  int i[3] = {(int)(cell % g.n[0]), (int)((cell / g.n[0]) % g.n[1]), (int)(cell / ((long)g.n[0] * g.n[1]))};
  double m = 0.0;
  bool flag;
  if (bg_in_box<D>(g, i)) {
    const double *wf = w + (long)(D + 2) * N * g.ncc;  // fine block; density is variable 0
#pragma unroll
    for (int a = 0; a < D; ++a) {
      double node = 0.0;
      for (int ch = 0; ch < NCH; ++ch) {
        const long f = bg_fine<D>(g, i, ch);
        for (int l = 0; l < N; ++l) node = fma(P[((long)ch * N + l) * N + 1 + a], wf[(long)l * g.ncf + f], node);
      }
      m = fmax(m, fabs(node / (double)NCH));
    }
    flag = m > thr_node;
  } else {
#pragma unroll
    for (int a = 0; a < D; ++a) m = fmax(m, fabs(w[(long)(1 + a) * g.ncc + cell]));
    flag = m > thr_cell;
  }
  flags[cell] = flag ? 1 : 0;
  if (flag) {
#pragma unroll
    for (int a = 0; a < D; ++a) {
      atomicMin(box + a, i[a]);
      atomicMax(box + 3 + a, i[a]);
    }
  }
}

__global__ void k_box_init(int *box) {
  if (threadIdx.x < 3) box[threadIdx.x] = 0x7fffffff;
  else if (threadIdx.x < 6) box[threadIdx.x] = -1;
}

// The refined box of the next mesh from the flagged range (min i, max i) per
// axis: the range grown by the one buffer layer of Sec. 4 (every flagged
// cell's neighbours are refined too), clipped to [1, n-1] so that the box
// keeps one coarse layer to the domain boundary; box = (lo[3], hi[3]) in
// refine_lo / refine_hi form, all zero when nothing is flagged or the
// clipped box is empty along some axis.
__global__ void k_box_final(int *box, int d, int nx, int ny, int nz) {
  if (threadIdx.x != 0) return;
  const int n[3] = {nx, ny, nz};
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  bool ok = true;
  for (int a = 0; a < d; ++a) {
    if (box[a] > box[3 + a]) ok = false;  // nothing flagged
    lo[a] = max(1, box[a] - 1);
    hi[a] = min(n[a] - 1, box[3 + a] + 2);
    if (hi[a] <= lo[a]) ok = false;
  }
  for (int a = 0; a < 3; ++a) {
    box[a] = ok ? lo[a] : 0;
    box[3 + a] = ok ? hi[a] : 0;
  }
}

// State on mesh B from a state on mesh A (same base grid): one thread per
// base cell of B, then per fine cell of B.  A base cell outside B's box is
// copied, or derefined (eq. deref_weights) if it was in A's box; one inside
// B's box is zeroed (a hole cell).  A fine cell of B is copied from A if its
// base cell was refined in A, else it is the refinement (eq. ref_weights) of
// the base cell's polynomial.
template <int D, int K>
__global__ __launch_bounds__(256) void k_amr_regrid(const double *__restrict__ wa, BoxGrid A,
                                                    const double *__restrict__ P, double *__restrict__ wb,
                                                    BoxGrid B) {
  constexpr int NV = D + 2, N = Cfg<D, K>::N, NCH = 1 << D;
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= B.ncc + B.ncf) return;
  const double *wa_f = wa + (long)NV * N * A.ncc;
  double *wb_f = wb + (long)NV * N * B.ncc;
  if (tid < B.ncc) {
    const long cell = tid;
    int i[3] = {(int)(cell % B.n[0]), (int)((cell / B.n[0]) % B.n[1]), (int)(cell / ((long)B.n[0] * B.n[1]))};
    if (bg_in_box<D>(B, i)) {
      for (int vl = 0; vl < NV * N; ++vl) wb[(long)vl * B.ncc + cell] = 0.0;
    } else if (bg_in_box<D>(A, i)) {
      long f[NCH];
#pragma unroll
      for (int ch = 0; ch < NCH; ++ch) f[ch] = bg_fine<D>(A, i, ch);
      for (int v = 0; v < NV; ++v)
        for (int j = 0; j < N; ++j) {
          double acc = 0.0;
#pragma unroll
          for (int ch = 0; ch < NCH; ++ch)
            for (int l = 0; l < N; ++l)
              acc = fma(P[((long)ch * N + l) * N + j], wa_f[(long)(v * N + l) * A.ncf + f[ch]], acc);
          wb[(long)(v * N + j) * B.ncc + cell] = acc / (double)NCH;
        }
    } else {
      for (int vl = 0; vl < NV * N; ++vl) wb[(long)vl * B.ncc + cell] = wa[(long)vl * A.ncc + cell];
    }
    return;
  }
  const long f = tid - B.ncc;
  const int fi[3] = {(int)(f % B.nf[0]), (int)((f / B.nf[0]) % B.nf[1]), (int)(f / ((long)B.nf[0] * B.nf[1]))};
  int i[3] = {0, 0, 0}, ch = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    i[a] = B.lo[a] + fi[a] / 2;
    ch |= (fi[a] & 1) << a;
  }
  if (bg_in_box<D>(A, i)) {
    const long fo = bg_fine<D>(A, i, ch);
    for (int vl = 0; vl < NV * N; ++vl) wb_f[(long)vl * B.ncf + f] = wa_f[(long)vl * A.ncf + fo];
  } else {
    const long cell = ((long)i[2] * A.n[1] + i[1]) * A.n[0] + i[0];
    for (int v = 0; v < NV; ++v)
      for (int j = 0; j < N; ++j) {
        double acc = 0.0;
        for (int l = 0; l < N; ++l) acc = fma(P[((long)ch * N + j) * N + l], wa[(long)(v * N + l) * A.ncc + cell], acc);
        wb_f[(long)(v * N + j) * B.ncf + f] = acc;
      }
  }
}

// Limiters on the refined mesh: neighbour means across the refinement
// boundary are the children's average (coarse side) or the coarse polynomial's
// mean over the adjacent child (fine side); coarse cells facing the fine block
// also check positivity at the hanging-face points (k_positivity).  One
// launch covers the ids [t0, t0 + tn) of the combined numbering (coarse
// cells, then fine cells): a fine cell on the block boundary reads the whole
// coarse neighbour polynomial, which the coarse cell's own pass rewrites, so
// the fine block is limited first and the coarse block after it (every
// neighbour value then comes from the state before limiting, as the
// limiter's definition has it; means are never written).
template <int D, int K, bool CHAR>
__global__ __launch_bounds__(256, 2) void k_limit_amr(const double *__restrict__ tab, double *__restrict__ w, AmrGrid g,
                                                      long t0, long tn, int slope, double beta, double mtilde,
                                                      int posit, double eps, int *__restrict__ flag,
                                                      int *__restrict__ plist) {
  using C = Cfg<D, K>;
  constexpr int NV = C::NV, N = C::N, NW = NV * N, NSUB = 1 << (D - 1);
  // lanes past the grid and on hole cells stay in the wave (the list of
  // troubled cells is appended per wave) and store nothing
  const long tid0 = t0 + (long)blockIdx.x * blockDim.x + threadIdx.x;
  const long tid = tid0 < t0 + tn ? tid0 : t0 + tn - 1;
  const bool fine = tid >= g.ncc;
  const long cell = fine ? tid - g.ncc : tid;
  const long ncb = fine ? g.ncf : g.ncc;
  double *wcb = w, *wfb = w + (long)NW * g.ncc;
  double *wb = fine ? wfb : wcb;
  const int bn0 = fine ? g.nf[0] : g.n[0], bn1 = fine ? g.nf[1] : g.n[1];
  int i[3] = {(int)(cell % bn0), (int)((cell / bn0) % bn1), (int)(cell / ((long)bn0 * bn1))};
  const bool act = tid0 < t0 + tn && (fine || !amr_in_hole<D>(g, i));
  constexpr int NL = D + 1 < N ? D + 1 : N;
  const double dx = fine ? g.dxf : g.dxc;
  if constexpr (!CHAR && D == 3 && K == 3) {
    // component-wise at 3D k = 3: one variable at a time (only its N
    // coefficients live, not all (D+2) N: 144 registers and three waves per
    // SIMD instead of 256 and two; at lower degree the compiler keeps the
    // all-variables form below in fewer registers).  Per side
    // of the cell, once: what the neighbour mean is (0 the own mean at a
    // wall, 1 the average of the 2^d children of a refined coarse neighbour,
    // first child fine cell snb, 2 the mean of cell snb of block sfine,
    // 3 the coarse polynomial of coarse cell snb over child sch)
    int sk[2 * D], sch[2 * D];
    long snb[2 * D];
    bool sfine[2 * D];
#pragma unroll
    for (int a = 0; a < D; ++a)
#pragma unroll
      for (int s = 0; s < 2; ++s) {
        const int f = 2 * a + s;
        sk[f] = 0; sch[f] = 0; snb[f] = 0; sfine[f] = fine;
        if (!fine) {
          int j[3];
          if (!amr_coarse_nb<D>(g, i, a, s ? 1 : -1, j)) {
            sk[f] = 0;
          } else if (amr_in_hole<D>(g, j)) {
            int fi[3] = {0, 0, 0};
#pragma unroll
            for (int b = 0; b < D; ++b) fi[b] = 2 * (j[b] - g.lo[b]);
            sk[f] = 1;
            snb[f] = ((long)fi[2] * g.nf[1] + fi[1]) * g.nf[0] + fi[0];
          } else {
            sk[f] = 2;
            snb[f] = ((long)j[2] * g.n[1] + j[1]) * g.n[0] + j[0];
          }
        } else {
          int f2[3] = {i[0], i[1], i[2]};
          f2[a] += s ? 1 : -1;
          if (f2[a] >= 0 && f2[a] < g.nf[a]) {
            sk[f] = 2;
            snb[f] = ((long)f2[2] * g.nf[1] + f2[1]) * g.nf[0] + f2[0];
          } else {
            int base[3] = {0, 0, 0}, j[3];
#pragma unroll
            for (int b = 0; b < D; ++b) base[b] = g.lo[b] + i[b] / 2;
            amr_coarse_nb<D>(g, base, a, s ? 1 : -1, j);
            sk[f] = 3;
            snb[f] = ((long)j[2] * g.n[1] + j[1]) * g.n[0] + j[0];
            int ch = 0;
#pragma unroll
            for (int b = 0; b < D; ++b) ch |= ((b == a) ? (s ? 0 : 1) : (i[b] & 1)) << b;
            sch[f] = ch;
          }
        }
      }
    const long cstr[3] = {1, (long)g.nf[0], (long)g.nf[0] * g.nf[1]};  // fine-cell strides of the children
    // what the positivity bounds need, accumulated in variable order (the
    // order of positivity_certain_mr): density mean and excursion, energy
    // mean and excursion, sum (|m_a| + R_a)^2 and |m|^2
    double m0 = 0.0, r0 = 0.0, mE = 0.0, rE = 0.0, m2 = 0.0, keb = 0.0;
#pragma unroll 1
    for (int v = 0; v < NV; ++v) {
      double c[N];
#pragma unroll
      for (int l = 0; l < NL; ++l) c[l] = wb[(long)(v * N + l) * ncb + cell];
      bool limited = false;
      if (slope && K >= 1) {
        double nbv[2 * D];
#pragma unroll
        for (int f = 0; f < 2 * D; ++f) {
          double m = c[0];
          if (sk[f] == 1) {
            m = 0.0;
#pragma unroll
            for (int ch = 0; ch < (1 << D); ++ch) {
              long o = snb[f];
#pragma unroll
              for (int b = 0; b < D; ++b) o += ((ch >> b) & 1) * cstr[b];
              m += wfb[(long)(v * N) * g.ncf + o];
            }
            m = m / (double)(1 << D);
          } else if (sk[f] == 2) {
            m = sfine[f] ? wfb[(long)(v * N) * g.ncf + snb[f]] : wcb[(long)(v * N) * g.ncc + snb[f]];
          } else if (sk[f] == 3) {
            m = 0.0;
#pragma unroll
            for (int l = 0; l < N; ++l) m = fma(wcb[(long)(v * N + l) * g.ncc + snb[f]], tab[C::CM + sch[f] * N + l], m);
          }
          nbv[f] = m;
        }
        const double r3 = sqrt(3.0), bound = mtilde * dx;
        const double mn = c[0];
        double mt[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          const double A = r3 * c[1 + a];
          const double m = (fabs(A) <= bound) ? A : minmod3(A, beta * (mn - nbv[2 * a]), beta * (nbv[2 * a + 1] - mn));
          mt[a] = m;
          limited |= (m != A);
        }
        if (limited) {
#pragma unroll
          for (int a = 0; a < D; ++a) c[1 + a] = mt[a] / r3;
        }
      }
#pragma unroll
      for (int l = NL; l < N; ++l) c[l] = limited ? 0.0 : wb[(long)(v * N + l) * ncb + cell];
      const double Rv = basis_excursion<D, N>(c);
      if (v == 0) {
        m0 = c[0];
        r0 = Rv;
      } else if (v == NV - 1) {
        mE = c[0];
        rE = Rv;
      } else {
        const double m = fabs(c[0]) + Rv;
        m2 = fma(m, m, m2);
        keb = fma(c[0], c[0], keb);
      }
      if (act && limited) {  // an unlimited variable is unchanged in memory
#pragma unroll
        for (int l = 1; l < N; ++l) wb[(long)(v * N + l) * ncb + cell] = c[l];
      }
    }
    if (posit) {
      keb *= vrcp(m0);
      const double pb = (g.gamma - 1.0) * (mE - 0.5 * keb);
      const bool bad = !(m0 > eps) || !(pb > eps);
      if (bad && act) atomicOr(flag, FLAG_NEGATIVE);
      // positivity_certain_mr on the accumulated quantities
      bool certain = false;
      const double rlo = m0 - r0;
      if (rlo > eps + 1e-10 * (fabs(m0) + r0)) {
        const double ke = 0.5 * m2 / rlo;
        const double plo = (g.gamma - 1.0) * ((mE - rE) - ke);
        const double scale = (g.gamma - 1.0) * (fabs(mE) + rE + ke);
        certain = plo > eps + 1e-10 * scale;
      }
      wave_append(act && !bad && !certain, (int)tid, plist);
    }
    return;
  }
  // characteristic: means and slopes first; the higher modes after the slope
  // pass (as in k_limit)
  double wc[NV][N];
  bool dropped[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    dropped[v] = false;
#pragma unroll
    for (int l = 0; l < NL; ++l) wc[v][l] = wb[(long)(v * N + l) * ncb + cell];
  }
  // neighbour means [2D][NV]
  double nbm[2 * D][NV];
#pragma unroll
  for (int a = 0; a < D; ++a)
#pragma unroll
    for (int s = 0; s < 2; ++s) {
      if (!fine) {
        int j[3];
        if (!amr_coarse_nb<D>(g, i, a, s ? 1 : -1, j)) {
#pragma unroll
          for (int v = 0; v < NV; ++v) nbm[2 * a + s][v] = wc[v][0];
        } else if (amr_in_hole<D>(g, j)) {
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            double m = 0.0;
            for (int ch = 0; ch < (1 << D); ++ch) {
              int fi[3] = {0, 0, 0};
#pragma unroll
              for (int b = 0; b < D; ++b) fi[b] = 2 * (j[b] - g.lo[b]) + ((ch >> b) & 1);
              m += wfb[(long)(v * N) * g.ncf + ((long)fi[2] * g.nf[1] + fi[1]) * g.nf[0] + fi[0]];
            }
            nbm[2 * a + s][v] = m / (double)(1 << D);
          }
        } else {
          const long nb = ((long)j[2] * g.n[1] + j[1]) * g.n[0] + j[0];
#pragma unroll
          for (int v = 0; v < NV; ++v) nbm[2 * a + s][v] = wcb[(long)(v * N) * g.ncc + nb];
        }
      } else {
        int f2[3] = {i[0], i[1], i[2]};
        f2[a] += s ? 1 : -1;
        if (f2[a] >= 0 && f2[a] < g.nf[a]) {
          const long nb = ((long)f2[2] * g.nf[1] + f2[1]) * g.nf[0] + f2[0];
#pragma unroll
          for (int v = 0; v < NV; ++v) nbm[2 * a + s][v] = wfb[(long)(v * N) * g.ncf + nb];
        } else {
          int base[3] = {0, 0, 0}, j[3];
#pragma unroll
          for (int b = 0; b < D; ++b) base[b] = g.lo[b] + i[b] / 2;
          amr_coarse_nb<D>(g, base, a, s ? 1 : -1, j);
          const long nb = ((long)j[2] * g.n[1] + j[1]) * g.n[0] + j[0];
          int ch = 0;
#pragma unroll
          for (int b = 0; b < D; ++b) ch |= ((b == a) ? (s ? 0 : 1) : (i[b] & 1)) << b;
#pragma unroll
          for (int v = 0; v < NV; ++v) {
            double m = 0.0;
#pragma unroll
            for (int l = 0; l < N; ++l) m = fma(wcb[(long)(v * N + l) * g.ncc + nb], tab[C::CM + ch * N + l], m);
            nbm[2 * a + s][v] = m;
          }
        }
      }
    }
  if (slope && K >= 1) {
    const double r3 = sqrt(3.0), bound = mtilde * dx;
    if constexpr (CHAR) {
      auto nbmean = [&](int a, int s, double *m) {
#pragma unroll
        for (int v = 0; v < NV; ++v) m[v] = nbm[2 * a + s][v];
      };
      const bool lim = char_limit_cell<D, N>(wc, nbmean, g.gamma, beta, bound);
#pragma unroll
      for (int v = 0; v < NV; ++v) dropped[v] = lim;
    } else
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const double mean = wc[v][0];
      double mt[D];
      bool limited = false;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        const double A = r3 * wc[v][1 + a];
        const double m = (fabs(A) <= bound) ? A
                                            : minmod3(A, beta * (mean - nbm[2 * a][v]), beta * (nbm[2 * a + 1][v] - mean));
        mt[a] = m;
        limited |= (m != A);
      }
      if (limited) {
#pragma unroll
        for (int a = 0; a < D; ++a) wc[v][1 + a] = mt[a] / r3;
      }
      dropped[v] = limited;
    }
  }
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int l = NL; l < N; ++l) wc[v][l] = dropped[v] ? 0.0 : wb[(long)(v * N + l) * ncb + cell];
  if (posit) {
    double Ub[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) Ub[v] = wc[v][0];
    double keb = 0.0;
#pragma unroll
    for (int b = 0; b < D; ++b) keb = fma(Ub[1 + b], Ub[1 + b], keb);
    keb *= vrcp(Ub[0]);
    const double pb = (g.gamma - 1.0) * (Ub[D + 1] - 0.5 * keb);
    const bool bad = !(Ub[0] > eps) || !(pb > eps);
    if (bad && act) atomicOr(flag, FLAG_NEGATIVE);
    // a cell whose bounds leave positivity open goes to k_positivity's list
    // (ids over both blocks: the coarse cells, then the fine cells)
    wave_append(act && !bad && !positivity_certain<D, N>(wc, g.gamma, eps), (int)tid, plist);
  }
  if (act) {  // the variables the slope pass changed (as in k_limit)
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (dropped[v])
#pragma unroll
        for (int l = 1; l < N; ++l) wb[(long)(v * N + l) * ncb + cell] = wc[v][l];
  }
}

__global__ void k_zero_count(int *p) { p[0] = 0; }

// The point loop of the positivity pass (Sec. 3.4) for every cell that
// k_limit or k_limit_amr listed (those whose bounds left positivity open),
// after those kernels have stored the cells' slope-limited coefficients: a
// wave takes one listed cell at a time and its 64 lanes share the cell's
// points (positivity_cell), so a troubled cell no longer holds its whole
// work-group while one lane walks ~150 points alone.  AMR: ids over both
// blocks (the coarse cells, then the fine cells); a coarse cell facing the
// fine block also checks the points of its hanging faces (table HG), all
// inside the reference cell.
template <int D, int K, bool AMR>
__global__ __launch_bounds__(256) void k_positivity(const double *__restrict__ tab, double *__restrict__ w, Grid g,
                                                    AmrGrid ag, const int *__restrict__ plist, double eps) {
  using C = Cfg<D, K>;
  constexpr int N = C::N, NW = C::NV * N, NSUB = 1 << (D - 1);
  const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
  const int cnt = plist[0];
  for (long t = wave; t < cnt; t += nwaves) {
    const long id = plist[1 + t];
    if constexpr (!AMR) {
      struct {
        const double *ps;
        __device__ int count(int) const { return C::NS; }
        __device__ const double *row(int, int i) const { return ps + i * N; }
      } pts{tab + C::PS};
      positivity_cell<D, N>(w + id, g.ncell, 0, pts, g.gamma, eps);
    } else {
      const bool fine = id >= ag.ncc;
      const long cell = fine ? id - ag.ncc : id;
      int hm = 0;  // bit 2a + s: side (a, s) is a hanging face
      if (!fine) {
        int i[3] = {(int)(cell % ag.n[0]), (int)((cell / ag.n[0]) % ag.n[1]),
                    (int)(cell / ((long)ag.n[0] * ag.n[1]))};
#pragma unroll
        for (int a = 0; a < D; ++a)
#pragma unroll
          for (int s = 0; s < 2; ++s) {
            int j[3];
            if (amr_coarse_nb<D>(ag, i, a, s ? 1 : -1, j) && amr_in_hole<D>(ag, j)) hm |= 1 << (2 * a + s);
          }
      }
      // point i >= NS: side = the (i - NS) / (NSUB QF)-th set bit of hm,
      // sub-face point (i - NS) mod (NSUB QF), rows of table HG
      struct {
        const double *t;
        __device__ int count(int h) const { return C::NS + __popc(h) * NSUB * C::QF; }
        __device__ const double *row(int h, int i) const {
          if (i < C::NS) return t + C::PS + i * N;
          const int e = i - C::NS, k = e / (NSUB * C::QF), rem = e % (NSUB * C::QF);
          int f = 0, seen = 0;
#pragma unroll
          for (int b = 0; b < 2 * D; ++b)
            if ((h >> b) & 1) {
              if (seen == k) f = b;
              ++seen;
            }
          return t + C::HG + (f * 4 + rem / C::QF) * C::QF * N + (rem % C::QF) * N;
        }
      } pts{tab};
      positivity_cell<D, N>(fine ? w + (long)NW * ag.ncc + cell : w + cell, fine ? ag.ncf : ag.ncc, hm, pts,
                            ag.gamma, eps);
    }
  }
}

}  // namespace dg

// ===========================================================================
// Quadtree meshes in 2D (Sec. 4): leaves of any level, the level jump across
// a face and a corner at most one.  One thread per leaf, FP64.  The leaf
// tables (built on the host by dg_tree_set) give per leaf its level and per
// side (a, s) the face kind: 0 one neighbour of the same level, 1 a
// transmissive wall, 2 two finer neighbours (this leaf is the coarse side:
// its trace at the mapped points (eta + sigma)/2 of each half, lifted with
// w_r / 2), 3 one coarser neighbour (whose trace is taken at this leaf's
// half of its face, `sub`).  Both leaves of a face form the traces from the
// same weights and tables in the same order, so they obtain the same flux.
// ===========================================================================
namespace dg {

struct TreeGrid {
  long nleaf;
  const int *lev;   // [nleaf]
  const int *info;  // [4][nleaf]: kind | sub << 2 | ch << 3, side 2a + s (ch: kind 3's child for the limiters)
  const int *nb;    // [8][nleaf]: neighbour (2 side + half)
  const int *grp;   // [4][nleaf]: the four leaves of this leaf's sibling group (child order), or -1
  double fac0;      // (2/dx) 2^-d of level 0
  double dx0;
  double gamma;
  const double *t1; // 1D tables (tables_1d)
};

// Right-hand side and fused stage on the quadtree, one thread per leaf.
// Volume integral as on uniform grids; each side is one face (same level,
// wall), two half faces (finer neighbours: this leaf's trace at the mapped
// nodes (eta + sigma)/2, lifted with w_r / 2) or one face against a coarser
// neighbour (its trace at this leaf's half).  The contractions are
// sum-factorised along one axis.  The total-degree basis is not a tensor product, but each of its
// modes is P~_ex(xi) P~_ey(eta): a trace on a face normal to x is
// sum_ey P~_ey(eta) [sum over the modes of that ey of w_l P~_ex(+-1)], the
// lift the transpose of that, and the volume integral goes one column of
// x-nodes at a time, contracting over ex first (tables_1d).  Both leaves of a
// face form a trace with the same function (tree_trace), weights and tables,
// so they obtain the same flux bit for bit.
// f(std::integral_constant<int, I>) for I = B .. E-1: the mode index is a
// compile-time constant, so register arrays indexed by a mode's exponents
// stay in registers
template <int B, int E, class F>
__device__ inline void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <int K>
struct Tree1D {
  static constexpr int n1 = K + 1, PG = 0, DG = n1 * n1, GW = 2 * n1 * n1, PB = GW + n1, PH = PB + 2 * n1;
};

// values of the four variables of weights ws at the n1 nodes of a face
// normal to axis a at xi_a = -1 (s = 0) or +1 (s = 1), the tangential node
// coordinates' Legendre values in rows of tt ([n1][n1]); out[r][v]
template <int K, int A>
__device__ inline void tree_trace(const double (&ws)[4][Cfg<2, K>::N], const double *t1, int s, const double *tt,
                                  double (&out)[K + 1][4]) {
  using T = Tree1D<K>;
  constexpr int N = Cfg<2, K>::N, n1 = K + 1;
  const double *pb = t1 + T::PB + s * n1;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    double c[n1];
#pragma unroll
    for (int e = 0; e < n1; ++e) c[e] = 0.0;
    static_for<0, N>([&](auto L_) {
      // normal and tangential exponents of mode l on a face normal to axis A
      constexpr int l = decltype(L_)::value, nrm = mode_exp<2>(l, A), tan = mode_exp<2>(l, 1 - A);
      c[tan] = fma(ws[v][l], pb[nrm], c[tan]);
    });
#pragma unroll
    for (int r = 0; r < n1; ++r) {
      double u = 0.0;
#pragma unroll
      for (int e = 0; e < n1; ++e) u = fma(c[e], tt[r * n1 + e], u);
      out[r][v] = u;
    }
  }
}

template <int K, int FX>
__global__ __launch_bounds__(256) void k_rhs_tree(const double *__restrict__ tab, const double *__restrict__ w,
                                                     double *__restrict__ out, const double *__restrict__ dtp,
                                                     TreeGrid g, int mode, Mix mx, int *__restrict__ flag) {
  using C = Cfg<2, K>;
  using T = Tree1D<K>;
  constexpr int NV = C::NV, N = C::N, n1 = K + 1;
  const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.nleaf) return;
  const long nl = g.nleaf;
  const double gm1 = g.gamma - 1.0;
  const double *t1 = g.t1;
  double wc[NV][N], acc[NV][N];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int l = 0; l < N; ++l) {
      wc[v][l] = w[(long)(v * N + l) * nl + cell];
      acc[v][l] = 0.0;
    }
  // volume integral (eq. dg_term2), one column of x-nodes (index i) at a time
#pragma unroll 1
  for (int i = 0; i < n1; ++i) {
    const double *pgi = t1 + T::PG + i * n1;
    const double *dgi = t1 + T::DG + i * n1;
    const double wi = t1[T::GW + i];
    // t[v][ey] = sum over the modes of exponent ey of w_l P~_ex(g_i)
    double tc[NV][n1], rx[NV][n1], ry[NV][n1];
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int e = 0; e < n1; ++e) {
        tc[v][e] = 0.0;
        rx[v][e] = 0.0;
        ry[v][e] = 0.0;
      }
#pragma unroll
    for (int v = 0; v < NV; ++v)
      static_for<0, N>([&](auto L_) {
        constexpr int l = decltype(L_)::value, ex = mode_exp<2>(l, 0), ey = mode_exp<2>(l, 1);
        tc[v][ey] = fma(wc[v][l], pgi[ex], tc[v][ey]);
      });
#pragma unroll 1
    for (int j = 0; j < n1; ++j) {
      const double *pgj = t1 + T::PG + j * n1;
      const double *dgj = t1 + T::DG + j * n1;
      const double wj = t1[T::GW + j];
      double U[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double u = 0.0;
#pragma unroll
        for (int e = 0; e < n1; ++e) u = fma(tc[v][e], pgj[e], u);
        U[v] = u;
      }
      double Fx[NV], Fy[NV];
      euler_flux<2, double>(U, 0, gm1, Fx);
      euler_flux<2, double>(U, 1, gm1, Fy);
      // rx[v][ey] += F_x P~_ey(g_j) w_j,  ry[v][ey] += F_y P~_ey'(g_j) w_j
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < n1; ++e) {
          rx[v][e] = fma(Fx[v] * wj, pgj[e], rx[v][e]);
          ry[v][e] = fma(Fy[v] * wj, dgj[e], ry[v][e]);
        }
    }
    // V_l += w_i (P~_ex'(g_i) rx[ey] + P~_ex(g_i) ry[ey])
#pragma unroll
    for (int v = 0; v < NV; ++v)
      static_for<1, N>([&](auto L_) {
        constexpr int l = decltype(L_)::value, ex = mode_exp<2>(l, 0), ey = mode_exp<2>(l, 1);
        acc[v][l] = fma(wi, fma(dgi[ex], rx[v][ey], pgi[ex] * ry[v][ey]), acc[v][l]);
      });
  }
  // face integrals (eq. dg_term3) over the sides' halves
#pragma unroll 1
  for (int side = 0; side < 4; ++side) {
    const int a = side >> 1, s = side & 1;
    const int inf = g.info[(long)side * nl + cell];
    const int kind = inf & 3, sub = (inf >> 2) & 1;
    const int nsub = (kind == 2) ? 2 : 1;
#pragma unroll 1
    for (int sb = 0; sb < nsub; ++sb) {
      const long nbc = (kind == 1) ? cell : (long)g.nb[(long)(2 * side + sb) * nl + cell];
      const int hs = (kind == 2) ? sb : sub;
      const double *tto = (kind == 2) ? t1 + T::PH + hs * n1 * n1 : t1 + T::PG;
      const double *ttn = (kind == 3) ? t1 + T::PH + hs * n1 * n1 : t1 + T::PG;
      double Uo[n1][NV], Un[n1][NV];
      if (a == 0)
        tree_trace<K, 0>(wc, t1, s, tto, Uo);
      else
        tree_trace<K, 1>(wc, t1, s, tto, Uo);
      {
        double wn[NV][N];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int l = 0; l < N; ++l) wn[v][l] = w[(long)(v * N + l) * nl + nbc];
        if (a == 0)
          tree_trace<K, 0>(wn, t1, 1 - s, ttn, Un);
        else
          tree_trace<K, 1>(wn, t1, 1 - s, ttn, Un);
      }
      const double half = (kind == 2) ? 0.5 : 1.0;
      double m[NV][n1];
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < n1; ++e) m[v][e] = 0.0;
#pragma unroll
      for (int r = 0; r < n1; ++r) {
        double UL[NV], UR[NV], F[NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double un = (kind == 1) ? Uo[r][v] : Un[r][v];
          UL[v] = s ? Uo[r][v] : un;
          UR[v] = s ? un : Uo[r][v];
        }
        hllc<double, 2, FX>(UL, UR, a, g.gamma, F);
        const double wr = half * t1[T::GW + r];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const double f = (s ? -F[v] : F[v]) * wr;
#pragma unroll
          for (int e = 0; e < n1; ++e) m[v][e] = fma(f, tto[r * n1 + e], m[v][e]);
        }
      }
      // lift: acc_l += P~_(normal exponent)(+-1) m[tangential exponent]
      const double *pb = t1 + T::PB + s * n1;
      if (a == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
          static_for<0, N>([&](auto L_) {
            constexpr int l = decltype(L_)::value, en = mode_exp<2>(l, 0), et = mode_exp<2>(l, 1);
            acc[v][l] = fma(pb[en], m[v][et], acc[v][l]);
          });
      } else {
#pragma unroll
        for (int v = 0; v < NV; ++v)
          static_for<0, N>([&](auto L_) {
            constexpr int l = decltype(L_)::value, en = mode_exp<2>(l, 0), et = mode_exp<2>(l, 1);
            acc[v][l] = fma(pb[et], m[v][en], acc[v][l]);
          });
      }
    }
  }
  const double fac = g.fac0 * (double)(1 << g.lev[cell]);
  const double cldt = (mode == 0) ? 0.0 : mx.cl * *dtp;
  bool bad = false;
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int l = 0; l < N; ++l) {
      const long ii = (long)(v * N + l) * nl + cell;
      const double L = fac * acc[v][l];
      bad |= (L != L);
      out[ii] = (mode == 0) ? L : mix_out(mx, w[ii], L, cldt, ii);
    }
  if (bad) atomicOr(flag, FLAG_NAN);
}

// largest signal rate of the leaves' means with each leaf's own edge
__global__ __launch_bounds__(256) void k_rate_tree(const double *__restrict__ w, TreeGrid g, int N,
                                                   unsigned long long *ratemax, int *__restrict__ flag) {
  double m = 0.0;
  bool bad = false;
  for (long cell = (long)blockIdx.x * blockDim.x + threadIdx.x; cell < g.nleaf; cell += (long)gridDim.x * blockDim.x) {
    double U[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) U[v] = w[(long)v * N * g.nleaf + cell];
    m = fmax(m, cell_rate<2>(U, g.gamma, g.dx0 / (double)(1 << g.lev[cell]), bad));
  }
  if (bad) atomicOr(flag, FLAG_NEGATIVE);
  m = block_max(m);
  if (threadIdx.x == 0) atomicMax(rate_slot(ratemax, blockIdx.x), (unsigned long long)__double_as_longlong(m));
}

// Refinement criterion per leaf (Sec. 4.1): bit 0 if max_a |w_rho,1+a| >
// thr_cell (eq. cell_ref); bit 1 if the node weights of the leaf's sibling
// group, 2^-d sum_c P_c^T w^c (eq. deref_weights), satisfy max_a > thr_node
// (eq. node_ref); bit 2 if the four siblings are all leaves.
template <int K>
__global__ __launch_bounds__(256) void k_tree_flags(const double *__restrict__ w, const double *__restrict__ P,
                                                    TreeGrid g, double thr_cell, double thr_node,
                                                    int *__restrict__ flags) {
  constexpr int N = Cfg<2, K>::N;
  const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (cell >= g.nleaf) return;
  const long nl = g.nleaf;
  double m = 0.0;
#pragma unroll
  for (int a = 0; a < 2; ++a) m = fmax(m, fabs(w[(long)(1 + a) * nl + cell]));
  int f = m > thr_cell ? 1 : 0;
  if (g.grp[cell] >= 0) {
    f |= 4;
    double mn = 0.0;
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      double node = 0.0;
      for (int ch = 0; ch < 4; ++ch) {
        const long s = g.grp[(long)ch * nl + cell];
        for (int l = 0; l < N; ++l) node = fma(P[((long)ch * N + l) * N + 1 + a], w[(long)l * nl + s], node);
      }
      mn = fmax(mn, fabs(node / 4.0));
    }
    if (mn > thr_node) f |= 2;
  }
  flags[cell] = f;
}

// New state after an adaptation (Sec. 4.2, 4.3): per new leaf rk = kind |
// child << 2 with kind 0 a copy of old leaf src[0], 1 child `child` of old
// leaf src[0] (eq. ref_weights, w^c = P_c w), 2 the merge of the old leaves
// src[0..3] in child order (eq. deref_weights, 2^-d sum_c P_c^T w^c).
template <int K>
__global__ __launch_bounds__(256) void k_tree_regrid(const double *__restrict__ wa, long na,
                                                     const double *__restrict__ P, const int *__restrict__ rk,
                                                     const int *__restrict__ src, double *__restrict__ wb, long nb) {
  constexpr int NV = 4, N = Cfg<2, K>::N;
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nb) return;
  const int kind = rk[i] & 3, ch = rk[i] >> 2;
  const long s0 = src[i];
  if (kind == 0) {
    for (int vl = 0; vl < NV * N; ++vl) wb[(long)vl * nb + i] = wa[(long)vl * na + s0];
  } else if (kind == 1) {
    for (int v = 0; v < NV; ++v)
      for (int j = 0; j < N; ++j) {
        double acc = 0.0;
        for (int l = 0; l < N; ++l) acc = fma(P[((long)ch * N + j) * N + l], wa[(long)(v * N + l) * na + s0], acc);
        wb[(long)(v * N + j) * nb + i] = acc;
      }
  } else {
    long sc[4];
#pragma unroll
    for (int c = 0; c < 4; ++c) sc[c] = src[(long)c * nb + i];
    for (int v = 0; v < NV; ++v)
      for (int j = 0; j < N; ++j) {
        double acc = 0.0;
#pragma unroll
        for (int c = 0; c < 4; ++c)
          for (int l = 0; l < N; ++l) acc = fma(P[((long)c * N + l) * N + j], wa[(long)(v * N + l) * na + sc[c]], acc);
        wb[(long)(v * N + j) * nb + i] = acc / 4.0;
      }
  }
}

}  // namespace dg

namespace dg {

// Neighbour values of the limiters on a quadtree (Sec. 4.4), from the state
// before limiting, per side (a, s) of each leaf: the mean over the cell of
// the leaf's own size there, i.e. the same-level leaf's mean, the coarser
// leaf's polynomial averaged over that cell (table CM, child `ch`), the
// area-weighted means of the finer leaves inside it (list `reg`), or at a
// transmissive wall the leaf's own mean.  nbm[(side NV + v) nleaf + leaf].
// plist (may be null): the positivity list, whose count this pass clears for
// the slope pass after it (kernel boundaries order the two).
template <int K>
__global__ __launch_bounds__(256) void k_tree_nbmean(const double *__restrict__ tab, const double *__restrict__ w,
                                                     TreeGrid g, const int *__restrict__ reg,
                                                     double *__restrict__ nbm, int *__restrict__ plist) {
  using C = Cfg<2, K>;
  constexpr int NV = C::NV, N = C::N;
  const long cell = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (plist && cell == 0) plist[0] = 0;
  if (cell >= g.nleaf) return;
  const long nl = g.nleaf;
  const int *roff = reg, *rcnt = reg + 4 * nl, *rlist = reg + 8 * nl;
  for (int side = 0; side < 4; ++side) {
    const int inf = g.info[(long)side * nl + cell];
    const int kind = inf & 3, ch = (inf >> 3) & 3;
    double m[NV];
    if (kind == 0 || kind == 1) {
      const long j = kind == 1 ? cell : (long)g.nb[(long)(2 * side) * nl + cell];
#pragma unroll
      for (int v = 0; v < NV; ++v) m[v] = w[(long)(v * N) * nl + j];
    } else if (kind == 3) {
      const long j = g.nb[(long)(2 * side) * nl + cell];
      const double *cm = tab + C::CM + ch * N;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        double s = 0.0;
#pragma unroll
        for (int l = 0; l < N; ++l) s = fma(w[(long)(v * N + l) * nl + j], cm[l], s);
        m[v] = s;
      }
    } else {
      const int o = roff[(long)side * nl + cell], n = rcnt[(long)side * nl + cell];
      const int l0 = g.lev[cell];
#pragma unroll
      for (int v = 0; v < NV; ++v) m[v] = 0.0;
      for (int e = 0; e < n; ++e) {
        const long j = rlist[o + e];
        const double frac = 1.0 / (double)(1L << (2 * (g.lev[j] - l0)));
#pragma unroll
        for (int v = 0; v < NV; ++v) m[v] = fma(w[(long)(v * N) * nl + j], frac, m[v]);
      }
    }
#pragma unroll
    for (int v = 0; v < NV; ++v) nbm[(long)(side * NV + v) * nl + cell] = m[v];
  }
}

// Slope limiter on a quadtree (component-wise, eq. comp_limiter, or on the
// characteristic variables, eq. char_limiter) against the neighbour values
// of k_tree_nbmean, with the TVB bound of the leaf's own edge (Sec. 3.3).
// With plist set it also does k_tree_poscheck's work on the limited leaf.
template <int K, bool CHAR>
__global__ __launch_bounds__(256) void k_limit_tree(double *__restrict__ w, TreeGrid g, const double *__restrict__ nbm,
                                                    double beta, double mtilde, double eps, int *__restrict__ flag,
                                                    int *__restrict__ plist) {
  using C = Cfg<2, K>;
  constexpr int NV = C::NV, N = C::N;
  // lanes past the mesh stay in the wave (the list is appended per wave) on a
  // copy of the last leaf, and store nothing
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = tid < g.nleaf;
  const long cell = act ? tid : g.nleaf - 1;
  const long nl = g.nleaf;
  const double bound = mtilde * (g.dx0 / (double)(1 << g.lev[cell]));
  double wc[NV][N];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int l = 0; l < N; ++l) wc[v][l] = w[(long)(v * N + l) * nl + cell];
  bool dropped[NV];
  if constexpr (CHAR) {
    auto nbmean = [&](int a, int s, double *m) {
#pragma unroll
      for (int v = 0; v < NV; ++v) m[v] = nbm[(long)((2 * a + s) * NV + v) * nl + cell];
    };
    const bool lim = char_limit_cell<2, N>(wc, nbmean, g.gamma, beta, bound);
#pragma unroll
    for (int v = 0; v < NV; ++v) dropped[v] = lim;
  } else {
    const double r3 = sqrt(3.0);
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      const double mean = wc[i][0];
      double mt[2];
      bool limited = false;
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const double mlo = nbm[(long)((2 * a) * NV + i) * nl + cell];
        const double mhi = nbm[(long)((2 * a + 1) * NV + i) * nl + cell];
        const double A = r3 * wc[i][1 + a];
        const double m = (fabs(A) <= bound) ? A : minmod3(A, beta * (mean - mlo), beta * (mhi - mean));
        mt[a] = m;
        limited |= (m != A);
      }
      if (limited) {
#pragma unroll
        for (int a = 0; a < 2; ++a) wc[i][1 + a] = mt[a] / r3;
#pragma unroll
        for (int l = 3; l < N; ++l) wc[i][l] = 0.0;
      }
      dropped[i] = limited;
    }
  }
  if (act)
#pragma unroll
    for (int v = 0; v < NV; ++v)
      if (dropped[v])
#pragma unroll
        for (int l = 1; l < N; ++l) w[(long)(v * N + l) * nl + cell] = wc[v][l];
  if (plist) {
    const double ke = (wc[1][0] * wc[1][0] + wc[2][0] * wc[2][0]) / wc[0][0];
    const double pb = (g.gamma - 1.0) * (wc[3][0] - 0.5 * ke);
    const bool bad = !(wc[0][0] > eps) || !(pb > eps);
    if (bad && act) atomicOr(flag, FLAG_NEGATIVE);
    wave_append(act && !bad && !positivity_certain<2, N>(wc, g.gamma, eps), (int)cell, plist);
  }
}

// Positivity limiter (Sec. 3.4) on a quadtree, in two passes as on uniform
// grids.  k_tree_poscheck, one thread per leaf: a mean without positive
// density and pressure (<= eps) sets the flag and is left alone; a leaf whose
// polynomial provably stays above eps everywhere in the cell (basis bounds,
// positivity_certain: theta_1 = theta_2 = 1 exactly) needs nothing; the
// others go to the list plist.  k_positivity_tree, one wave per listed leaf:
// the points S and, on each side with finer neighbours, the leaf's trace
// points on the two half faces (table HG; Sec. 4.4).
template <int K>
__global__ __launch_bounds__(256) void k_tree_poscheck(const double *__restrict__ w, TreeGrid g, double eps,
                                                       int *__restrict__ flag, int *__restrict__ plist) {
  using C = Cfg<2, K>;
  constexpr int NV = C::NV, N = C::N;
  // lanes past the mesh stay in the wave (the list is appended per wave) on a
  // copy of the last leaf, and append nothing
  const long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool act = tid < g.nleaf;
  const long cell = act ? tid : g.nleaf - 1;
  const long nl = g.nleaf;
  double wc[NV][N];
#pragma unroll
  for (int v = 0; v < NV; ++v)
#pragma unroll
    for (int l = 0; l < N; ++l) wc[v][l] = w[(long)(v * N + l) * nl + cell];
  const double ke = (wc[1][0] * wc[1][0] + wc[2][0] * wc[2][0]) / wc[0][0];
  const double pb = (g.gamma - 1.0) * (wc[3][0] - 0.5 * ke);
  const bool bad = !(wc[0][0] > eps) || !(pb > eps);
  if (bad && act) atomicOr(flag, FLAG_NEGATIVE);
  wave_append(act && !bad && !positivity_certain<2, N>(wc, g.gamma, eps), (int)cell, plist);
}

template <int K>
__global__ __launch_bounds__(256) void k_positivity_tree(const double *__restrict__ tab, double *__restrict__ w,
                                                         TreeGrid g, const int *__restrict__ plist, double eps) {
  using C = Cfg<2, K>;
  constexpr int N = C::N;
  const long wave = ((long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const long nwaves = ((long)gridDim.x * blockDim.x) >> 6;
  const long nl = g.nleaf;
  const int cnt = plist[0];
  for (long t = wave; t < cnt; t += nwaves) {
    const long cell = plist[1 + t];
    int hm = 0;
#pragma unroll
    for (int side = 0; side < 4; ++side)
      if ((g.info[(long)side * nl + cell] & 3) == 2) hm |= 1 << side;
    struct {
      const double *t;
      __device__ int count(int h) const { return C::NS + __popc(h) * 2 * C::QF; }
      __device__ const double *row(int h, int i) const {
        if (i < C::NS) return t + C::PS + i * N;
        const int e = i - C::NS, k = e / (2 * C::QF), rem = e % (2 * C::QF);
        int f = 0, seen = 0;
#pragma unroll
        for (int b = 0; b < 4; ++b)
          if ((h >> b) & 1) {
            if (seen == k) f = b;
            ++seen;
          }
        return t + C::HG + (f * 4 + rem / C::QF) * C::QF * N + (rem % C::QF) * N;
      }
    } pts{tab};
    positivity_cell<2, N>(w + cell, nl, hm, pts, g.gamma, eps);
  }
}

}  // namespace dg

// ===========================================================================
// C ABI
// ===========================================================================

using dg::Cfg;

// Scratch of dg_rhs_noalloc: the FP32 volume term of the BF16 path in a
// file-scope device array instead of the context's allocation.  Each GPU
// holds its own copy; host code reaches it only through the address that
// hipGetSymbolAddress returns for the current device (the array's name in
// host code is not a device address).
__device__ __align__(256) float scratch[DG_STATIC_SCRATCH_FLOATS];

namespace {

constexpr int kBlock = 256;

thread_local char g_hip_msg[256];

// per-device address of `scratch`, looked up once per device (in dg_init,
// with that device current)
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float *g_scratch_ptr[kMaxDevices] = {};

int hip_fail(hipError_t e) {
  std::snprintf(g_hip_msg, sizeof(g_hip_msg), "%s", hipGetErrorString(e));
  return DG_EHIP;
}

#define HIP_TRY(expr)                     \
  do {                                    \
    hipError_t e_ = (expr);               \
    if (e_ != hipSuccess) return hip_fail(e_); \
  } while (0)

dg::Grid make_grid(const dg_ctx *c) {
  dg::Grid g;
  g.nx = (int)c->nx;
  g.ny = (int)c->ny;
  g.nz = (int)c->nz;
  g.ncell = c->ncell;
  for (int a = 0; a < 3; ++a) g.bc[a] = c->cfg.bc[a];
  g.fac = 2.0 / c->dx / (double)(1 << c->sh.d);
  g.gamma = c->cfg.gamma;
  g.xg = g.xzc = g.xp = 0;
  const long plane = c->nx * c->ny;
  if (c->sh.d == 3 && plane % 64 == 0 && c->nz % 8 == 0) {
    const long xg = c->nx % 64 == 0 ? c->nx / 64 : 1;
    if ((plane / 64) % xg == 0) {
      g.xg = (int)xg;
      g.xzc = (int)(c->nz / 8);
      g.xp = (int)(plane / 64);
    }
  }
  return g;
}

unsigned nblocks(long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// every axis of the context's grid periodic (no wall faces)
bool periodic(const dg_ctx *c) {
  for (int a = 0; a < c->sh.d; ++a)
    if (c->cfg.bc[a] != DG_BC_PERIODIC) return false;
  return true;
}

dg::AmrGrid make_amr_grid(const dg_ctx *c) {
  dg::AmrGrid g;
  g.n[0] = (int)c->nx;
  g.n[1] = (int)c->ny;
  g.n[2] = (int)c->nz;
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = c->lo[a];
    g.hi[a] = c->hi[a];
    g.nf[a] = (int)c->nf[a];
    g.bc[a] = c->cfg.bc[a];
  }
  g.ncc = c->ncc;
  g.ncf = c->ncf;
  g.dxc = c->dx;
  g.dxf = 0.5 * c->dx;
  g.facc = 2.0 / g.dxc / (double)(1 << c->sh.d);
  g.facf = 2.0 / g.dxf / (double)(1 << c->sh.d);
  g.gamma = c->cfg.gamma;
  return g;
}

// The uniform grid as a refined box with no fine block and an empty hole.
dg::AmrGrid make_uniform_amr_grid(const dg_ctx *c) {
  dg::AmrGrid g = make_amr_grid(c);
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = 0;
    g.hi[a] = 0;
    g.nf[a] = 1;
  }
  g.ncc = c->ncell;
  g.ncf = 0;
  return g;
}

// Calls F::template run<D, K>() for the context's (dim, k).
template <class F>
int dispatch(const dg_ctx *c, F &&f) {
  const int d = c->sh.d, k = c->sh.k;
  if (d == 2 && k == 1) return f.template run<2, 1>();
  if (d == 2 && k == 2) return f.template run<2, 2>();
  if (d == 2 && k == 3) return f.template run<2, 3>();
  if (d == 2 && k == 4) return f.template run<2, 4>();  // uniform grids, FP64/FP32 (dg_init checks)
  if (d == 3 && k == 1) return f.template run<3, 1>();
  if (d == 3 && k == 2) return f.template run<3, 2>();
  if (d == 3 && k == 3) return f.template run<3, 3>();
  return DG_EUNSUPPORTED;
}

struct LayoutCheck {
  const dg_ctx *c;
  template <int D, int K>
  int run() {
    using C = Cfg<D, K>;
    const dg::Layout &l = c->lay;
    bool ok = l.B == C::B && l.DW == C::DW && l.TF == C::TF && l.TW == C::TW && l.WQ == C::WQ &&
              l.PS == C::PS && l.XQ == C::XQ && l.HG == C::HG && l.HW == C::HW && l.CM == C::CM && l.total == C::TOTAL &&
              c->sh.N == C::N && c->sh.NS == C::NS;
    return ok ? DG_OK : DG_EINVAL;
  }
};

int check_layout(const dg_ctx *c) { return dispatch(c, LayoutCheck{c}); }

struct StageLaunch {
  dg_ctx *c;
  const double *w, *dt;
  double *out;
  int mode;  // 0: out = L(w); 1: out = the combination mx
  dg::Mix mx;
  hipStream_t s;
  dg::RateOp ro = {nullptr, nullptr, 0.0, 0.0, dg::RATE_NONE};  // only the 2D tile kernel takes one
  float *vs = nullptr;  // volume-term scratch of the BF16 path (null: the context's)
  template <int D, int K, class R>
  int launch(const R *tabr, const float *vext) {
    return c->cfg.flux == DG_HLLC_DAVIS ? launch_fx<D, K, R, DG_HLLC_DAVIS>(tabr, vext)
                                        : launch_fx<D, K, R, DG_HLLC_BATTEN>(tabr, vext);
  }
  template <int D, int K, class R, int FX>
  int launch_fx(const R *tabr, const float *vext) {
    if ((c->amr || D != 2) && ro.op != dg::RATE_NONE) return DG_EINVAL;
    if (c->amr) {
      if constexpr (K > 3) {
        return DG_EUNSUPPORTED;
      } else if constexpr (D == 3 && (K == 2 || K == 3) && sizeof(R) == sizeof(float)) {
        if (c->tabmf32 && !vext) {
          // contractions on FP32 MFMA: coarse-block cells, then fine-block cells
          const unsigned nb = (unsigned)((c->ncc + 63) / 64 + (c->ncf + 63) / 64);
          hipLaunchKernelGGL((dg::k_rhs_mfma3d<K, FX, true, float>), dim3(nb), dim3(kBlock), 0, s, c->tabmf32,
                             c->tablw, nullptr, w, out, dt, make_grid(c), make_amr_grid(c), mode, mx, c->flag);
        } else {
          hipLaunchKernelGGL((dg::k_rhs_amr<D, K, R, FX>), dim3(nblocks(c->ncc + c->ncf)), dim3(kBlock), 0, s,
                             c->tab, tabr, w, out, dt, vext, make_amr_grid(c), mode, mx, c->flag);
        }
      } else if constexpr (D == 3 && (K == 2 || K == 3) && sizeof(R) == sizeof(double)) {
        if (c->tabmf && !vext) {
          // contractions on FP64 MFMA: coarse-block cells, then fine-block cells
          const unsigned nb = (unsigned)((c->ncc + 63) / 64 + (c->ncf + 63) / 64);
          hipLaunchKernelGGL((dg::k_rhs_mfma3d<K, FX, true>), dim3(nb), dim3(kBlock), 0, s, c->tabmf, nullptr,
                             nullptr, w, out, dt, make_grid(c), make_amr_grid(c), mode, mx, c->flag);
        } else if constexpr (K == 3) {
          // four lanes per cell (the one-thread kernel would spill)
          hipLaunchKernelGGL((dg::k_rhs_amr_quad<K, FX, false>), dim3(nblocks(4 * (c->ncc + c->ncf))), dim3(kBlock),
                             0, s, c->tab, w, out, dt, make_amr_grid(c), mode, mx, c->flag);
        } else {
          hipLaunchKernelGGL((dg::k_rhs_amr<D, K, R, FX>), dim3(nblocks(c->ncc + c->ncf)), dim3(kBlock), 0, s,
                             c->tab, tabr, w, out, dt, vext, make_amr_grid(c), mode, mx, c->flag);
        }
      } else if constexpr (D == 3 && K == 3 && sizeof(R) == 8) {
        // four lanes per cell (the one-thread kernel would spill)
        hipLaunchKernelGGL((dg::k_rhs_amr_quad<K, FX, false>), dim3(nblocks(4 * (c->ncc + c->ncf))), dim3(kBlock), 0,
                           s, c->tab, w, out, dt, make_amr_grid(c), mode, mx, c->flag);
      } else {
        hipLaunchKernelGGL((dg::k_rhs_amr<D, K, R, FX>), dim3(nblocks(c->ncc + c->ncf)), dim3(kBlock), 0, s, c->tab,
                           tabr, w, out, dt, vext, make_amr_grid(c), mode, mx, c->flag);
      }
    } else if constexpr (D == 2) {
      using T = dg::Tile2D<K>;
      dim3 grid((unsigned)(((c->nx + T::TX - 1) / T::TX) * ((c->ny + T::TY - 1) / T::TY)));
      dg::RateOp r2 = ro;
      if (r2.op == dg::RATE_FOLD && c->gravity) {
        r2.gmax = c->gmax;
        r2.gk = c->grav_k;
      }
      const bool small = dg::tile2d_small(K, (long)grid.x, c->tile_small);
      using T1 = dg::Tile2D<K, 1>;
      const dim3 grid1((unsigned)(((c->nx + T1::TX - 1) / T1::TX) * ((c->ny + T1::TY - 1) / T1::TY)));
      if (c->gravity) {
        if constexpr (sizeof(R) == sizeof(double)) {
          if (small)
            hipLaunchKernelGGL((dg::k_rhs_tile2d<K, R, FX, true, 1>), grid1, dim3(4 * T1::TX * T1::TY), 0, s, c->tab,
                               tabr, w, out, dt, vext, make_grid(c), mode, mx, c->flag, r2, c->grav);
          else
            hipLaunchKernelGGL((dg::k_rhs_tile2d<K, R, FX, true>), grid, dim3(4 * T::TX * T::TY), 0, s, c->tab, tabr,
                               w, out, dt, vext, make_grid(c), mode, mx, c->flag, r2, c->grav);
        } else {
          return DG_EUNSUPPORTED;
        }
      } else if (small) {
        hipLaunchKernelGGL((dg::k_rhs_tile2d<K, R, FX, false, 1>), grid1, dim3(4 * T1::TX * T1::TY), 0, s, c->tab,
                           tabr, w, out, dt, vext, make_grid(c), mode, mx, c->flag, r2, nullptr);
      } else {
        hipLaunchKernelGGL((dg::k_rhs_tile2d<K, R, FX>), grid, dim3(4 * T::TX * T::TY), 0, s, c->tab, tabr, w, out,
                           dt, vext, make_grid(c), mode, mx, c->flag, r2, nullptr);
      }
    } else if (D == 3 && K == 3 && sizeof(R) == sizeof(double) && !c->gravity && !vext && c->tabmf) {
      // contractions on FP64 MFMA, 16 cells per wave
      if (periodic(c))
        hipLaunchKernelGGL((dg::k_rhs_mfma3d<3, FX, false, double, false, true>),
                           dim3((unsigned)((c->ncell + 63) / 64)), dim3(kBlock), 0, s, c->tabmf, nullptr, nullptr, w,
                           out, dt, make_grid(c), dg::AmrGrid{}, mode, mx, c->flag);
      else
        hipLaunchKernelGGL((dg::k_rhs_mfma3d<3, FX, false>), dim3((unsigned)((c->ncell + 63) / 64)), dim3(kBlock), 0,
                           s, c->tabmf, nullptr, nullptr, w, out, dt, make_grid(c), dg::AmrGrid{}, mode, mx, c->flag);
    } else if (D == 3 && K == 3 && sizeof(R) == sizeof(float) && !c->gravity && !vext && c->tabmf32) {
      // contractions on FP32 MFMA, 16 cells per wave, the mean's lift in FP64
      // (at k = 2 the one-thread-per-cell FP32 kernel is faster: 1.77 ms
      // against 2.4 ms per 128^3 launch)
      hipLaunchKernelGGL((dg::k_rhs_mfma3d<3, FX, false, float>), dim3((unsigned)((c->ncell + 63) / 64)),
                         dim3(kBlock), 0, s, c->tabmf32, c->tablw, nullptr, w, out, dt, make_grid(c), dg::AmrGrid{},
                         mode, mx, c->flag);
    } else if constexpr (D == 3 && K == 3 && sizeof(R) == 8) {
      // four lanes per cell: one thread per cell would hold two 100-double
      // register sets (the weights and the accumulators) and spill 632 B per
      // lane (at k = 2 the one-thread kernel, at one wave per SIMD, is twice
      // as fast as this one, whose rounds of four nodes waste a quarter of the
      // nine face nodes)
      if (vext || c->gravity) return DG_EUNSUPPORTED;
      hipLaunchKernelGGL((dg::k_rhs_amr_quad<K, FX, true>), dim3(nblocks(4 * c->ncell)), dim3(kBlock), 0, s, c->tab,
                         w, out, dt, make_uniform_amr_grid(c), mode, mx, c->flag);
    } else if (D == 3 && K == 2 && sizeof(R) == sizeof(double) && !c->gravity && !vext && c->tabmf) {
      // contractions on FP64 MFMA, 16 cells per wave
      if (periodic(c))
        hipLaunchKernelGGL((dg::k_rhs_mfma3d<2, FX, false, double, false, true>),
                           dim3((unsigned)((c->ncell + 63) / 64)), dim3(kBlock), 0, s, c->tabmf, nullptr, nullptr, w,
                           out, dt, make_grid(c), dg::AmrGrid{}, mode, mx, c->flag);
      else
        hipLaunchKernelGGL((dg::k_rhs_mfma3d<2, FX, false>), dim3((unsigned)((c->ncell + 63) / 64)), dim3(kBlock), 0,
                           s, c->tabmf, nullptr, nullptr, w, out, dt, make_grid(c), dg::AmrGrid{}, mode, mx, c->flag);
    } else {
      if (c->gravity) {
        if constexpr (sizeof(R) == sizeof(double)) {
          hipLaunchKernelGGL((dg::k_rhs_stage<D, K, R, FX, true>), dim3(nblocks(c->ncell)), dim3(kBlock), 0, s, c->tab,
                             tabr, w, out, dt, vext, make_grid(c), mode, mx, c->flag, c->grav);
        } else {
          return DG_EUNSUPPORTED;
        }
      } else {
        hipLaunchKernelGGL((dg::k_rhs_stage<D, K, R, FX>), dim3(nblocks(c->ncell)), dim3(kBlock), 0, s, c->tab, tabr,
                           w, out, dt, vext, make_grid(c), mode, mx, c->flag, nullptr);
      }
    }
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
  template <int D, int K>
  int volume_bf16(float *v) {
    const __bf16 *tb = reinterpret_cast<const __bf16 *>(c->tabbf);
    if (!c->amr) {
      hipLaunchKernelGGL((dg::k_volume_bf16<D, K>), dim3((unsigned)((c->ncell + 63) / 64)), dim3(256), 0, s, tb, w,
                         c->ncell, v, c->cfg.gamma);
    } else {
      const long nw = (long)c->sh.nv * c->sh.N;
      hipLaunchKernelGGL((dg::k_volume_bf16<D, K>), dim3((unsigned)((c->ncc + 63) / 64)), dim3(256), 0, s, tb, w,
                         c->ncc, v, c->cfg.gamma);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL((dg::k_volume_bf16<D, K>), dim3((unsigned)((c->ncf + 63) / 64)), dim3(256), 0, s, tb,
                         w + nw * c->ncc, c->ncf, v + nw * c->ncc, c->cfg.gamma);
    }
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
  // BF16 path on 3D grids at k = 2, 3: the volume term fused into the FP32
  // MFMA stage kernel (no scratch)
  template <int K, int FX>
  int launch_vb() {
    const dg::bf16x8 *tv = static_cast<const dg::bf16x8 *>(c->tabvb);
    if (c->amr) {
      const unsigned nb = (unsigned)((c->ncc + 63) / 64 + (c->ncf + 63) / 64);
      hipLaunchKernelGGL((dg::k_rhs_mfma3d<K, FX, true, float, true>), dim3(nb), dim3(kBlock), 0, s, c->tabmf32,
                         c->tablw, tv, w, out, dt, make_grid(c), make_amr_grid(c), mode, mx, c->flag);
    } else {
      hipLaunchKernelGGL((dg::k_rhs_mfma3d<K, FX, false, float, true>), dim3((unsigned)((c->ncell + 63) / 64)),
                         dim3(kBlock), 0, s, c->tabmf32, c->tablw, tv, w, out, dt, make_grid(c), dg::AmrGrid{}, mode,
                         mx, c->flag);
    }
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
  template <int D, int K>
  int run() {
    if (c->cfg.precision == DG_BF16_VOL && c->tabvb) {
      if constexpr (D == 3 && (K == 2 || K == 3)) {
        if (ro.op != dg::RATE_NONE) return DG_EINVAL;
        return c->cfg.flux == DG_HLLC_DAVIS ? launch_vb<K, DG_HLLC_DAVIS>() : launch_vb<K, DG_HLLC_BATTEN>();
      } else {
        return DG_EUNSUPPORTED;
      }
    }
    if (c->cfg.precision == DG_BF16_VOL) {
      if constexpr (K > 3) {
        return DG_EUNSUPPORTED;
      } else {
        float *v = vs ? vs : c->vscratch;
        int st = volume_bf16<D, K>(v);
        if (st != DG_OK) return st;
        return launch<D, K, float>(c->tab32, v);
      }
    }
    if (c->cfg.precision == DG_FP32) return launch<D, K, float>(c->tab32, nullptr);
    return launch<D, K, double>(c->tab, nullptr);
  }
};

struct ProjectLaunch {
  dg_ctx *c;
  const double *prim;
  double *w;
  hipStream_t s;
  template <int D, int K>
  int run() {
    if (c->tree) {
      const long nl = (long)c->tleaves.size() / 3;
      hipLaunchKernelGGL((dg::k_project<D, K>), dim3(nblocks(nl)), dim3(kBlock), 0, s, c->tab, prim, nl, 0L, w, nl,
                         c->cfg.gamma);
    } else if (!c->amr) {
      hipLaunchKernelGGL((dg::k_project<D, K>), dim3(nblocks(c->ncell)), dim3(kBlock), 0, s, c->tab, prim, c->ncell,
                         0L, w, c->ncell, c->cfg.gamma);
    } else {
      const long nt = c->ncc + c->ncf;
      hipLaunchKernelGGL((dg::k_project<D, K>), dim3(nblocks(c->ncc)), dim3(kBlock), 0, s, c->tab, prim, nt, 0L, w,
                         c->ncc, c->cfg.gamma);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL((dg::k_project<D, K>), dim3(nblocks(c->ncf)), dim3(kBlock), 0, s, c->tab, prim, nt, c->ncc,
                         w + (long)c->sh.nv * c->sh.N * c->ncc, c->ncf, c->cfg.gamma);
    }
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
};

struct LimitLaunch {
  dg_ctx *c;
  double *w;
  hipStream_t s;
  template <int D, int K>
  int run() {
    const bool chr = c->cfg.slope_limiter == DG_LIM_CHAR;
    const int slope = c->cfg.slope_limiter != DG_LIM_NONE;
    const int posit = c->cfg.positivity;
    if constexpr (K > 3) {
      if (c->amr) return DG_EUNSUPPORTED;
    }
    // positivity: the limiter lists the cells that need the point loop,
    // k_positivity runs it (a fill kernel clears the count: no memset, so
    // the sequence can be captured in a graph)
    if (posit) {
      hipLaunchKernelGGL(dg::k_zero_count, dim3(1), dim3(1), 0, s, c->plist);
      HIP_TRY(hipGetLastError());
    }
    // waves of the point-loop kernel: a grid-stride over the listed cells
    const unsigned npos = (unsigned)std::min<long>(1024, std::max<long>(1, (c->ncell + 255) / 256));
    if constexpr (K <= 3) {
      if (c->amr) {
        // the fine block first: its boundary cells read whole coarse polynomials
        const long part[2][2] = {{c->ncc, c->ncf}, {0, c->ncc}};
        for (const auto &pt : part) {
          hipLaunchKernelGGL((chr ? dg::k_limit_amr<D, K, true> : dg::k_limit_amr<D, K, false>),
                             dim3(nblocks(pt[1])), dim3(kBlock), 0, s, c->tab, w, make_amr_grid(c), pt[0], pt[1],
                             slope, c->cfg.beta, c->cfg.m_tilde, posit, c->cfg.eps, c->flag, c->plist);
          HIP_TRY(hipGetLastError());
        }
        if (posit)
          hipLaunchKernelGGL((dg::k_positivity<D, K, true>), dim3(npos), dim3(kBlock), 0, s, c->tab, w, make_grid(c),
                             make_amr_grid(c), c->plist, c->cfg.eps);
        HIP_TRY(hipGetLastError());
        return DG_OK;
      }
    }
    hipLaunchKernelGGL((chr ? dg::k_limit<D, K, true> : dg::k_limit<D, K, false>), dim3(nblocks(c->ncell)),
                       dim3(kBlock), 0, s, c->tab, w, make_grid(c), slope, c->cfg.beta, c->cfg.m_tilde * c->dx,
                       posit, c->cfg.eps, c->flag, c->plist);
    HIP_TRY(hipGetLastError());
    if (posit)
      hipLaunchKernelGGL((dg::k_positivity<D, K, false>), dim3(npos), dim3(kBlock), 0, s, c->tab, w, make_grid(c),
                         dg::AmrGrid{}, c->plist, c->cfg.eps);
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
};

struct AdjointLaunch {
  dg_ctx *c;
  const double *w, *lam, *acc;
  double *out, *acc_out;
  const double *dt;
  int mode;
  double ca, cb;
  hipStream_t s;
  template <int D, int K>
  int run() {
    return c->cfg.flux == DG_HLLC_DAVIS ? run_fx<D, K, DG_HLLC_DAVIS>() : run_fx<D, K, DG_HLLC_BATTEN>();
  }
  template <int D, int K, int FX>
  int run_fx() {
    if constexpr (K > 3) {
      return DG_EUNSUPPORTED;
    } else if constexpr (D == 2) {  // four lanes per cell
      hipLaunchKernelGGL((dg::k_adjoint_quad2d<K, FX>), dim3(nblocks(4 * c->ncell)), dim3(kBlock), 0, s, c->tab, w, lam,
                         acc, out, acc_out, dt, make_grid(c), mode, ca, cb, c->flag);
    } else {
      hipLaunchKernelGGL((dg::k_adjoint<D, K, FX>), dim3(nblocks(c->ncell)), dim3(kBlock), 0, s, c->tab, w, lam, acc,
                         out, acc_out, dt, make_grid(c), mode, ca, cb, c->flag);
    }
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
};

// Round-to-nearest-even conversion of a float to BF16 bits.
uint16_t to_bf16(float f) {
  uint32_t u;
  std::memcpy(&u, &f, sizeof(u));
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

float from_bf16(uint16_t h) {
  const uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, sizeof(f));
  return f;
}

struct Bf16Tables {
  const dg_ctx *c;
  std::vector<uint16_t> *out;
  template <int D, int K>
  int run() {
    if constexpr (K > 3) {
      return DG_EUNSUPPORTED;
    } else {
      using C = Cfg<D, K>;
      using M = dg::Mfma<D, K>;
      std::vector<uint16_t> &t = *out;
      t.assign(M::TOTAL, 0);
      const std::vector<double> &h = c->host_tab;
      // each table value x as hi = bf16(x) at offset o and lo = bf16(x - hi)
      // at offset LO + o
      auto put = [&](long o, double x) {
        const uint16_t hi = to_bf16((float)x);
        t[o] = hi;
        t[M::LO + o] = to_bf16((float)(x - (double)from_bf16(hi)));
      };
      for (int q = 0; q < C::Q; ++q)
        for (int m = 0; m < C::N; ++m) put(M::PB + q * M::NP + m, h[C::B + q * C::N + m]);
      for (int a = 0; a < D; ++a)
        for (int m = 0; m < C::N; ++m)
          for (int q = 0; q < C::Q; ++q)
            put(M::DB + (a * M::NP + m) * M::QP + q, h[C::DW + (a * C::Q + q) * C::N + m]);
      return DG_OK;
    }
  }
};

int bf16_tables(const dg_ctx *c, std::vector<uint16_t> &out) { return dispatch(c, Bf16Tables{c, &out}); }

// A operands of k_rhs_mfma3d, 64 doubles per operand block: lane l holds
// A[i = l % 16][k = l / 16] (evaluation: rows = points, k = modes 4 ks + k;
// projection and lifting: rows = modes j, k = points 4 r + k).  The lifting
// tables carry the side's sign (- on the +a side of the cell).
template <int K>
std::vector<double> mf3_tables(const dg_ctx *c) {
  using C = Cfg<3, K>;
  using M = dg::Mf3<K>;
  std::vector<double> t((size_t)(c->amr ? M::AOPS : M::OPS) * 64, 0.0);
  const std::vector<double> &h = c->host_tab;
  for (int l = 0; l < 64; ++l) {
    const int i = l % 16, k = l / 16;
    for (int tt = 0; tt < M::NQT; ++tt)
      for (int ks = 0; ks < M::NKS; ++ks) {
        const int q = 16 * tt + i, m = 4 * ks + k;
        t[(size_t)(M::EV + tt * M::NKS + ks) * 64 + l] = (q < C::Q && m < C::N) ? h[C::B + q * C::N + m] : 0.0;
      }
    for (int fs = 0; fs < 6; ++fs)
      for (int ft = 0; ft < M::NFT; ++ft)
        for (int ks = 0; ks < M::NKS; ++ks) {
          const int pt = 16 * ft + i, m = 4 * ks + k;
          t[(size_t)(M::EF + (fs * M::NFT + ft) * M::NKS + ks) * 64 + l] =
              (pt < C::QF && m < C::N) ? h[C::TF + (fs * C::QF + pt) * C::N + m] : 0.0;
        }
    for (int a = 0; a < 3; ++a)
      for (int tt = 0; tt < M::NQT; ++tt)
        for (int r = 0; r < 4; ++r)
          for (int mt = 0; mt < M::NMT; ++mt) {
            const int q = 16 * tt + 4 * r + k, j = 16 * mt + i;
            t[(size_t)(M::PV + ((a * M::NQT + tt) * 4 + r) * M::NMT + mt) * 64 + l] =
                (q < C::Q && j < C::N && j >= 1) ? h[C::DW + (a * C::Q + q) * C::N + j] : 0.0;
          }
    for (int fs = 0; fs < 6; ++fs)
      for (int ft = 0; ft < M::NFT; ++ft)
        for (int r = 0; r < 4; ++r)
          for (int mt = 0; mt < M::NMT; ++mt) {
            const int pt = 16 * ft + 4 * r + k, j = 16 * mt + i;
            const double sg = (fs & 1) ? -1.0 : 1.0;
            t[(size_t)(M::LF + (((fs * M::NFT + ft) * 4 + r) * M::NMT + mt)) * 64 + l] =
                (pt < C::QF && j < C::N) ? sg * h[C::TW + (fs * C::QF + pt) * C::N + j] : 0.0;
          }
    if (!c->amr) continue;
    // refined box: per side and sub-face, the coarse basis at the sub-face's
    // points (table HG) and the signed sub-face lift (table HW)
    for (int fs = 0; fs < 6; ++fs)
      for (int sb = 0; sb < 4; ++sb)
        for (int ft = 0; ft < M::NFT; ++ft) {
          for (int ks = 0; ks < M::NKS; ++ks) {
            const int pt = 16 * ft + i, m = 4 * ks + k;
            t[(size_t)(M::HGA + ((fs * 4 + sb) * M::NFT + ft) * M::NKS + ks) * 64 + l] =
                (pt < C::QF && m < C::N) ? h[C::HG + ((fs * 4 + sb) * C::QF + pt) * C::N + m] : 0.0;
          }
          for (int r = 0; r < 4; ++r)
            for (int mt = 0; mt < M::NMT; ++mt) {
              const int pt = 16 * ft + 4 * r + k, j = 16 * mt + i;
              const double sg = (fs & 1) ? -1.0 : 1.0;
              t[(size_t)(M::HWA + (((fs * 4 + sb) * M::NFT + ft) * 4 + r) * M::NMT + mt) * 64 + l] =
                  (pt < C::QF && j < C::N) ? sg * h[C::HW + ((fs * 4 + sb) * C::QF + pt) * C::N + j] : 0.0;
            }
        }
  }
  return t;
}

// The FP32 kernel's tables from the FP64 ones: operand row 4 g + r holds the
// FP64 operand's row 4 r + g (the FP32 MFMA's result rows are transposed
// within groups of four), and the FP64 weights of mode 0 of every lift
// operand, per K step r and lane group g, for the mean's FP64 lift.
template <int K>
void mf3_tables_f32(const std::vector<double> &T, bool amr, std::vector<float> &t32, std::vector<double> &lw) {
  using M = dg::Mf3<K, float>;
  t32.assign(T.size(), 0.0f);
  for (size_t o = 0; o < T.size() / 64; ++o)
    for (int l = 0; l < 64; ++l) {
      const int k = l / 16, i = l % 16, ip = 4 * (i % 4) + i / 4;
      t32[o * 64 + l] = (float)T[o * 64 + 16 * k + ip];
    }
  lw.assign(M::LWTOT, 0.0);
  for (int fs = 0; fs < 6; ++fs)
    for (int ft = 0; ft < M::NFT; ++ft)
      for (int r = 0; r < 4; ++r)
        for (int g = 0; g < 4; ++g) {
          // row j = 0 of the lift operand of K step r sits in lane 16 g
          lw[((fs * M::NFT + ft) * 4 + r) * 4 + g] = T[(size_t)(M::LF + ((fs * M::NFT + ft) * 4 + r) * M::NMT) * 64 + 16 * g];
          if (!amr) continue;
          for (int sb = 0; sb < 4; ++sb)
            lw[M::LWH + (((fs * 4 + sb) * M::NFT + ft) * 4 + r) * 4 + g] =
                T[(size_t)(M::HWA + (((fs * 4 + sb) * M::NFT + ft) * 4 + r) * M::NMT) * 64 + 16 * g];
        }
}

// BF16 volume operands of the fused BF16 kernel (k_rhs_mfma3d, VB): per lane
// (g = lane / 16, row = lane % 16) eight BF16 values of A[row][8 g + e] as
// pairs hi, lo; rows in the FP32 result order (row 4 g' + i stands for node
// or mode 4 i + g' of its tile).  Evaluation: nodes x modes (table B);
// projection: modes j >= 1 x nodes 16 (2 tp + e / 4) + 4 (e % 4) + g (table DW).
template <int K>
std::vector<uint16_t> mf3_tables_bf16(const dg_ctx *c) {
  using C = Cfg<3, K>;
  using M = dg::Mf3<K, float>;
  std::vector<uint16_t> t((size_t)M::BOPS * 64 * 8, 0);
  const std::vector<double> &h = c->host_tab;
  auto put = [&](int o, int lane, int e, double x) {
    const uint16_t hi = to_bf16((float)x);
    t[((size_t)o * 64 + lane) * 8 + e] = hi;
    t[((size_t)(o + 1) * 64 + lane) * 8 + e] = to_bf16((float)(x - (double)from_bf16(hi)));
  };
  for (int lane = 0; lane < 64; ++lane) {
    const int row = lane % 16, g = lane / 16, pr = 4 * (row % 4) + row / 4;
    for (int tt = 0; tt < M::NQT; ++tt)
      for (int e = 0; e < 8; ++e) {
        const int q = 16 * tt + pr, m = 8 * g + e;
        put(M::BEV + 2 * tt, lane, e, (q < C::Q && m < C::N) ? h[C::B + q * C::N + m] : 0.0);
      }
    for (int a = 0; a < 3; ++a)
      for (int tp = 0; tp < M::NQC; ++tp)
        for (int mt = 0; mt < M::NMT; ++mt)
          for (int e = 0; e < 8; ++e) {
            const int q = 16 * (2 * tp + e / 4) + 4 * (e % 4) + g, j = 16 * mt + pr;
            put(M::BPV + ((a * M::NQC + tp) * M::NMT + mt) * 2, lane, e,
                (q < C::Q && j < C::N && j >= 1) ? h[C::DW + (a * C::Q + q) * C::N + j] : 0.0);
          }
  }
  return t;
}

// Folds the maximum signal rate of w's cell means into *rm (atomic max).
int rate_fold(dg_ctx *c, const double *w, unsigned long long *rm, hipStream_t s) {
  if (c->amr) {
    if (c->sh.d == 2)
      hipLaunchKernelGGL(dg::k_rate_amr<2>, dim3(c->npartial), dim3(kBlock), 0, s, w, make_amr_grid(c), c->sh.N, rm,
                         c->flag);
    else
      hipLaunchKernelGGL(dg::k_rate_amr<3>, dim3(c->npartial), dim3(kBlock), 0, s, w, make_amr_grid(c), c->sh.N, rm,
                         c->flag);
  } else {
    const double *gm = c->gravity ? c->gmax : nullptr;
    if (c->sh.d == 2)
      hipLaunchKernelGGL(dg::k_rate<2>, dim3(c->npartial), dim3(kBlock), 0, s, w, c->ncell, c->sh.N, c->cfg.gamma,
                         c->dx, rm, c->flag, gm, c->grav_k);
    else
      hipLaunchKernelGGL(dg::k_rate<3>, dim3(c->npartial), dim3(kBlock), 0, s, w, c->ncell, c->sh.N, c->cfg.gamma,
                         c->dx, rm, c->flag, gm, c->grav_k);
  }
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

bool limited(const dg_ctx *c) { return c->cfg.slope_limiter != DG_LIM_NONE || c->cfg.positivity; }

// Shu-Osher form of an explicit tableau with the derivative on the previous
// stage only (see dg_set_tableau).  Writing each stage value as w^n + dt
// sum_l Abar_jl k_l (Abar: a with b appended as row s), stage m needs
// beta_m = Abar_{m,m-1} and sum_{j>l} alpha_mj Abar_jl = Abar_ml for l < m-1;
// the equation of l = j-1 is the first one in which alpha_mj appears, so
// sweeping j downwards fixes alpha_mj from that equation and removes its
// share from the residuals of the lower equations.
int shu_osher_form(dg_ctx *c, int s, const double *a, const double *b) {
  if (s < 1 || s > DG_MAX_STAGES) return DG_EINVAL;
  double Ab[DG_MAX_STAGES + 1][DG_MAX_STAGES];
  for (int i = 0; i <= s; ++i)
    for (int j = 0; j < s; ++j) {
      const double v = (i < s) ? a[i * s + j] : b[j];
      if (!std::isfinite(v) || (i < s && j >= i && v != 0.0)) return DG_EINVAL;
      Ab[i][j] = v;
    }
  for (int i = 0; i < s; ++i)
    if (Ab[i + 1][i] == 0.0) return DG_EINVAL;
  double al[DG_MAX_STAGES + 1][DG_MAX_STAGES + 1] = {}, be[DG_MAX_STAGES + 1] = {};
  for (int m = 1; m <= s; ++m) {
    be[m] = Ab[m][m - 1];
    double res[DG_MAX_STAGES] = {};
    for (int l = 0; l + 1 < m; ++l) res[l] = Ab[m][l];
    double rest = 0.0;
    for (int j = m - 1; j >= 1; --j) {
      al[m][j] = res[j - 1] / Ab[j][j - 1];
      rest += al[m][j];
      for (int l = 0; l < j - 1; ++l) res[l] -= al[m][j] * Ab[j][l];
    }
    al[m][0] = 1.0 - rest;
  }
  c->rk_s = s;
  std::memcpy(c->rk_alpha, al, sizeof(al));
  std::memcpy(c->rk_beta, be, sizeof(be));
  return DG_OK;
}

// The stage combination of SSP-RK3 (table RK_3): 1, 1; 1/4, 1/4 with 3/4 w^n;
// 2/3, 2/3 with 1/3 w^n.
dg::Mix rk3_mix(int stage, const double *wn) {
  static const double A[3] = {0.0, 0.75, 1.0 / 3.0};
  static const double B[3] = {1.0, 0.25, 2.0 / 3.0};
  dg::Mix m{};
  m.cu = m.cl = B[stage - 1];
  if (stage > 1) {
    m.y[0] = wn;
    m.a[0] = A[stage - 1];
    m.n = 1;
  }
  return m;
}

struct GravSetup {
  dg_ctx *c;
  const double *accel;
  hipStream_t s;
  template <int D, int K>
  int run() {
    hipLaunchKernelGGL((dg::k_grav_setup<D, K>), dim3(nblocks(c->ncell)), dim3(kBlock), 0, s, c->tab, accel, c->ncell,
                       0.5 * c->dx, c->grav, c->gmax);
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
};

dg::BoxGrid box_grid(const dg_ctx *c) {
  dg::BoxGrid g{};
  g.n[0] = (int)c->nx;
  g.n[1] = (int)c->ny;
  g.n[2] = (int)c->nz;
  for (int a = 0; a < 3; ++a) {
    g.lo[a] = c->amr ? c->lo[a] : 0;
    g.hi[a] = c->amr ? c->hi[a] : 0;
    g.nf[a] = c->amr ? (int)c->nf[a] : 1;
  }
  g.ncc = c->amr ? c->ncc : c->ncell;
  g.ncf = c->amr ? c->ncf : 0;
  g.box = c->amr ? 1 : 0;
  return g;
}

struct AmrFlagsLaunch {
  dg_ctx *c;
  const double *w;
  double thr_cell, thr_node;
  int *flags, *box;
  hipStream_t s;
  template <int D, int K>
  int run() {
    const dg::BoxGrid g = box_grid(c);
    hipLaunchKernelGGL(dg::k_box_init, dim3(1), dim3(64), 0, s, box);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL((dg::k_amr_flags<D, K>), dim3(nblocks(g.ncc)), dim3(kBlock), 0, s, w, c->prmat, g, thr_cell,
                       thr_node, flags, box);
    HIP_TRY(hipGetLastError());
    hipLaunchKernelGGL(dg::k_box_final, dim3(1), dim3(64), 0, s, box, D, g.n[0], g.n[1], g.n[2]);
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
};

struct AmrRegridLaunch {
  const dg_ctx *a;
  const double *wa;
  dg_ctx *b;
  double *wb;
  hipStream_t s;
  template <int D, int K>
  int run() {
    const dg::BoxGrid ga = box_grid(a), gb = box_grid(b);
    hipLaunchKernelGGL((dg::k_amr_regrid<D, K>), dim3(nblocks(gb.ncc + gb.ncf)), dim3(kBlock), 0, s, wa, ga,
                       b->prmat, wb, gb);
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
};

// Stage m of the configured tableau from the stage values y[0..m-1]: the
// input is y[m-1]; earlier values with a nonzero weight are the extra terms.
dg::Mix tableau_mix(const dg_ctx *c, int m, const double *const *y) {
  dg::Mix mx{};
  mx.cu = c->rk_alpha[m][m - 1];
  mx.cl = c->rk_beta[m];
  for (int j = 0; j + 1 < m; ++j)
    if (c->rk_alpha[m][j] != 0.0) {
      mx.y[mx.n] = y[j];
      mx.a[mx.n] = c->rk_alpha[m][j];
      ++mx.n;
    }
  return mx;
}

}  // namespace

extern "C" {

const char *dg_strerror(int code) {
  switch (code) {
    case DG_OK: return "success";
    case DG_EINVAL: return "invalid argument";
    case DG_EUNSUPPORTED: return "unsupported dimension, degree or option";
    case DG_ENOMEM: return "out of memory";
    case DG_EHIP: return g_hip_msg[0] ? g_hip_msg : "HIP runtime error";
    case DG_ENEGATIVE: return "non-positive mean density or pressure";
    case DG_ENAN: return "NaN in the right-hand side";
    case DG_ESCRATCH: return "state larger than the static scratch of dg_rhs_noalloc";
    default: return "unknown error";
  }
}

int dg_init(const dg_config *cfg, dg_ctx **out) {
  if (!cfg || !out) return DG_EINVAL;
  *out = nullptr;
  if (cfg->dim != 2 && cfg->dim != 3) return DG_EUNSUPPORTED;
  if (cfg->k < 1 || cfg->k > 4) return DG_EUNSUPPORTED;
  if (cfg->k == 4 && (cfg->dim != 2 || cfg->precision == DG_BF16_VOL)) return DG_EUNSUPPORTED;
  for (int a = 0; a < cfg->dim; ++a) {
    if (cfg->n[a] < 1 || !(cfg->len[a] > 0.0)) return DG_EINVAL;
    if (cfg->bc[a] != DG_BC_PERIODIC && cfg->bc[a] != DG_BC_TRANSMISSIVE) return DG_EINVAL;
  }
  if (!(cfg->gamma > 1.0) || !(cfg->cfl > 0.0)) return DG_EINVAL;
  if (cfg->flux != DG_HLLC_BATTEN && cfg->flux != DG_HLLC_DAVIS) return DG_EINVAL;
  if (cfg->precision != DG_FP64 && cfg->precision != DG_FP32 && cfg->precision != DG_BF16_VOL)
    return DG_EUNSUPPORTED;
  if (cfg->slope_limiter != DG_LIM_NONE && cfg->slope_limiter != DG_LIM_MINMOD && cfg->slope_limiter != DG_LIM_CHAR)
    return DG_EUNSUPPORTED;
  if (cfg->positivity != 0 && cfg->positivity != 1) return DG_EINVAL;
  if (cfg->tile2d != DG_TILE2D_AUTO && cfg->tile2d != DG_TILE2D_8X8 && cfg->tile2d != DG_TILE2D_LARGE)
    return DG_EINVAL;
  if (cfg->path3d != DG_PATH3D_AUTO && cfg->path3d != DG_PATH3D_VALU) return DG_EINVAL;
  if (cfg->positivity && !(cfg->eps > 0.0)) return DG_EINVAL;
  bool amr = false;
  for (int a = 0; a < cfg->dim; ++a)
    if (cfg->refine_lo[a] != cfg->refine_hi[a]) amr = true;
  if (amr)
    for (int a = 0; a < cfg->dim; ++a)
      if (cfg->refine_lo[a] < 1 || cfg->refine_hi[a] > cfg->n[a] - 1 || cfg->refine_hi[a] <= cfg->refine_lo[a])
        return DG_EINVAL;
  if (amr && cfg->k == 4) return DG_EUNSUPPORTED;
  const double dx = cfg->len[0] / cfg->n[0];
  for (int a = 1; a < cfg->dim; ++a)
    if (std::fabs(cfg->len[a] / cfg->n[a] - dx) > 1e-12 * dx) return DG_EINVAL;
  long long cells = 1;
  for (int a = 0; a < cfg->dim; ++a) cells *= cfg->n[a];
  if (cells > (1LL << 31)) return DG_EUNSUPPORTED;

  dg_ctx *c = new (std::nothrow) dg_ctx();
  if (!c) return DG_ENOMEM;
  c->cfg = *cfg;
  c->sh = dg::make_shape(cfg->dim, cfg->k);
  c->lay = dg::make_layout(c->sh);
  c->nx = cfg->n[0];
  c->ny = cfg->n[1];
  c->nz = cfg->dim == 3 ? cfg->n[2] : 1;
  c->ncell = c->nx * c->ny * c->nz;
  c->dx = dx;
  if (amr) {
    c->amr = true;
    c->ncc = c->ncell;
    c->ncf = 1;
    for (int a = 0; a < cfg->dim; ++a) {
      c->lo[a] = cfg->refine_lo[a];
      c->hi[a] = cfg->refine_hi[a];
      c->nf[a] = 2L * (c->hi[a] - c->lo[a]);
      c->ncf *= c->nf[a];
    }
    c->ncell = c->ncc + c->ncf;  // cells of both blocks (hole cells included)
    if (c->ncf > (1L << 31)) {  // kernels index a block's cells in 32 bits
      delete c;
      return DG_EUNSUPPORTED;
    }
  }
  try {
    c->host_tab = dg::build_tables(c->sh, &c->gll_w1);
  } catch (...) {
    delete c;
    return DG_EUNSUPPORTED;
  }
  if (check_layout(c) != DG_OK) {
    delete c;
    return DG_EINVAL;
  }
  double fk = 1.0 / (2.0 * cfg->k + 1.0);
  if (cfg->positivity && c->gll_w1 / 2.0 < fk) fk = c->gll_w1 / 2.0;
  c->cfl_fk = cfg->cfl * fk;
  c->tile_small = cfg->tile2d == DG_TILE2D_8X8 ? 1 : cfg->tile2d == DG_TILE2D_LARGE ? 0 : -1;
  {
    static const double a3[9] = {0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.25, 0.25, 0.0};
    static const double b3[3] = {1.0 / 6.0, 1.0 / 6.0, 2.0 / 3.0};
    shu_osher_form(c, 3, a3, b3);
  }
  c->npartial = (int)std::min<long>(1024, (c->ncell + kBlock - 1) / kBlock);

  auto fail = [&](hipError_t e) {
    int r = hip_fail(e);
    dg_destroy(c);
    return r;
  };
  hipError_t e;
  if ((e = hipGetDevice(&c->device)) != hipSuccess) return fail(e);
  if (c->device >= 0 && c->device < kMaxDevices) {
    // the address of this device's copy of the static scratch (dg_rhs_noalloc)
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[c->device]) {
      void *p = nullptr;
      if ((e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch))) != hipSuccess) return fail(e);
      g_scratch_ptr[c->device] = static_cast<float *>(p);
    }
  }
  const size_t nt = c->host_tab.size();
  if ((e = hipMalloc((void **)&c->tab, nt * sizeof(double))) != hipSuccess) return fail(e);
  if ((e = hipMalloc((void **)&c->tab32, nt * sizeof(float))) != hipSuccess) return fail(e);
  if ((e = hipMalloc((void **)&c->partial, DG_RATE_STATE * sizeof(double))) != hipSuccess) return fail(e);
  if ((e = hipMalloc((void **)&c->flag, sizeof(int))) != hipSuccess) return fail(e);
  if (cfg->positivity && (e = hipMalloc((void **)&c->plist, (size_t)(c->ncell + 1) * sizeof(int))) != hipSuccess)
    return fail(e);
  std::vector<float> t32(nt);
  for (size_t i = 0; i < nt; ++i) t32[i] = (float)c->host_tab[i];
  if ((e = hipMemcpy(c->tab, c->host_tab.data(), nt * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e);
  if ((e = hipMemcpy(c->tab32, t32.data(), nt * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
  int zero = 0;
  if ((e = hipMemcpy(c->flag, &zero, sizeof(int), hipMemcpyHostToDevice)) != hipSuccess) return fail(e);
  // the fused BF16 stage kernel (3D, k = 2, 3) needs no separate volume pass
  const bool vb_fused = cfg->precision == DG_BF16_VOL && cfg->dim == 3 && (cfg->k == 2 || cfg->k == 3) &&
                        cfg->path3d != DG_PATH3D_VALU;
  if (cfg->precision == DG_BF16_VOL && !vb_fused) {
    std::vector<uint16_t> tb;
    int st = bf16_tables(c, tb);
    if (st != DG_OK) {
      dg_destroy(c);
      return st;
    }
    if ((e = hipMalloc((void **)&c->tabbf, tb.size() * sizeof(uint16_t))) != hipSuccess) return fail(e);
    if ((e = hipMemcpy(c->tabbf, tb.data(), tb.size() * sizeof(uint16_t), hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e);
    const size_t nv = (size_t)c->sh.nv * c->sh.N * c->ncell;
    if ((e = hipMalloc((void **)&c->vscratch, nv * sizeof(float))) != hipSuccess) return fail(e);
  }
  const std::vector<double> zeros(DG_RATE_STATE, 0.0);
  if ((e = hipMemcpy(c->partial, zeros.data(), DG_RATE_STATE * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
    return fail(e);
  if (cfg->dim == 3 && (cfg->k == 2 || cfg->k == 3) && cfg->path3d != DG_PATH3D_VALU &&
      (cfg->precision == DG_FP64 || (cfg->precision == DG_FP32 && (cfg->k == 3 || amr)) || vb_fused)) {
    const std::vector<double> T = cfg->k == 2 ? mf3_tables<2>(c) : mf3_tables<3>(c);
    if (cfg->precision == DG_FP64) {
      if ((e = hipMalloc((void **)&c->tabmf, T.size() * sizeof(double))) != hipSuccess) return fail(e);
      if ((e = hipMemcpy(c->tabmf, T.data(), T.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    } else {
      std::vector<float> t32;
      std::vector<double> lw;
      if (cfg->k == 2)
        mf3_tables_f32<2>(T, c->amr, t32, lw);
      else
        mf3_tables_f32<3>(T, c->amr, t32, lw);
      if ((e = hipMalloc((void **)&c->tabmf32, t32.size() * sizeof(float))) != hipSuccess) return fail(e);
      if ((e = hipMemcpy(c->tabmf32, t32.data(), t32.size() * sizeof(float), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
      if ((e = hipMalloc((void **)&c->tablw, lw.size() * sizeof(double))) != hipSuccess) return fail(e);
      if ((e = hipMemcpy(c->tablw, lw.data(), lw.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    }
    if (vb_fused) {
      const std::vector<uint16_t> tv = cfg->k == 2 ? mf3_tables_bf16<2>(c) : mf3_tables_bf16<3>(c);
      if ((e = hipMalloc(&c->tabvb, tv.size() * sizeof(uint16_t))) != hipSuccess) return fail(e);
      if ((e = hipMemcpy(c->tabvb, tv.data(), tv.size() * sizeof(uint16_t), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    }
  }
  if (cfg->k <= 3) {
    // refinement matrices of dg_amr_flags / dg_amr_regrid (eq. ref_pa_integral)
    const std::vector<double> P = dg::refine_matrices(c->sh);
    if ((e = hipMalloc((void **)&c->prmat, P.size() * sizeof(double))) != hipSuccess) return fail(e);
    if ((e = hipMemcpy(c->prmat, P.data(), P.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
      return fail(e);
    if (cfg->dim == 2) {
      // 1D tables of the quadtree stage kernel
      const std::vector<double> t1 = dg::tables_1d(cfg->k);
      if ((e = hipMalloc((void **)&c->t1d, t1.size() * sizeof(double))) != hipSuccess) return fail(e);
      if ((e = hipMemcpy(c->t1d, t1.data(), t1.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
        return fail(e);
    }
  }
  *out = c;
  return DG_OK;
}

void dg_destroy(dg_ctx *c) {
  if (!c) return;
  if (c->tab) (void)hipFree(c->tab);
  if (c->tab32) (void)hipFree(c->tab32);
  if (c->tabbf) (void)hipFree(c->tabbf);
  if (c->vscratch) (void)hipFree(c->vscratch);
  if (c->partial) (void)hipFree(c->partial);
  if (c->flag) (void)hipFree(c->flag);
  if (c->plist) (void)hipFree(c->plist);
  if (c->grav) (void)hipFree(c->grav);
  if (c->gmax) (void)hipFree(c->gmax);
  if (c->prmat) (void)hipFree(c->prmat);
  if (c->tabmf) (void)hipFree(c->tabmf);
  if (c->tabmf32) (void)hipFree(c->tabmf32);
  if (c->tablw) (void)hipFree(c->tablw);
  if (c->tabvb) (void)hipFree(c->tabvb);
  if (c->ttab) (void)hipFree(c->ttab);
  if (c->tmap) (void)hipFree(c->tmap);
  if (c->tflags) (void)hipFree(c->tflags);
  if (c->treg) (void)hipFree(c->treg);
  if (c->tplist) (void)hipFree(c->tplist);
  if (c->t1d) (void)hipFree(c->t1d);
  if (c->tnbm) (void)hipFree(c->tnbm);
  delete c;
}

int dg_state_size(const dg_ctx *c, int64_t *n) {
  if (!c || !n) return DG_EINVAL;
  *n = (int64_t)c->sh.nv * c->sh.N * (c->tree ? (long)c->tleaves.size() / 3 : c->ncell);
  return DG_OK;
}

int dg_sizes(const dg_ctx *c, int64_t out[6]) {
  if (!c || !out) return DG_EINVAL;
  out[0] = c->sh.nv;
  out[1] = c->sh.N;
  out[2] = c->sh.Q;
  out[3] = c->sh.QF;
  out[4] = c->ncell;
  out[5] = c->sh.NS;
  return DG_OK;
}

int dg_amr_sizes(const dg_ctx *c, int64_t out[5]) {
  if (!c || !out) return DG_EINVAL;
  out[0] = c->amr ? c->ncc : c->ncell;
  out[1] = c->amr ? c->ncf : 0;
  for (int a = 0; a < 3; ++a) out[2 + a] = c->amr ? c->nf[a] : 0;
  return DG_OK;
}

int dg_quadrature(const dg_ctx *c, double *xi, double *w) {
  if (!c || !xi || !w) return DG_EINVAL;
  for (int q = 0; q < c->sh.Q; ++q) {
    for (int a = 0; a < 3; ++a) xi[3 * q + a] = c->host_tab[c->lay.XQ + 3 * q + a];
    w[q] = c->host_tab[c->lay.WQ + q];
  }
  return DG_OK;
}

int dg_project(dg_ctx *c, const double *prim, double *w, void *stream) {
  if (!c || !prim || !w) return DG_EINVAL;
  return dispatch(c, ProjectLaunch{c, prim, w, (hipStream_t)stream});
}

int dg_rhs(dg_ctx *c, const double *w, double *L, void *stream) {
  if (!c || !w || !L || w == L || c->tree) return DG_EINVAL;
  return dispatch(c, StageLaunch{c, w, nullptr, L, 0, dg::Mix{}, (hipStream_t)stream});
}

int dg_rhs_noalloc(dg_ctx *c, const double *w, double *L, void *stream) {
  if (!c || !w || !L || w == L || c->tree) return DG_EINVAL;
  if (c->cfg.precision != DG_BF16_VOL) return DG_EINVAL;
  // the fused 3D kernel keeps its volume term in registers: nothing to stage
  if (c->tabvb) return dispatch(c, StageLaunch{c, w, nullptr, L, 0, dg::Mix{}, (hipStream_t)stream});
  if ((long long)c->sh.nv * c->sh.N * c->ncell > (long long)DG_STATIC_SCRATCH_FLOATS) return DG_ESCRATCH;
  if (c->device < 0 || c->device >= kMaxDevices) return DG_EUNSUPPORTED;
  float *vs;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    vs = g_scratch_ptr[c->device];
  }
  if (!vs) return DG_EHIP;  // dg_init failed to look it up (it returned an error then)
  StageLaunch sl{c, w, nullptr, L, 0, dg::Mix{}, (hipStream_t)stream};
  sl.vs = vs;
  return dispatch(c, sl);
}

int dg_rk_stage(dg_ctx *c, int stage, const double *dt, const double *wn, const double *wp, double *out,
                void *stream) {
  if (!c || !dt || !wp || !out || stage < 1 || stage > 3 || c->tree) return DG_EINVAL;
  if (stage > 1 && !wn) return DG_EINVAL;
  if (out == wp || out == wn) return DG_EINVAL;
  return dispatch(c, StageLaunch{c, wp, dt, out, 1, rk3_mix(stage, wn), (hipStream_t)stream});
}

int dg_set_tableau(dg_ctx *c, int stages, const double *a, const double *b) {
  if (!c || !a || !b || stages < 1 || stages > DG_MAX_STAGES) return DG_EINVAL;
  return shu_osher_form(c, stages, a, b);  // leaves c alone on error
}

int dg_tableau_stage(dg_ctx *c, int m, const double *dt, const double *const *y, double *out, void *stream) {
  if (!c || !dt || !y || !out || m < 1 || m > c->rk_s || c->tree) return DG_EINVAL;
  for (int j = 0; j < m; ++j)
    if (!y[j] || y[j] == out) return DG_EINVAL;
  return dispatch(c, StageLaunch{c, y[m - 1], dt, out, 1, tableau_mix(c, m, y), (hipStream_t)stream});
}


int dg_max_dt(dg_ctx *c, const double *w, double *dt, void *stream) {
  if (!c || !w || !dt || c->tree) return DG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long *rm = reinterpret_cast<unsigned long long *>(c->partial);
  int st = rate_fold(c, w, rm, s);
  if (st != DG_OK) return st;
  hipLaunchKernelGGL(dg::k_dt_final, dim3(1), dim3(64), 0, s, rm, c->cfl_fk, dt);
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

int dg_max_rate(dg_ctx *c, const double *w, double *rate, void *stream) {
  if (!c || !w || !rate || c->tree) return DG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long *rm = reinterpret_cast<unsigned long long *>(rate);
  hipLaunchKernelGGL(dg::k_rate_zero, dim3(1), dim3(64), 0, s, rm);
  HIP_TRY(hipGetLastError());
  return rate_fold(c, w, rm, s);
}

int dg_rk_step(dg_ctx *c, const double *w, double *u1, double *u2, double *out, double *dt, double *rate,
               void *stream) {
  if (!c || !w || !u1 || !u2 || !out || !dt || !rate || c->tree) return DG_EINVAL;
  const void *st_ptr[4] = {w, u1, u2, out};
  for (int i = 0; i < 4; ++i)
    for (int j = i + 1; j < 4; ++j)
      if (st_ptr[i] == st_ptr[j]) return DG_EINVAL;
  if (dt >= rate && dt < rate + DG_RATE_STATE) return DG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long *rm = reinterpret_cast<unsigned long long *>(rate);
  const bool fused = !c->amr && c->sh.d == 2;
  if (!fused) {
    // dt from the carried rate (the word is cleared for the fold below)
    hipLaunchKernelGGL(dg::k_dt_final, dim3(1), dim3(64), 0, s, rm, c->cfl_fk, dt);
    HIP_TRY(hipGetLastError());
  }
  auto op = [&](int k) { return dg::RateOp{rm, dt, c->cfl_fk, c->dx, fused ? k : dg::RATE_NONE}; };
  const double *wp[3] = {w, u1, u2};
  double *wo[3] = {u1, u2, out};
  static const int R[3] = {dg::RATE_DT, dg::RATE_CLEAR, dg::RATE_FOLD};
  for (int k = 0; k < 3; ++k) {
    int st = dispatch(c, StageLaunch{c, wp[k], dt, wo[k], 1, rk3_mix(k + 1, w), s, op(R[k])});
    if (st != DG_OK) return st;
    if (limited(c) && (st = dispatch(c, LimitLaunch{c, wo[k], s})) != DG_OK) return st;
  }
  return fused ? DG_OK : rate_fold(c, out, rm, s);
}

int dg_tableau_step(dg_ctx *c, const double *w, double *const *stage, double *out, double *dt, double *rate,
                    void *stream) {
  if (!c || !w || !out || !dt || !rate || c->tree) return DG_EINVAL;
  const int ns = c->rk_s;
  if (ns > 1 && !stage) return DG_EINVAL;
  const double *Y[DG_MAX_STAGES + 1];
  Y[0] = w;
  for (int m = 1; m < ns; ++m) Y[m] = stage[m - 1];
  Y[ns] = out;
  for (int i = 0; i <= ns; ++i) {
    if (!Y[i]) return DG_EINVAL;
    for (int j = i + 1; j <= ns; ++j)
      if (Y[i] == Y[j]) return DG_EINVAL;
  }
  if (dt >= rate && dt < rate + DG_RATE_STATE) return DG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  unsigned long long *rm = reinterpret_cast<unsigned long long *>(rate);
  // the stage kernels carry the time-step work on 2D grids: the first takes
  // dt from the slots, the second clears them (or a clear kernel runs before
  // the last stage of a two-stage method), the last folds the new rate in
  const bool fused = !c->amr && c->sh.d == 2 && ns >= 2;
  if (!fused) {
    hipLaunchKernelGGL(dg::k_dt_final, dim3(1), dim3(64), 0, s, rm, c->cfl_fk, dt);
    HIP_TRY(hipGetLastError());
  }
  for (int m = 1; m <= ns; ++m) {
    int op = dg::RATE_NONE;
    if (fused) {
      if (m == 1) op = dg::RATE_DT;
      else if (m == ns) op = dg::RATE_FOLD;
      else if (m == 2) op = dg::RATE_CLEAR;
      if (m == ns && ns == 2) {
        hipLaunchKernelGGL(dg::k_rate_zero, dim3(1), dim3(64), 0, s, rm);
        HIP_TRY(hipGetLastError());
      }
    }
    double *o = const_cast<double *>(Y[m]);
    int st = dispatch(c, StageLaunch{c, Y[m - 1], dt, o, 1, tableau_mix(c, m, Y), s,
                                     dg::RateOp{rm, dt, c->cfl_fk, c->dx, op}});
    if (st != DG_OK) return st;
    if (limited(c) && (st = dispatch(c, LimitLaunch{c, o, s})) != DG_OK) return st;
  }
  return fused ? DG_OK : rate_fold(c, out, rm, s);
}

int dg_limit(dg_ctx *c, double *w, void *stream) {
  if (!c || !w || c->tree) return DG_EINVAL;
  if (c->cfg.slope_limiter == DG_LIM_NONE && !c->cfg.positivity) return DG_OK;
  return dispatch(c, LimitLaunch{c, w, (hipStream_t)stream});
}

int dg_set_gravity(dg_ctx *c, const double *accel, void *stream) {
  if (!c || c->tree) return DG_EINVAL;
  if (!accel) {
    c->gravity = false;
    return DG_OK;
  }
  // the source is fused into the FP64 one-lane and tile stage kernels
  if (c->amr || c->cfg.precision != DG_FP64 || (c->sh.d == 3 && c->sh.k > 2)) return DG_EUNSUPPORTED;
  const size_t n = (size_t)c->sh.d * c->sh.Q * c->ncell;
  HIP_TRY(hipSetDevice(c->device));
  if (!c->grav) {
    hipError_t e = hipMalloc(&c->grav, n * sizeof(double));
    if (e != hipSuccess) {
      c->grav = nullptr;
      return e == hipErrorOutOfMemory ? DG_ENOMEM : DG_EHIP;
    }
  }
  if (!c->gmax) {
    hipError_t e = hipMalloc(&c->gmax, (size_t)c->ncell * sizeof(double));
    if (e != hipSuccess) {
      c->gmax = nullptr;
      return e == hipErrorOutOfMemory ? DG_ENOMEM : DG_EHIP;
    }
  }
  const int st = dispatch(c, GravSetup{c, accel, (hipStream_t)stream});
  if (st != DG_OK) return st;
  c->gravity = true;
  c->grav_k = c->cfl_fk * std::sqrt(2.0 * c->cfg.gamma * (c->cfg.gamma - 1.0));
  return DG_OK;
}

int dg_amr_flags(dg_ctx *c, const double *w, double wt, double alpha, int *flags, int *box, void *stream) {
  if (!c || !w || !flags || !box || !(wt > 0.0) || !(alpha >= 1.0) || c->tree) return DG_EINVAL;
  if (c->sh.k > 3) return DG_EUNSUPPORTED;
  return dispatch(c, AmrFlagsLaunch{c, w, alpha * wt, wt / alpha, flags, box, (hipStream_t)stream});
}

int dg_amr_regrid(const dg_ctx *from, const double *w_from, dg_ctx *to, double *w_to, void *stream) {
  if (!from || !to || !w_from || !w_to || w_from == w_to || from->tree || to->tree) return DG_EINVAL;
  if (from->sh.d != to->sh.d || from->sh.k != to->sh.k || from->nx != to->nx || from->ny != to->ny ||
      from->nz != to->nz || from->dx != to->dx || from->device != to->device)
    return DG_EINVAL;
  for (int a = 0; a < 3; ++a)
    if (from->cfg.x0[a] != to->cfg.x0[a]) return DG_EINVAL;
  if (to->sh.k > 3) return DG_EUNSUPPORTED;
  return dispatch(to, AmrRegridLaunch{from, w_from, to, w_to, (hipStream_t)stream});
}

int dg_adjoint_rhs(dg_ctx *c, const double *w, const double *lam, double *mu, void *stream) {
  if (!c || !w || !lam || !mu || mu == w || mu == lam || c->tree) return DG_EINVAL;
  if (c->amr || c->gravity) return DG_EUNSUPPORTED;
  return dispatch(c, AdjointLaunch{c, w, lam, nullptr, mu, nullptr, nullptr, 0, 0.0, 0.0, (hipStream_t)stream});
}

int dg_adjoint_rk_stage(dg_ctx *c, int stage, const double *dt, const double *u, const double *lam,
                        const double *acc, double *lam_out, double *acc_out, void *stream) {
  if (!c || !dt || !u || !lam || !lam_out || stage < 1 || stage > 3 || c->tree) return DG_EINVAL;
  if (c->amr || c->gravity) return DG_EUNSUPPORTED;
  if (lam_out == lam || lam_out == u || (acc && lam_out == acc)) return DG_EINVAL;
  if (stage != 3 && !acc) return DG_EINVAL;
  if (stage != 1 && !acc_out) return DG_EINVAL;
  if (acc_out && (acc_out == lam || acc_out == u || acc_out == lam_out)) return DG_EINVAL;
  const int mode = stage == 3 ? 3 : stage == 2 ? 2 : 1;
  const double ca = stage == 3 ? 1.0 / 3.0 : 0.75;
  const double cb = stage == 3 ? 2.0 / 3.0 : 0.25;
  return dispatch(c, AdjointLaunch{c, u, lam, acc, lam_out, acc_out, dt, mode, ca, cb, (hipStream_t)stream});
}

int dg_status(dg_ctx *c, void *stream) {
  if (!c) return DG_EINVAL;
  HIP_TRY(hipStreamSynchronize((hipStream_t)stream));
  int f = 0, zero = 0;
  HIP_TRY(hipMemcpy(&f, c->flag, sizeof(int), hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(c->flag, &zero, sizeof(int), hipMemcpyHostToDevice));
  if (f & dg::FLAG_NEGATIVE) return DG_ENEGATIVE;
  if (f & dg::FLAG_NAN) return DG_ENAN;
  return DG_OK;
}

}  // extern "C"

// ===========================================================================
// Quadtree meshes (host side): leaf tables, adaptation, C ABI
// ===========================================================================
namespace {

// Tree kernels run one thread per leaf; a mesh of tens of thousands of
// leaves is a few hundred waves, so blocks of one wave spread them over all
// 256 CUs (256-thread blocks left a third of the CUs without work).
constexpr int kTreeBlock = 64;
unsigned tree_blocks(long n) { return (unsigned)((n + kTreeBlock - 1) / kTreeBlock); }

inline uint64_t tkey(int l, long x, long y) { return ((uint64_t)l << 58) | ((uint64_t)x << 29) | (uint64_t)y; }

constexpr int kTreeInts = 17;  // per leaf: level, 4 face infos, 8 neighbours, 4 group members

struct TreeIndex {
  std::unordered_map<uint64_t, int> m;
  long nx = 0, ny = 0;
  int bc[2] = {0, 0};
  // level-l cell (x, y) wrapped onto the periodic domain; false outside a wall
  bool wrap(int l, long &x, long &y) const {
    const long nxl = nx << l, nyl = ny << l;
    if (x < 0 || x >= nxl) {
      if (bc[0] != DG_BC_PERIODIC) return false;
      x = ((x % nxl) + nxl) % nxl;
    }
    if (y < 0 || y >= nyl) {
      if (bc[1] != DG_BC_PERIODIC) return false;
      y = ((y % nyl) + nyl) % nyl;
    }
    return true;
  }
  int find(int l, long x, long y) const {
    auto it = m.find(tkey(l, x, y));
    return it == m.end() ? -1 : it->second;
  }
  // the leaf that covers level-l cell (x, y) if it is that cell or coarser, else -1
  int covering(int l, long x, long y) const {
    for (int q = l; q >= 0; --q) {
      const int j = find(q, x >> (l - q), y >> (l - q));
      if (j >= 0) return j;
    }
    return -1;
  }
};

// Validates a leaf set (a tiling of the base grid, the level jump across every
// face at most one) and builds its device tables: level [nl], face info
// [4][nl] (kind | sub << 2), neighbours [8][nl], sibling groups [4][nl].
int tree_tables(const dg_ctx *c, const std::vector<int32_t> &lv, TreeIndex &ix, std::vector<int> &T) {
  const long nl = (long)lv.size() / 3;
  if (nl < 1 || nl > (1L << 30)) return DG_EINVAL;
  ix.m.clear();
  ix.m.reserve((size_t)nl * 2);
  ix.nx = c->nx;
  ix.ny = c->ny;
  ix.bc[0] = c->cfg.bc[0];
  ix.bc[1] = c->cfg.bc[1];
  int L = 0;
  for (long i = 0; i < nl; ++i) {
    const int l = lv[3 * i];
    const long x = lv[3 * i + 1], y = lv[3 * i + 2];
    if (l < 0 || l > 24 || (c->nx << l) >= (1L << 29) || (c->ny << l) >= (1L << 29)) return DG_EINVAL;
    if (x < 0 || y < 0 || x >= (c->nx << l) || y >= (c->ny << l)) return DG_EINVAL;
    if (!ix.m.emplace(tkey(l, x, y), (int)i).second) return DG_EINVAL;
    L = l > L ? l : L;
  }
  unsigned __int128 area = 0;
  for (long i = 0; i < nl; ++i) {
    const int l = lv[3 * i];
    for (int q = 0; q < l; ++q)  // no leaf inside another
      if (ix.find(q, lv[3 * i + 1] >> (l - q), lv[3 * i + 2] >> (l - q)) >= 0) return DG_EINVAL;
    area += (unsigned __int128)1 << (2 * (L - l));
  }
  if (area != ((unsigned __int128)(c->nx * c->ny) << (2 * L))) return DG_EINVAL;
  T.assign((size_t)kTreeInts * nl, -1);
  int *lev = T.data(), *info = lev + nl, *nb = info + 4 * nl, *grp = nb + 8 * nl;
  for (long i = 0; i < nl; ++i) {
    const int l = lv[3 * i];
    const long x = lv[3 * i + 1], y = lv[3 * i + 2];
    lev[i] = l;
    for (int side = 0; side < 4; ++side) {
      const int a = side >> 1, s = side & 1;
      long X = x + (a == 0 ? (s ? 1 : -1) : 0), Y = y + (a == 1 ? (s ? 1 : -1) : 0);
      int kind, sub = 0, n0 = -1, n1 = -1;
      if (!ix.wrap(l, X, Y)) {
        kind = 1;
      } else if ((n0 = ix.find(l, X, Y)) >= 0) {
        kind = 0;
      } else if (l > 0 && (n0 = ix.find(l - 1, X >> 1, Y >> 1)) >= 0) {
        kind = 3;
        sub = (int)((a == 0 ? y : x) & 1);
        // the child of the coarse leaf that the same-level cell (X, Y) is (limiters)
        sub |= (int)(((X & 1) | ((Y & 1) << 1)) << 1);
      } else {
        kind = 2;
        // the two children of the same-level neighbour that touch this face
        const long cx = 2 * X + (a == 0 ? (s ? 0 : 1) : 0), cy = 2 * Y + (a == 1 ? (s ? 0 : 1) : 0);
        n0 = ix.find(l + 1, cx, cy);
        n1 = ix.find(l + 1, cx + (a == 0 ? 0 : 1), cy + (a == 0 ? 1 : 0));
        if (n0 < 0 || n1 < 0) return DG_EINVAL;  // a level jump above one
      }
      info[(long)side * nl + i] = kind | (sub << 2);
      nb[(long)(2 * side) * nl + i] = n0;
      nb[(long)(2 * side + 1) * nl + i] = n1;
    }
    if (l > 0) {
      int g[4];
      bool all = true;
      for (int ch = 0; ch < 4; ++ch) {
        g[ch] = ix.find(l, 2 * (x >> 1) + (ch & 1), 2 * (y >> 1) + (ch >> 1));
        all &= g[ch] >= 0;
      }
      if (all)
        for (int ch = 0; ch < 4; ++ch) grp[(long)ch * nl + i] = g[ch];
    }
  }
  return DG_OK;
}

dg::TreeGrid make_tree_grid(const dg_ctx *c) {
  dg::TreeGrid g;
  g.nleaf = (long)c->tleaves.size() / 3;
  g.lev = c->ttab;
  g.info = c->ttab + g.nleaf;
  g.nb = c->ttab + 5 * g.nleaf;
  g.grp = c->ttab + 13 * g.nleaf;
  g.fac0 = 2.0 / c->dx / 4.0;
  g.dx0 = c->dx;
  g.gamma = c->cfg.gamma;
  g.t1 = c->t1d;
  return g;
}

// grow a device int buffer to at least n ints
int grow_ints(int *&p, long &cap, long n) {
  if (n <= cap) return DG_OK;
  if (p) (void)hipFree(p);
  p = nullptr;
  cap = 0;
  HIP_TRY(hipMalloc((void **)&p, (size_t)n * sizeof(int)));
  cap = n;
  return DG_OK;
}

int tree_upload(dg_ctx *c, std::vector<int32_t> &lv, TreeIndex &ix, const std::vector<int> &T);

// makes `lv` the context's mesh (device tables replaced after the device is
// idle).  An invalid mesh leaves the context as it was; a failure while the
// device tables are replaced leaves it without a mesh (the tree calls then
// refuse with DG_EINVAL) rather than with tables of one mesh and leaves of
// another.
int tree_install(dg_ctx *c, std::vector<int32_t> lv) {
  TreeIndex ix;
  std::vector<int> T;
  int st = tree_tables(c, lv, ix, T);
  if (st != DG_OK) return st;
  st = tree_upload(c, lv, ix, T);
  if (st != DG_OK) {
    c->tree = false;
    c->tleaves.clear();
    c->tnext.clear();
  }
  return st;
}

int tree_upload(dg_ctx *c, std::vector<int32_t> &lv, TreeIndex &ix, const std::vector<int> &T) {
  int st = DG_OK;
  HIP_TRY(hipDeviceSynchronize());
  st = grow_ints(c->ttab, c->ttab_cap, (long)T.size());
  if (st != DG_OK) return st;
  HIP_TRY(hipMemcpy(c->ttab, T.data(), T.size() * sizeof(int), hipMemcpyHostToDevice));
  // limiters: per side with finer neighbours the leaves inside the same-level
  // cell there, in leaf order ([4][nl] offsets, [4][nl] counts, the lists)
  const long nl = (long)lv.size() / 3;
  std::vector<int> R((size_t)8 * nl, 0);
  const int *info = T.data() + nl;
  for (long i = 0; i < nl; ++i)
    for (int side = 0; side < 4; ++side) {
      if ((info[(long)side * nl + i] & 3) != 2) continue;
      const int a = side >> 1, sd = side & 1, l = lv[3 * i];
      long X = lv[3 * i + 1] + (a == 0 ? (sd ? 1 : -1) : 0), Y = lv[3 * i + 2] + (a == 1 ? (sd ? 1 : -1) : 0);
      ix.wrap(l, X, Y);
      std::vector<int> in;
      std::vector<std::pair<int, std::pair<long, long>>> st{{l, {X, Y}}};
      while (!st.empty()) {
        const auto e = st.back();
        st.pop_back();
        const int j = ix.find(e.first, e.second.first, e.second.second);
        if (j >= 0) {
          in.push_back(j);
          continue;
        }
        if (e.first >= 24) return DG_EINVAL;
        for (int ch = 0; ch < 4; ++ch)
          st.push_back({e.first + 1, {2 * e.second.first + (ch & 1), 2 * e.second.second + (ch >> 1)}});
      }
      std::sort(in.begin(), in.end());
      R[(size_t)(side * nl + i)] = (int)(R.size() - 8 * nl);
      R[(size_t)(4 * nl + side * nl + i)] = (int)in.size();
      R.insert(R.end(), in.begin(), in.end());
    }
  st = grow_ints(c->tplist, c->tplist_cap, nl + 1);
  if (st != DG_OK) return st;
  st = grow_ints(c->treg, c->treg_cap, (long)R.size());
  if (st != DG_OK) return st;
  HIP_TRY(hipMemcpy(c->treg, R.data(), R.size() * sizeof(int), hipMemcpyHostToDevice));
  if (16 * nl > c->tnbm_cap) {
    if (c->tnbm) (void)hipFree(c->tnbm);
    c->tnbm = nullptr;
    c->tnbm_cap = 0;
    HIP_TRY(hipMalloc((void **)&c->tnbm, (size_t)16 * nl * sizeof(double)));
    c->tnbm_cap = 16 * nl;
  }
  c->tleaves = std::move(lv);
  c->tree = true;
  c->tnext.clear();
  return DG_OK;
}

// Morton order of the leaves' lower-left corners on the finest level
void tree_sort(std::vector<int32_t> &lv, std::vector<int> *perm_src = nullptr) {
  const long nl = (long)lv.size() / 3;
  int L = 0;
  for (long i = 0; i < nl; ++i) L = lv[3 * i] > L ? lv[3 * i] : L;
  std::vector<std::pair<unsigned __int128, long>> keys((size_t)nl);
  for (long i = 0; i < nl; ++i) {
    const uint64_t x = (uint64_t)lv[3 * i + 1] << (L - lv[3 * i]), y = (uint64_t)lv[3 * i + 2] << (L - lv[3 * i]);
    unsigned __int128 k = 0;
    for (int b = 0; b < 60; ++b)
      k |= ((unsigned __int128)((x >> b) & 1) << (2 * b)) | ((unsigned __int128)((y >> b) & 1) << (2 * b + 1));
    keys[(size_t)i] = {k, i};
  }
  std::sort(keys.begin(), keys.end());
  std::vector<int32_t> out(lv.size());
  std::vector<int> ps;
  for (long j = 0; j < nl; ++j) {
    const long i = keys[(size_t)j].second;
    for (int e = 0; e < 3; ++e) out[3 * j + e] = lv[3 * i + e];
    ps.push_back((int)i);
  }
  lv.swap(out);
  if (perm_src) *perm_src = ps;
}

// The next mesh from the current leaves and their flags (k_tree_flags):
//  1. leaves flagged by eq. cell_ref below max_level are split, and with them
//     the leaves of the same or a coarser level among the eight neighbour
//     cells of each flagged leaf (the one buffer layer of Sec. 4);
//  2. split leaves force the split of any coarser face or corner neighbour
//     (level jump at most one to all neighbours, Sec. 4), until none is left;
//  3. a complete sibling group of unsplit leaves whose node weights fail
//     eq. node_ref is merged, if no face or corner neighbour of its members is
//     finer than them in the mesh of step 2 (all such merges at once).
// New leaves in Morton order; rk/src: the regrid map of k_tree_regrid.
int tree_plan(const dg_ctx *c, const std::vector<int> &flags, int max_level, std::vector<int32_t> &next,
              std::vector<int> &rk, std::vector<int> &src) {
  const std::vector<int32_t> &lv = c->tleaves;
  const long nl = (long)lv.size() / 3;
  TreeIndex ix;
  std::vector<int> T;
  int st = tree_tables(c, lv, ix, T);
  if (st != DG_OK) return st;
  auto L = [&](long i) { return lv[3 * i]; };
  auto X = [&](long i) { return (long)lv[3 * i + 1]; };
  auto Y = [&](long i) { return (long)lv[3 * i + 2]; };
  std::vector<char> split((size_t)nl, 0);
  std::vector<long> work;
  for (long i = 0; i < nl; ++i) {
    if (!(flags[(size_t)i] & 1) || L(i) >= max_level) continue;
    if (!split[(size_t)i]) { split[(size_t)i] = 1; work.push_back(i); }
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy) {
        long xx = X(i) + dx, yy = Y(i) + dy;
        if ((dx == 0 && dy == 0) || !ix.wrap(L(i), xx, yy)) continue;
        const long j = ix.covering(L(i), xx, yy);
        if (j >= 0 && L(j) < max_level && !split[(size_t)j]) { split[(size_t)j] = 1; work.push_back(j); }
      }
  }
  while (!work.empty()) {
    const long i = work.back();
    work.pop_back();
    for (int dx = -1; dx <= 1; ++dx)
      for (int dy = -1; dy <= 1; ++dy) {
        long xx = X(i) + dx, yy = Y(i) + dy;
        if ((dx == 0 && dy == 0) || !ix.wrap(L(i), xx, yy)) continue;
        const long j = ix.covering(L(i), xx, yy);
        if (j >= 0 && L(j) < L(i) && !split[(size_t)j]) { split[(size_t)j] = 1; work.push_back(j); }
      }
  }
  // level of level-l cell (x, y) after step 2: finer than l -> l + 1
  auto level_after = [&](int l, long x, long y) {
    const long j = ix.covering(l, x, y);
    if (j < 0) return l + 1;
    return L(j) + split[(size_t)j];
  };
  std::vector<char> merge((size_t)nl, 0);
  for (long i = 0; i < nl; ++i) {
    if (!(flags[(size_t)i] & 4) || (flags[(size_t)i] & 2) || L(i) < 1) continue;
    const int *grp = T.data() + 13 * nl;
    if (grp[i] != i) continue;  // the group's child 0 decides
    bool ok = true;
    for (int ch = 0; ch < 4 && ok; ++ch) {
      const long m = grp[(long)ch * nl + i];
      if (split[(size_t)m] || (flags[(size_t)m] & 2)) { ok = false; break; }
      for (int dx = -1; dx <= 1 && ok; ++dx)
        for (int dy = -1; dy <= 1 && ok; ++dy) {
          long xx = X(m) + dx, yy = Y(m) + dy;
          if ((dx == 0 && dy == 0) || !ix.wrap(L(m), xx, yy)) continue;
          if (level_after(L(m), xx, yy) > L(m)) ok = false;
        }
    }
    if (ok)
      for (int ch = 0; ch < 4; ++ch) merge[(size_t)grp[(long)ch * nl + i]] = 1;
  }
  // new leaves with their sources, then Morton order
  std::vector<int32_t> nx;
  std::vector<int> k0, s0;  // kind | child << 2, and 4 sources
  for (long i = 0; i < nl; ++i) {
    if (split[(size_t)i]) {
      for (int ch = 0; ch < 4; ++ch) {
        nx.insert(nx.end(), {L(i) + 1, (int32_t)(2 * X(i) + (ch & 1)), (int32_t)(2 * Y(i) + (ch >> 1))});
        k0.push_back(1 | (ch << 2));
        s0.insert(s0.end(), {(int)i, -1, -1, -1});
      }
    } else if (merge[(size_t)i]) {
      const int *grp = T.data() + 13 * nl;
      if (grp[i] != i) continue;
      nx.insert(nx.end(), {L(i) - 1, (int32_t)(X(i) >> 1), (int32_t)(Y(i) >> 1)});
      k0.push_back(2);
      s0.insert(s0.end(), {grp[i], grp[nl + i], grp[2 * nl + i], grp[3 * nl + i]});
    } else {
      nx.insert(nx.end(), {L(i), (int32_t)X(i), (int32_t)Y(i)});
      k0.push_back(0);
      s0.insert(s0.end(), {(int)i, -1, -1, -1});
    }
  }
  std::vector<int> perm;
  tree_sort(nx, &perm);
  const long nn = (long)perm.size();
  rk.assign((size_t)nn, 0);
  src.assign((size_t)4 * nn, -1);
  for (long j = 0; j < nn; ++j) {
    const long i = perm[(size_t)j];
    rk[(size_t)j] = k0[(size_t)i];
    for (int e = 0; e < 4; ++e) src[(size_t)(e * nn + j)] = s0[(size_t)(4 * i + e)];
  }
  next.swap(nx);
  return DG_OK;
}

bool tree_ok(const dg_ctx *c) {
  return c->sh.d == 2 && c->sh.k <= 3 && !c->amr && !c->gravity && c->cfg.precision == DG_FP64;
}

template <class F>
int tree_dispatch(const dg_ctx *c, F &&f) {
  switch (c->sh.k) {
    case 1: return f.template run<1>();
    case 2: return f.template run<2>();
    case 3: return f.template run<3>();
    default: return DG_EUNSUPPORTED;
  }
}

struct TreeStage {
  dg_ctx *c;
  const double *w, *dt;
  double *out;
  int mode;
  dg::Mix mx;
  hipStream_t s;
  template <int K>
  int run() {
    const dg::TreeGrid g = make_tree_grid(c);
    if (c->cfg.flux == DG_HLLC_DAVIS)
      hipLaunchKernelGGL((dg::k_rhs_tree<K, DG_HLLC_DAVIS>), dim3(tree_blocks(g.nleaf)), dim3(kTreeBlock), 0, s,
                         c->tab, w, out, dt, g, mode, mx, c->flag);
    else
      hipLaunchKernelGGL((dg::k_rhs_tree<K, DG_HLLC_BATTEN>), dim3(tree_blocks(g.nleaf)), dim3(kTreeBlock), 0, s,
                         c->tab, w, out, dt, g, mode, mx, c->flag);
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
};

struct TreeFlags {
  dg_ctx *c;
  const double *w;
  double tc, tn;
  hipStream_t s;
  template <int K>
  int run() {
    const dg::TreeGrid g = make_tree_grid(c);
    hipLaunchKernelGGL((dg::k_tree_flags<K>), dim3(nblocks(g.nleaf)), dim3(kBlock), 0, s, w, c->prmat, g, tc, tn,
                       c->tflags);
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
};

struct TreeRegrid {
  dg_ctx *c;
  const double *wa;
  double *wb;
  long na, nb;
  hipStream_t s;
  template <int K>
  int run() {
    hipLaunchKernelGGL((dg::k_tree_regrid<K>), dim3(nblocks(nb)), dim3(kBlock), 0, s, wa, na, c->prmat, c->tmap,
                       c->tmap + nb, wb, nb);
    HIP_TRY(hipGetLastError());
    return DG_OK;
  }
};

struct TreeLimit {
  dg_ctx *c;
  double *w;
  hipStream_t s;
  template <int K>
  int run() {
    const dg::TreeGrid g = make_tree_grid(c);
    const bool posit = c->cfg.positivity != 0;
    // the positivity list's count is cleared by a kernel (no memset), so the
    // pass can be captured; with the slope limiter on, its two kernels clear
    // the count and fill the list themselves
    int *pl = posit ? c->tplist : nullptr;
    if (c->cfg.slope_limiter != DG_LIM_NONE) {
      hipLaunchKernelGGL((dg::k_tree_nbmean<K>), dim3(tree_blocks(g.nleaf)), dim3(kTreeBlock), 0, s, c->tab, w, g,
                         c->treg, c->tnbm, pl);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL((c->cfg.slope_limiter == DG_LIM_CHAR ? dg::k_limit_tree<K, true> : dg::k_limit_tree<K, false>),
                         dim3(tree_blocks(g.nleaf)), dim3(kTreeBlock), 0, s, w, g, c->tnbm, c->cfg.beta,
                         c->cfg.m_tilde, c->cfg.eps, c->flag, pl);
      HIP_TRY(hipGetLastError());
    } else if (posit) {
      hipLaunchKernelGGL(dg::k_zero_count, dim3(1), dim3(1), 0, s, c->tplist);
      HIP_TRY(hipGetLastError());
      hipLaunchKernelGGL((dg::k_tree_poscheck<K>), dim3(tree_blocks(g.nleaf)), dim3(kTreeBlock), 0, s, w, g,
                         c->cfg.eps, c->flag, c->tplist);
      HIP_TRY(hipGetLastError());
    }
    if (posit) {
      const unsigned nb = (unsigned)std::min<long>(1024, std::max<long>(1, (g.nleaf + 255) / 256));
      hipLaunchKernelGGL((dg::k_positivity_tree<K>), dim3(nb), dim3(kBlock), 0, s, c->tab, w, g, c->tplist,
                         c->cfg.eps);
      HIP_TRY(hipGetLastError());
    }
    return DG_OK;
  }
};

}  // namespace

extern "C" {

int dg_tree_limit(dg_ctx *c, double *w, void *stream) {
  if (!c || !w || !c->tree) return DG_EINVAL;
  return tree_dispatch(c, TreeLimit{c, w, (hipStream_t)stream});
}

int dg_tree_set(dg_ctx *c, int64_t nleaf, const int32_t *leaves) {
  if (!c || !leaves || nleaf < 1) return DG_EINVAL;
  if (!tree_ok(c)) return DG_EUNSUPPORTED;
  return tree_install(c, std::vector<int32_t>(leaves, leaves + 3 * nleaf));
}

int dg_tree_size(const dg_ctx *c, int64_t *nleaf) {
  if (!c || !nleaf || !c->tree) return DG_EINVAL;
  *nleaf = (int64_t)c->tleaves.size() / 3;
  return DG_OK;
}

int dg_tree_leaves(const dg_ctx *c, int32_t *leaves) {
  if (!c || !leaves || !c->tree) return DG_EINVAL;
  std::memcpy(leaves, c->tleaves.data(), c->tleaves.size() * sizeof(int32_t));
  return DG_OK;
}

int dg_tree_rhs(dg_ctx *c, const double *w, double *L, void *stream) {
  if (!c || !w || !L || w == L || !c->tree) return DG_EINVAL;
  return tree_dispatch(c, TreeStage{c, w, nullptr, L, 0, dg::Mix{}, (hipStream_t)stream});
}

int dg_tree_rk_stage(dg_ctx *c, int stage, const double *dt, const double *wn, const double *wp, double *out,
                     void *stream) {
  if (!c || !dt || !wp || !out || stage < 1 || stage > 3 || !c->tree) return DG_EINVAL;
  if (stage > 1 && !wn) return DG_EINVAL;
  if (out == wp || out == wn) return DG_EINVAL;
  return tree_dispatch(c, TreeStage{c, wp, dt, out, 1, rk3_mix(stage, wn), (hipStream_t)stream});
}

int dg_tree_max_dt(dg_ctx *c, const double *w, double *dt, void *stream) {
  if (!c || !w || !dt || !c->tree) return DG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const dg::TreeGrid g = make_tree_grid(c);
  unsigned long long *rm = reinterpret_cast<unsigned long long *>(c->partial);
  const unsigned nb = nblocks(g.nleaf) < 1024u ? nblocks(g.nleaf) : 1024u;
  hipLaunchKernelGGL(dg::k_rate_tree, dim3(nb), dim3(kBlock), 0, s, w, g, c->sh.N, rm, c->flag);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(dg::k_dt_final, dim3(1), dim3(64), 0, s, rm, c->cfl_fk, dt);
  HIP_TRY(hipGetLastError());
  return DG_OK;
}

int dg_tree_adapt(dg_ctx *c, const double *w, double wt, double alpha, int max_level, int64_t *nleaf_new,
                  void *stream) {
  if (!c || !w || !nleaf_new || !c->tree || !(wt > 0.0) || !(alpha >= 1.0) || max_level < 0 || max_level > 24)
    return DG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const long nl = (long)c->tleaves.size() / 3;
  int st = grow_ints(c->tflags, c->tflags_cap, nl);
  if (st != DG_OK) return st;
  st = tree_dispatch(c, TreeFlags{c, w, alpha * wt, wt / alpha, s});
  if (st != DG_OK) return st;
  std::vector<int> flags((size_t)nl);
  HIP_TRY(hipStreamSynchronize(s));
  HIP_TRY(hipMemcpy(flags.data(), c->tflags, (size_t)nl * sizeof(int), hipMemcpyDeviceToHost));
  std::vector<int32_t> next;
  st = tree_plan(c, flags, max_level, next, c->trk, c->tsrc);
  if (st != DG_OK) return st;
  c->tnext.swap(next);
  *nleaf_new = (int64_t)c->tnext.size() / 3;
  return DG_OK;
}

int dg_tree_regrid(dg_ctx *c, const double *w_old, double *w_new, void *stream) {
  if (!c || !w_old || !w_new || w_old == w_new || !c->tree || c->tnext.empty()) return DG_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const long na = (long)c->tleaves.size() / 3, nb = (long)c->tnext.size() / 3;
  HIP_TRY(hipStreamSynchronize(s));
  int st = grow_ints(c->tmap, c->tmap_cap, 5 * nb);
  if (st != DG_OK) return st;
  HIP_TRY(hipMemcpy(c->tmap, c->trk.data(), (size_t)nb * sizeof(int), hipMemcpyHostToDevice));
  HIP_TRY(hipMemcpy(c->tmap + nb, c->tsrc.data(), (size_t)4 * nb * sizeof(int), hipMemcpyHostToDevice));
  st = tree_dispatch(c, TreeRegrid{c, w_old, w_new, na, nb, s});
  if (st != DG_OK) return st;
  return tree_install(c, c->tnext);
}

}  // extern "C"
