// Internal declarations of libdg: table layout shared by the host set-up and
// the device kernels, and the context structure behind the opaque dg_ctx.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/dg.h"

namespace dg {

// Sizes of one (dim, k) discretisation.
struct Shape {
  int d, k;
  int n1;   // Gauss points per axis, k + 1
  int nv;   // conserved variables, d + 2
  int N;    // modes per variable
  int Q;    // volume nodes (k+1)^d
  int QF;   // nodes per face (k+1)^(d-1)
  int M;    // GLL points of the positivity rule, smallest m >= (k+3)/2
  int NS;   // positivity points per cell, d * M * QF
};

Shape make_shape(int d, int k);

// Offsets (in doubles) of the tables in one contiguous buffer:
//   B  [Q][N]        phi_l at the volume nodes
//   DW [d][Q][N]     d phi_l / d xi_a at the volume nodes, times the node weight
//   TF [d][2][QF][N] phi_l at the face nodes (side 0: xi_a = -1, side 1: +1)
//   TW [d][2][QF][N] TF times the face-node weight
//   WQ [Q]           volume-node weights
//   PS [NS][N]       phi_l at the positivity points
//   XQ [Q][3]        volume-node coordinates
//   HG [d][2][4][QF][N] coarse basis at the nodes of the 2^(d-1) fine faces
//                    covering a coarse face (static 2:1 refinement)
//   HW [d][2][4][QF][N] HG times the fine-face weight / 2^(d-1) (coarse lift)
//   CM [8][N]        mean of phi_l over each child subcell
struct Layout {
  int B, DW, TF, TW, WQ, PS, XQ, HG, HW, CM, total;
};

Layout make_layout(const Shape &s);

// Host tables for (d, k); also returns the first GLL weight.
std::vector<double> build_tables(const Shape &s, double *gll_w1);
std::vector<double> refine_matrices(const Shape &s);  // [2^d][N][N] (eq. ref_pa_integral)
std::vector<double> tables_1d(int k);  // 1D tables of the quadtree stage kernel (2D)

// Exponent triples of the modes in the library's mode order.
std::vector<int> mode_exponents(int d, int k);

}  // namespace dg

struct dg_ctx {
  dg_config cfg;
  dg::Shape sh;
  dg::Layout lay;
  long nx, ny, nz, ncell;
  double dx;
  double gll_w1;
  double cfl_fk;  // CFL times the order factor of the time step
  std::vector<double> host_tab;
  double *tab = nullptr;     // FP64 tables on the device
  float *tab32 = nullptr;    // FP32 copy
  void *tabbf = nullptr;     // BF16 tables of the MFMA volume kernel (padded)
  float *vscratch = nullptr; // volume term from the MFMA kernel (BF16 path)
  double *partial = nullptr; // rate slots of dg_max_dt (DG_RATE_STATE doubles)
  int npartial = 0;          // blocks of the time-step reduction
  int *flag = nullptr;       // sticky device error flag
  int device = 0;
  // static 2:1 refined box (amr = true): base grid nx,ny,nz is the coarse
  // block, base cells [lo, hi) are covered by the fine block of nf cells
  bool amr = false;
  int lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  long nf[3] = {1, 1, 1};
  long ncc = 0, ncf = 0;
  // time integrator of dg_tableau_stage / dg_tableau_step: stage m = 1..rk_s
  // of the tableau's Shu-Osher form, Y_m = sum_{j<m} rk_alpha[m][j] Y_j +
  // rk_beta[m] dt L(Y_{m-1}); SSP-RK3 (table RK_3) until dg_set_tableau
  int rk_s = 0;
  double rk_alpha[DG_MAX_STAGES + 1][DG_MAX_STAGES + 1] = {};
  double rk_beta[DG_MAX_STAGES + 1] = {};
  // external gravity (dg_set_gravity): (dx/2) w_q a at the volume nodes
  // [d][Q][ncell], the largest |a| per cell, and CFL f_k sqrt(2 gamma (gamma-1))
  bool gravity = false;
  double *grav = nullptr, *gmax = nullptr;
  double grav_k = 0.0;
  double *prmat = nullptr;  // refinement matrices on the device (dg_amr_flags, dg_amr_regrid)
  double *tabmf = nullptr;  // A-operand tables of the 3D MFMA stage kernel (null: the VALU kernel)
  float *tabmf32 = nullptr; // the same in FP32, rows in the FP32 MFMA's order (FP32 path)
  double *tablw = nullptr;  // FP64 mode-0 lift weights of the FP32 MFMA kernel
  void *tabvb = nullptr;    // BF16 volume operands of the fused BF16 MFMA kernel (3D, k = 2, 3)
  int *plist = nullptr;     // positivity: count, then the ids of the cells that need the point loop
  // 2D tile size: -1 automatic (dg::tile2d_small: 8x8 tiles for k <= 3, and
  // for k = 4 on grids with fewer 16x8 tiles than CUs), 0 always the large
  // tiles, 1 always 8x8 (dg_config.tile2d)
  int tile_small = -1;
  // 2D quadtree mesh (dg_tree_set): the leaves (level, ix, iy) on the host,
  // their device tables (level, face kinds, neighbours, sibling groups), and
  // the next mesh of dg_tree_adapt with its regrid map until dg_tree_regrid
  bool tree = false;
  std::vector<int32_t> tleaves, tnext;
  std::vector<int> trk, tsrc;
  int *ttab = nullptr, *tmap = nullptr, *tflags = nullptr, *treg = nullptr;
  int *tplist = nullptr;  // positivity: count, then the leaves that need the point loop
  long ttab_cap = 0, tmap_cap = 0, tflags_cap = 0, treg_cap = 0, tplist_cap = 0;
  double *tnbm = nullptr;  // limiters' neighbour values [4][nvar][nleaf]
  double *t1d = nullptr;   // 1D tables of the quadtree stage kernel (dg::tables_1d; 2D, k <= 3)
  long tnbm_cap = 0;
};
