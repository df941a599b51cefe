/*
 * dg.h -- C ABI of the MI355X modal discontinuous Galerkin library (libdg.so).
 *
 * The library evaluates the right-hand side of the semi-discrete modal DG
 * scheme for the compressible Euler equations on Cartesian cells and advances
 * it with the third-order SSP Runge-Kutta method, following Schaal et al.
 * (2015), "Astrophysical hydrodynamics with a high order discontinuous
 * Galerkin scheme and adaptive mesh refinement":
 *   - state and basis ............ Sec. 2.2 (eqs. solution_representation,
 *                                  weights, set_basis_functions)
 *   - right-hand side ............ Sec. 2.4 (eqs. dg_projected, dg_term2,
 *                                  dg_term3, spatial_discretisation)
 *   - time step .................. Sec. 2.5 (eq. time_step), Sec. 3.4
 *                                  (eq. time_step_pos)
 *   - SSP-RK3 .................... App. D (table RK_3)
 *   - limiters ................... Sec. 3.1, 3.2 (with App. E), 3.3, 3.4
 *   - other Runge-Kutta methods .. App. D (tables butcher, RK_2, RK_4)
 *   - gravity source and step .... Sec. 2.4 (eq. gravity_term), Sec. 2.5
 *   - adaptive refinement ........ Sec. 4.1-4.3 (eqs. cell_ref, node_ref,
 *                                  ref_pa_integral, ref_weights, deref_weights)
 *   - 2D quadtree meshes ......... Sec. 4 (leaves of any depth, hanging faces)
 * and a hand-written discrete adjoint of the right-hand side and of the
 * SSP-RK3 stages (not part of the paper).
 *
 * Conventions shared by every call:
 *   - A *state* is a device array of doubles with layout
 *     [nvar][N][nz][ny][nx] (x fastest; nz = 1 in 2D), nvar = dim + 2
 *     conserved variables (rho, m_x, m_y[, m_z], E) and N = N(k) modal
 *     weights per variable.  Modes are ordered by total degree, then by
 *     x-exponent descending, then by y-exponent descending, so mode 0 is the
 *     cell mean and modes 1..dim are the x, y(, z) slopes.  The scaled
 *     Legendre basis is orthonormal: (1/|K|) int_K phi_i phi_j = delta_ij.
 *   - The caller allocates and owns every state, dt and output buffer; the
 *     library never frees them.  The context owns its tables and scratch.
 *   - `stream` is a hipStream_t (0 = the null stream).  Calls enqueue work
 *     and return without synchronising; the time step stays on the device.
 *   - Outputs must not alias inputs unless a call says so.
 *   - One context may be used from one stream at a time.
 *   - Every call returns DG_OK (0) or a negative DG_E* code and never
 *     throws.  Conditions detected on the device (a non-positive mean
 *     density or pressure, a NaN) set a sticky flag read by dg_status().
 */
#ifndef DG_MI355X_H
#define DG_MI355X_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  DG_OK = 0,
  DG_EINVAL = -1,       /* invalid argument (bad config, null pointer, stage) */
  DG_EUNSUPPORTED = -2, /* dim, degree or option outside the built set       */
  DG_ENOMEM = -3,       /* device or host allocation failed                  */
  DG_EHIP = -4,         /* a HIP runtime call failed                         */
  DG_ENEGATIVE = -5,    /* a cell mean has rho <= eps or p <= eps             */
  DG_ENAN = -6,         /* a NaN appeared in a right-hand side                */
  DG_ESCRATCH = -7      /* input larger than the static scratch (dg_rhs_noalloc) */
};

/* Floats in the library's static device scratch (32 MiB per GPU, held from
 * the library's load until the process ends). */
#define DG_STATIC_SCRATCH_FLOATS (8 * 1024 * 1024)

enum { DG_BC_PERIODIC = 0, DG_BC_TRANSMISSIVE = 1 };
enum { DG_HLLC_BATTEN = 0, DG_HLLC_DAVIS = 1 };
enum { DG_FP64 = 0, DG_FP32 = 1, DG_BF16_VOL = 2 };
enum { DG_LIM_NONE = 0, DG_LIM_MINMOD = 1, DG_LIM_CHAR = 2 };
enum { DG_TILE2D_AUTO = 0, DG_TILE2D_8X8 = 1, DG_TILE2D_LARGE = 2 };
enum { DG_PATH3D_AUTO = 0, DG_PATH3D_VALU = 1 };

typedef struct dg_ctx dg_ctx;

/* Run description (all fields read by dg_init only). */
typedef struct {
  int dim;            /* 2 or 3                                              */
  int k;              /* polynomial degree, 1..3 (spatial order k+1); 4 on 2D
                         grids without refinement in DG_FP64 or DG_FP32     */
  int n[3];           /* cells per axis (n[2] ignored in 2D)                  */
  double x0[3];       /* lower corner of the box                              */
  double len[3];      /* box edge lengths; cells must be cubes (len/n equal)  */
  double gamma;       /* adiabatic index of the ideal-gas EOS (eq. eos)       */
  double cfl;         /* CFL number of eq. time_step                          */
  int bc[3];          /* DG_BC_* per axis                                     */
  int flux;           /* DG_HLLC_BATTEN (Roe-averaged speed bounds) or DAVIS  */
  int precision;      /* DG_FP64, DG_FP32 (contractions and fluxes in FP32),
                         DG_BF16_VOL (volume contraction BF16 on MFMA, faces
                         FP32; on 3D grids at k = 2, 3 fused into the FP32
                         MFMA stage kernel, else a separate volume pass)     */
  int slope_limiter;  /* DG_LIM_NONE, DG_LIM_MINMOD (component-wise, TVB,
                         Sec. 3.1) or DG_LIM_CHAR (characteristic, TVB,
                         Sec. 3.2 with the App. E eigenvectors)               */
  double beta;        /* minmod parameter beta in [0.5, 1] (Sec. 3.1)          */
  double m_tilde;     /* TVB bound Mtilde; slopes |a| <= Mtilde dx kept (3.3)  */
  int positivity;     /* 1: Zhang-Shu positivity limiter (Sec. 3.4)            */
  double eps;         /* positivity floor (the paper uses about 1e-10)         */
  int refine_lo[3];   /* static 2:1 refined box: the base cells [lo, hi) per   */
  int refine_hi[3];   /* axis are covered by 2(hi-lo) fine cells per axis of   */
                      /* half the edge (Sec. 4); lo == hi (e.g. all zero) for  */
                      /* a uniform grid.  Requires 1 <= lo < hi <= n-1.        */
  int tile2d;         /* 2D uniform grids: cell tile of the stage kernel,      */
                      /* DG_TILE2D_AUTO (0, the rule of dg_init),              */
                      /* DG_TILE2D_8X8 or DG_TILE2D_LARGE (16 x 16 for k <= 2, */
                      /* 16 x 8 for k = 3, 4); results equal to rounding       */
  int path3d;         /* 3D, k = 2 or 3, no gravity: DG_PATH3D_AUTO (0) runs   */
                      /* the stage kernel's contractions on MFMA: FP64 on     */
                      /* FP64 MFMA; FP32 on FP32 MFMA at k = 3 and on refined */
                      /* boxes (FP32 at k = 2 on a uniform grid keeps the     */
                      /* one-thread-per-cell kernel, faster there);           */
                      /* DG_PATH3D_VALU runs them on the vector ALU (one      */
                      /* thread per cell; FP64 at k = 3 four lanes per cell); */
                      /* results equal to rounding                            */
} dg_config;

/* Builds the basis and quadrature tables (Gauss-Legendre nodes by Newton
 * iteration, App. B; GLL nodes, App. C; scaled Legendre values, App. A) and,
 * for k <= 3, the refinement matrices of Sec. 4.2 (eq. ref_pa_integral),
 * copies them to the current device and allocates scratch.  Host-to-device
 * copies happen here only.  *out receives the context.  With
 * cfg->tile2d = DG_TILE2D_AUTO, on 2D grids without refinement the stage
 * kernel works on tiles of 8 x 8 cells for k <= 3; at k = 4 on tiles of
 * 16 x 8 cells, or of 8 x 8 when the grid has fewer 16 x 8 tiles than the GPU
 * has compute units.  DG_EUNSUPPORTED for a base grid or a fine block of more
 * than 2^31 cells (kernels index a block's cells in 32 bits). */
int dg_init(const dg_config *cfg, dg_ctx **out);

/* Number of doubles in one state array (nvar * N * cells). */
int dg_state_size(const dg_ctx *ctx, int64_t *n_fp64);

/* Sizes: out[0..5] = nvar, N, Q (volume nodes), Qf (face nodes), cells, nS
 * (positivity check points per cell).  With a refined box, cells counts
 * both blocks. */
int dg_sizes(const dg_ctx *ctx, int64_t out[6]);

/* Refined-box geometry: out[0] = cells of the coarse block (the base grid,
 * hole included), out[1] = cells of the fine block, out[2..4] = fine block
 * cells per axis (0 without a refined box).  With a refined box a state is
 * the coarse block [nvar][N][coarse cells] followed by the fine block
 * [nvar][N][fine cells]; the hole cells of the coarse block are ignored.
 * Coarse faces next to the fine block are integrated at the Gauss points of
 * the fine faces that cover them (Sec. 4, hanging faces); the limiters use
 * the projected neighbour means of Sec. 4.4.  The adjoint calls return
 * DG_EUNSUPPORTED with a refined box. */
int dg_amr_sizes(const dg_ctx *ctx, int64_t out[5]);

/* Reference coordinates of the (k+1)^dim Gauss volume nodes, xi[Q][3]
 * (x index fastest; unused axes 0), and their weights w[Q] (host memory). */
int dg_quadrature(const dg_ctx *ctx, double *xi, double *w);

/* L2 projection of initial data (Sec. 2.3): prim is a device array
 * [5][Q][cells] of primitive values (rho, v_x, v_y, v_z, p) at the Gauss
 * volume nodes of every cell (with a refined box: the coarse block's cells,
 * then the fine block's; on a quadtree mesh set by dg_tree_set: the leaves
 * in mesh order); w receives the state. */
int dg_project(dg_ctx *ctx, const double *prim, double *w, void *stream);

/* L = dw/dt = -R_K of eq. spatial_discretisation for every cell: volume
 * integral (eq. dg_term2) minus surface integral (eq. dg_term3) with the HLLC
 * flux, times (2/dx) 2^-dim.  w and L are states; L must not alias w. */
int dg_rhs(dg_ctx *ctx, const double *w, double *L, void *stream);

/* dg_rhs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same kernels and result as dg_rhs on a DG_BF16_VOL context, with the FP32
 * volume term that dg_rhs keeps in the context's scratch held instead in
 * the library's static device scratch of DG_STATIC_SCRATCH_FLOATS floats
 * (3D grids at k = 2, 3 with path3d = DG_PATH3D_AUTO keep the volume term in
 * registers of the fused stage kernel and use no scratch at all).
 * The call allocates nothing and frees nothing.  Where it stages the volume
 * term it needs nvar * N * cells (both blocks with a refined box) <=
 * DG_STATIC_SCRATCH_FLOATS, else it returns DG_ESCRATCH; DG_EINVAL for a
 * context of another precision.  Every
 * call on one GPU shares that GPU's scratch, so calls that overlap in time
 * on one GPU (different streams, or different host threads) race and must
 * be ordered by the caller; each call writes every scratch entry it reads
 * before reading it. */
int dg_rhs_noalloc(dg_ctx *ctx, const double *w, double *L, void *stream);

/* Global time step of eq. time_step (eq. time_step_pos with the positivity
 * limiter) from the cell means of w, written to dt_dev[0] on the device. */
int dg_max_dt(dg_ctx *ctx, const double *w, double *dt_dev, void *stream);

/* One SSP-RK3 stage in convex-combination form (App. D, table RK_3):
 *   stage 1: w_out = w_prev + dt L(w_prev)              (w_n unused)
 *   stage 2: w_out = 3/4 w_n + 1/4 (w_prev + dt L(w_prev))
 *   stage 3: w_out = 1/3 w_n + 2/3 (w_prev + dt L(w_prev))
 * dt is read from dt_dev[0].  w_out must not alias w_prev or w_n. */
int dg_rk_stage(dg_ctx *ctx, int stage, const double *dt_dev, const double *w_n,
                const double *w_prev, double *w_out, void *stream);

/* Doubles in the rate state that dg_max_rate writes and dg_rk_step carries:
 * 8 slots at a stride of 16 doubles (one 128-byte line each, so that
 * workgroups on different XCDs fold into different lines).  Each slot holds
 * a partial maximum of the signal rate; the rate of the state is the largest
 * slot (slots are non-negative doubles).  Which slot holds the overall
 * maximum depends on the kernel that wrote the state. */
#define DG_RATE_STATE 128

/* Maximum over cells of the signal rate sum_a (|v_a| + c)/dx of the cell
 * means of w (the denominator of eq. time_step), written as a rate state
 * (DG_RATE_STATE doubles on the device, caller-owned): the input dg_rk_step
 * expects for the state it starts from.  Sets DG_ENEGATIVE for a
 * non-positive mean density or pressure. */
int dg_max_rate(dg_ctx *ctx, const double *w, double *rate_dev, void *stream);

/* One full SSP-RK3 step (App. D, table RK_3) with the configured limiters
 * after every stage (Sec. 4.5 without refinement):
 *   dt = CFL f_k / (maximum signal rate of w)  (eq. time_step / time_step_pos),
 *   u1 = stage 1 of w, u2 = stage 2, w_out = stage 3.
 * On entry rate_dev (DG_RATE_STATE doubles) must hold the rate state of w, as
 * written by dg_max_rate(w) or by the dg_rk_step that produced w; on return
 * it holds that of w_out (the limiters keep cell means, so it is also the
 * rate of the limited state), so that steps chain without a separate
 * time-step pass.  dt_dev[0] receives the step's dt.  Results equal
 * dg_max_dt, three dg_rk_stage and dg_limit calls bit for bit.  w, u1, u2
 * and w_out must be four distinct states, dt_dev and rate_dev distinct;
 * otherwise DG_EINVAL.  On a 2D grid without refinement the time-step work
 * rides in the three stage kernels; elsewhere two small kernels carry it.
 * Two calls that share rate_dev must not run concurrently. */
int dg_rk_step(dg_ctx *ctx, const double *w, double *u1, double *u2, double *w_out,
               double *dt_dev, double *rate_dev, void *stream);

/* Most stages of a time integrator given to dg_set_tableau. */
#define DG_MAX_STAGES 5

/* Time integrator of dg_tableau_stage and dg_tableau_step: the explicit
 * Runge-Kutta method of the Butcher tableau (App. D, table butcher: w^{n+1} =
 * w^n + dt sum_i b_i k_i, k_i = L(w^n + dt sum_{j<i} a_ij k_j)), e.g. table
 * RK_2 (Heun), RK_3 or the five-stage RK_4.  a is stages x stages, row-major,
 * host memory, strictly lower triangular (entries on or above the diagonal
 * must be zero); b has `stages` entries.  The method is run in its Shu-Osher
 * form with a derivative term on the previous stage only,
 *   Y_0 = w^n,  Y_m = sum_{j<m} alpha_mj Y_j + beta_m dt L(Y_{m-1}),  w^{n+1} = Y_s,
 * whose stage values Y_m are what the limiters act on (the main loop of
 * Sec. 4.5 limits after every stage); the form exists and is unique when
 * a_{i+1,i} != 0 for every i and b_s != 0.  Returns DG_EINVAL for a NULL
 * pointer, stages outside 1..DG_MAX_STAGES, a non-finite entry, an entry on
 * or above the diagonal, or a zero a_{i+1,i} or b_s; the previous integrator
 * is then kept.  Host-only: enqueues nothing.  dg_init sets table RK_3;
 * dg_rk_stage and dg_rk_step are SSP-RK3 whatever is set here. */
int dg_set_tableau(dg_ctx *ctx, int stages, const double *a, const double *b);

/* Stage value Y_m (1 <= m <= stages) of the integrator set by
 * dg_set_tableau: y is a host array of m device pointers to the states Y_0
 * (= w^n) .. Y_{m-1}; out receives Y_m; dt_dev is the step on the device.
 * Unlimited.  out must differ from every y[j]; otherwise, or for a NULL
 * pointer or m out of range, DG_EINVAL. */
int dg_tableau_stage(dg_ctx *ctx, int m, const double *dt_dev, const double *const *y, double *out,
                     void *stream);

/* One full step of the integrator set by dg_set_tableau with the configured
 * limiters after every stage, like dg_rk_step: dt from the rate carried in
 * rate_dev (written to dt_dev), the stage values into stage[0..s-2] (a host
 * array of s-1 device states; may be NULL when s = 1), w^{n+1} into w_out,
 * and rate_dev updated for the next step.  w, the stage states and w_out
 * must all be distinct, dt_dev outside rate_dev; otherwise DG_EINVAL.  On a
 * 2D grid without refinement (and s >= 2) the time-step work rides in the
 * first and last stage kernels. */
int dg_tableau_step(dg_ctx *ctx, const double *w, double *const *stage, double *w_out, double *dt_dev,
                    double *rate_dev, void *stream);

/* External gravity: the source s = (0, rho a, m . a) of eq. gravity_term
 * (Sec. 2.4), projected with the volume rule, is added to the right-hand side
 * of every later dg_rhs / stage / step call, and the time step becomes the
 * smaller of the CFL step and c / (sqrt(2 gamma (gamma-1)) |grad Phi|) per
 * cell (Sec. 2.5; c of the cell mean, |grad Phi| the largest over the cell's
 * volume nodes).  accel: device array of the acceleration a = -grad Phi at
 * the volume nodes, [dim][Q][ncell] with the node order of dg_quadrature; it
 * is read on `stream` before the call's work completes and may be freed or
 * reused after that; NULL switches gravity off.  The library keeps its own
 * copy (allocated on the first call: dim * Q + 1 doubles per cell).
 * DG_EUNSUPPORTED for a refined box, a precision other than DG_FP64, or 3D
 * with k = 3; dg_adjoint_rhs and dg_adjoint_rk_stage return DG_EUNSUPPORTED
 * while gravity is on. */
int dg_set_gravity(dg_ctx *ctx, const double *accel, void *stream);

/* Refinement criterion on the one-box mesh (Sec. 4.1): flags[b] = 1 for
 * each base cell b that should be refined: an unrefined base cell if its
 * largest density slope coefficient |w_rho,1+a| (the change across the half
 * cell over sqrt(3)) exceeds alpha * wt (eq. cell_ref); a refined one if that
 * of its node weights, the derefined projection of its children (eq.
 * deref_weights), exceeds wt / alpha (eq. node_ref).  flags: device, one int
 * per base cell (base-grid order, x fastest); box: device, 6 ints, receives
 * the refined box of the next mesh in refine_lo[3], refine_hi[3] form: the
 * range of the flagged cells grown by one buffer layer of cells on every
 * side (Sec. 4: the neighbours of a refined cell are refined too, which
 * keeps the level jump across every face at one), clipped to [1, n-1]; all
 * six zero when no cell is flagged or the clipped range is empty (2D: the
 * z entries are zero).  Pass it to dg_init's refine_lo / refine_hi and move
 * the state with dg_amr_regrid.  The paper's values are wt = 0.01,
 * alpha = 1.1.  DG_EINVAL for wt <= 0 or alpha < 1; DG_EUNSUPPORTED for
 * k = 4. */
int dg_amr_flags(dg_ctx *ctx, const double *w, double wt, double alpha, int *flags, int *box, void *stream);

/* Moves a state between two meshes over the same base grid (same dim, k,
 * cells, edge and origin; each with or without a refined box): a base cell
 * that stays unrefined is copied, one that leaves the box is derefined from
 * its children by L2 projection (Sec. 4.3 eq. deref_weights), the children
 * of a newly refined base cell are the L2 projections of its polynomial
 * (Sec. 4.2 eq. ref_weights), children present in both boxes are copied.
 * Hole cells of the new mesh are set to zero.  Mass, momentum and energy
 * are kept to rounding.  w_to must not alias w_from; DG_EINVAL for meshes
 * that do not share the base grid. */
int dg_amr_regrid(const dg_ctx *from, const double *w_from, dg_ctx *to, double *w_to, void *stream);

/* Slope limiter (minmod with TVB bound, Sec. 3.3: component-wise on the
 * conserved variables, Sec. 3.1, or on the characteristic variables of the
 * cell mean, Sec. 3.2 eq. char_limiter) then positivity limiter (Sec. 3.4),
 * in place, as configured.  Cell means are never changed.  A cell whose mean
 * density or pressure is <= eps sets the DG_ENEGATIVE flag and is left
 * unlimited; the characteristic limiter also leaves alone a mean without a
 * positive density and pressure.  With positivity on, the call runs the
 * point loop of the cells it cannot prove positive in a second pass, through
 * a list in the context: calls on one context (dg_limit, dg_rk_step,
 * dg_tableau_step) must be ordered, not overlapped on different streams. */
int dg_limit(dg_ctx *ctx, double *w, void *stream);

/* Discrete adjoint of dg_rhs: mu = (dL/dw)^T lam at the state w (all
 * states).  Exact transpose of the discrete operator, including the HLLC
 * branch taken at w.  mu must not alias w or lam. */
int dg_adjoint_rhs(dg_ctx *ctx, const double *w, const double *lam, double *mu, void *stream);

/* Transpose of one SSP-RK3 stage, applied from stage 3 down to stage 1 with
 * u the stage input state of that stage (u0, u1, u2) and dt fixed:
 *   stage 3: lam_out = 2/3 (lam + dt J(u)^T lam);  acc_out = 1/3 lam
 *   stage 2: lam_out = 1/4 (lam + dt J(u)^T lam);  acc_out = acc + 3/4 lam
 *   stage 1: lam_out = acc + lam + dt J(u)^T lam    (acc_out unused)
 * where J = dL/dw.  After stage 1, lam_out is dJ/dw_n of the step. */
int dg_adjoint_rk_stage(dg_ctx *ctx, int stage, const double *dt_dev, const double *u,
                        const double *lam, const double *acc, double *lam_out,
                        double *acc_out, void *stream);

/* ---- 2D quadtree meshes (Sec. 4) ------------------------------------------
 * A tree-based mesh of leaf cells: every cell can be split into four children
 * at any level (Sec. 4), leaf (level, ix, iy) covering
 * [x0 + ix h, x0 + (ix+1) h) x [y0 + iy h, y0 + (iy+1) h) with h = dx / 2^level
 * over the context's base grid (level 0).  Once dg_tree_set has given a
 * context a tree, the grid calls above (dg_rhs, dg_rk_stage, dg_max_dt,
 * dg_max_rate, dg_rk_step, dg_tableau_*, dg_limit, dg_set_gravity,
 * dg_amr_*, dg_adjoint_*, dg_rhs_noalloc) return DG_EINVAL on it, and
 * dg_state_size and dg_project count leaves.  Across a face the level jump is
 * at most one: a side has one neighbour or two finer ones, whose faces are
 * integrated with the coarse trace at the mapped nodes (eta + sigma)/2 and the
 * weight w_r / 2 on the coarse side (Sec. 4).  A tree *state* is a device
 * array [nvar][N][nleaf] in leaf order, same modes as above.  FP64, dim = 2,
 * k = 1..3, no refined box, no gravity (else DG_EUNSUPPORTED). */

/* Makes `leaves` (host, [nleaf][3] ints: level, ix, iy; any order) the
 * context's mesh.  DG_EINVAL unless the leaves tile the base grid without
 * overlap and every face sees a level jump of at most one (periodic axes
 * wrap).  Builds and uploads the neighbour tables: allocates on growth and
 * waits for the device to be idle (a mesh change, not a per-step call). */
int dg_tree_set(dg_ctx *ctx, int64_t nleaf, const int32_t *leaves);

/* Number of leaves of the current mesh, and the leaves themselves (host
 * [nleaf][3]: level, ix, iy, in the mesh's order). */
int dg_tree_size(const dg_ctx *ctx, int64_t *nleaf);
int dg_tree_leaves(const dg_ctx *ctx, int32_t *leaves);

/* dw/dt on every leaf (Sec. 2.4 eqs. dg_term2, dg_term3 with each leaf's own
 * edge in the factor (2/h) 2^-d; hanging faces as above).  L must not alias w. */
int dg_tree_rhs(dg_ctx *ctx, const double *w, double *L, void *stream);

/* One SSP-RK3 stage (App. D, table RK_3) on the tree, as dg_rk_stage. */
int dg_tree_rk_stage(dg_ctx *ctx, int stage, const double *dt_dev, const double *w_n,
                     const double *w_prev, double *w_out, void *stream);

/* Time step of the tree (Sec. 2.5 eq. time_step with each leaf's own edge):
 * CFL f_k / max over leaves of sum_a (|v_a| + c)/h into the device scalar. */
int dg_tree_max_dt(dg_ctx *ctx, const double *w, double *dt_dev, void *stream);

/* Slope limiter then positivity limiter on the tree, in place, as
 * configured (as dg_limit), with the AMR rules of Sec. 4.4: the neighbour
 * value on each side of a leaf is the mean of the solution over the cell of
 * the leaf's own size there (a same-level leaf's mean, a coarser leaf's
 * polynomial averaged over that cell, or the area-weighted means of the finer
 * leaves inside it), all taken from the state before limiting; the TVB bound
 * uses the leaf's own edge; a leaf with finer neighbours also checks
 * positivity at its trace points on the half faces to them.  A mean density
 * or pressure <= eps sets the DG_ENEGATIVE flag and is left alone.  Uses the
 * context's neighbour-value scratch: calls on one context must be ordered. */
int dg_tree_limit(dg_ctx *ctx, double *w, void *stream);

/* Plans the next mesh (Sec. 4.1): on the device, per leaf, the refinement
 * criterion max_a |w_rho,1+a| > alpha wt (eq. cell_ref) and, for a complete
 * group of four sibling leaves, whether its node weights (eq. deref_weights)
 * keep it refined, max_a > wt / alpha (eq. node_ref); then on the host:
 * flagged leaves below max_level are split together with the neighbour
 * leaves of the same or a coarser level among their eight face and corner
 * neighbours (the buffer layer of Sec. 4); splits propagate to coarser face
 * and corner neighbours until every jump is at most one; a complete group of
 * unsplit siblings that fails eq. node_ref and has no finer face or corner
 * neighbour is merged.  New leaves are in Morton order of their lower-left
 * corners.  Synchronises `stream`; *nleaf_new receives the new count: the
 * caller allocates the new state and calls dg_tree_regrid.  The paper's
 * values are wt = 0.01, alpha = 1.1.  DG_EINVAL for wt <= 0, alpha < 1 or
 * max_level outside 0..24. */
int dg_tree_adapt(dg_ctx *ctx, const double *w, double wt, double alpha, int max_level,
                  int64_t *nleaf_new, void *stream);

/* Moves the state onto the mesh planned by dg_tree_adapt and makes that mesh
 * current: kept leaves are copied, children of a split leaf are the L2
 * projections of its polynomial (Sec. 4.2 eq. ref_weights), a merged group
 * becomes the projection of its four children (Sec. 4.3 eq. deref_weights).
 * w_new ([nvar][N][nleaf_new]) must not alias w_old.  Synchronises. */
int dg_tree_regrid(dg_ctx *ctx, const double *w_old, double *w_new, void *stream);

/* Synchronises `stream`, returns the sticky device flag (DG_OK,
 * DG_ENEGATIVE or DG_ENAN) and clears it. */
int dg_status(dg_ctx *ctx, void *stream);

/* Frees the context's device tables and scratch. */
void dg_destroy(dg_ctx *ctx);

/* Static description of an error code. */
const char *dg_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* DG_MI355X_H */
