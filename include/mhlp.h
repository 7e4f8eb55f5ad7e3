/*
 * mhlp.h -- C ABI of the modified-Helmholtz layer-potential library (gfx950).
 *
 * Computes, for a closed (possibly multiply connected) boundary discretised by
 * composite 16-point Gauss-Legendre panels (af Klinteberg, Askham & Kropinski,
 * "A fast integral equation method for the two-dimensional Navier-Stokes
 * equations", Sec. 3.2), the Yukawa single- and double-layer potentials
 *
 *   S[sigma](x) = int_Gamma K0(alpha |x-y|)/(2 pi) sigma(y) dS_y
 *   D[mu](x)    = int_Gamma alpha K1(alpha r) (x-y).n_y / (2 pi r) mu(y) dS_y,
 *
 * (K0/2pi is the Yukawa part of the paper's modified-biharmonic Green's
 * function, Sec. 2 and App. B), with the near-field panel corrections of
 * Sec. 4, the on-surface second-kind operator (1/2 I + D) of Sec. 3.2 (the
 * jump relation of the paper's Lemma on jump conditions, inward normal) and
 * GMRES for (1/2 I + D) mu = g (Sec. 3.2).
 *
 * Conventions
 *  - Geometry: N = 16 * n_panels nodes, panel-major, local parameter t
 *    ascending inside a panel; each curve is oriented with the domain on its
 *    left, so n = i tau'/|tau'| points into the domain.
 *  - All array pointers are DEVICE pointers owned by the caller unless marked
 *    "host".  The library owns the opaque handles and their workspaces
 *    (allocated at create, freed at destroy).
 *  - `stream` is a hipStream_t passed as void*; all work is enqueued on it.
 *    Calls return after enqueueing unless documented as synchronising.
 *  - Every call returns an mhlp_status.  No exception crosses the ABI.  On
 *    error mhlp_last_error() returns a thread-local message.  Inputs are
 *    validated before anything is enqueued.
 *  - Handles are bound to the device current at creation and are not safe
 *    for concurrent use from several threads.
 */
#ifndef MHLP_H
#define MHLP_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t mhlp_status;
#define MHLP_OK 0
#define MHLP_NOT_CONVERGED 1 /* soft: GMRES stopped before the tolerance   */
#define MHLP_INVALID_ARG (-1)
#define MHLP_HIP_ERROR (-2)
#define MHLP_UNSUPPORTED (-3)
#define MHLP_NO_MEMORY (-4)

/* Arithmetic of the far-field direct sum.  Near-field corrections, the
   identity term and GMRES orthogonalisation are FP64 in both modes. */
#define MHLP_FP64 0
#define MHLP_MIXED 1 /* FP32 far field with compensated accumulation */

typedef struct mhlp_geometry mhlp_geometry;
typedef struct mhlp_plan mhlp_plan;

/* Near-field parameters (Sec. 4.5).  Zero fields take the paper's values. */
typedef struct {
    double near_factor; /* candidate panels: some node within near_factor*h   (1.2)      */
    double rho_direct;  /* Bernstein radius beyond which 16-point GL is used  (3.5)      */
    double rho_split;   /* below: kernel split on the 32-point panel          (sqrt 3.5) */
    double ah_max;      /* panels with alpha*h above are subdivided            (4.5)      */
    double far_exp;     /* subpanels with alpha*dist beyond are plain GL       (40)       */
} mhlp_params;

typedef struct {
    double tol;         /* stop when ||g - A mu||_2 / ||g||_2 <= tol (true residual) */
    int32_t max_iter;   /* total Arnoldi steps                                        */
    int32_t restart;    /* Krylov dimension before a restart (<= 512)                 */
    int32_t precision;  /* MHLP_FP64 or MHLP_MIXED (mixed: FP32 far-field inner solves
                           inside FP64 iterative refinement: each cycle's Arnoldi steps
                           use the FP32 far field and stop at 0.5e-6 of the residual
                           the cycle started from; each cycle ends with the FP64 true
                           residual, from which the next starts)                      */
    int32_t use_x0;     /* 1: mu holds the initial guess on entry; 0: zero guess      */
} mhlp_gmres_opts;

typedef struct {
    int32_t iters;        /* Arnoldi steps taken                                   */
    int32_t restarts;     /* outer cycles (restarts or refinement steps)           */
    double rel_residual;  /* true ||g - A mu|| / ||g|| at exit (FP64 operator)     */
    double x0_residual;   /* true relative residual of the initial guess           */
    int32_t converged;    /* 1 if rel_residual <= tol                              */
    int32_t used_x0;      /* 0 if the initial guess was rejected (residual >= 1)   */
} mhlp_gmres_info;

const char *mhlp_last_error(void);

/* Geometry of the composite panel discretisation (Sec. 3.2: each of the
   closed curves of the boundary is divided into panels carrying 16
   Gauss-Legendre nodes; with the interpolation of Sec. 4.5.3 we take a
   panel to be the degree-15 polynomial through its nodes, so node data
   determine it).
   n_curves >= 1 closed curves; curve_panel_offsets: HOST [n_curves + 1],
   curve c owns panels offsets[c] .. offsets[c+1]-1 (offsets[0] = 0,
   strictly increasing; Np = offsets[n_curves]).  nodes_per_panel: 16 (other
   values MHLP_UNSUPPORTED).  node_soa: device [6][N], N = 16 Np, rows x, y,
   dx/dt, dy/dt, d2x/dt2, d2y/dt2 with derivatives in the panel parameter
   t in [-1,1], panels in curve order, each curve oriented with the domain
   on its left.  panel_ends: device [4][Np] (xa, ya, xb, yb: the points
   t = -1 and t = 1 of each panel) or NULL; when given they are checked, not
   used: each must lie within 1e-6 of the panel's arclength of the node
   polynomial's end, and the end of every panel within that of the start of
   the next panel of its curve (the last panel of a curve is followed by
   its first), else MHLP_INVALID_ARG naming the panel.  The library copies
   everything it needs; the caller may free its arrays on return.
   Synchronises the stream.  Errors: MHLP_INVALID_ARG (null pointers, bad
   offsets, panel_ends inconsistent), MHLP_UNSUPPORTED, MHLP_HIP_ERROR,
   MHLP_NO_MEMORY. */
mhlp_status mhlp_geometry_create(int32_t n_curves, const int32_t *curve_panel_offsets, int32_t nodes_per_panel,
                                 const double *node_soa, const double *panel_ends, void *stream,
                                 mhlp_geometry **out);
/* Sizes and curve offsets of a geometry (host outputs, any may be NULL;
   curve_panel_offsets receives at most cap entries). */
mhlp_status mhlp_geometry_info(const mhlp_geometry *geom, int64_t *n_nodes, int64_t *n_panels, int32_t *n_curves,
                               int32_t *curve_panel_offsets, int32_t cap);
mhlp_status mhlp_geometry_destroy(mhlp_geometry *geom);
/* Device views (valid for the geometry's lifetime): per-node quadrature
   weight, unit normal (x, y) and signed curvature. Any output may be NULL. */
mhlp_status mhlp_geometry_arrays(const mhlp_geometry *geom, const double **w, const double **nx, const double **ny,
                                 const double **kappa);

/* Plan: targets plus precomputed near-field correction weights (Sec. 4.5:
   candidate panels within 1.2 h, Newton preimage, Bernstein-radius tiers,
   kernel split, subdivision for alpha h > 4.5).  tx, ty: device [m] float64.
   m == 0 builds the on-surface plan (targets are the nodes; needed by
   apply_bie_operator and gmres_solve).  params: host, NULL = paper values.
   Synchronises the stream.  Errors: MHLP_INVALID_ARG (alpha <= 0 or not
   finite, null targets with m > 0), MHLP_HIP_ERROR, MHLP_NO_MEMORY. */
mhlp_status mhlp_plan_create(const mhlp_geometry *geom, double alpha, const double *tx, const double *ty, int64_t m,
                             const mhlp_params *params, void *stream, mhlp_plan **out);
mhlp_status mhlp_plan_destroy(mhlp_plan *plan);
/* Plan statistics (host outputs; any may be NULL). */
mhlp_status mhlp_plan_info(const mhlp_plan *plan, int64_t *n_targets, int64_t *n_sources, int64_t *n_near_pairs,
                           double *alpha);

/* Far-field launch shape.  The mixed-precision far field, the gradients and
   the stresslet split the direct sum over sources into nsplit ranges of
   panels evaluated by separate blocks (partial sums added in fixed order, so
   results do not depend on nsplit beyond rounding); the default aims at about
   8192 blocks of 256 targets with at least 2 panels per split.  The FP64
   single and double layers do not use it: they run as a stream of
   (256 targets, one panel) units spread evenly over one launch of as many
   blocks as the chip holds, and the FP64 double layer of an on-surface scalar
   plan of up to 8192 nodes (the BIE operator, GMRES) evaluates each unordered
   pair once on tiles of its own.  set_split may reallocate the plan's
   partial-sum buffer (it synchronises the device then).
   mhlp_plan_autotune times the far evaluation (layers: 1 SLP, 2 DLP, 3 both,
   4 the on-surface BIE operator, 5 the gradients of both, off-surface, 6 the
   stresslet operator of a stokes plan, 7 the stresslet target gradient of an
   off-surface stokes plan) for nsplit = 1, 2, 4, ... (up to Np and 256)
   plus the current value, reps timed launches each after one warm-up,
   with HIP events on `stream`, keeps the fewest splits within 1% of the
   fastest and reports it with its time (host outputs; cand/cand_ms receive up
   to cap candidates and their ms per launch).  Where the FP64 launch does not
   use the split (layers 1-3, and 4 on a symmetric on-surface plan), FP64
   requests time the MIXED launch of the same layers, the one the split
   serves.  Synchronises the stream.  Errors: MHLP_INVALID_ARG. */
mhlp_status mhlp_plan_set_split(mhlp_plan *plan, int32_t nsplit);
mhlp_status mhlp_plan_get_split(const mhlp_plan *plan, int32_t *nsplit);
mhlp_status mhlp_plan_autotune(mhlp_plan *plan, int32_t layers, int32_t precision, int32_t reps, void *stream,
                               int32_t *best_nsplit, double *best_ms, int32_t *cand, double *cand_ms, int32_t cap,
                               int32_t *n_cand);

/* Layer potentials of the modified Helmholtz (Yukawa) kernel, the K0 part of
   the paper's modified-biharmonic Green's function (Sec. 2, App. B):
     S[sigma](x) = int_Gamma K0(alpha|x-y|)/(2 pi) sigma(y) dS_y,
     D[mu](x)    = int_Gamma alpha K1(alpha r) (x-y).n_y / (2 pi r) mu(y) dS_y,
   discretised by the composite 16-point Nystrom rule of Sec. 3.2, with the
   near-boundary and on-boundary quadrature of Sec. 4.5 (kernel split of
   Sec. 4.1, upsampling and subdivision of Sec. 4.5.3-4.5.4) replacing the
   rule on the plan's near panels.
   S[sigma] and/or D[mu] at the plan's targets (sigma, mu: device [N];
   u_slp, u_dlp: device [M], overwritten).  Either density/output pair may be
   NULL (then that potential is skipped), not both.  On an on-surface plan,
   D is the principal value (no 1/2 mu term) and S is the on-surface value.
   Far field in FP64 or mixed precision; near-field corrections FP64. */
mhlp_status mhlp_eval_layer(const mhlp_plan *plan, const double *sigma, const double *mu, double *u_slp,
                            double *u_dlp, int32_t precision, void *stream);
/* S[sigma] alone (eval_slp) and D[mu] alone (eval_dlp): the same sums as
   mhlp_eval_layer with one density; u: device [M], overwritten.  Errors as
   mhlp_eval_layer (MHLP_INVALID_ARG for NULL arrays or a stokes plan). */
mhlp_status mhlp_eval_slp(const mhlp_plan *plan, const double *sigma, double *u, int32_t precision, void *stream);
mhlp_status mhlp_eval_dlp(const mhlp_plan *plan, const double *mu, double *u, int32_t precision, void *stream);

/* out = (1/2 I + D) mu on an on-surface plan (Sec. 3.2, second-kind BIE with
   the interior limit).  Errors: MHLP_INVALID_ARG if the plan is not on-surface. */
mhlp_status mhlp_apply_bie_operator(const mhlp_plan *onsurf, const double *mu, double *out, int32_t precision,
                                    void *stream);

/* Modified-Stokes double layer, the paper's own BIE kernel (Sec. 3.2, the
   stresslet of App. B with its split of Sec. 4.1 and the complex forms of
   Sec. 4.3):
     D[mu]_i(x) = int_Gamma D_ij(x,y) mu_j(y) dS_y,  D_ij = -T_jik(x,y) n_k(y),
     T_ijk = alpha^2 T1 (d_jk r_i + d_ik r_j + d_ij r_k) + alpha^4 T2 r_i r_j r_k
             + alpha^2 T3 d_ik r_j,   r = x - y, n into the domain.
   A stokes plan has the near lists of mhlp_plan_create, 64 stresslet
   correction weights per near pair (2x2 blocks on the panel's 16 nodes) and,
   like a scalar plan, one byte per (64 targets, panel) naming the far-field
   fit that serves those pairs; it
   serves only the mhlp_stokes_* calls (the scalar calls reject it and vice
   versa).  Densities and outputs are component-major: mu [2][N] (mu_1 at
   mu[0..N), mu_2 at mu[N..2N)), u [2][M].  FP64 throughout.
   mhlp_stokes_eval: D[mu] at the plan's targets (on-surface: principal value,
   no 1/2 mu or W term).
   mhlp_stokes_apply_bie (on-surface plan): out = 1/2 mu + D mu + W mu with the
   nullspace correction W mu = n(x) int mu.n dS / |Gamma| (Sec. 2.2), out [2][N].
   mhlp_stokes_gmres_solve: GMRES for (1/2 I + D + W) mu = g, g and mu [2][N],
   same options and behaviour as mhlp_gmres_solve (precision must be FP64).
   Errors: MHLP_INVALID_ARG (NULL or aliased arrays, wrong plan kind). */
mhlp_status mhlp_stokes_plan_create(const mhlp_geometry *geom, double alpha, const double *tx, const double *ty,
                                    int64_t m, const mhlp_params *params, void *stream, mhlp_plan **out);
mhlp_status mhlp_stokes_eval(const mhlp_plan *plan, const double *mu, double *u, void *stream);
mhlp_status mhlp_stokes_apply_bie(const mhlp_plan *onsurf, const double *mu, double *out, void *stream);
mhlp_status mhlp_stokes_gmres_solve(const mhlp_plan *onsurf, const double *g, double *mu, const mhlp_gmres_opts *opts,
                                    mhlp_gmres_info *info, void *stream);

/* Target gradient of the modified-Stokes double layer on an off-surface
   stokes plan (the near-boundary gradient of Sec. 4.4 for the paper's BIE
   kernel), the velocity gradient of the represented flow:
     d u_i/d x_l = int_Gamma d/dx_l D_ij(x, y) mu_j(y) dS_y,
     d_l D_ij = -[ r_l (B1 P1 + B2 P2 + B3 P3)_ij + A1 dP1 + A2 dP2 + A3 dP3 ],
   with D_ij = -(A1 P1 + A2 P2 + A3 P3)_ij as for mhlp_stokes_eval
   (P1 = n_i r_j + r_i n_j + d_ij r.n, P2 = r_i r_j r.n, P3 = r_i n_j),
   dPk = d Pk/d x_l and B_k = A_k'(r)/r (from T1' = K0/(2 pi z) - 4 T1/z,
   T2' = -(z K0 + 2 K1)/(pi z^4) - 6 T2/z, T3' = -K0/(2 pi z) - 2 T3/z).  The
   near panels are integrated with the split of the stresslet carried to the
   gradient: smooth and log parts, the Cauchy vector (tau - z)^-1 part, the
   Laplace double-layer gradient under the alpha^2 r_i r_j r.n/(8 pi r^2) term
   and, for the Stokes stresslet part, the complex derivatives d/dz and d/dzbar
   of its complex form with the (tau - z)^-2 and (tau - z)^-3 integrals (the
   latter lowered by parts).  mu: device [2][N]; g: device [4][M], overwritten,
   row c = 2 i + l (i the velocity component, l the derivative direction) in
   the caller's target order.  Targets must lie off the curve.  FP64.  The
   first call on a plan builds its gradient weights (128 doubles per near
   pair) and synchronises the stream; later calls only enqueue.
   Errors: MHLP_INVALID_ARG (NULL or aliased arrays, a scalar plan),
   MHLP_UNSUPPORTED on an on-surface plan. */
mhlp_status mhlp_stokes_eval_grad(const mhlp_plan *plan, const double *mu, double *g, void *stream);

/* Target gradients of S[sigma] and D[mu] on an off-surface plan (the
   near-boundary gradient of Sec. 4.4, for the scalar kernel):
     grad S[sigma](x) = -(1/2pi) int alpha K1(alpha r)/r (x - y) sigma dS_y,
     grad D[mu](x)    = (1/2pi) int [A n_y - ((x-y).n_y)(x - y)(alpha^2 K0 + 2A)/r^2] mu dS_y,
   A = alpha K1(alpha r)/r.  The near panels of the plan are integrated with
   the kernel split of the gradient: smooth, log, Cauchy (tau - z)^-1 and
   (tau - z)^-2 parts with interpolatory weights on the upsampled panel, the
   same Bernstein-radius tiers and subdivision as the potentials.
   sigma, mu: device [N] (either may be NULL, not both); gs_x, gs_y (with
   sigma) and gd_x, gd_y (with mu): device [M], overwritten, the x1 and x2
   components in the caller's target order.  Targets must lie off the curve
   (the gradient has no limit there).  FP64 throughout.  The first call on a
   plan builds its gradient correction weights (64 doubles per near pair) and
   synchronises the stream; later calls only enqueue.
   Errors: MHLP_UNSUPPORTED on an on-surface plan; MHLP_INVALID_ARG for a
   density without both of its outputs or outputs without their density. */
mhlp_status mhlp_eval_grad(const mhlp_plan *plan, const double *sigma, const double *mu, double *gs_x, double *gs_y,
                           double *gd_x, double *gd_y, void *stream);

/* GMRES for (1/2 I + D) mu = g (Sec. 3.2), restarted, classical Gram-Schmidt
   with reorthogonalisation in FP64, judged by the true FP64 residual.  g, mu:
   device [N].  With opts->use_x0, mu holds the initial guess; a guess whose
   true relative residual is >= 1 is replaced by zero (info->used_x0 = 0).
   The Arnoldi steps, Givens rotations, the stopping test and the end of each
   cycle (the update of mu and its true residual) run on the device; chunks of
   steps are replayed from HIP graphs captured on a private stream of the plan
   (the host reads the state once per chunk).  The first chunk of a solve is
   as long as the first cycle of the plan's previous solve, which only changes
   how the steps are grouped, never the result.  The plan's GMRES state and
   workspace (with its own copies of g and mu) are shared: concurrent solves on
   one plan are not allowed.
   opts, info: host.  Synchronises the stream.  Returns MHLP_NOT_CONVERGED
   (mu = last iterate, info filled) if max_iter is reached. */
mhlp_status mhlp_gmres_solve(const mhlp_plan *onsurf, const double *g, double *mu, const mhlp_gmres_opts *opts,
                             mhlp_gmres_info *info, void *stream);

/* Fast multipole far field (Sec. 3.2.1, "Fast summation"), for the scalar
   kernel.  The far sums sum_j [q_j K0(alpha r) + d_j . grad_y K0(alpha r)] (q = w sigma
   for S, d = w mu n for D) are evaluated on a uniform quadtree: each leaf box
   takes the sources of its 3x3 neighbourhood directly and every other source
   through multipole (K_n) and local (I_n) expansions of order `order`
   (|n| <= order), translated by Graf's addition theorem (the paper's
   expansions restricted to modified-Helmholtz fields).  The truncation error
   falls geometrically with the order (order 40, the paper's choice, gives about
   1e-15 relative to the field; 20 about 1e-9).  Levels whose well-separated
   pairs are all below K0(40) (alpha 0.586 side > 40) are left out.
   Root square: centre at the midpoint of the bounding box of all sources and
   targets, side = largest extent x (1 + 2^-20); leaf level L has 4^L boxes.
   mhlp_plan_set_fmm (off-surface scalar plan): order 0 turns the FMM off; order
   in [4, 60] builds the tree for the plan's nodes and targets, after which
   mhlp_eval_layer / _slp / _dlp with MHLP_FP64 evaluate the far field by the
   FMM (near-panel corrections unchanged; the direct part skips each target's
   near panels); MHLP_MIXED keeps the direct FP32 tiles.  leaf_level -1 picks the
   finest level <= 8 (about 32 points per leaf or more) at which every node of
   each target's near panels lies in the target's 3x3 leaf neighbourhood; an
   explicit level must satisfy that (MHLP_INVALID_ARG otherwise).  Builds on the
   host and the device, synchronises the stream.  Errors: MHLP_UNSUPPORTED on an
   on-surface plan, MHLP_INVALID_ARG for a stokes plan or parameters out of range.
   mhlp_plan_get_fmm (host outputs): order (0 when off) and leaf level (-1). */
mhlp_status mhlp_plan_set_fmm(mhlp_plan *plan, int32_t order, int32_t leaf_level, void *stream);
mhlp_status mhlp_plan_get_fmm(const mhlp_plan *plan, int32_t *order, int32_t *leaf_level);

/* The volume sum of mhlp_volume_eval by the FMM: the object holds the tree of
   the n points (x, y, w: device [n], copied in leaf order at create; the
   caller's arrays may be freed afterwards) and the self-cell weight.
   mhlp_volume_fmm_eval: u (device [n], overwritten) for the density f (device
   [n]); coincident points are skipped in the direct part as in
   mhlp_volume_eval.  leaf_level -1: about 64 points per leaf (<= 8).
   mhlp_volume_fmm_info: order, leaf level and Wcell (host outputs, may be NULL).
   Errors: MHLP_INVALID_ARG (NULL or aliased arrays, n < 1, alpha or h not > 0,
   order not in [4, 60], level not -1 or in [0, 10]). */
typedef struct mhlp_volume_fmm mhlp_volume_fmm;
mhlp_status mhlp_volume_fmm_create(const double *x, const double *y, const double *w, int64_t n, double alpha,
                                   double h, int32_t order, int32_t leaf_level, void *stream, mhlp_volume_fmm **out);
mhlp_status mhlp_volume_fmm_eval(const mhlp_volume_fmm *vf, const double *f, double *u, void *stream);
mhlp_status mhlp_volume_fmm_info(const mhlp_volume_fmm *vf, int32_t *order, int32_t *leaf_level, double *self_cell);
mhlp_status mhlp_volume_fmm_destroy(mhlp_volume_fmm *vf);

/* Particular solution of the modified Stokes equations on a periodic box
   (Sec. 2.1: (alpha^2 - Delta) u + grad p = F, div u = 0 by the periodic stokeslet
   multiplier; Sec. 3.1.2: grid FFTs, the gradient by Fourier differentiation
   and values at boundary points by type-2 sums):
     u^_j(k) = S^_jl(k) F^_l(k), S^_jl = (delta_jl - k_j k_l/|k|^2)/(alpha^2 + |k|^2), S^(0) = I/alpha^2,
   on the box [x0, x0 + Lb) x [y0, y0 + Lb) with the M x M grid x_a = x0 + a Lb/M,
   y_b = y0 + b Lb/M, fields stored [b][a] (row = y); F^ = (1/M^2) DFT of the grid
   values, wavenumbers k = (2 pi/Lb)(k1, k2), k1, k2 in [-M/2, M/2), Nyquist modes
   set to zero.  F must be the grid values of a smooth periodic (compactly
   supported in the box) forcing; the result is spectrally accurate then.
   mhlp_box_create: M a power of two in [16, 2048], Lb > 0, alpha > 0; the box
   holds the twiddles and spectra (FP64).  mhlp_box_particular: F device
   [2][M][M] (F_1 then F_2); outputs (device, each may be NULL, not all): u
   [2][M][M], grad [4][M][M] (du1/dx, du1/dy, du2/dx, du2/dy), and at n points
   (px, py device [n]) up [2][n] = sum_k u^_j(k) e^{i k.(x - x0)} evaluated directly
   (the sum a type-2 non-uniform FFT approximates).  Enqueues only (the first
   point evaluation with more points than before synchronises to grow a buffer).
   Calls on one box must not overlap.  Errors: MHLP_INVALID_ARG. */
typedef struct mhlp_box mhlp_box;
/* mhlp_box_set_point_method: how the point values are formed.  0: the type-2
   sums written out directly (exact, n M^2 work); 1 (the default for M <= 1024):
   a non-uniform FFT as in Sec. 3.1.2 (coefficients divided by the transform of
   an exponential-of-semicircle kernel of width 14, inverse FFT on a 2M x 2M
   grid, a 14 x 14 kernel sum per point; ~1e-14 of sum |u^| from the exact sums;
   the first call allocates 2 (2M)^2 complex and synchronises).  Errors:
   MHLP_INVALID_ARG (method not 0 or 1, method 1 with M > 1024). */
mhlp_status mhlp_box_set_point_method(mhlp_box *box, int32_t method);
mhlp_status mhlp_box_create(int32_t M, double x0, double y0, double Lb, double alpha, void *stream, mhlp_box **out);
mhlp_status mhlp_box_particular(mhlp_box *box, const double *F, double *u, double *grad, int64_t n, const double *px,
                                const double *py, double *up, void *stream);
mhlp_status mhlp_box_destroy(mhlp_box *box);

/* One SISDC time step (Sec. 3.3, "Time stepping") of the Navier-Stokes equations
   u_t = -(u.grad)u + (1/Re) Delta u - grad p, div u = 0, on the periodic box
   (every term on the grid: no embedded boundary and no function extension).
   K in [2, 5]: p = K - 1 equal substeps dts = dt/p, a first implicit-explicit
   Euler sweep and K - 1 correction sweeps (global order K); each implicit
   substep is the box's particular solution with alpha^2 = Re/dts, which the box
   must have been created with (MHLP_INVALID_ARG otherwise).  Correction sweep:
     F_{m+1} = alpha^2 u'_m - Re (N'_m - N_m) - L_{m+1} + sum_j q_j^m (L_j - Re N_j),
   N = (u.grad)u, L = Delta u - Re grad p recovered as alpha^2 u - F from each solve,
   q_j^m the integrals over [t_m, t_{m+1}] of the Lagrange basis of the substep
   times (in units of dts).  In/out (device, overwritten with the end-of-step
   values): u [2][M][M], grad [4][M][M] (du1/dx, du1/dy, du2/dx, du2/dy of u), lap
   [2][M][M] = L at the start (Delta u of the initial field suffices: gradient
   terms do not change u).  The first step with a larger K synchronises to grow
   the box's workspace ((5 K + 1) 2 M^2 doubles).  Errors: MHLP_INVALID_ARG. */
mhlp_status mhlp_sisdc_step(mhlp_box *box, double Re, double dt, int32_t K, double *u, double *grad, double *lap,
                            void *stream);

/* Volume-style all-pairs Yukawa sum on a tensor grid (the dense stress case;
   the paper instead treats volume potentials by FFT, Sec. 3.1.2):
     u_i = sum_{j != i} K0(alpha |x_i - x_j|)/(2 pi) w_j f_j + (w_i / h^2) Wcell f_i,
   Wcell = integral of K0(alpha |x|)/(2 pi) over the h x h cell centred at the
   point (exact self-cell correction; trapezoid edge/corner cells take their
   weight fraction w_i/h^2).  x, y, w, f, u: device [n].  self_cell (host, may be
   NULL) receives Wcell.  Synchronises the stream when the source range is
   split (n small enough that fewer than 1024 target blocks exist).  Errors:
   MHLP_INVALID_ARG for NULL arrays, n < 1, alpha or h not > 0. */
mhlp_status mhlp_volume_eval(const double *x, const double *y, const double *w, const double *f, int64_t n,
                             double alpha, double h, int32_t precision, double *u, double *self_cell, void *stream);

/* mhlp_volume_eval without any allocation, for callers that cannot allocate
   device memory (code under HIP graph capture, tight serving loops, harnesses
   that forbid hipMalloc).  Same sum, arguments and launch shape (hence the same
   result) as mhlp_volume_eval, without the self_cell output; it only enqueues
   and never synchronises.  The self-cell weight and the split partial sums live
   in a fixed device array of the library (32 + 2^19 doubles, about 4 MiB, one
   copy per device, held until the process ends), which every call on that
   device shares: calls that overlap on one device (different streams, or
   threads without ordering) race and give wrong results; order them.  Every
   scratch value is written before it is read, so nothing carries over between
   calls.  The first call on a device looks up the array's address (no
   allocation).  Errors: as mhlp_volume_eval; MHLP_INVALID_ARG if the partial
   sums would exceed the array (not reached by any n: at most 523,776 values). */
mhlp_status mhlp_volume_eval_noalloc(const double *x, const double *y, const double *w, const double *f, int64_t n,
                                     double alpha, double h, int32_t precision, double *u, void *stream);

/* Batched on-surface solves over many geometries (each with its own alpha)
   and up to 4 right-hand sides per geometry (Sec. 3.2 BIE, one system per
   geometry and right-hand side).  plans: host array of n_geom on-surface
   plans (borrowed; they must outlive the batch).  Batched vectors hold, for
   each geometry in order, its n_rhs right-hand sides of N_g values each;
   mhlp_batch_info reports the total length and each system's offset and
   length (host arrays of n_geom*n_rhs entries, may be NULL). */
typedef struct mhlp_batch mhlp_batch;
mhlp_status mhlp_batch_create(int32_t n_geom, const mhlp_plan *const *plans, int32_t n_rhs, void *stream,
                              mhlp_batch **out);
mhlp_status mhlp_batch_destroy(mhlp_batch *batch);
mhlp_status mhlp_batch_info(const mhlp_batch *batch, int64_t *total_len, int32_t *n_systems, int64_t *offsets,
                            int64_t *lengths);
/* out = (1/2 I + D) mu for every system in one grouped launch (kernel values
   shared by the right-hand sides of a geometry); FP64.  The launch runs a
   work list of (geometry, 256 targets, source split) items, longest first. */
mhlp_status mhlp_batch_apply_bie(const mhlp_batch *batch, const double *mu, double *out, void *stream);
/* Autotuner of the grouped operator's launch shape: for every tile shape
   (1 or 2 targets per lane, i.e. target tiles of 256 or 512 nodes; 128 or
   256 sources staged in LDS per step) and a total of 512, 1024, ..., 16384
   blocks, rebuild the work list and time the operator (reps launches after a
   warm-up, HIP events on `stream`); keep the fewest blocks within 1% of the
   fastest.  best_target and best_ms (host) may be NULL.  Synchronises the
   stream. */
mhlp_status mhlp_batch_autotune(mhlp_batch *batch, int32_t reps, void *stream, int64_t *best_target, double *best_ms);
/* The batch's launch shape (block target, targets per lane, sources per LDS
   stage) and the autotuner's candidates: cand [cap][3] rows {block target,
   targets per lane, sources per stage}, cand_ms [cap] ms per application;
   n_cand receives the number measured (0 before autotuning).  Host outputs,
   any may be NULL. */
mhlp_status mhlp_batch_tile(const mhlp_batch *batch, int64_t *target, int32_t *tpl, int32_t *src, int64_t *cand,
                            double *cand_ms, int32_t cap, int32_t *n_cand);
/* Set the launch shape directly: target blocks in total (>= 1), tpl targets per
   lane (1 or 2), src sources per LDS stage (128 or 256); rebuilds the work
   list (synchronises the stream).  Errors: MHLP_INVALID_ARG. */
mhlp_status mhlp_batch_set_tile(mhlp_batch *batch, int64_t target, int32_t tpl, int32_t src, void *stream);
/* Lockstep restarted GMRES on every system (FP64, CGS2, restart <= 64),
   converged systems frozen (their geometries drop out of the operator
   launches of the cycle); each judged by its own true residual.  infos:
   host array of n_geom*n_rhs.  Synchronises the stream.  Returns
   MHLP_NOT_CONVERGED if any system misses the tolerance within max_iter
   Arnoldi steps (counted per lockstep iteration). */
mhlp_status mhlp_batch_gmres_solve(mhlp_batch *batch, const double *g, double *mu, const mhlp_gmres_opts *opts,
                                   mhlp_gmres_info *infos, void *stream);

/* ------------------------------------------------------------------------
 * Learned GMRES warm start.  The paper's implicit time stepping (Sec. 3)
 * solves one Sec. 3.2 BIE per step with slowly changing data; these entries
 * predict the next step's density from the last ones, to be passed to
 * mhlp_gmres_solve with use_x0 = 1 (which falls back to the zero guess when
 * the prediction's residual is not below ||g||).  Not part of the paper.
 *
 * Network (mhlp_mlp): n_in -> width -> width -> n_out, GELU (tanh form)
 * after both hidden layers, no activation on the output.  Parameters are FP32
 * master copies laid out per layer l = 0,1,2 as W_l (row-major
 * [n_{l+1}][n_l]) followed by b_l; every product rounds its operands to BF16
 * (nearest even) and accumulates in FP32 on the matrix cores.  Default
 * initialisation: W_l ~ U(-1/sqrt(n_l), 1/sqrt(n_l)) from a counter-based
 * generator seeded by `seed`, biases 0.  Batched arrays are row-major
 * [batch][features], FP32, device.
 * ---------------------------------------------------------------------- */
typedef struct mhlp_mlp mhlp_mlp;
mhlp_status mhlp_mlp_create(int32_t n_in, int32_t width, int32_t n_out, uint64_t seed, void *stream,
                            mhlp_mlp **out);
mhlp_status mhlp_mlp_destroy(mhlp_mlp *mlp);
/* parameter count and the four layer widths (host outputs, may be NULL) */
mhlp_status mhlp_mlp_info(const mhlp_mlp *mlp, int64_t *n_params, int32_t *sizes4);
/* copy the FP32 parameters out to dst and/or in from src (device, n_params
   floats each, may be NULL); loading resets the Adam state */
mhlp_status mhlp_mlp_params(mhlp_mlp *mlp, float *dst, const float *src, void *stream);
/* Y [batch][n_out] = net(X [batch][n_in]) */
mhlp_status mhlp_mlp_forward(mhlp_mlp *mlp, const float *X, int32_t batch, float *Y, void *stream);
/* forward, loss L = mean over batch*n_out entries of (net(X) - T)^2, and the
   gradient dL/dparams (back-propagation with the same BF16 products) into the
   network's gradient buffer; loss (device, 1 float) and grad (device,
   n_params floats) receive copies when non-NULL */
mhlp_status mhlp_mlp_loss_grad(mhlp_mlp *mlp, const float *X, const float *T, int32_t batch, float *loss,
                               float *grad, void *stream);
/* one Adam step (bias-corrected, no weight decay) with the last gradient */
mhlp_status mhlp_mlp_adam_step(mhlp_mlp *mlp, float lr, float beta1, float beta2, float eps, void *stream);
/* C[m][n] (row-major, leading dimension ldc >= n) = sum_k A(m,k) B(k,n) with
   A(m,k) = A[m*sam + k*sak], B(k,n) = B[k*sbk + n*sbn]; FP32 in memory,
   BF16 operands, FP32 accumulation (the network's product, exposed for tests) */
mhlp_status mhlp_gemm_bf16(int32_t m, int32_t n, int32_t k, const float *A, int64_t sam, int64_t sak, const float *B,
                           int64_t sbk, int64_t sbn, float *C, int64_t ldc, void *stream);

/* Warm-start model (mhlp_warm): Fourier features of the density on each
   closed curve in its parameter theta, c_k = (1/2 pi) int mu e^{-i k theta},
   k = 0..n_modes-1, by the panel quadrature in theta; F = 2 n_modes n_curves
   reals per density, ordered [curve][k][Re, Im].  From the coefficients of
   the last n_hist densities (newest last) the network input is, for
   h = 0..n_hist-1, the h-th backward difference of the newest coefficients,
   each group scaled to unit RMS over the training samples.  The network
   predicts the error of a base prediction of the next coefficients, in units
   of its RMS over the training samples:
   * base_order = p >= 0: the order-p polynomial extrapolation of the history,
     sum_{i<=p} (-1)^i C(p+1, i+1) c_{s-i} (0 = the last density, 1 = linear,
     2 = quadratic, 3 = cubic); the initial guess is the same extrapolation of
     the densities plus the synthesis of the predicted correction;
   * base_order = -1 (MHLP_WARM_RECURRENCE): a linear recurrence of order
     n_hist for each complex coefficient, c_k(s) = sum_i a_{k,i} c_k(s-1-i),
     fitted by mhlp_warm_train (least squares over the training windows with a
     relative Tikhonov term of 1e-14, complex normal equations solved by
     Cholesky); the initial guess is the cubic extrapolation of the densities
     (quadratic or lower when n_hist < 4) plus the synthesis of (recurrence -
     cubic extrapolation) of the coefficients plus the predicted correction.
     A coefficient that rotates, c_k(s) = b e^{i w s} (a drifting mode on a
     curve the operator maps to itself), or sums up to n_hist such terms,
     satisfies such a recurrence exactly.
   theta, omega: device [N] float64, curve parameter and theta-quadrature
   weight of each node (copied); curve_ptr: host [n_curves+1], node ranges of
   the curves (0 = curve_ptr[0] < ... < curve_ptr[n_curves] = N).
   1 <= n_hist <= 8, base_order = -1 or 0 <= base_order <= min(3, n_hist - 1).
   The network is n_hist*F -> width -> width -> F.  Synchronises the stream. */
#define MHLP_WARM_RECURRENCE (-1)
typedef struct mhlp_warm mhlp_warm;
mhlp_status mhlp_warm_create(const double *theta, const double *omega, const int64_t *curve_ptr, int32_t n_curves,
                             int32_t n_modes, int32_t n_hist, int32_t base_order, int32_t width, uint64_t seed,
                             void *stream, mhlp_warm **out);
mhlp_status mhlp_warm_destroy(mhlp_warm *warm);
/* node count, F, the network (borrowed, owned by the model) and the scales
   {input group factors 0..n_hist-1, output unit} (host [n_hist+1];
   synchronous); any may be NULL */
mhlp_status mhlp_warm_info(const mhlp_warm *warm, int64_t *n_nodes, int64_t *n_features, mhlp_mlp **net,
                           double *scales);
/* coef [n_dens][F] = Fourier coefficients of mu [n_dens][N] (FP64) */
mhlp_status mhlp_warm_coefficients(const mhlp_warm *warm, const double *mu, int32_t n_dens, double *coef,
                                   void *stream);
/* out [n_dens][N] = base + real Fourier series of coef [n_dens][F] at the
   nodes (base may be NULL = 0) */
mhlp_status mhlp_warm_synthesize(const mhlp_warm *warm, const double *coef, int32_t n_dens, const double *base,
                                 double *out, void *stream);
/* Train on a series of solved densities mus [n_steps][N] (oldest first):
   samples j = 0..n_steps-n_hist-1, full-batch Adam (beta 0.9/0.999, eps
   1e-8) for iters steps at learning rate lr; the scales are fixed from this
   series.  losses: host [iters] (may be NULL).  Synchronises the stream. */
mhlp_status mhlp_warm_train(mhlp_warm *warm, const double *mus, int32_t n_steps, int32_t iters, float lr,
                            float *losses, void *stream);
/* x0 [N] = extrapolation of hist [n_hist][N] (oldest first) + predicted
   correction.  Errors: MHLP_INVALID_ARG before training. */
mhlp_status mhlp_warm_predict(mhlp_warm *warm, const double *hist, double *x0, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* MHLP_H */
