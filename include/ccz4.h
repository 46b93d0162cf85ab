/*
 * ccz4.h -- C ABI of the MI355X (gfx950) CCZ4 FD4 hot-path library.
 *
 * The library evaluates the first-order CCZ4 right-hand side of the Einstein equations
 * (3+1 split; 1+log or harmonic slicing; Gamma-driver or frozen shift) with fourth-order
 * central finite differences and Kreiss-Oliger dissipation on block-structured Cartesian
 * patches, and combines the stages of the classical RK4 integrator.  Paper:
 * "ExaGRyPE: Numerical General Relativity Solvers Based upon the Hyperbolic PDEs Solver
 * Engine ExaHyPE" (arXiv:2406.11626): the evolution system and its closing relations are its
 * App. B, the stencils its App. D, the coarse-fine transfer matrices its App. E, the patch
 * and halo layout its section on spatial discretisation, the boundary treatment its section
 * on boundary conditions.
 *
 * Conventions shared by every call:
 *  - A state holds 59 double slots per cell: the 58 first-order variables in the paper's
 *    order -- gt_ij(0-5) alpha(6) beta^i(7-9) phi(10) At_ij(11-16) K(17) Theta(18)
 *    Ghat^i(19-21) b^i(22-24) A_k(25-27) B_k^i(28+3k+i) D_kij(37+6k+sym(ij)) P_k(55-57) --
 *    plus slot 58 = K_0, the constant of the slicing condition.  Symmetric pairs are ordered
 *    xx,xy,xz,yy,yz,zz.
 *  - Device layout (the caller allocates with the size from ccz4_layout): one slot of
 *    212400 doubles per leaf patch, leaves in canonical order (level, then k, j, i index);
 *    inside a patch, slot-major boxes of 15 x 15 x 16 doubles: element (v, z, y, x) at
 *    v*3600 + z*240 + y*16 + x, with x, y, z in 0..14, the 9^3 interior at 3..11 and 3 halo
 *    layers per face; x = 15 is padding.  Edge and corner cells of the box are never read
 *    or written.
 *  - All pointers named Q, k, acc, Qn, Qnext, HM, tags, indicator are device pointers owned
 *    by the caller; the library never frees caller memory.  `stream` is a hipStream_t (NULL:
 *    the null stream).  Calls are asynchronous on `stream` unless stated otherwise.
 *  - Every call returns a ccz4_status; on failure a message is available from
 *    ccz4_last_error() (thread-local, valid until the next failing call of that thread).
 *    Argument errors are reported before anything is launched.  Asynchronous device errors
 *    surface at the next call that synchronises.
 */
#ifndef CCZ4_H
#define CCZ4_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    CCZ4_OK = 0,
    CCZ4_EINVAL = 1,     /* invalid argument (null pointer, bad size or index, dt <= 0, ...) */
    CCZ4_ENOMEM = 2,     /* host or device allocation inside the library failed */
    CCZ4_ELAYOUT = 3,    /* mesh violates an assumption (e.g. a level jump > 1 across a face) */
    CCZ4_EHIP = 4,       /* a HIP runtime call failed */
    CCZ4_ENONFINITE = 5, /* ccz4_constraints found non-finite values (norms are still written) */
    CCZ4_ESTATE = 6      /* call not valid in the context's current state */
} ccz4_status;

enum { CCZ4_BC_PERIODIC = 0, CCZ4_BC_NEUMANN = 1, CCZ4_BC_SOMMERFELD = 2 };
enum { CCZ4_SLICING_HARMONIC = 0, CCZ4_SLICING_ONE_PLUS_LOG = 1 };
enum { CCZ4_SHIFT_FROZEN = 0, CCZ4_SHIFT_GAMMA_DRIVER = 1 };
enum { CCZ4_PREC_FP64 = 0, CCZ4_PREC_MIXED = 1 };
enum { CCZ4_SCEN_GAUGE_WAVE = 0, CCZ4_SCEN_PUNCTURE = 1, CCZ4_SCEN_BL_BY = 2 };

/* Parameters of App. B (kappa1..3, tau, e, c, mu, f, eta), the KO strength epsilon of
   App. D, the slicing function g(alpha) (harmonic: 1; 1+log: 2/alpha), the shift
   condition (frozen: beta, b, B do not evolve; Gamma-driver: s = 1) and the formulation
   (Sec. 2.2): first order (all 58 variables evolve, with the red constraint-addition terms of
   App. B) or second order (the 24 primaries evolve without the red terms; the auxiliaries
   A, B, D, P are recomputed from the primaries after every update, ccz4_reconstruct_aux), and
   the derivative taken in the advection terms beta^k d_k Q (App. D): the central FD4 difference,
   or one of the two lopsided fourth-order stencils chosen per axis by the sign of beta^k, either
   biased towards +x_k where beta^k > 0 (the upwind reading of d_t Q = beta^k d_k Q + ...) or with
   the pairing as printed (biased towards -x_k where beta^k > 0). */
enum { CCZ4_FORMULATION_FIRST_ORDER = 0, CCZ4_FORMULATION_SECOND_ORDER = 1 };
enum { CCZ4_ADVECTION_CENTRAL = 0, CCZ4_ADVECTION_LOPSIDED_UPWIND = 1, CCZ4_ADVECTION_LOPSIDED_PRINTED = 2 };
/* transfer selects the coarse-fine halo operators of every fill: the App. E operators as printed
   (linear P_par x P_par x P_perp prolongation, R_avg x R_avg x R_perp restriction by average and
   linear extrapolation), or higher-order ones (the remedy the paper names for reflections at
   refinement boundaries): restriction injects the fine cell whose centre coincides with the
   coarse halo centre, prolongation interpolates with three-point Lagrange quadratics along each
   axis (coarse layers c1, c2 and the restricted c3 along the normal); both reproduce quadratic
   fields exactly.  Regrid transfers are unaffected. */
enum { CCZ4_TRANSFER_APP_E = 0, CCZ4_TRANSFER_HIGHER_ORDER = 1 };
typedef struct {
    double kappa1, kappa2, kappa3, tau, e, c, mu, f, eta, ko_eps;
    int32_t slicing, shift;
    int32_t formulation;
    int32_t advection;
    int32_t transfer;
} ccz4_params;

/* Forest of n0[0] x n0[1] x n0[2] level-0 cubes over [origin, origin + extent], every cube
   holding a 9^3 patch.  A refined cube is split into 3^3 children (the paper's
   tri-partitioning); `refined` lists every refined cube as (level, i, j, k) with indices
   counted at that level.  Leaves carry data.  Faces between a leaf and finer leaves are
   coupled by restriction, between a leaf and a coarser leaf by prolongation; leaves that
   share a face may differ by one level at most.  bc applies to all six domain faces. */
typedef struct {
    int32_t n0[3];
    double origin[3];
    double extent[3];
    int32_t bc;
    int32_t n_refined;
    const int32_t *refined; /* host array of n_refined x 4 int32, may be NULL if n_refined = 0 */
} ccz4_grid_desc;

typedef struct ccz4_ctx ccz4_ctx;

/* Builds the leaf table, the face-task plan of the halo fill and the per-level spacings,
   and uploads them to the current HIP device.  The context owns those tables only. */
ccz4_status ccz4_create(ccz4_ctx **out, const ccz4_grid_desc *grid, const ccz4_params *prm);
/* Frees the context (waits for the device).  NULL is accepted. */
void ccz4_destroy(ccz4_ctx *ctx);
/* Replaces the parameters used by later calls. */
ccz4_status ccz4_set_params(ccz4_ctx *ctx, const ccz4_params *prm);

/* n_patches: number of leaves; patch_doubles: doubles per patch slot (212400);
   bytes_per_state: bytes of one state buffer (n_patches * patch_doubles * 8). */
ccz4_status ccz4_layout(const ccz4_ctx *ctx, int64_t *n_patches, int64_t *patch_doubles,
                        int64_t *bytes_per_state);
/* Host copies of the leaf table: ids[n][4] = (level, i, j, k); geom[n][6] = lower corner of
   the patch interior (x, y, z) and cell spacing (dx, dy, dz).  Either may be NULL. */
ccz4_status ccz4_patch_table(const ccz4_ctx *ctx, int32_t *ids, double *geom);

/* Initial data.  Pointwise initial data on every interior cell and, with the Sommerfeld condition, on
   the ghost layers of domain-boundary faces (which are evolved, not filled).  Interior cells
   are then projected (det gt = 1, tr At = 0).  Also records the Sommerfeld background Q_ini.
   scenario / scen (host array of n_scen doubles):
     CCZ4_SCEN_GAUGE_WAVE: {A, k}: H = 1 - A sin(k pi x) (paper's gauge-wave test, t = 0);
     CCZ4_SCEN_PUNCTURE:   {M, x0, y0, z0, lapse}: psi = 1 + M/(2r), phi = psi^-2, gt = delta,
                           K_ij = 0, beta = 0; lapse 0: psi^-2, 1: the paper's averaged lapse,
                           2: (1 - M/2r)/(1 + M/2r);
     CCZ4_SCEN_BL_BY:      {m, x, y, z, Px, Py, Pz} per hole, two holes: Brill-Lindquist
                           conformal factor with Bowen-York curvature, K = 0, alpha = psi^-2.
   Does not fill halos. */
ccz4_status ccz4_init_patches(ccz4_ctx *ctx, double *Q, int32_t scenario, const double *scen,
                              int32_t n_scen, void *stream);
/* Records the Sommerfeld ghost values of Q as the background Q_ini (no-op for other bcs). */
ccz4_status ccz4_set_background(ccz4_ctx *ctx, const double *Q, void *stream);

/* Halo fill.  Fills the six face halos of every leaf from the current values of Q: same-level copy
   (periodic wrap included), homogeneous Neumann copied layer by layer outwards, restriction
   of fine interiors into coarse halos (R_avg x R_avg x R_perp of App. E), then prolongation
   of coarse interiors and restricted halos into fine halos (P_par x P_par x P_perp).
   Sommerfeld ghosts are left untouched. */
ccz4_status ccz4_fill_halos(ccz4_ctx *ctx, double *Q, void *stream);

/* Halo fill restricted to some kinds of face (same semantics per face as ccz4_fill_halos):
   CCZ4_FILL_SAME_LEVEL (copy from a same-level leaf, periodic wrap included), CCZ4_FILL_NEUMANN,
   CCZ4_FILL_LEVELS (all restrictions, then all prolongations).  kinds = CCZ4_FILL_ALL is
   ccz4_fill_halos.  EINVAL on unknown bits.  Pairs with CCZ4_STAGE_FILL_SAME_LEVEL below, which
   leaves only the Neumann and coarse-fine faces to fill between stages. */
enum { CCZ4_FILL_SAME_LEVEL = 1, CCZ4_FILL_NEUMANN = 2, CCZ4_FILL_LEVELS = 4, CCZ4_FILL_ALL = 7 };
ccz4_status ccz4_fill_halos_kinds(ccz4_ctx *ctx, double *Q, int32_t kinds, void *stream);

/* Face counts of the fill plan: counts[0..4] = same-level faces, Neumann faces, restriction
   faces (coarse side), prolongation faces (fine side), Sommerfeld faces.  Host call. */
ccz4_status ccz4_plan_counts(const ccz4_ctx *ctx, int64_t *counts);

/* Right-hand side.  k = RHS(Q) on every interior cell: FD4 central derivatives of slots 11..57,
   the pointwise first-order CCZ4 algebra of App. B, plus the Kreiss-Oliger sum over the axes
   on the 58 evolved slots (frozen-shift slots get 0; slot 58 gets 0).  On Sommerfeld faces
   the ghost slots receive G_L = -(r/|x_n|)(Q_L - Q_{L-1})/dx - (Q_L - Q_ini)/r.  Requires
   filled halos; never modifies Q.  Q and k must not alias.  precision: CCZ4_PREC_FP64, or
   CCZ4_PREC_MIXED (stencil differences in FP64, nonlinear algebra in FP32, the inverse
   metric, det gt and every factor of 1/phi in FP64, result promoted to FP64).  In the
   second-order formulation the red terms are off and the interior slots of A, B, D, P get 0
   (the Sommerfeld ghost slots keep G_L for every slot). */
ccz4_status ccz4_rhs(ccz4_ctx *ctx, const double *Q, double *k, int32_t precision, void *stream);

/* RK4 stage (Sec. 3.2: Runge-Kutta time stepping of the FD4 solver up to fourth order, with a
   global time step over all levels; the algebraic post-processing of Sec. 4.2.1 after each step).
   Stage s (0..3) of classical RK4 in two-register form, on interior cells and
   Sommerfeld ghosts:  s=0: acc = Qn + dt/6 k, Qnext = Qn + dt/2 k;  s=1: acc += dt/3 k,
   Qnext = Qn + dt/2 k;  s=2: acc += dt/3 k, Qnext = Qn + dt k;  s=3: Qnext = acc + dt/6 k,
   then gt <- gt/det(gt)^(1/3) and At <- At - gt tr(At)/3 on interior cells.  dt > 0.
   Qnext may alias Qn only at s = 3. */
ccz4_status ccz4_rk4_stage(ccz4_ctx *ctx, int32_t s, double dt, const double *Qn,
                           const double *k, double *acc, double *Qnext, void *stream);

/* Fused stage.  One launch over every leaf of every level: the right-hand
   side of Qs exactly as ccz4_rhs computes it, folded slot by slot into stage s of RK4 exactly as
   ccz4_rk4_stage combines it (interior cells and Sommerfeld ghosts; projection at s = 3), without
   storing the right-hand side.  Qnext must not alias Qs (other cells still read it), may alias
   Qn only at s = 3; acc aliases none of them.  acc is a state-sized accumulator private to this
   call: its layout (interior cells slab by slab, then the Sommerfeld ghost slabs, so that every
   access covers whole cache lines) is not the state layout, and only s = 0 needs no prior
   contents; it is not interchangeable with the acc of ccz4_rk4_stage.  A step is
   s = 0: (Qn -> Q1), 1: (Q1 -> Q2), 2: (Q2 -> Q1), 3: (Q1 -> Qn).  flags, any combination of:
     CCZ4_STAGE_FILL_SAME_LEVEL: the stage also writes every new interior value that lies within
       three layers of a face shared with a same-level leaf into that leaf's face halo of Qnext
       (what CCZ4_FILL_SAME_LEVEL would copy there afterwards);
     CCZ4_STAGE_FILL_SAME_LEVEL_X: the same for the faces normal to x only;
     CCZ4_STAGE_GATHER_SAME_LEVEL: the stage reads every y and z face halo of Qs that a same-level
       leaf covers straight from that leaf's interior, so those halos of Qs need not be filled
       (all other halos must be).  LDS kernel only (EINVAL if the context's kernel for this
       precision is the phased one).
   Without GATHER, Qs needs filled halos.  EINVAL on unknown flags.  In the second-order
   formulation the interior slots of A, B, D, P in acc and Qnext are not written: after the halo
   fill of Qnext, call ccz4_reconstruct_aux on it (and fill again). */
enum { CCZ4_STAGE_FILL_SAME_LEVEL = 1, CCZ4_STAGE_GATHER_SAME_LEVEL = 2, CCZ4_STAGE_FILL_SAME_LEVEL_X = 4 };
ccz4_status ccz4_rhs_rk4_stage(ccz4_ctx *ctx, int32_t s, double dt, const double *Qs, const double *Qn,
                               double *acc, double *Qnext, int32_t precision, int32_t flags, void *stream);

/* The flags the step graph passes to stage s (0..3), and in the second-order formulation to the
   reconstruction after it, with the context's current kernel for this precision, into *flags
   (host).  LDS kernel: GATHER at every stage, FILL_SAME_LEVEL_X at s = 0..2 and FILL_SAME_LEVEL
   at s = 3 (between stages only the x-face halos are copied; the y and z ones are read from the
   neighbours, and the step leaves complete halos).  Phased kernel: FILL_SAME_LEVEL at every
   stage.  Between stages only ccz4_fill_halos_kinds(NEUMANN | LEVELS) is needed either way, and
   Qn must enter the step with filled halos.  EINVAL on a NULL pointer, bad precision or stage. */
ccz4_status ccz4_step_stage_flags(ccz4_ctx *ctx, int32_t precision, int32_t s, int32_t *flags);

/* Second-order formulation, explicit gradient reconstruction (Sec. 3.2 and Algorithm 2): on every
   interior cell of every leaf, A_k = d_k alpha, B_k^i = d_k beta^i, D_kij = d_k gt_ij / 2 and
   P_k = d_k phi (eq. auxiliary-variables) from the central FD4 difference of the primaries.
   Q (device, a state of this context) is updated in place; the primaries' halos must be filled
   (gt, alpha, beta, phi), and no primary is modified.  flags, any combination of
   CCZ4_STAGE_FILL_SAME_LEVEL (the new values within three layers of a face shared with a
   same-level leaf are also written into that leaf's face halo; then only
   ccz4_fill_halos_kinds(NEUMANN | LEVELS) remains for the auxiliaries' halos),
   CCZ4_STAGE_FILL_SAME_LEVEL_X (the same for the faces normal to x only) and
   CCZ4_STAGE_GATHER_SAME_LEVEL (the primaries' y and z face halos that a same-level leaf covers
   are read from that leaf's interior and need not be filled).  Independent of the context's
   formulation setting and kernel.  EINVAL on a NULL pointer or unknown flags. */
ccz4_status ccz4_reconstruct_aux(ccz4_ctx *ctx, double *Q, int32_t flags, void *stream);

/* Tracers (Sec. 3.8, data probes).  For each of n points pos[n][3] (device, float64), the leaf
   that holds it (the leaf whose cube contains the point's cube at the finest level, that cube's
   index being floor((x - origin) / edge): every point of the domain is in exactly one leaf), then
   for each of the nslots slots (host array, values 0..58) the trilinear interpolation of the 2^3
   cell centres around the point at that leaf's spacing.  A centre outside the leaf's interior is
   read from the interior of the same-level leaf that holds it, else (outside the domain, or in a
   leaf of another level) from the leaf's face halo, so Q's halos must be filled (edge and corner
   regions of halos are never read).  out[n][nslots] (device).  A point outside the domain samples
   NaN.  n = 0 does nothing.  EINVAL on NULL pointers, n < 0, nslots outside 1..59 or a slot
   outside 0..58. */
ccz4_status ccz4_tracers_sample(ccz4_ctx *ctx, const double *Q, int64_t n, const double *pos, int32_t nslots,
                                const int32_t *slots, double *out, void *stream);

/* Puncture trackers (Sec. 4.2.3: tracers moved by the reversed shift).  One explicit Euler step of the
   Sec. 3.8 rule x <- x + dt v with v = -beta(x), beta interpolated as in ccz4_tracers_sample; pos
   (device) is updated in place; a point outside every leaf stays.  Q's halos must be filled. */
ccz4_status ccz4_tracers_advance(ccz4_ctx *ctx, const double *Q, int64_t n, double *pos, double dt, void *stream);

/* Refinement tags by coordinates (Sec. 4.2.1, dynamic refinement based on coordinates): with the
   per-level radii r[0..nradii-1] (host), a leaf of level l < min(max_level, nradii) whose closed
   cube lies within r[l] of one of the n tracers pos[n][3] (device) is tagged REFINE (1); a leaf of
   level l >= 1 whose parent cube lies farther than r[l-1] from every tracer COARSEN (-1); every
   other leaf KEEP (0).  tags[n_patches] (device, int8), in the form ccz4_regrid_plan takes once
   copied to the host.  A mesh refined by spheres of these radii around the tracers is a fixed
   point.  EINVAL on NULL pointers or nradii outside 0..16. */
ccz4_status ccz4_tag_tracers(ccz4_ctx *ctx, int64_t n, const double *pos, int32_t nradii, const double *radii,
                             int32_t max_level, int8_t *tags, void *stream);

/* Launch configuration of ccz4_rhs and ccz4_rhs_rk4_stage, per precision (CCZ4_PREC_FP64 or
   CCZ4_PREC_MIXED): CCZ4_KERNEL_PHASED or CCZ4_KERNEL_LDS, optionally with
   CCZ4_KERNEL_LINEAR_ORDER added, plus one CCZ4_KERNEL_ORDER_* value.  Both kernels evaluate the
   same right-hand side (App. B algebra, App. D FD4 and KO stencils) and agree up to
   floating-point rounding order; they differ only in how the stencil footprints reach the
   registers.  CCZ4_KERNEL_PHASED reads every stencil point from the state in six phases;
   CCZ4_KERNEL_LDS copies each slot's slab footprint once into LDS per evaluation, in four rounds.
   The work-groups of consecutive logical patches run on one XCD unless CCZ4_KERNEL_LINEAR_ORDER
   is given (plain block order).  The leaf order sets which leaf each logical patch is, level by
   level: canonical (i fastest), z-pencils (k fastest, then j, then i), bricks of 4^3 cubes, or
   Morton (bits of i, j, k interleaved); neighbours across y and z faces, whose halos a stage
   reads, are then processed closer in time.  No configuration changes the arithmetic of a cell.
   Default after ccz4_create: CCZ4_KERNEL_LDS (canonical order) for both precisions.  EINVAL on an
   unknown precision or value (0..15), or a NULL out pointer. */
typedef enum {
    CCZ4_KERNEL_PHASED = 0,
    CCZ4_KERNEL_LDS = 1,
    CCZ4_KERNEL_LINEAR_ORDER = 2,
    CCZ4_KERNEL_ORDER_CANONICAL = 0,
    CCZ4_KERNEL_ORDER_Z_PENCILS = 4,
    CCZ4_KERNEL_ORDER_BRICKS = 8,
    CCZ4_KERNEL_ORDER_MORTON = 12,
    CCZ4_KERNEL_CONFIGS = 16
} ccz4_kernel;
ccz4_status ccz4_set_kernel(ccz4_ctx *ctx, int32_t precision, int32_t kernel);
ccz4_status ccz4_get_kernel(const ccz4_ctx *ctx, int32_t precision, int32_t *kernel);

/* Autotuner: times one fused stage (s = 1, with the flags ccz4_step_stage_flags gives that
   configuration) of every launch configuration (0..CCZ4_KERNEL_CONFIGS-1 above: kernel, block
   order and leaf order) on this context's mesh, `reps` launches each after one warm-up, with
   events on `stream`, and selects the fastest for `precision`.  Q: a state with filled halos
   (read only); acc and Qx: state-sized scratch (overwritten).  ms (host, may be NULL) receives the
   CCZ4_KERNEL_CONFIGS average launch times in milliseconds, indexed by configuration.
   Synchronises `stream`. */
ccz4_status ccz4_autotune(ccz4_ctx *ctx, const double *Q, double *acc, double *Qx, int32_t precision,
                          int32_t reps, double *ms, void *stream);

/* A fused RK4 step captured as a HIP graph: the four stages of ccz4_rhs_rk4_stage with the
   flags of ccz4_step_stage_flags, (Qn -> Q1), (Q1 -> Q2), (Q2 -> Q1), (Q1 -> Qn), each followed
   by ccz4_fill_halos_kinds(NEUMANN | LEVELS) of its output (in the second-order formulation then
   ccz4_reconstruct_aux with the same flags and the same fill again), with the launch
   configuration current at creation.  Buffers and dt are fixed at creation; Qn must enter each launch with all halos filled
   and leaves with them filled.  The graph uses the context's tables: destroy it before the
   context.  Launch is asynchronous on `stream`. */
typedef struct ccz4_graph ccz4_graph;
ccz4_status ccz4_step_graph_create(ccz4_ctx *ctx, double *Qn, double *Q1, double *Q2, double *acc, double dt,
                                   int32_t precision, ccz4_graph **out);
ccz4_status ccz4_step_graph_launch(ccz4_graph *graph, void *stream);
void ccz4_step_graph_destroy(ccz4_graph *graph);

/* Constraint monitor.  Hamiltonian H = R + 2/3 K^2 - At_ij At^ij and momentum M_i (App. B) on every interior
   cell (FD4 derivatives; requires filled halos).  HM (device, may be NULL) receives
   HM[(p*4 + q)*729 + c] for q = H, Mx, My, Mz and interior cell c = (z*9 + y)*9 + x.
   norms_host (host, may be NULL): {sqrt(sum H^2/n), sqrt(sum |M|^2/n), count of cells with a
   non-finite slot or constraint}, sums over finite cells with r >= r_excise.  With
   norms_host the call synchronises `stream` and returns CCZ4_ENONFINITE if the count is > 0. */
ccz4_status ccz4_constraints(ccz4_ctx *ctx, const double *Q, double *HM, double r_excise,
                             double *norms_host, void *stream);

/* Refinement tags (Sec. 3.6: feature-based refinement by the largest difference between two
   adjacent volumes of a patch).  Plain refinement criterion per leaf (requires filled halos): indicator[p] =
   (max |chi_a - chi_b|, max |alpha_a - alpha_b| over face-adjacent interior cells a, b with
   chi = phi^2, dx^2 max |H|) and e = the largest of the three.  tags[p] = +1 (refine) if
   e >= theta_r and level < max_level; -1 (coarsen) if level > 0, e < theta_c and all 27
   siblings are leaves with e < theta_c; else 0.  indicator (device, n x 3) may be NULL. */
ccz4_status ccz4_tag_refine(ccz4_ctx *ctx, const double *Q, double theta_r, double theta_c,
                            int32_t max_level, int8_t *tags, double *indicator, void *stream);

/* Regrid plan (dynamic AMR on the refinement-criterion hook): the refined cubes of the mesh that
   results from per-leaf tags (host, +1 refine, -1 coarsen, 0 keep; e.g. from ccz4_tag_refine or
   ccz4_tag_learned): every leaf tagged +1 below max_level is refined; a family of 27 leaves all
   tagged -1 is merged into its parent unless a face neighbour of one of them outside the family
   stays refined; then cubes are refined until no face joins leaves two levels apart.
   refined_out (host, cap x 4 int32: lev, i, j, k, sorted by level, k, j, i) receives the list
   for ccz4_create; *n_out its length (also when cap is too small, which returns EINVAL). */
ccz4_status ccz4_regrid_plan(const ccz4_ctx *ctx, const int8_t *tags_host, int32_t max_level,
                             int32_t *refined_out, int64_t cap, int64_t *n_out);

/* State transfer onto the leaves of another mesh of the same domain whose leaves differ from the
   old ones by at most one level (a mesh from ccz4_regrid_plan): a leaf present in both is copied
   whole; a new leaf inside an old leaf one level coarser takes, at each fine cell centre, the
   tensor product over the axes of the linear interpolation of App. E's P-parallel rule on the old
   leaf's interior; a new leaf covering 27 old leaves takes the mean of the 3^3 fine cells at
   each cell.  Halos and ghost slabs of interpolated or averaged leaves keep what Qnew held (the
   analytic initial data after ccz4_init_patches on the new context); fill the halos afterwards.
   Synchronises `stream`. */
ccz4_status ccz4_regrid_transfer(const ccz4_ctx *old_ctx, const double *Qold, const ccz4_ctx *new_ctx,
                                 double *Qnew, void *stream);

/* ---------------------------------------------------------------------------------------
   Learned refinement indicator (a project addition on the refinement-criterion hook of the
   paper's Sec. 3.6): a small perceptron, trained on tags of the plain criterion, that can add
   refinement ahead of the plain criterion and veto its coarsening; the plain criterion stays
   the fallback.  Parameter vector of CCZ4_MLP_NPARAM floats, row-major (out x in):
     W1[64][81] b1[64] W2[64][64] b2[64] W3[3][64] b3[3].
   Inputs are standardised as x = (feat - mu) * inv_sigma in FP32 (norm = mu[81] followed by
   inv_sigma[81]), then every matrix operand (x, weights, ReLU outputs; in the backward pass the
   pre-activation gradients) is rounded to BF16 for the matrix cores, which accumulate in FP32.
   All buffers are device memory owned by the caller; no call allocates. */
enum { CCZ4_MLP_NIN = 81, CCZ4_MLP_NH = 64, CCZ4_MLP_NOUT = 3, CCZ4_MLP_NPARAM = 9603 };

/* Per-leaf features (requires filled halos and HM from ccz4_constraints of the same Q): the
   interior of each leaf is split into 3^3 blocks of 3^3 cells, b = (bz*3 + by)*3 + bx; feat[p*81
   + 3b + q] = log10(max over the block of v_q + 1e-12) with v_0 = dx |grad chi| (chi = phi^2, FD4
   of chi), v_1 = dx |grad alpha| (FD4), v_2 = dx^2 |H|, dx the leaf's spacing (the scaling of the
   plain criterion's indicators, so that leaves of all levels are comparable).  feat: n_leaves x
   81 floats. */
ccz4_status ccz4_features(ccz4_ctx *ctx, const double *Q, const double *HM, float *feat, void *stream);

/* logits[n][3] (classes COARSEN, KEEP, REFINE) of n standardised feature rows. */
ccz4_status ccz4_mlp_forward(const float *params, const float *norm, const float *feat, int64_t n,
                             float *logits, void *stream);

/* Floats of workspace that ccz4_mlp_grad needs for n rows. */
ccz4_status ccz4_mlp_workspace(int64_t n, int64_t *floats);

/* Mean softmax cross-entropy of the logits of n rows against tags in {-1, 0, 1} (COARSEN,
   KEEP, REFINE) and its gradient with respect to every parameter (grad: CCZ4_MLP_NPARAM floats;
   loss: one float, may be NULL).  work: at least ccz4_mlp_workspace(n) floats.  With
   work_floats >= ccz4_mlp_workspace(n) + CCZ4_MLP_TRACE * n the call also leaves, for row r at
   work + ccz4_mlp_workspace(n) + CCZ4_MLP_TRACE * r, the operands of its matrix products as FP32
   values (for checking the gradient layer by layer): the BF16 standardised input x[81], the
   BF16 activations a1[64] and a2[64], and the FP32 pre-activation gradients d3[3] (softmax minus
   one-hot, divided by n), d2[64] and d1[64] before their BF16 rounding. */
enum { CCZ4_MLP_TRACE = 340 };
ccz4_status ccz4_mlp_grad(const float *params, const float *norm, const float *feat, const int8_t *tags,
                          int64_t n, float *work, int64_t work_floats, float *grad, float *loss, void *stream);

/* ccz4_mlp_grad without a workspace, for callers that cannot allocate (code under HIP graph
   capture, tight serving or training loops, harnesses that forbid hipMalloc): the same kernels
   and the same result, bit for bit, with the per-tile partials in an array that the library
   holds on each GPU until the process ends (CCZ4_MLP_NOALLOC_MAX_ROWS / 64 tiles of
   CCZ4_MLP_NPARAM + 1 floats, 2.5 MB).  The call allocates nothing: no hipMalloc, no host or
   device allocation of any library.  n must be 1..CCZ4_MLP_NOALLOC_MAX_ROWS, else EINVAL (use
   ccz4_mlp_grad with a workspace).  Every call on a GPU shares that array: calls that overlap on
   one GPU (on different streams, or from several threads) race and give wrong gradients; calls
   ordered on one stream do not.  No trace is written. */
enum { CCZ4_MLP_NOALLOC_MAX_ROWS = 4096 };
ccz4_status ccz4_mlp_grad_noalloc(const float *params, const float *norm, const float *feat, const int8_t *tags,
                                  int64_t n, float *grad, float *loss, void *stream);

/* One Adam step t >= 1 on every parameter (FP32): m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2,
   params -= lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps). */
ccz4_status ccz4_mlp_adam(float *params, float *m, float *v, const float *grad, int32_t step, float lr,
                          float beta1, float beta2, float eps, void *stream);

/* Combined tags per leaf from the network's logits and the plain criterion's tags: a plain
   REFINE stays; a REFINE predicted with softmax probability >= conf is added (below max_level);
   a plain COARSEN survives unless the network predicts KEEP or REFINE with probability >= conf,
   and a family coarsens only if all 27 of its leaves still do; otherwise KEEP.  Arg-max ties go
   to the higher class. */
ccz4_status ccz4_tag_learned(ccz4_ctx *ctx, const float *logits, const int8_t *plain_tags, float conf,
                             int32_t max_level, int8_t *tags, void *stream);

/* Message of the last failing call of this thread ("" if none). */
const char *ccz4_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
