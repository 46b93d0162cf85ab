/*
 * ccz4_oracle.h -- plain FP64 CPU oracle for the first-order CCZ4 FD4 + Kreiss-Oliger
 * hot path of "ExaGRyPE: Numerical General Relativity Solvers Based upon the Hyperbolic
 * PDEs Solver Engine ExaHyPE" (arXiv:2406.11626).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library may include, link or call this
 * code; only the test-suite, the smoke check and the CPU-baseline leg of the benchmark use it.
 * It shares no code with the HIP path.
 *
 * Conventions (oracle's own):
 *   - 59 slots per cell: the 58 first-order variables in the order of the paper's eq.
 *     (first-order-variables) -- gt_ij(6) alpha beta^i(3) phi At_ij(6) K Theta Ghat^i(3)
 *     b^i(3) A_k(3) B_k^i(9, slot 28+3k+i) D_kij(18, slot 37+6k+sym(ij)) P_k(3) -- plus
 *     slot 58 = K_0 (the constant of the slicing condition, never evolved).
 *   - symmetric pairs ordered xx,xy,xz,yy,yz,zz.
 *   - a patch box is 15^3 cells (9^3 interior + 3 halo layers per face), stored
 *     cell-major: box[(z*15 + y)*15 + x][slot]  (array-of-structures).
 */
#ifndef CCZ4_ORACLE_H
#define CCZ4_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_NV 59
#define ORC_P 9
#define ORC_H 3
#define ORC_NB 15
#define ORC_BOXCELLS (ORC_NB * ORC_NB * ORC_NB)

typedef struct {
    double kappa1, kappa2, kappa3; /* Z4 damping (kappa1, kappa2) and kappa3 of the Gamma eq. */
    double tau;                    /* relaxation time of det(gt)=1 */
    double e;                      /* Hamiltonian-constraint cleaning speed */
    double c;                      /* CCZ4 source switch c */
    double mu;                     /* constraint-term weight in the B equation */
    double f, eta;                 /* Gamma-driver parameters */
    double ko_eps;                 /* Kreiss-Oliger strength epsilon */
    int slicing;                   /* 0: harmonic g(alpha)=1, 1: 1+log g(alpha)=2/alpha */
    int shift;                     /* 0: frozen (static) shift, 1: Gamma-driver (s=1) */
    int formulation;               /* 0: first order (FO, all 58 evolve, red terms on);
                                      1: second order (SO, the 24 primaries evolve, red terms
                                      off, A, B, D, P reconstructed after every update) */
    int advection;                 /* derivative of the advection terms beta^k d_k Q (App. D):
                                      0: central FD4; 1: lopsided FD4, the stencil biased towards
                                      +x_k where beta^k > 0 (upwind reading); 2: lopsided FD4 with
                                      the pairing as printed (biased towards -x_k where beta^k > 0) */
} orc_params;

/* ---- pointwise algebra (App. B) ---- */
void orc_rhs_point(const orc_params *pr, const double *q, const double *dq /* [3][59] */,
                   double *out /* [59] */);
void orc_constraints_point(const double *q, const double *dq /* [3][59] */, double *hm /* [4] */);

/* ---- one-dimensional stencils (App. D) ---- */
double orc_fd4(const double *v5 /* Q--,Q-,Q,Q+,Q++ */, double dx);
double orc_ko(const double *v7 /* Q---..Q+++ */, double dx, double eps);
/* the lopsided fourth-order first derivatives of App. D on Q---..Q+++: right = 1 uses
   Q-..Q+++, right = 0 uses Q---..Q+ */
double orc_fd4_lop(const double *v7, double dx, int right);

/* ---- one patch box with filled halos ---- */
void orc_rhs_box(const orc_params *pr, const double dx[3], const double *box, double *out);
void orc_constraints_box(const double dx[3], const double *box, double *hm /* [729][4] */);

/* ---- mesh of patches ---- */
typedef struct orc_mesh orc_mesh;

enum { ORC_BC_PERIODIC = 0, ORC_BC_NEUMANN = 1, ORC_BC_SOMMERFELD = 2 };

orc_mesh *orc_mesh_create(const int n0[3], const double origin[3], const double extent[3],
                          int bc, int n_refined, const int *refined /* [n][4]: lev,i,j,k */);
void orc_mesh_destroy(orc_mesh *m);
/* Coarse-fine halo operators.  0: App. E as printed (P_par x P_par x P_perp linear, R_avg x
   R_avg x R_perp average and linear extrapolation).  1: higher order (the paper's suggested
   remedy for reflections at refinement boundaries, Sec. 5.2): restriction injects the fine cell
   whose centre coincides with the coarse halo centre (tangentially the middle of three fine
   cells, along the normal the fine interior depth 2, 5 or 8), and prolongation interpolates
   with three-point Lagrange quadratics along each axis (coarse layers c1, c2 and the restricted
   c3 along the normal).  Both reproduce quadratic fields exactly. */
void orc_mesh_set_transfer(orc_mesh *m, int transfer);
int64_t orc_mesh_npatches(const orc_mesh *m);
/* per leaf: lev, i, j, k */
void orc_mesh_patch_ids(const orc_mesh *m, int *ids /* [n][4] */);
/* per leaf: origin xyz (lower corner of the interior) and dx xyz */
void orc_mesh_patch_geom(const orc_mesh *m, double *geom /* [n][6] */);

/* scenario 0 gauge wave (sp: A, k); 1 single puncture (sp: M, x0,y0,z0, lapse kind);
   2 Brill-Lindquist + Bowen-York (sp: m1,x1,y1,z1,Px1,Py1,Pz1, m2,...)  */
int orc_init_point(int scenario, const double *sp, const double x[3], double *q /* [59] */);
int orc_init(const orc_mesh *m, double *Q, int scenario, const double *sp);

void orc_set_background(orc_mesh *m, const double *Q);
void orc_fill_halos(const orc_mesh *m, double *Q);
void orc_rhs(const orc_mesh *m, const orc_params *pr, const double *Q, double *kout);
/* host threads of the patch loops of orc_rhs, orc_rhs_subset and orc_rk4_stage (OpenMP) */
void orc_set_threads(int n);
int orc_max_threads(void);
/* Second-order formulation: the auxiliaries A_k = d_k alpha, B_k^i = d_k beta^i,
   D_kij = d_k gt_ij / 2, P_k = d_k phi on every leaf interior cell, from central FD4
   differences of the primaries (whose halos must be filled); halos are left as they are. */
void orc_reconstruct_aux(const orc_mesh *m, double *Q);
void orc_rhs_subset(const orc_mesh *m, const orc_params *pr, const double *Q, double *kout,
                    int64_t n_sel, const int64_t *sel);
int orc_rk4_stage(const orc_mesh *m, int s, double dt, const double *Qn, const double *k,
                  double *acc, double *Qnext);
void orc_project_point(double *q);
int64_t orc_constraints(const orc_mesh *m, const double *Q, double *HM /* [n][729][4] or NULL */,
                        double r_excise, double norms[3]);
void orc_tag_indicator(const orc_mesh *m, const double *Q, double *ind /* [n][3] */);

/* ---- tracers (Sec. 3.8) and puncture trackers (Sec. 4.2.3, puncture tracking) ---- */
/* the leaf whose interior box [o, o + 9 dx) holds x, or -1 */
int64_t orc_find_leaf(const orc_mesh *m, const double x[3]);
/* trilinear interpolation of nslot slots at n points pos[n][3] from the 2^3 cell centres around
   each (the leaf's filled halos supply the centres beyond its interior); out[n][nslot];
   returns the number of points outside every leaf (their samples are NaN) */
int64_t orc_tracer_sample(const orc_mesh *m, const double *Q, int64_t n, const double *pos, int nslot,
                          const int *slots, double *out);
/* one explicit Euler step of puncture trackers: x <- x + dt v with v = -beta(x) interpolated as
   above; points outside every leaf stay; returns their number */
int64_t orc_tracer_advance(const orc_mesh *m, const double *Q, int64_t n, double *pos, double dt);
/* Tracker-based refinement tags (Sec. 4.2.1, refinement by coordinates): with R_l = radii[l],
   a leaf of level l < min(max_level, nrad) whose cube lies within R_l of a tracer gets REFINE (1);
   a leaf of level l >= 1 whose parent cube lies farther than R_(l-1) from every tracer gets
   COARSEN (-1); every other leaf KEEP (0).  Distances are from the tracer to the nearest point
   of the closed cube.  A mesh refined by concentric spheres of these radii around the tracers
   is a fixed point (all KEEP). */
void orc_tag_tracers(const orc_mesh *m, int64_t n, const double *pos, int nrad, const double *radii, int max_level,
                     int8_t *tags);
void orc_tag_refine(const orc_mesh *m, const double *Q, double theta_r, double theta_c,
                    int max_level, int8_t *tags);

/* ---- regrid ---- */
int64_t orc_regrid_plan(const orc_mesh *m, const int8_t *tags, int max_level, int *out /* [cap][4] */,
                        int64_t cap);
void orc_regrid_transfer(const orc_mesh *mo, const double *Qo, const orc_mesh *mn, double *Qn);

/* ---- learned refinement indicator (ccz4_mlp.c) ---- */
#define ORC_MLP_NIN 81
#define ORC_MLP_NH 64
#define ORC_MLP_NOUT 3
#define ORC_MLP_NPARAM 9603 /* W1[64][81] b1[64] W2[64][64] b2[64] W3[3][64] b3[3] */
void orc_features(const orc_mesh *m, const double *Q, double *feat /* [n][81] */);
double orc_bf16_round(double x);
void orc_mlp_standardize(int64_t n, const float *feat, const float *norm /* mu[81], inv_sigma[81] */,
                         double *x);
void orc_mlp_forward(int64_t n, const double *x, const double *prm, int bf16, double *a1, double *a2,
                     double *z3);
double orc_mlp_loss_grad(int64_t n, const double *x, const int32_t *labels, const double *prm, int bf16,
                         double *grad);
void orc_tag_learned(const orc_mesh *m, const float *logits /* [n][3] */, const int8_t *plain, float conf,
                     int max_level, int8_t *tags);
void orc_adam_step(int64_t n, double *p, double *mom, double *vel, const double *g, int t, double lr, double b1,
                   double b2, double eps);

#ifdef __cplusplus
}
#endif
#endif
