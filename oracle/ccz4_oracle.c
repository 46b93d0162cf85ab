/*
 * Oracle (test infrastructure only): stencils, patch boxes, mesh of patches, initial data,
 * halo filling, RK4 stage combine, algebraic projection, constraints and tagging for the
 * first-order CCZ4 FD4 hot path of arXiv:2406.11626.  Plain loops in FP64; nothing here is
 * blocked, fused or reordered beyond what the paper's definitions state.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include "ccz4_oracle.h"

#define NV ORC_NV
#define NB ORC_NB
#define PP ORC_P
#define HH ORC_H

static int64_t cix(int x, int y, int z) { return ((int64_t)z * NB + y) * NB + x; }

/* ----------------------------------------------------------------------------------------
 * One-dimensional stencils (App. D).
 * Central fourth-order first derivative, eq. (eq_exa_fd4_central_difference):
 *   dQ/dx = [8 (Q+ - Q-) - (Q++ - Q--)] / (12 dx).
 * Kreiss-Oliger dissipation of order N = 3, eq. (eq_exa_fd4_ko):
 *   KO = eps/(64 dx) (Q--- - 6Q-- + 15Q- - 20Q + 15Q+ - 6Q++ + Q+++).
 * ---------------------------------------------------------------------------------------- */
double orc_fd4(const double *v, double dx)
{
    return (8.0 * (v[3] - v[1]) - (v[4] - v[0])) / (12.0 * dx);
}

double orc_ko(const double *v, double dx, double eps)
{
    return eps / (64.0 * dx) *
           (v[0] - 6.0 * v[1] + 15.0 * v[2] - 20.0 * v[3] + 15.0 * v[4] - 6.0 * v[5] + v[6]);
}

double orc_fd4_lop(const double *v, double dx, int right)
{
    if (right) return (-3.0 * v[2] - 10.0 * v[3] + 18.0 * v[4] - 6.0 * v[5] + v[6]) / (12.0 * dx);
    return (-v[0] + 6.0 * v[1] - 18.0 * v[2] + 10.0 * v[3] + 3.0 * v[4]) / (12.0 * dx);
}

static int frozen_slot(const orc_params *pr, int v)
{
    /* beta^i (7-9), b^i (22-24), B_k^i (28-36) do not evolve with the static shift */
    if (pr->shift) return 0;
    return (v >= 7 && v <= 9) || (v >= 22 && v <= 24) || (v >= 28 && v <= 36);
}

/* Right-hand side on the 9^3 interior of one box whose halos are filled.  Algorithm 1 of
   the paper (FD4 first-order step): per volume, the source and the non-conservative
   products from the central FD4 derivatives along x, y, z, plus the KO sum over the axes.
   Slots 11..57 are differentiated; KO acts on the 58 evolved slots. */
void orc_rhs_box(const orc_params *pr, const double dx[3], const double *box, double *out)
{
    int x, y, z, a, v, s;
    double dq[3 * NV], q[NV], r[NV], w[7];
    for (z = HH; z < HH + PP; z++)
        for (y = HH; y < HH + PP; y++)
            for (x = HH; x < HH + PP; x++) {
                const int64_t c = cix(x, y, z);
                memcpy(q, box + c * NV, sizeof(q));
                memset(dq, 0, sizeof(dq));
                for (a = 0; a < 3; a++) {
                    for (v = 11; v <= 57; v++) {
                        for (s = -2; s <= 2; s++) {
                            int xx = x + (a == 0 ? s : 0), yy = y + (a == 1 ? s : 0),
                                zz = z + (a == 2 ? s : 0);
                            w[s + 2] = box[cix(xx, yy, zz) * NV + v];
                        }
                        dq[a * NV + v] = orc_fd4(w, dx[a]);
                    }
                }
                orc_rhs_point(pr, q, dq, r);
                /* Lopsided advection (App. D): in every equation of a differentiated slot the
                   advection term is +beta^k d_k Q_v with the slot's own derivative (App. B; in the
                   b equation the two Ghat advection terms cancel).  The algebra above used the
                   central difference there; replace it by the lopsided one along each axis. */
                if (pr->advection)
                    for (v = 11; v <= 57; v++) {
                        if (frozen_slot(pr, v) || (pr->formulation && v >= 25)) continue;
                        for (a = 0; a < 3; a++) {
                            const double be = q[7 + a];
                            const int right = pr->advection == 1 ? be > 0.0 : !(be > 0.0);
                            for (s = -3; s <= 3; s++) {
                                int xx = x + (a == 0 ? s : 0), yy = y + (a == 1 ? s : 0),
                                    zz = z + (a == 2 ? s : 0);
                                w[s + 3] = box[cix(xx, yy, zz) * NV + v];
                            }
                            r[v] += be * (orc_fd4_lop(w, dx[a], right) - dq[a * NV + v]);
                        }
                    }
                for (v = 0; v < 58; v++) {
                    double ko = 0;
                    if (frozen_slot(pr, v)) continue;
                    if (pr->formulation && v >= 25) continue; /* SO: KO on the primaries only */
                    for (a = 0; a < 3; a++) {
                        for (s = -3; s <= 3; s++) {
                            int xx = x + (a == 0 ? s : 0), yy = y + (a == 1 ? s : 0),
                                zz = z + (a == 2 ? s : 0);
                            w[s + 3] = box[cix(xx, yy, zz) * NV + v];
                        }
                        ko += orc_ko(w, dx[a], pr->ko_eps);
                    }
                    r[v] += ko;
                }
                r[58] = 0.0;
                memcpy(out + c * NV, r, sizeof(r));
            }
}

/* Constraints on the 9^3 interior of one box: hm[cell][4] = (H, M_x, M_y, M_z), interior
   cells in x-fastest order.  Derivatives are the same central FD4 differences. */
void orc_constraints_box(const double dx[3], const double *box, double *hm)
{
    int x, y, z, a, v, s;
    double dq[3 * NV], w[5];
    int64_t n = 0;
    for (z = HH; z < HH + PP; z++)
        for (y = HH; y < HH + PP; y++)
            for (x = HH; x < HH + PP; x++, n++) {
                memset(dq, 0, sizeof(dq));
                for (a = 0; a < 3; a++)
                    for (v = 11; v <= 57; v++) {
                        for (s = -2; s <= 2; s++) {
                            int xx = x + (a == 0 ? s : 0), yy = y + (a == 1 ? s : 0),
                                zz = z + (a == 2 ? s : 0);
                            w[s + 2] = box[cix(xx, yy, zz) * NV + v];
                        }
                        dq[a * NV + v] = orc_fd4(w, dx[a]);
                    }
                orc_constraints_point(box + cix(x, y, z) * NV, dq, hm + 4 * n);
            }
}

/* ----------------------------------------------------------------------------------------
 * Mesh of patches: a forest of n0 level-0 cubes over [origin, origin+extent], each refined
 * cube split into 3^3 children (tri-partitioning, ratio 3).  Leaves carry the data.  The
 * leaves are ordered by (level, k, j, i).
 * ---------------------------------------------------------------------------------------- */
struct orc_mesh {
    int n0[3];
    double origin[3], extent[3];
    int bc;
    int nref;
    int *ref;      /* refined cubes: lev,i,j,k */
    int64_t np;
    int *id;       /* leaves: lev,i,j,k */
    double *bg;    /* Sommerfeld background: one full box per leaf touching the boundary */
    int64_t *bgix; /* leaf -> background box index or -1 */
    int transfer;  /* coarse-fine operators: 0 as printed in App. E, 1 higher order */
};

void orc_mesh_set_transfer(orc_mesh *m, int transfer) { m->transfer = transfer; }

static int lev_n(const orc_mesh *m, int lev, int a)
{
    int n = m->n0[a];
    while (lev-- > 0) n *= 3;
    return n;
}

/* keys are (lev, k, j, i) compared lexicographically: the canonical leaf order */
static int cmp4(const void *pa, const void *pb)
{
    const int *x = (const int *)pa, *y = (const int *)pb;
    static const int ord[4] = {0, 3, 2, 1};
    int t;
    for (t = 0; t < 4; t++)
        if (x[ord[t]] != y[ord[t]]) return x[ord[t]] < y[ord[t]] ? -1 : 1;
    return 0;
}

static int is_refined(const orc_mesh *m, int lev, int i, int j, int k)
{
    int key[4] = {lev, i, j, k};
    return m->nref > 0 && bsearch(key, m->ref, m->nref, sizeof(int) * 4, cmp4) != NULL;
}

/* A cube exists if it is level 0 or its parent is refined. */
static int exists(const orc_mesh *m, int lev, int i, int j, int k)
{
    if (i < 0 || j < 0 || k < 0 || i >= lev_n(m, lev, 0) || j >= lev_n(m, lev, 1) ||
        k >= lev_n(m, lev, 2))
        return 0;
    if (lev == 0) return 1;
    return is_refined(m, lev - 1, i / 3, j / 3, k / 3) && exists(m, lev - 1, i / 3, j / 3, k / 3);
}

static int64_t find_leaf(const orc_mesh *m, int lev, int i, int j, int k)
{
    int key[4] = {lev, i, j, k};
    const int *hit;
    if (m->np == 0) return -1;
    hit = (const int *)bsearch(key, m->id, m->np, sizeof(int) * 4, cmp4);
    return hit ? (int64_t)(hit - m->id) / 4 : -1;
}

static void push4(int **arr, int64_t *n, int64_t *cap, int l, int i, int j, int k)
{
    if (*n == *cap) {
        *cap = *cap ? 2 * *cap : 1024;
        *arr = (int *)realloc(*arr, sizeof(int) * 4 * *cap);
    }
    (*arr)[4 * *n] = l;
    (*arr)[4 * *n + 1] = i;
    (*arr)[4 * *n + 2] = j;
    (*arr)[4 * *n + 3] = k;
    (*n)++;
}

orc_mesh *orc_mesh_create(const int n0[3], const double origin[3], const double extent[3],
                          int bc, int n_refined, const int *refined)
{
    orc_mesh *m = (orc_mesh *)calloc(1, sizeof(orc_mesh));
    int a, i, j, k, u, v, w;
    int64_t cap = 0, r;
    for (a = 0; a < 3; a++) {
        m->n0[a] = n0[a];
        m->origin[a] = origin[a];
        m->extent[a] = extent[a];
    }
    m->bc = bc;
    m->nref = n_refined > 0 ? n_refined : 0;
    m->ref = (int *)malloc(sizeof(int) * 4 * (m->nref > 0 ? m->nref : 1));
    if (m->nref > 0) memcpy(m->ref, refined, sizeof(int) * 4 * (size_t)m->nref);
    qsort(m->ref, m->nref, sizeof(int) * 4, cmp4);
    m->id = NULL;
    m->np = 0;
    /* level-0 cubes, then the children of every refined cube; keep the unrefined ones */
    for (k = 0; k < n0[2]; k++)
        for (j = 0; j < n0[1]; j++)
            for (i = 0; i < n0[0]; i++)
                if (!is_refined(m, 0, i, j, k)) push4(&m->id, &m->np, &cap, 0, i, j, k);
    for (r = 0; r < m->nref; r++) {
        const int *c = m->ref + 4 * r;
        if (!exists(m, c[0], c[1], c[2], c[3])) continue;
        for (w = 0; w < 3; w++)
            for (v = 0; v < 3; v++)
                for (u = 0; u < 3; u++)
                    if (!is_refined(m, c[0] + 1, 3 * c[1] + u, 3 * c[2] + v, 3 * c[3] + w))
                        push4(&m->id, &m->np, &cap, c[0] + 1, 3 * c[1] + u, 3 * c[2] + v,
                              3 * c[3] + w);
    }
    qsort(m->id, m->np, sizeof(int) * 4, cmp4);
    m->bgix = (int64_t *)malloc(sizeof(int64_t) * (m->np ? m->np : 1));
    for (r = 0; r < m->np; r++) m->bgix[r] = -1;
    return m;
}

void orc_mesh_destroy(orc_mesh *m)
{
    if (!m) return;
    free(m->ref);
    free(m->id);
    free(m->bg);
    free(m->bgix);
    free(m);
}

int64_t orc_mesh_npatches(const orc_mesh *m) { return m->np; }

void orc_mesh_patch_ids(const orc_mesh *m, int *ids) { memcpy(ids, m->id, sizeof(int) * 4 * m->np); }

static void patch_geom(const orc_mesh *m, int64_t p, double org[3], double dx[3])
{
    int a, lev = m->id[4 * p];
    for (a = 0; a < 3; a++) {
        double L = m->extent[a] / lev_n(m, lev, a);
        org[a] = m->origin[a] + L * m->id[4 * p + 1 + a];
        dx[a] = L / PP;
    }
}

void orc_mesh_patch_geom(const orc_mesh *m, double *geom)
{
    int64_t p;
    for (p = 0; p < m->np; p++) patch_geom(m, p, geom + 6 * p, geom + 6 * p + 3);
}

/* centre of box cell (x,y,z) (box coordinates 0..14, interior 3..11) */
static void cell_center(const orc_mesh *m, int64_t p, int x, int y, int z, double out[3])
{
    double org[3], dx[3];
    int c[3] = {x, y, z}, a;
    patch_geom(m, p, org, dx);
    for (a = 0; a < 3; a++) out[a] = org[a] + (c[a] - HH + 0.5) * dx[a];
}

/* ----------------------------------------------------------------------------------------
 * Initial data.
 *  0: gauge wave (the paper's gauge-wave section): H = 1 - A sin(k pi (x - t)) at t = 0,
 *     alpha = sqrt(H), gamma = diag(H,1,1), phi = H^(-1/6), K_xx = -d_t H/(2 alpha),
 *     K = K_xx/H; conformal variables and the auxiliaries A, D, P follow from their
 *     definitions; Ghat = Gt (Z = 0), Theta = 0, zero shift.
 *  1: single puncture (the paper's single black hole section): psi = 1 + M/(2r),
 *     phi = psi^-2, gt = delta, K_ij = 0; lapse kind sp[4]: 0 -> alpha = psi^-2,
 *     1 -> alpha = ((1 - M/2r)/(1 + M/2r) + 1)/2 (the paper's averaged lapse),
 *     2 -> alpha = (1 - M/2r)/(1 + M/2r) (static isotropic Schwarzschild).
 *  2: two Brill-Lindquist punctures with Bowen-York extrinsic curvature (no spin, no
 *     puncture correction): psi = 1 + sum m_a/(2 r_a), At = psi^-6 Ahat,
 *     Ahat_ij = sum 3/(2 r_a^2) [P_i n_j + P_j n_i - (delta_ij - n_i n_j) P.n], K = 0,
 *     alpha = psi^-2.
 * ---------------------------------------------------------------------------------------- */
int orc_init_point(int scenario, const double *sp, const double xx[3], double *q)
{
    int i, j, k;
    memset(q, 0, sizeof(double) * NV);
    if (scenario == 0) {
        const double A = sp[0], kk = sp[1], pi = 3.14159265358979323846;
        const double Hh = 1.0 - A * sin(kk * pi * xx[0]);
        const double Hp = -A * kk * pi * cos(kk * pi * xx[0]); /* dH/dx (= -dH/dt) */
        const double al = sqrt(Hh);
        const double Kxx = Hp / (2.0 * al); /* -d_t H / (2 alpha) with d_t H = -H' */
        const double Kt = Kxx / Hh;
        q[0] = pow(Hh, 2.0 / 3.0);           /* gt_xx */
        q[3] = pow(Hh, -1.0 / 3.0);          /* gt_yy */
        q[5] = pow(Hh, -1.0 / 3.0);          /* gt_zz */
        q[6] = al;
        q[10] = pow(Hh, -1.0 / 6.0);
        q[11] = 2.0 / 3.0 * pow(Hh, -1.0 / 3.0) * Kxx;  /* At_xx */
        q[14] = -1.0 / 3.0 * pow(Hh, -4.0 / 3.0) * Kxx; /* At_yy */
        q[16] = -1.0 / 3.0 * pow(Hh, -4.0 / 3.0) * Kxx; /* At_zz */
        q[17] = Kt;
        q[19] = 2.0 / 3.0 * pow(Hh, -5.0 / 3.0) * Hp;   /* Ghat^x = Gt^x */
        q[25] = Hp / (2.0 * al);                        /* A_x */
        q[37 + 0] = 1.0 / 3.0 * pow(Hh, -1.0 / 3.0) * Hp;  /* D_xxx */
        q[37 + 3] = -1.0 / 6.0 * pow(Hh, -4.0 / 3.0) * Hp; /* D_xyy */
        q[37 + 5] = -1.0 / 6.0 * pow(Hh, -4.0 / 3.0) * Hp; /* D_xzz */
        q[55] = -1.0 / 6.0 * pow(Hh, -7.0 / 6.0) * Hp;     /* P_x */
        return 0;
    }
    if (scenario == 1) {
        const double M = sp[0];
        double d[3], r, psi, dpsi[3], al, dal[3];
        for (i = 0; i < 3; i++) d[i] = xx[i] - sp[1 + i];
        r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        psi = 1.0 + M / (2.0 * r);
        for (i = 0; i < 3; i++) dpsi[i] = -M * d[i] / (2.0 * r * r * r);
        q[0] = q[3] = q[5] = 1.0;
        q[10] = 1.0 / (psi * psi);
        for (i = 0; i < 3; i++) q[55 + i] = -2.0 / (psi * psi * psi) * dpsi[i];
        if ((int)sp[4] == 0) {
            al = 1.0 / (psi * psi);
            for (i = 0; i < 3; i++) dal[i] = -2.0 / (psi * psi * psi) * dpsi[i];
        } else {
            /* alpha_s = (1 - M/2r)/(1 + M/2r) = (2 - psi)/psi,  d alpha_s = -2 dpsi / psi^2 */
            double as = (2.0 - psi) / psi;
            double w = ((int)sp[4] == 1) ? 0.5 : 1.0;
            al = ((int)sp[4] == 1) ? 0.5 * (as + 1.0) : as;
            for (i = 0; i < 3; i++) dal[i] = w * (-2.0 / (psi * psi)) * dpsi[i];
        }
        q[6] = al;
        for (i = 0; i < 3; i++) q[25 + i] = dal[i];
        return 0;
    }
    if (scenario == 2) {
        double psi = 1.0, dpsi[3] = {0, 0, 0}, Ah[3][3] = {{0}};
        int a;
        for (a = 0; a < 2; a++) {
            const double *s = sp + 7 * a;
            double d[3], r, n[3], Pn = 0;
            for (i = 0; i < 3; i++) d[i] = xx[i] - s[1 + i];
            r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
            for (i = 0; i < 3; i++) n[i] = d[i] / r;
            psi += s[0] / (2.0 * r);
            for (i = 0; i < 3; i++) dpsi[i] += -s[0] * d[i] / (2.0 * r * r * r);
            for (i = 0; i < 3; i++) Pn += s[4 + i] * n[i];
            for (i = 0; i < 3; i++)
                for (j = 0; j < 3; j++)
                    Ah[i][j] += 3.0 / (2.0 * r * r) *
                                (s[4 + i] * n[j] + s[4 + j] * n[i] -
                                 ((i == j ? 1.0 : 0.0) - n[i] * n[j]) * Pn);
        }
        q[0] = q[3] = q[5] = 1.0;
        q[10] = 1.0 / (psi * psi);
        q[6] = 1.0 / (psi * psi);
        for (i = 0; i < 3; i++) {
            q[55 + i] = -2.0 / (psi * psi * psi) * dpsi[i];
            q[25 + i] = q[55 + i];
        }
        k = 11;
        for (i = 0; i < 3; i++)
            for (j = i; j < 3; j++) q[k++] = pow(psi, -6.0) * Ah[i][j];
        return 0;
    }
    return -1;
}

static int on_phys_boundary(const orc_mesh *m, int64_t p, int a, int side)
{
    int lev = m->id[4 * p], i = m->id[4 * p + 1 + a];
    if (m->bc == ORC_BC_PERIODIC) return 0;
    return side < 0 ? (i == 0) : (i == lev_n(m, lev, a) - 1);
}

/* Initial data on the interior of every leaf and, with the Sommerfeld condition, on the
   ghost layers of faces on the domain boundary (those ghosts are evolved, not filled).
   The interior and the Sommerfeld ghosts are then projected (det gt = 1, tr At = 0). */
int orc_init(const orc_mesh *m, double *Q, int scenario, const double *sp)
{
    int64_t p;
    int x, y, z;
    for (p = 0; p < m->np; p++) {
        double *box = Q + p * (int64_t)ORC_BOXCELLS * NV;
        for (z = 0; z < NB; z++)
            for (y = 0; y < NB; y++)
                for (x = 0; x < NB; x++) {
                    int c[3] = {x, y, z}, a, nin = 0, ghost_ok = 0;
                    double xx[3];
                    for (a = 0; a < 3; a++) nin += (c[a] >= HH && c[a] < HH + PP);
                    if (nin == 3) ghost_ok = 1;
                    else if (nin == 2 && m->bc == ORC_BC_SOMMERFELD) {
                        for (a = 0; a < 3; a++) {
                            if (c[a] < HH && on_phys_boundary(m, p, a, -1)) ghost_ok = 1;
                            if (c[a] >= HH + PP && on_phys_boundary(m, p, a, +1)) ghost_ok = 1;
                        }
                    }
                    if (!ghost_ok) continue;
                    cell_center(m, p, x, y, z, xx);
                    if (orc_init_point(scenario, sp, xx, box + cix(x, y, z) * NV)) return -1;
                    if (nin == 3) orc_project_point(box + cix(x, y, z) * NV);
                }
    }
    orc_set_background((orc_mesh *)m, Q);
    return 0;
}

/* Snapshot the Sommerfeld ghost values of every boundary leaf as Q_ini. */
void orc_set_background(orc_mesh *m, const double *Q)
{
    int64_t p, nb = 0;
    int a;
    free(m->bg);
    m->bg = NULL;
    for (p = 0; p < m->np; p++) {
        int any = 0;
        for (a = 0; a < 3; a++) any |= on_phys_boundary(m, p, a, -1) | on_phys_boundary(m, p, a, 1);
        m->bgix[p] = any ? nb++ : -1;
    }
    if (!nb) return;
    m->bg = (double *)malloc(sizeof(double) * nb * ORC_BOXCELLS * NV);
    for (p = 0; p < m->np; p++)
        if (m->bgix[p] >= 0)
            memcpy(m->bg + m->bgix[p] * ORC_BOXCELLS * NV, Q + p * (int64_t)ORC_BOXCELLS * NV,
                   sizeof(double) * ORC_BOXCELLS * NV);
}

/* ----------------------------------------------------------------------------------------
 * Halo filling (paper: patch/face data layout, boundary treatment, AMR and App. E).
 * For every leaf and each of its six faces (axis a, side s):
 *   - same-level leaf neighbour (with periodic wrap): copy its three interior layers;
 *   - domain boundary: Neumann copies the boundary layer outwards layer by layer,
 *     Sommerfeld leaves the ghosts alone (they are evolved by the RHS and RK stage);
 *   - neighbour refined (finer leaves behind the face): RESTRICT, coarse halo layers
 *     c3,c4,c5 = (R_avg x R_avg x R_perp) of the fine interior layers f3,f4,f5;
 *   - neighbour covered by a coarser leaf: PROLONG, fine halo layers f0,f1,f2 =
 *     (P_par x P_par x P_perp) of the coarse layers c0..c5 (c3..c5 = coarse halo).
 * All restrictions are done before any prolongation because P_perp reads c3.
 * Edges and corners of the box are never filled (the stencils are axis-aligned).
 * ---------------------------------------------------------------------------------------- */

/* P_parallel (3p x p): row F maps to coarse u = (F+1/2)/3 - 1/2, linear between
   l = clamp(floor(u), 0, p-2) and l+1 (rows of App. E, with extrapolation at both ends). */
static void build_P_par(double Ppar[3 * PP][PP])
{
    int F, l;
    memset(Ppar, 0, sizeof(double) * 3 * PP * PP);
    for (F = 0; F < 3 * PP; F++) {
        double u = (F + 0.5) / 3.0 - 0.5;
        l = (int)floor(u);
        if (l < 0) l = 0;
        if (l > PP - 2) l = PP - 2;
        Ppar[F][l] = 1.0 - (u - l);
        Ppar[F][l + 1] = u - l;
    }
}

static const double P_perp[3][6] = {{0, 1.0 / 3, 2.0 / 3, 0, 0, 0},
                                    {0, 0, 1, 0, 0, 0},
                                    {0, 0, 2.0 / 3, 1.0 / 3, 0, 0}};
static const double R_perp[3][6] = {{0, 0, 0, 1.0 / 3, 1.0 / 3, 1.0 / 3},
                                    {0, 0, 0, 0, -2, 3},
                                    {0, 0, 0, 0, -5, 6}};

/* box coordinate of a cell at "depth" d from a face: d = 1..3 inside (1 adjacent to the
   face), d = -1..-3 outside (ghost layer -d, -1 adjacent) */
static int layer_coord(int side, int d)
{
    if (side > 0) return d > 0 ? HH + PP - d : HH + PP - 1 - d;
    return d > 0 ? HH - 1 + d : HH + d;
}

static double *cellp(double *Q, int64_t p, int c[3])
{
    return Q + (p * (int64_t)ORC_BOXCELLS + cix(c[0], c[1], c[2])) * NV;
}

static void fill_face_copy(const orc_mesh *m, double *Q, int64_t p, int a, int side, int64_t nb)
{
    int t1, t2, L, c[3], cn[3];
    const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
    for (L = 1; L <= 3; L++)
        for (t2 = HH; t2 < HH + PP; t2++)
            for (t1 = HH; t1 < HH + PP; t1++) {
                c[b1] = cn[b1] = t1;
                c[b2] = cn[b2] = t2;
                c[a] = layer_coord(side, -L);
                cn[a] = layer_coord(-side, L); /* neighbour's interior layer L from the shared face */
                memcpy(cellp(Q, p, c), cellp(Q, nb, cn), sizeof(double) * NV);
            }
    (void)m;
}

static void fill_face_neumann(double *Q, int64_t p, int a, int side)
{
    /* Q_out = Q_in layer by layer outwards: ghost L takes the value of ghost L-1, ghost 1
       that of the boundary interior layer, so every ghost equals the boundary layer. */
    int t1, t2, L, c[3], ci[3];
    const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
    for (L = 1; L <= 3; L++)
        for (t2 = HH; t2 < HH + PP; t2++)
            for (t1 = HH; t1 < HH + PP; t1++) {
                c[b1] = ci[b1] = t1;
                c[b2] = ci[b2] = t2;
                c[a] = layer_coord(side, -L);
                ci[a] = (L == 1) ? layer_coord(side, 1) : layer_coord(side, -(L - 1));
                memcpy(cellp(Q, p, c), cellp(Q, p, ci), sizeof(double) * NV);
            }
}

/* coarse leaf p (level lev) face (a, side) whose neighbour cube is refined: restrict from
   the 9 fine children that touch the face. */
static void fill_face_restrict(const orc_mesh *m, double *Q, int64_t p, int a, int side,
                               int ni[3])
{
    const int b1 = (a + 1) % 3, b2 = (a + 2) % 3, lev = m->id[4 * p];
    int64_t kids[3][3];
    int u1, u2, L, v, F1, F2, m6, c[3];
    /* fine children of the neighbour cube adjacent to the shared face */
    for (u2 = 0; u2 < 3; u2++)
        for (u1 = 0; u1 < 3; u1++) {
            int ci[3];
            ci[a] = 3 * ni[a] + (side > 0 ? 0 : 2);
            ci[b1] = 3 * ni[b1] + u1;
            ci[b2] = 3 * ni[b2] + u2;
            kids[u2][u1] = find_leaf(m, lev + 1, ci[0], ci[1], ci[2]);
        }
    if (m->transfer == 1) {
        /* injection: coarse halo layer c_{2+L} at normal distance (L - 1/2) coarse cells from
           the face = (3L - 3/2) fine cells: fine interior depth 3L - 1; tangentially the
           middle fine cell 3u + 1 of the three under coarse cell u */
        for (L = 1; L <= 3; L++)
            for (u2 = 0; u2 < PP; u2++)
                for (u1 = 0; u1 < PP; u1++) {
                    const int Fa = 3 * u1 + 1, Fb = 3 * u2 + 1;
                    int cf[3];
                    cf[b1] = HH + Fa % PP;
                    cf[b2] = HH + Fb % PP;
                    cf[a] = layer_coord(-side, 3 * L - 1);
                    c[b1] = HH + u1;
                    c[b2] = HH + u2;
                    c[a] = layer_coord(side, -L);
                    memcpy(cellp(Q, p, c), cellp(Q, kids[Fb / PP][Fa / PP], cf), sizeof(double) * NV);
                }
        return;
    }
    for (L = 1; L <= 3; L++)           /* coarse halo layer c_{2+L} */
        for (u2 = 0; u2 < PP; u2++)    /* coarse tangential index along b2 */
            for (u1 = 0; u1 < PP; u1++) {
                double acc[NV];
                memset(acc, 0, sizeof(acc));
                /* sum over fine tangential F1, F2 in [0,27) and fine layers f0..f5 */
                for (F2 = 0; F2 < 3 * PP; F2++)
                    for (F1 = 0; F1 < 3 * PP; F1++) {
                        double w1 = (F1 / 3 == u1) ? 1.0 / 3.0 : 0.0; /* R_avg */
                        double w2 = (F2 / 3 == u2) ? 1.0 / 3.0 : 0.0;
                        if (w1 == 0.0 || w2 == 0.0) continue;
                        for (m6 = 3; m6 < 6; m6++) {
                            double w = w1 * w2 * R_perp[L - 1][m6];
                            int64_t kid = kids[F2 / PP][F1 / PP];
                            int cf[3];
                            if (w == 0.0) continue;
                            cf[b1] = HH + F1 % PP;
                            cf[b2] = HH + F2 % PP;
                            /* fine layer f_{m6}, m6 = 3..5: fine interior depth m6-2 from the
                               face shared with the coarse leaf (that face is -side for the kid) */
                            cf[a] = layer_coord(-side, m6 - 2);
                            const double *src = cellp(Q, kid, cf);
                            for (v = 0; v < NV; v++) acc[v] += w * src[v];
                        }
                    }
                c[b1] = HH + u1;
                c[b2] = HH + u2;
                c[a] = layer_coord(side, -L);
                memcpy(cellp(Q, p, c), acc, sizeof(acc));
            }
}

/* P-parallel, built once before any fill runs (orc_fill_halos) */
static double Ppar[3 * PP][PP];
static int Ppar_built = 0;

/* fine leaf p face (a, side) whose neighbour region is covered by the coarse leaf cp */
static void fill_face_prolong(const orc_mesh *m, double *Q, int64_t p, int a, int side,
                              int64_t cp, const int ni[3])
{
    const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
    int L, t1, t2, l1, l2, m6, v, c[3];
    int o1, o2;
    /* position of this fine patch inside the coarse face: fine index minus 3 * coarse index */
    o1 = ni[b1] - 3 * m->id[4 * cp + 1 + b1];
    o2 = ni[b2] - 3 * m->id[4 * cp + 1 + b2];
    if (m->transfer == 1) {
        /* three-point Lagrange quadratics.  Tangentially: fine cell F sits at coarse coordinate
           u = (F + 1/2)/3 - 1/2; the three coarse centres l-1, l, l+1 with l the nearest, kept
           inside 1..p-2.  Along the normal: fine ghost L sits at (1/2 - (L - 1/2)/3) coarse
           cells from the centre of c2 towards the face, interpolated from c1, c2, c3. */
        for (L = 1; L <= 3; L++) {
            const double sn = 0.5 - (L - 0.5) / 3.0;
            double wn[3];
            wn[0] = sn * (sn - 1.0) / 2.0;
            wn[1] = 1.0 - sn * sn;
            wn[2] = sn * (sn + 1.0) / 2.0;
            for (t2 = 0; t2 < PP; t2++)
                for (t1 = 0; t1 < PP; t1++) {
                    double acc[NV], w1[3], w2[3], s1, s2;
                    int k1, k2, kn, j1, j2;
                    const double u1 = (PP * o1 + t1 + 0.5) / 3.0 - 0.5, u2 = (PP * o2 + t2 + 0.5) / 3.0 - 0.5;
                    j1 = (int)floor(u1 + 0.5);
                    j2 = (int)floor(u2 + 0.5);
                    if (j1 < 1) j1 = 1;
                    if (j1 > PP - 2) j1 = PP - 2;
                    if (j2 < 1) j2 = 1;
                    if (j2 > PP - 2) j2 = PP - 2;
                    s1 = u1 - j1;
                    s2 = u2 - j2;
                    w1[0] = s1 * (s1 - 1.0) / 2.0; w1[1] = 1.0 - s1 * s1; w1[2] = s1 * (s1 + 1.0) / 2.0;
                    w2[0] = s2 * (s2 - 1.0) / 2.0; w2[1] = 1.0 - s2 * s2; w2[2] = s2 * (s2 + 1.0) / 2.0;
                    memset(acc, 0, sizeof(acc));
                    for (kn = 0; kn < 3; kn++)          /* c1, c2, c3 */
                        for (k2 = 0; k2 < 3; k2++)
                            for (k1 = 0; k1 < 3; k1++) {
                                const double w = wn[kn] * w2[k2] * w1[k1];
                                int cc[3];
                                cc[b1] = HH + j1 - 1 + k1;
                                cc[b2] = HH + j2 - 1 + k2;
                                /* c1, c2: coarse interior depth 2, 1 from the shared face; c3: halo 1 */
                                cc[a] = kn < 2 ? layer_coord(-side, 2 - kn) : layer_coord(-side, -1);
                                const double *src = cellp(Q, cp, cc);
                                for (v = 0; v < NV; v++) acc[v] += w * src[v];
                            }
                    c[b1] = HH + t1;
                    c[b2] = HH + t2;
                    c[a] = layer_coord(side, -L);
                    memcpy(cellp(Q, p, c), acc, sizeof(acc));
                }
        }
        return;
    }
    for (L = 1; L <= 3; L++) {        /* fine ghost layer L -> f_{3-L} */
        const int frow = 3 - L;
        for (t2 = 0; t2 < PP; t2++)
            for (t1 = 0; t1 < PP; t1++) {
                double acc[NV];
                const int F1 = PP * o1 + t1, F2 = PP * o2 + t2;
                memset(acc, 0, sizeof(acc));
                for (l2 = 0; l2 < PP; l2++)
                    for (l1 = 0; l1 < PP; l1++) {
                        double w12 = Ppar[F1][l1] * Ppar[F2][l2];
                        if (w12 == 0.0) continue;
                        for (m6 = 0; m6 < 6; m6++) {
                            double w = w12 * P_perp[frow][m6];
                            int cc[3];
                            if (w == 0.0) continue;
                            cc[b1] = HH + l1;
                            cc[b2] = HH + l2;
                            /* coarse layer c_{m6}: c0..c2 interior depth 3..1 from the shared face
                               (which is face -side of the coarse leaf), c3..c5 its halo 1..3 */
                            cc[a] = m6 < 3 ? layer_coord(-side, 3 - m6) : layer_coord(-side, -(m6 - 2));
                            const double *src = cellp(Q, cp, cc);
                            for (v = 0; v < NV; v++) acc[v] += w * src[v];
                        }
                    }
                c[b1] = HH + t1;
                c[b2] = HH + t2;
                c[a] = layer_coord(side, -L);
                memcpy(cellp(Q, p, c), acc, sizeof(acc));
            }
    }
}

typedef struct { int kind; int64_t nb; int ni[3]; } face_t; /* 0 copy 1 bc 2 restrict 3 prolong */

static face_t classify(const orc_mesh *m, int64_t p, int a, int side)
{
    face_t f;
    int lev = m->id[4 * p], n[3], b;
    memset(&f, 0, sizeof(f));
    for (b = 0; b < 3; b++) n[b] = m->id[4 * p + 1 + b];
    n[a] += side;
    if (n[a] < 0 || n[a] >= lev_n(m, lev, a)) {
        if (m->bc != ORC_BC_PERIODIC) { f.kind = 1; return f; }
        n[a] = (n[a] + lev_n(m, lev, a)) % lev_n(m, lev, a);
    }
    for (b = 0; b < 3; b++) f.ni[b] = n[b];
    f.nb = find_leaf(m, lev, n[0], n[1], n[2]);
    if (f.nb >= 0) { f.kind = 0; return f; }
    if (exists(m, lev, n[0], n[1], n[2]) && is_refined(m, lev, n[0], n[1], n[2])) {
        f.kind = 2;
        return f;
    }
    f.kind = 3;
    f.nb = find_leaf(m, lev - 1, n[0] / 3, n[1] / 3, n[2] / 3);
    return f;
}

/* Every face task writes only its own leaf's halo and reads interiors (the prolongation also
   reads coarse halos, which the first sweep completes), so each sweep may run over the leaves on
   several host threads (OpenMP) with the same result. */
void orc_fill_halos(const orc_mesh *m, double *Q)
{
    int64_t p;
    if (!Ppar_built) {
        build_P_par(Ppar);
        Ppar_built = 1;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (p = 0; p < m->np; p++) {
        int a, side;
        for (a = 0; a < 3; a++)
            for (side = -1; side <= 1; side += 2) {
                face_t f = classify(m, p, a, side);
                if (f.kind == 0) fill_face_copy(m, Q, p, a, side, f.nb);
                else if (f.kind == 1) { if (m->bc == ORC_BC_NEUMANN) fill_face_neumann(Q, p, a, side); }
                else if (f.kind == 2) fill_face_restrict(m, Q, p, a, side, f.ni);
            }
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (p = 0; p < m->np; p++) {
        int a, side;
        for (a = 0; a < 3; a++)
            for (side = -1; side <= 1; side += 2) {
                face_t f = classify(m, p, a, side);
                if (f.kind == 3) fill_face_prolong(m, Q, p, a, side, f.nb, f.ni);
            }
    }
}

/* ----------------------------------------------------------------------------------------
 * Right-hand side over the mesh.  Interior cells per orc_rhs_box; on faces at the domain
 * boundary with the Sommerfeld condition, every ghost layer L is an ODE unknown with
 *   G_L = -c (r/|x_n|) (Q_L - Q_{L-1})/dx_n - (c/r)(Q_L - Q_ini,L),   c = 1,
 * the layered finite-difference form of the paper's radiative condition
 * (eq_exa_sommerfeld_inter), r and x_n taken at the ghost itself, Q_{L-1} the next layer
 * inwards (L = 1: the last interior layer).  K_0 and frozen-shift slots get 0.
 * ---------------------------------------------------------------------------------------- */
static void sommerfeld_box(const orc_mesh *m, const orc_params *pr, int64_t p, const double *box,
                           double *out)
{
    int a, side, L, t1, t2, v, c[3], ci[3];
    double org[3], dx[3];
    const double *bg;
    if (m->bc != ORC_BC_SOMMERFELD || m->bgix[p] < 0) return;
    bg = m->bg + m->bgix[p] * ORC_BOXCELLS * NV;
    patch_geom(m, p, org, dx);
    for (a = 0; a < 3; a++)
        for (side = -1; side <= 1; side += 2) {
            const int b1 = (a + 1) % 3, b2 = (a + 2) % 3;
            if (!on_phys_boundary(m, p, a, side)) continue;
            for (L = 1; L <= 3; L++)
                for (t2 = HH; t2 < HH + PP; t2++)
                    for (t1 = HH; t1 < HH + PP; t1++) {
                        double xx[3], r;
                        c[b1] = ci[b1] = t1;
                        c[b2] = ci[b2] = t2;
                        c[a] = layer_coord(side, -L);
                        ci[a] = (L == 1) ? layer_coord(side, 1) : layer_coord(side, -(L - 1));
                        cell_center(m, p, c[0], c[1], c[2], xx);
                        r = sqrt(xx[0] * xx[0] + xx[1] * xx[1] + xx[2] * xx[2]);
                        const double *qL = box + cix(c[0], c[1], c[2]) * NV;
                        const double *qI = box + cix(ci[0], ci[1], ci[2]) * NV;
                        const double *q0 = bg + cix(c[0], c[1], c[2]) * NV;
                        double *o = out + cix(c[0], c[1], c[2]) * NV;
                        for (v = 0; v < 58; v++) {
                            if (frozen_slot(pr, v)) { o[v] = 0.0; continue; }
                            o[v] = -1.0 * (r / fabs(xx[a])) * (qL[v] - qI[v]) / dx[a] -
                                   (1.0 / r) * (qL[v] - q0[v]);
                        }
                        o[58] = 0.0;
                    }
        }
}

/* Patches are independent here, so the loop may run on several host threads (OpenMP, see
   orc_set_threads): each patch's arithmetic is the same whichever thread takes it. */
void orc_rhs_subset(const orc_mesh *m, const orc_params *pr, const double *Q, double *kout,
                    int64_t n_sel, const int64_t *sel)
{
    int64_t s;
#pragma omp parallel for schedule(dynamic, 1)
    for (s = 0; s < n_sel; s++) {
        int64_t p = sel[s];
        double org[3], dx[3];
        const double *box = Q + p * (int64_t)ORC_BOXCELLS * NV;
        double *out = kout + p * (int64_t)ORC_BOXCELLS * NV;
        patch_geom(m, p, org, dx);
        orc_rhs_box(pr, dx, box, out);
        sommerfeld_box(m, pr, p, box, out);
    }
}

void orc_rhs(const orc_mesh *m, const orc_params *pr, const double *Q, double *kout)
{
    int64_t p, *all = (int64_t *)malloc(sizeof(int64_t) * (m->np ? m->np : 1));
    for (p = 0; p < m->np; p++) all[p] = p;
    orc_rhs_subset(m, pr, Q, kout, m->np, all);
    free(all);
}

/* Host threads of the patch loops (OpenMP; 1 without it). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    omp_set_num_threads(n > 0 ? n : 1);
#else
    (void)n;
#endif
}

int orc_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ----------------------------------------------------------------------------------------
 * Tracers (Sec. 3.8): a point's value is the trilinear interpolation of the 2^3 cell centres
 * around it in the leaf that holds it; puncture trackers (Sec. 4.2.3) move with velocity -beta by
 * the explicit Euler rule x <- x + dt v.
 * ---------------------------------------------------------------------------------------- */
/* The leaf holding x.  The point's cube at the mesh's finest level has the index
   K = floor((x - origin) / edge) along each axis, and the leaf of level l holding x is the one
   whose cube (l, i) satisfies i * 3^(L - l) <= K < (i + 1) * 3^(L - l), L the finest level.  One
   rounded index serves every level, so the leaves tile the domain without gaps or overlaps even
   for points within rounding of a face (testing x against each leaf's own floating-point box,
   or flooring at each level separately, can leave such a point in no leaf). */
int64_t orc_find_leaf(const orc_mesh *m, const double x[3])
{
    int64_t p;
    int a, top = 0;
    double K[3];
    for (p = 0; p < m->np; p++)
        if (m->id[4 * p] > top) top = m->id[4 * p];
    for (a = 0; a < 3; a++) K[a] = floor((x[a] - m->origin[a]) / (m->extent[a] / lev_n(m, top, a)));
    for (p = 0; p < m->np; p++) {
        int in = 1, l;
        double s = 1.0;
        for (l = m->id[4 * p]; l < top; l++) s *= 3.0;
        for (a = 0; a < 3 && in; a++) {
            const double i = (double)m->id[4 * p + 1 + a];
            if (!(K[a] >= i * s && K[a] < (i + 1.0) * s)) in = 0;
        }
        if (in) return p;
    }
    return -1;
}

/* Trilinear interpolation (Sec. 3.8) at x: the weights come from the cell-centre coordinate
   u = (x - o)/dx - 1/2 of the leaf holding x, in interior units.  Each of the eight cells is read
   from the interior of the leaf that holds its centre when that leaf has the same level (so that
   no value is taken from an edge or corner region of a halo, which no fill writes); a cell whose
   centre lies outside the domain or in a leaf of another level is read from the holding leaf's
   own box (its face halo, filled by the boundary or coarse-fine fill). */
static int tracer_interp(const orc_mesh *m, const double *Q, const double x[3], int nslot, const int *slots,
                         double *out)
{
    const int64_t p = orc_find_leaf(m, x);
    double org[3], dx[3], t[3];
    int i0[3], a, s, c;
    const double *cellv[8];
    if (p < 0) return 0;
    patch_geom(m, p, org, dx);
    for (a = 0; a < 3; a++) {
        const double u = (x[a] - org[a]) / dx[a] - 0.5;
        const double f = floor(u);
        i0[a] = (int)f + HH; /* box index of the lower centre: 2..11 */
        t[a] = u - f;
    }
    for (c = 0; c < 8; c++) {
        const int b[3] = {i0[0] + (c & 1), i0[1] + ((c >> 1) & 1), i0[2] + ((c >> 2) & 1)};
        int64_t q = p;
        int bq[3] = {b[0], b[1], b[2]};
        if (b[0] < HH || b[0] >= HH + PP || b[1] < HH || b[1] >= HH + PP || b[2] < HH || b[2] >= HH + PP) {
            double xc[3], oq[3], dq[3];
            for (a = 0; a < 3; a++) xc[a] = org[a] + ((double)(b[a] - HH) + 0.5) * dx[a];
            q = orc_find_leaf(m, xc);
            if (q >= 0 && m->id[4 * q] == m->id[4 * p]) {
                patch_geom(m, q, oq, dq);
                for (a = 0; a < 3; a++) bq[a] = (int)floor((xc[a] - oq[a]) / dq[a]) + HH;
            } else {
                q = p;
            }
        }
        cellv[c] = Q + q * (int64_t)ORC_BOXCELLS * NV + cix(bq[0], bq[1], bq[2]) * NV;
    }
    for (s = 0; s < nslot; s++) {
        double v = 0.0;
        for (c = 0; c < 8; c++) {
            const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
            const double w = (cx ? t[0] : 1.0 - t[0]) * (cy ? t[1] : 1.0 - t[1]) * (cz ? t[2] : 1.0 - t[2]);
            v += w * cellv[c][slots[s]];
        }
        out[s] = v;
    }
    return 1;
}

int64_t orc_tracer_sample(const orc_mesh *m, const double *Q, int64_t n, const double *pos, int nslot,
                          const int *slots, double *out)
{
    int64_t i, missing = 0;
    int s;
    for (i = 0; i < n; i++)
        if (!tracer_interp(m, Q, pos + 3 * i, nslot, slots, out + i * nslot)) {
            for (s = 0; s < nslot; s++) out[i * nslot + s] = NAN;
            missing++;
        }
    return missing;
}

int64_t orc_tracer_advance(const orc_mesh *m, const double *Q, int64_t n, double *pos, double dt)
{
    static const int beta[3] = {7, 8, 9};
    int64_t i, missing = 0;
    int a;
    for (i = 0; i < n; i++) {
        double b[3];
        if (!tracer_interp(m, Q, pos + 3 * i, 3, beta, b)) {
            missing++;
            continue;
        }
        for (a = 0; a < 3; a++) pos[3 * i + a] += dt * (-b[a]);
    }
    return missing;
}

/* distance from the nearest of n points to the closed cube [lo, lo + L] */
static double cube_distance(const double lo[3], const double L[3], int64_t n, const double *pos)
{
    double best = HUGE_VAL;
    int64_t i;
    int a;
    for (i = 0; i < n; i++) {
        double d2 = 0.0;
        for (a = 0; a < 3; a++) {
            const double x = pos[3 * i + a];
            const double c = x < lo[a] ? lo[a] : (x > lo[a] + L[a] ? lo[a] + L[a] : x);
            d2 += (c - x) * (c - x);
        }
        if (sqrt(d2) < best) best = sqrt(d2);
    }
    return best;
}

void orc_tag_tracers(const orc_mesh *m, int64_t n, const double *pos, int nrad, const double *radii, int max_level,
                     int8_t *tags)
{
    int64_t p;
    int a;
    for (p = 0; p < m->np; p++) {
        const int lev = m->id[4 * p];
        double lo[3], L[3];
        tags[p] = 0;
        for (a = 0; a < 3; a++) {
            L[a] = m->extent[a] / lev_n(m, lev, a);
            lo[a] = m->origin[a] + L[a] * m->id[4 * p + 1 + a];
        }
        if (lev < max_level && lev < nrad && cube_distance(lo, L, n, pos) <= radii[lev]) {
            tags[p] = 1;
            continue;
        }
        if (lev >= 1) {
            for (a = 0; a < 3; a++) {
                L[a] = m->extent[a] / lev_n(m, lev - 1, a);
                lo[a] = m->origin[a] + L[a] * (m->id[4 * p + 1 + a] / 3);
            }
            if (lev - 1 >= nrad || cube_distance(lo, L, n, pos) > radii[lev - 1]) tags[p] = -1;
        }
    }
}

/* ----------------------------------------------------------------------------------------
 * Second-order formulation (Sec. 2.2; Sec. 3.2, explicit gradient reconstruction; Algorithm 2):
 * after each update the auxiliaries are recomputed from the primaries with the central FD4
 * difference, by their definitions A_i = d_i alpha, B_k^i = d_k beta^i,
 * D_kij = d_k gt_ij / 2, P_i = d_i phi (eq. auxiliary-variables).  Interior cells of every
 * leaf; the primaries' halos must be filled; no halo is written.
 * ---------------------------------------------------------------------------------------- */
void orc_reconstruct_aux(const orc_mesh *m, double *Q)
{
    int64_t p;
    int x, y, z, a, s, i, v;
    double w[5], d[11];
    for (p = 0; p < m->np; p++) {
        double org[3], dx[3];
        double *box = Q + p * (int64_t)ORC_BOXCELLS * NV;
        patch_geom(m, p, org, dx);
        for (z = HH; z < HH + PP; z++)
            for (y = HH; y < HH + PP; y++)
                for (x = HH; x < HH + PP; x++) {
                    double *q = box + cix(x, y, z) * NV;
                    for (a = 0; a < 3; a++) {
                        /* FD4 along axis a of gt (slots 0-5), alpha (6), beta (7-9), phi (10) */
                        for (v = 0; v <= 10; v++) {
                            for (s = -2; s <= 2; s++) {
                                int xx = x + (a == 0 ? s : 0), yy = y + (a == 1 ? s : 0),
                                    zz = z + (a == 2 ? s : 0);
                                w[s + 2] = box[cix(xx, yy, zz) * NV + v];
                            }
                            d[v] = orc_fd4(w, dx[a]);
                        }
                        q[25 + a] = d[6];                                       /* A_a */
                        for (i = 0; i < 3; i++) q[28 + 3 * a + i] = d[7 + i];   /* B_a^i */
                        for (i = 0; i < 6; i++) q[37 + 6 * a + i] = 0.5 * d[i]; /* D_a(ij) */
                        q[55 + a] = d[10];                                      /* P_a */
                    }
                }
    }
}

/* ----------------------------------------------------------------------------------------
 * Algebraic constraints det(gt) = 1 and tr(At) = 0 enforced pointwise after a time step
 * (the paper's post-processing): gt <- gt / det(gt)^(1/3), then At <- At - gt (gt^kl At_kl)/3
 * with the rescaled metric.
 * ---------------------------------------------------------------------------------------- */
void orc_project_point(double *q)
{
    double g[3][3], ig[3][3], d, s, tr = 0;
    int i, j;
    static const int si[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) g[i][j] = q[si[i][j]];
    d = g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1]) -
        g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0]) +
        g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
    s = 1.0 / cbrt(d);
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) g[i][j] *= s;
    d = g[0][0] * (g[1][1] * g[2][2] - g[1][2] * g[2][1]) -
        g[0][1] * (g[1][0] * g[2][2] - g[1][2] * g[2][0]) +
        g[0][2] * (g[1][0] * g[2][1] - g[1][1] * g[2][0]);
    ig[0][0] = (g[1][1] * g[2][2] - g[1][2] * g[2][1]) / d;
    ig[0][1] = (g[0][2] * g[2][1] - g[0][1] * g[2][2]) / d;
    ig[0][2] = (g[0][1] * g[1][2] - g[0][2] * g[1][1]) / d;
    ig[1][0] = (g[1][2] * g[2][0] - g[1][0] * g[2][2]) / d;
    ig[1][1] = (g[0][0] * g[2][2] - g[0][2] * g[2][0]) / d;
    ig[1][2] = (g[0][2] * g[1][0] - g[0][0] * g[1][2]) / d;
    ig[2][0] = (g[1][0] * g[2][1] - g[1][1] * g[2][0]) / d;
    ig[2][1] = (g[0][1] * g[2][0] - g[0][0] * g[2][1]) / d;
    ig[2][2] = (g[0][0] * g[1][1] - g[0][1] * g[1][0]) / d;
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) tr += ig[i][j] * q[11 + si[i][j]];
    for (i = 0; i < 3; i++)
        for (j = i; j < 3; j++) {
            q[si[i][j]] = g[i][j];
            q[11 + si[i][j]] -= g[i][j] * tr / 3.0;
        }
}

/* ----------------------------------------------------------------------------------------
 * Classical RK4 (the paper allows Runge-Kutta up to order four; the classical tableau is
 * the reading here), in two-register form over interior cells and Sommerfeld ghosts:
 *   s=0: acc = Qn + dt/6 k0, Qnext = Qn + dt/2 k0
 *   s=1: acc += dt/3 k1,     Qnext = Qn + dt/2 k1
 *   s=2: acc += dt/3 k2,     Qnext = Qn + dt k2
 *   s=3: Qnext = acc + dt/6 k3, then the projection on interior cells.
 * ---------------------------------------------------------------------------------------- */
int orc_rk4_stage(const orc_mesh *m, int s, double dt, const double *Qn, const double *k,
                  double *acc, double *Qnext)
{
    static const double bw[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
    static const double aw[3] = {0.5, 0.5, 1.0};
    int64_t p;
    if (s < 0 || s > 3 || !(dt > 0)) return -1;
#pragma omp parallel for schedule(static)
    for (p = 0; p < m->np; p++) {
        int x, y, z, v;
        for (z = 0; z < NB; z++)
            for (y = 0; y < NB; y++)
                for (x = 0; x < NB; x++) {
                    int c[3] = {x, y, z}, a, nin = 0, active = 0;
                    for (a = 0; a < 3; a++) nin += (c[a] >= HH && c[a] < HH + PP);
                    if (nin == 3) active = 1;
                    else if (nin == 2 && m->bc == ORC_BC_SOMMERFELD)
                        for (a = 0; a < 3; a++) {
                            if (c[a] < HH && on_phys_boundary(m, p, a, -1)) active = 1;
                            if (c[a] >= HH + PP && on_phys_boundary(m, p, a, 1)) active = 1;
                        }
                    if (!active) continue;
                    int64_t o = (p * (int64_t)ORC_BOXCELLS + cix(x, y, z)) * NV;
                    for (v = 0; v < NV; v++) {
                        if (s == 0) acc[o + v] = Qn[o + v] + bw[0] * dt * k[o + v];
                        else if (s < 3) acc[o + v] = acc[o + v] + bw[s] * dt * k[o + v];
                        if (s < 3) Qnext[o + v] = Qn[o + v] + aw[s] * dt * k[o + v];
                        else Qnext[o + v] = acc[o + v] + bw[3] * dt * k[o + v];
                    }
                    if (s == 3 && nin == 3) orc_project_point(Qnext + o);
                }
    }
    return 0;
}

/* ----------------------------------------------------------------------------------------
 * Constraint monitor: H and M_i on every interior leaf cell, the norms
 * L2(H) = sqrt(sum H^2 / n) (the paper's L2 error of the Hamiltonian constraint with
 * H_theoretical = 0) and L2(|M|) = sqrt(sum |M|^2 / n) over cells with r >= r_excise, and the
 * count of cells with a non-finite state slot or constraint.  Returns that count.
 * ---------------------------------------------------------------------------------------- */
int64_t orc_constraints(const orc_mesh *m, const double *Q, double *HM, double r_excise,
                        double norms[3])
{
    int64_t p, nbad = 0, ncell = 0;
    double sH = 0, sM = 0;
    double *hm = (double *)malloc(sizeof(double) * 729 * 4);
    for (p = 0; p < m->np; p++) {
        double org[3], dx[3];
        const double *box = Q + p * (int64_t)ORC_BOXCELLS * NV;
        int x, y, z, n = 0, v;
        patch_geom(m, p, org, dx);
        orc_constraints_box(dx, box, hm);
        for (z = HH; z < HH + PP; z++)
            for (y = HH; y < HH + PP; y++)
                for (x = HH; x < HH + PP; x++, n++) {
                    double xx[3], r;
                    int bad = 0;
                    const double *q = box + cix(x, y, z) * NV;
                    for (v = 0; v < NV; v++) bad |= !isfinite(q[v]);
                    for (v = 0; v < 4; v++) bad |= !isfinite(hm[4 * n + v]);
                    nbad += bad;
                    if (HM) memcpy(HM + (p * 729 + n) * 4, hm + 4 * n, sizeof(double) * 4);
                    cell_center(m, p, x, y, z, xx);
                    r = sqrt(xx[0] * xx[0] + xx[1] * xx[1] + xx[2] * xx[2]);
                    if (r < r_excise || bad) continue;
                    sH += hm[4 * n] * hm[4 * n];
                    sM += hm[4 * n + 1] * hm[4 * n + 1] + hm[4 * n + 2] * hm[4 * n + 2] +
                          hm[4 * n + 3] * hm[4 * n + 3];
                    ncell++;
                }
    }
    free(hm);
    norms[0] = ncell ? sqrt(sH / ncell) : 0.0;
    norms[1] = ncell ? sqrt(sM / ncell) : 0.0;
    norms[2] = (double)nbad;
    return nbad;
}

/* ----------------------------------------------------------------------------------------
 * Plain refinement indicator per leaf: the paper's feature-based criterion (largest
 * difference between two adjacent volumes of a patch) applied to chi = phi^2 and alpha,
 * and a constraint term dx^2 max|H| over the patch interior.
 *   ind[p] = (max adjacent |d chi|, max adjacent |d alpha|, dx^2 max |H|)
 * Tags: e = max of the three; REFINE (+1) if e >= theta_r and lev < max_level; COARSEN (-1)
 * if lev > 0, e < theta_c, and all 27 siblings are leaves with e < theta_c; else KEEP (0).
 * ---------------------------------------------------------------------------------------- */
void orc_tag_indicator(const orc_mesh *m, const double *Q, double *ind)
{
    int64_t p;
    double *hm = (double *)malloc(sizeof(double) * 729 * 4);
    for (p = 0; p < m->np; p++) {
        double org[3], dx[3], gc = 0, ga = 0, hmax = 0;
        const double *box = Q + p * (int64_t)ORC_BOXCELLS * NV;
        int x, y, z, a, n;
        patch_geom(m, p, org, dx);
        for (z = HH; z < HH + PP; z++)
            for (y = HH; y < HH + PP; y++)
                for (x = HH; x < HH + PP; x++)
                    for (a = 0; a < 3; a++) {
                        int c2[3] = {x, y, z};
                        c2[a] += 1;
                        if (c2[a] >= HH + PP) continue;
                        const double *q1 = box + cix(x, y, z) * NV;
                        const double *q2 = box + cix(c2[0], c2[1], c2[2]) * NV;
                        double dc = fabs(q2[10] * q2[10] - q1[10] * q1[10]);
                        double da = fabs(q2[6] - q1[6]);
                        if (dc > gc) gc = dc;
                        if (da > ga) ga = da;
                    }
        orc_constraints_box(dx, box, hm);
        for (n = 0; n < 729; n++)
            if (fabs(hm[4 * n]) > hmax) hmax = fabs(hm[4 * n]);
        ind[3 * p] = gc;
        ind[3 * p + 1] = ga;
        ind[3 * p + 2] = dx[0] * dx[0] * hmax;
    }
    free(hm);
}

void orc_tag_refine(const orc_mesh *m, const double *Q, double theta_r, double theta_c,
                    int max_level, int8_t *tags)
{
    int64_t p;
    double *ind = (double *)malloc(sizeof(double) * 3 * (m->np ? m->np : 1));
    double *e = (double *)malloc(sizeof(double) * (m->np ? m->np : 1));
    orc_tag_indicator(m, Q, ind);
    for (p = 0; p < m->np; p++) {
        double v = ind[3 * p];
        if (ind[3 * p + 1] > v) v = ind[3 * p + 1];
        if (ind[3 * p + 2] > v) v = ind[3 * p + 2];
        e[p] = v;
    }
    for (p = 0; p < m->np; p++) {
        int lev = m->id[4 * p];
        tags[p] = 0;
        if (e[p] >= theta_r) { if (lev < max_level) tags[p] = 1; continue; }
        if (lev > 0 && e[p] < theta_c) {
            int ok = 1, u, v, w;
            int pi = m->id[4 * p + 1] / 3, pj = m->id[4 * p + 2] / 3, pk = m->id[4 * p + 3] / 3;
            for (w = 0; w < 3 && ok; w++)
                for (v = 0; v < 3 && ok; v++)
                    for (u = 0; u < 3 && ok; u++) {
                        int64_t s = find_leaf(m, lev, 3 * pi + u, 3 * pj + v, 3 * pk + w);
                        if (s < 0 || !(e[s] < theta_c)) ok = 0;
                    }
            if (ok) tags[p] = -1;
        }
    }
    free(ind);
    free(e);
}

/* Learned tags (the combination rule of the learned indicator with the plain criterion):
   per leaf, the softmax of the three logits (COARSEN, KEEP, REFINE) and its arg-max class, ties
   to the higher class, evaluated in FP32 as on the GPU; a plain REFINE stays, a REFINE predicted
   with probability >= conf is added below max_level, a plain COARSEN survives unless KEEP or
   REFINE is predicted with probability >= conf, and a family coarsens only if all 27 of its
   leaves still do. */
void orc_tag_learned(const orc_mesh *m, const float *logits, const int8_t *plain, float conf, int max_level,
                     int8_t *tags)
{
    int64_t p;
    int8_t *pre = (int8_t *)malloc(m->np ? (size_t)m->np : 1);
    for (p = 0; p < m->np; p++) {
        const float z0 = logits[3 * p], z1 = logits[3 * p + 1], z2 = logits[3 * p + 2];
        const float zm = fmaxf(fmaxf(z0, z1), z2);
        const float se = expf(z0 - zm) + expf(z1 - zm) + expf(z2 - zm);
        const float pm = 1.0f / se;
        const int cls = z2 >= zm ? 1 : (z1 >= zm ? 0 : -1);
        const int sure = pm >= conf;
        int8_t tg = 0;
        if (plain[p] == 1) tg = 1;
        else if (sure && cls == 1 && m->id[4 * p] < max_level) tg = 1;
        else if (plain[p] == -1 && !(sure && cls != -1)) tg = -1;
        pre[p] = tg;
    }
    for (p = 0; p < m->np; p++) {
        int8_t tg = pre[p];
        const int lev = m->id[4 * p];
        if (tg == -1) {
            int u, v, w;
            const int pi = m->id[4 * p + 1] / 3, pj = m->id[4 * p + 2] / 3, pk = m->id[4 * p + 3] / 3;
            if (lev == 0) tg = 0;
            for (w = 0; w < 3 && tg; w++)
                for (v = 0; v < 3 && tg; v++)
                    for (u = 0; u < 3 && tg; u++) {
                        const int64_t s = lev > 0 ? find_leaf(m, lev, 3 * pi + u, 3 * pj + v, 3 * pk + w) : -1;
                        if (s < 0 || pre[s] != -1) tg = 0;
                    }
        }
        tags[p] = tg;
    }
    free(pre);
}

/* ----------------------------------------------------------------------------------------
 * Regrid (dynamic AMR on the refinement-criterion hook, Sec. 3.6): the refined cubes of the mesh
 * after per-leaf tags, and the transfer of a state onto the new leaves.
 * ---------------------------------------------------------------------------------------- */
typedef struct {
    int *c; /* [n][4] */
    int64_t n, cap;
} cubeset;

static int cs_has(const cubeset *s, int l, int i, int j, int k)
{
    int64_t r;
    for (r = 0; r < s->n; r++)
        if (s->c[4 * r] == l && s->c[4 * r + 1] == i && s->c[4 * r + 2] == j && s->c[4 * r + 3] == k) return 1;
    return 0;
}

static void cs_add(cubeset *s, int l, int i, int j, int k)
{
    if (cs_has(s, l, i, j, k)) return;
    push4(&s->c, &s->n, &s->cap, l, i, j, k);
}

static void cs_del(cubeset *s, int l, int i, int j, int k)
{
    int64_t r;
    for (r = 0; r < s->n; r++)
        if (s->c[4 * r] == l && s->c[4 * r + 1] == i && s->c[4 * r + 2] == j && s->c[4 * r + 3] == k) {
            memmove(s->c + 4 * r, s->c + 4 * (r + 1), sizeof(int) * 4 * (size_t)(s->n - r - 1));
            s->n--;
            return;
        }
}

/* the face neighbour of cube (l, c) along axis a, side sd, wrapped if periodic; 0 if outside */
static int face_nb(const orc_mesh *m, int l, const int c[3], int a, int sd, int out[3])
{
    const int na = lev_n(m, l, a);
    out[0] = c[0];
    out[1] = c[1];
    out[2] = c[2];
    out[a] += sd;
    if (out[a] < 0 || out[a] >= na) {
        if (m->bc != ORC_BC_PERIODIC) return 0;
        out[a] = (out[a] + na) % na;
    }
    return 1;
}

/* Rules: a leaf tagged +1 below max_level is refined; a refined cube whose 27 children are all
   leaves tagged -1 is coarsened unless a face neighbour of one of those children (outside the
   cube) is refined; then, while some refined cube of level L >= 1 has a face neighbour at level L
   whose parent is not refined, that parent is refined (no face joins leaves two levels apart).
   Writes the refined cubes, sorted, to out (cap entries); returns their number, or -1 if cap is
   too small. */
int64_t orc_regrid_plan(const orc_mesh *m, const int8_t *tags, int max_level, int *out, int64_t cap)
{
    cubeset R = {NULL, 0, 0};
    int64_t r, p;
    int a, sd, u, v, w, changed;
    for (r = 0; r < m->nref; r++) {
        const int *c = m->ref + 4 * r;
        if (exists(m, c[0], c[1], c[2], c[3])) cs_add(&R, c[0], c[1], c[2], c[3]);
    }
    const int64_t nold = R.n;
    int *old = (int *)malloc(sizeof(int) * 4 * (size_t)(nold ? nold : 1));
    memcpy(old, R.c, sizeof(int) * 4 * (size_t)nold);
    for (p = 0; p < m->np; p++)
        if (tags[p] == 1 && m->id[4 * p] < max_level)
            cs_add(&R, m->id[4 * p], m->id[4 * p + 1], m->id[4 * p + 2], m->id[4 * p + 3]);
    for (r = 0; r < nold; r++) {
        const int *P = old + 4 * r;
        const int L = P[0] + 1;
        int all = 1;
        for (w = 0; w < 3 && all; w++)
            for (v = 0; v < 3 && all; v++)
                for (u = 0; u < 3 && all; u++) {
                    const int64_t q = find_leaf(m, L, 3 * P[1] + u, 3 * P[2] + v, 3 * P[3] + w);
                    if (q < 0 || tags[q] != -1) all = 0;
                }
        for (w = 0; w < 3 && all; w++)
            for (v = 0; v < 3 && all; v++)
                for (u = 0; u < 3 && all; u++) {
                    const int ch[3] = {3 * P[1] + u, 3 * P[2] + v, 3 * P[3] + w};
                    for (a = 0; a < 3 && all; a++)
                        for (sd = -1; sd <= 1 && all; sd += 2) {
                            int nb[3];
                            if (!face_nb(m, L, ch, a, sd, nb)) continue;
                            if (nb[0] / 3 == P[1] && nb[1] / 3 == P[2] && nb[2] / 3 == P[3]) continue;
                            if (cs_has(&R, L, nb[0], nb[1], nb[2])) all = 0;
                        }
                }
        if (all) cs_del(&R, P[0], P[1], P[2], P[3]);
    }
    do {
        changed = 0;
        for (r = 0; r < R.n; r++) {
            const int L = R.c[4 * r];
            const int c[3] = {R.c[4 * r + 1], R.c[4 * r + 2], R.c[4 * r + 3]};
            if (L == 0) continue;
            for (a = 0; a < 3; a++)
                for (sd = -1; sd <= 1; sd += 2) {
                    int nb[3];
                    if (!face_nb(m, L, c, a, sd, nb)) continue;
                    if (!cs_has(&R, L - 1, nb[0] / 3, nb[1] / 3, nb[2] / 3)) {
                        cs_add(&R, L - 1, nb[0] / 3, nb[1] / 3, nb[2] / 3);
                        changed = 1;
                    }
                }
        }
    } while (changed);
    free(old);
    if (R.n > cap) {
        free(R.c);
        return -1;
    }
    qsort(R.c, R.n, sizeof(int) * 4, cmp4);
    if (R.n) memcpy(out, R.c, sizeof(int) * 4 * (size_t)R.n);
    free(R.c);
    return R.n;
}

/* Transfer of Qo (mesh mo) to the leaves of mn (same domain, levels differing by at most one
   leaf-wise): a leaf of both meshes is copied (whole box); a new leaf inside an old leaf one
   level coarser takes, at each fine cell centre, the tensor product along the three axes of the
   linear interpolation of App. E's P-parallel rule (fine index f in 0..26 across the old leaf,
   u = (f + 1/2)/3 - 1/2, l = clamp(floor(u), 0, 7), weights 1 - (u - l) and u - l on the old
   interior cells l and l+1); a new leaf covering 27 old leaves one level finer takes at each
   cell the mean of the 3^3 fine cells it covers.  Halos and ghost slabs of interpolated or
   averaged leaves keep the values Qn held. */
void orc_regrid_transfer(const orc_mesh *mo, const double *Qo, const orc_mesh *mn, double *Qn)
{
    const int64_t bs = (int64_t)ORC_BOXCELLS * NV;
    int64_t p;
    for (p = 0; p < mn->np; p++) {
        const int L = mn->id[4 * p], I[3] = {mn->id[4 * p + 1], mn->id[4 * p + 2], mn->id[4 * p + 3]};
        double *dst = Qn + p * bs;
        const int64_t same = find_leaf(mo, L, I[0], I[1], I[2]);
        int x, y, z, v;
        if (same >= 0) {
            memcpy(dst, Qo + same * bs, sizeof(double) * (size_t)bs);
            continue;
        }
        const int64_t par = L > 0 ? find_leaf(mo, L - 1, I[0] / 3, I[1] / 3, I[2] / 3) : -1;
        if (par >= 0) {
            const double *src = Qo + par * bs;
            for (z = 0; z < PP; z++)
                for (y = 0; y < PP; y++)
                    for (x = 0; x < PP; x++) {
                        const int fc[3] = {x, y, z};
                        int l[3];
                        double wt[3];
                        for (int a = 0; a < 3; a++) {
                            const int f = 9 * (I[a] % 3) + fc[a];
                            const double uu = (f + 0.5) / 3.0 - 0.5;
                            int ll = (int)floor(uu);
                            if (ll < 0) ll = 0;
                            if (ll > PP - 2) ll = PP - 2;
                            l[a] = ll;
                            wt[a] = uu - ll;
                        }
                        double *q = dst + cix(x + HH, y + HH, z + HH) * NV;
                        for (v = 0; v < NV; v++) {
                            double s = 0.0;
                            for (int dz = 0; dz < 2; dz++)
                                for (int dy = 0; dy < 2; dy++)
                                    for (int dx = 0; dx < 2; dx++) {
                                        const double wgt = (dz ? wt[2] : 1.0 - wt[2]) * (dy ? wt[1] : 1.0 - wt[1]) *
                                                           (dx ? wt[0] : 1.0 - wt[0]);
                                        s += wgt * src[cix(l[0] + dx + HH, l[1] + dy + HH, l[2] + dz + HH) * NV + v];
                                    }
                            q[v] = s;
                        }
                    }
            continue;
        }
        /* the 27 finer leaves */
        for (z = 0; z < PP; z++)
            for (y = 0; y < PP; y++)
                for (x = 0; x < PP; x++) {
                    const int64_t kid = find_leaf(mo, L + 1, 3 * I[0] + x / 3, 3 * I[1] + y / 3, 3 * I[2] + z / 3);
                    double *q = dst + cix(x + HH, y + HH, z + HH) * NV;
                    if (kid < 0) continue; /* cannot happen for a valid pair of meshes */
                    const double *src = Qo + kid * bs;
                    for (v = 0; v < NV; v++) {
                        double s = 0.0;
                        for (int dz = 0; dz < 3; dz++)
                            for (int dy = 0; dy < 3; dy++)
                                for (int dx = 0; dx < 3; dx++)
                                    s += src[cix(3 * (x % 3) + dx + HH, 3 * (y % 3) + dy + HH, 3 * (z % 3) + dz + HH) * NV + v];
                        q[v] = s / 27.0;
                    }
                }
    }
}
