/*
 * Oracle (test infrastructure only): pointwise first-order CCZ4 right-hand side and the
 * ADM constraints, written out index by index from App. B of arXiv:2406.11626
 * ("Spacetime Foliation and Evolution Equations").  Every left-hand-side term other than
 * the time derivative is moved to the right.  Readings of the paper (all listed in the
 * design notes of the repository):
 *   - trace of At is taken with the conformal metric, [X]^TF = X - gt gt^kl X_kl / 3;
 *   - s = 1 for the Gamma-driver shift, and with the frozen shift the right-hand sides of
 *     beta, b and B are zero;
 *   - d_k K_0 = 0 (K_0 is a constant); g(alpha) = 1 (harmonic) or 2/alpha (1+log);
 *   - d_(k D_i)jl = (d_k D_ijl + d_i D_kjl)/2, d_(k P_i) = (d_k P_i + d_i P_k)/2,
 *     d_(k B_l)^i = (d_k B_l^i + d_l B_k^i)/2, d_(i A_j) = (d_i A_j + d_j A_i)/2;
 *   - the Ricci tensor R_ij is evaluated for all nine index pairs from the relations of
 *     App. B and its symmetric part enters the At equation (its trace uses all nine);
 *   - second-order formulation (pr->formulation = 1, Sec. 2.2 and Algorithm 2): the same
 *     equations for the primaries with the red terms removed (App. B: they are used in the
 *     first-order formulation only), and zero right-hand sides for A, B, D, P.
 * dq[k][v] is the derivative along axis k of slot v; only slots 11..57 are ever read.
 */
#include <math.h>
#include <string.h>
#include "ccz4_oracle.h"

static int sym(int i, int j)
{
    static const int t[3][3] = {{0, 1, 2}, {1, 3, 4}, {2, 4, 5}};
    return t[i][j];
}

#define S_G(i, j) (0 + sym(i, j))
#define S_ALPHA 6
#define S_BETA(i) (7 + (i))
#define S_PHI 10
#define S_AT(i, j) (11 + sym(i, j))
#define S_K 17
#define S_THETA 18
#define S_GHAT(i) (19 + (i))
#define S_BB(i) (22 + (i))
#define S_A(k) (25 + (k))
#define S_B(k, i) (28 + 3 * (k) + (i))
#define S_D(k, i, j) (37 + 6 * (k) + sym(i, j))
#define S_P(k) (55 + (k))
#define S_K0 58

static double det3(double m[3][3])
{
    return m[0][0] * (m[1][1] * m[2][2] - m[1][2] * m[2][1]) -
           m[0][1] * (m[1][0] * m[2][2] - m[1][2] * m[2][0]) +
           m[0][2] * (m[1][0] * m[2][1] - m[1][1] * m[2][0]);
}

static void inv3(double m[3][3], double r[3][3])
{
    double d = det3(m);
    r[0][0] = (m[1][1] * m[2][2] - m[1][2] * m[2][1]) / d;
    r[0][1] = (m[0][2] * m[2][1] - m[0][1] * m[2][2]) / d;
    r[0][2] = (m[0][1] * m[1][2] - m[0][2] * m[1][1]) / d;
    r[1][0] = (m[1][2] * m[2][0] - m[1][0] * m[2][2]) / d;
    r[1][1] = (m[0][0] * m[2][2] - m[0][2] * m[2][0]) / d;
    r[1][2] = (m[0][2] * m[1][0] - m[0][0] * m[1][2]) / d;
    r[2][0] = (m[1][0] * m[2][1] - m[1][1] * m[2][0]) / d;
    r[2][1] = (m[0][1] * m[2][0] - m[0][0] * m[2][1]) / d;
    r[2][2] = (m[0][0] * m[1][1] - m[0][1] * m[1][0]) / d;
}

/* All fields of one cell, unpacked from the slot vector, plus the first derivatives. */
typedef struct {
    double g[3][3], ig[3][3], alpha, beta[3], phi, At[3][3], K, Theta, Ghat[3], b[3];
    double A[3], B[3][3] /* B[k][i] = d_k beta^i */, D[3][3][3] /* D[k][i][j] */, P[3], K0;
    double dAt[3][3][3] /* dAt[k][i][j] = d_k At_ij */, dK[3], dTheta[3], dGhat[3][3], db[3][3];
    double dA[3][3] /* dA[k][i] = d_k A_i */, dB[3][3][3] /* dB[k][l][i] = d_k B_l^i */;
    double dD[3][3][3][3] /* dD[k][l][i][j] = d_k D_lij */, dP[3][3] /* dP[k][i] = d_k P_i */;
} cell_t;

static void unpack(const double *q, const double *dq, cell_t *c)
{
    int i, j, k, l;
    memset(c, 0, sizeof(*c));
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) {
            c->g[i][j] = q[S_G(i, j)];
            c->At[i][j] = q[S_AT(i, j)];
        }
    c->alpha = q[S_ALPHA];
    c->phi = q[S_PHI];
    c->K = q[S_K];
    c->Theta = q[S_THETA];
    c->K0 = q[S_K0];
    for (i = 0; i < 3; i++) {
        c->beta[i] = q[S_BETA(i)];
        c->Ghat[i] = q[S_GHAT(i)];
        c->b[i] = q[S_BB(i)];
        c->A[i] = q[S_A(i)];
        c->P[i] = q[S_P(i)];
        for (j = 0; j < 3; j++) {
            c->B[i][j] = q[S_B(i, j)];
            for (k = 0; k < 3; k++) c->D[i][j][k] = q[S_D(i, j, k)];
        }
    }
    inv3(c->g, c->ig);
    if (!dq) return;
    for (k = 0; k < 3; k++) {
        const double *d = dq + 59 * k;
        c->dK[k] = d[S_K];
        c->dTheta[k] = d[S_THETA];
        for (i = 0; i < 3; i++) {
            c->dGhat[k][i] = d[S_GHAT(i)];
            c->db[k][i] = d[S_BB(i)];
            c->dA[k][i] = d[S_A(i)];
            c->dP[k][i] = d[S_P(i)];
            for (j = 0; j < 3; j++) {
                c->dAt[k][i][j] = d[S_AT(i, j)];
                c->dB[k][i][j] = d[S_B(i, j)];
                for (l = 0; l < 3; l++) c->dD[k][i][j][l] = d[S_D(i, j, l)];
            }
        }
    }
}

/* Quantities of the closing relations of App. B that both the RHS and the constraints use. */
typedef struct {
    double Dup[3][3][3];       /* D_k^{ij} */
    double Gt[3][3][3];        /* conformal Christoffel Gt^k_ij, index [k][i][j] */
    double dGt[3][3][3][3];    /* d_k Gt^m_ij, index [k][m][i][j] */
    double Gam[3][3][3];       /* physical Christoffel Gamma^k_ij */
    double dGam[3][3][3][3];   /* d_k Gamma^m_ij, index [k][m][i][j] */
    double Ric[3][3];          /* R_ij (all nine) */
    double trAt;
} rel_t;

static double sdD(const cell_t *c, int k, int i, int j, int l) /* d_(k D_i)jl */
{
    return 0.5 * (c->dD[k][i][j][l] + c->dD[i][k][j][l]);
}

static double sdP(const cell_t *c, int k, int i) /* d_(k P_i) */
{
    return 0.5 * (c->dP[k][i] + c->dP[i][k]);
}

static void relations(const cell_t *c, rel_t *r)
{
    int i, j, k, l, m, n;
    const double iphi = 1.0 / c->phi;
    memset(r, 0, sizeof(*r));
    for (k = 0; k < 3; k++)
        for (i = 0; i < 3; i++)
            for (j = 0; j < 3; j++) {
                double s = 0;
                for (n = 0; n < 3; n++)
                    for (m = 0; m < 3; m++) s += c->ig[i][n] * c->ig[m][j] * c->D[k][n][m];
                r->Dup[k][i][j] = s;
            }
    /* Gt^k_ij = gt^kl (D_ijl + D_jil - D_lij) */
    for (k = 0; k < 3; k++)
        for (i = 0; i < 3; i++)
            for (j = 0; j < 3; j++) {
                double s = 0;
                for (l = 0; l < 3; l++)
                    s += c->ig[k][l] * (c->D[i][j][l] + c->D[j][i][l] - c->D[l][i][j]);
                r->Gt[k][i][j] = s;
            }
    /* d_k Gt^m_ij = -2 D_k^ml (D_ijl + D_jil - D_lij)
                     + gt^ml (d_(k D_i)jl + d_(k D_j)il - d_(k D_l)ij) */
    for (k = 0; k < 3; k++)
        for (m = 0; m < 3; m++)
            for (i = 0; i < 3; i++)
                for (j = 0; j < 3; j++) {
                    double s = 0;
                    for (l = 0; l < 3; l++) {
                        s += -2.0 * r->Dup[k][m][l] *
                             (c->D[i][j][l] + c->D[j][i][l] - c->D[l][i][j]);
                        s += c->ig[m][l] *
                             (sdD(c, k, i, j, l) + sdD(c, k, j, i, l) - sdD(c, k, l, i, j));
                    }
                    r->dGt[k][m][i][j] = s;
                }
    /* Gamma^k_ij = Gt^k_ij - (1/phi) gt^kl (gt_jl P_i + gt_il P_j - gt_ij P_l) */
    for (k = 0; k < 3; k++)
        for (i = 0; i < 3; i++)
            for (j = 0; j < 3; j++) {
                double s = 0;
                for (l = 0; l < 3; l++)
                    s += c->ig[k][l] *
                         (c->g[j][l] * c->P[i] + c->g[i][l] * c->P[j] - c->g[i][j] * c->P[l]);
                r->Gam[k][i][j] = r->Gt[k][i][j] - iphi * s;
            }
    /* d_k Gamma^m_ij, the six-line relation of App. B */
    for (k = 0; k < 3; k++)
        for (m = 0; m < 3; m++)
            for (i = 0; i < 3; i++)
                for (j = 0; j < 3; j++) {
                    double s = 0;
                    for (l = 0; l < 3; l++) {
                        s += -2.0 * r->Dup[k][m][l] *
                             (c->D[i][j][l] + c->D[j][i][l] - c->D[l][i][j]);
                        s += c->ig[m][l] *
                             (sdD(c, k, i, j, l) + sdD(c, k, j, i, l) - sdD(c, k, l, i, j));
                        s += 2.0 * iphi * r->Dup[k][m][l] *
                             (c->g[j][l] * c->P[i] + c->g[i][l] * c->P[j] -
                              c->g[i][j] * c->P[l]);
                        s += -2.0 * iphi * c->ig[m][l] *
                             (c->D[k][j][l] * c->P[i] + c->D[k][i][l] * c->P[j] -
                              c->D[k][i][j] * c->P[l]);
                        s += -iphi * c->ig[m][l] *
                             (c->g[j][l] * sdP(c, k, i) + c->g[i][l] * sdP(c, k, j) -
                              c->g[i][j] * sdP(c, k, l));
                        s += iphi * iphi * c->ig[m][l] *
                             (c->g[j][l] * c->P[i] * c->P[k] + c->g[i][l] * c->P[j] * c->P[k] -
                              c->g[i][j] * c->P[k] * c->P[l]);
                    }
                    r->dGam[k][m][i][j] = s;
                }
    /* R^m_ikj = d_k Gamma^m_ij - d_j Gamma^m_ik + Gamma^l_ij Gamma^m_lk - Gamma^l_ik Gamma^m_lj,
       R_ij = R^m_imj */
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) {
            double s = 0;
            for (m = 0; m < 3; m++) {
                s += r->dGam[m][m][i][j] - r->dGam[j][m][i][m];
                for (l = 0; l < 3; l++)
                    s += r->Gam[l][i][j] * r->Gam[m][l][m] - r->Gam[l][i][m] * r->Gam[m][l][j];
            }
            r->Ric[i][j] = s;
        }
    r->trAt = 0;
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) r->trAt += c->ig[i][j] * c->At[i][j];
}

void orc_rhs_point(const orc_params *pr, const double *q, const double *dq, double *out)
{
    cell_t C, *c = &C;
    rel_t R, *r = &R;
    int i, j, k, l, m, n;
    double g_a, dg_a, s_on, Aup[3][3], Gtv[3], dGtv[3][3], Z[3], Zup[3], nZ[3][3], RpZ, DDa[3][3];
    double X[3][3], trX, trB, AA, DA[3], trdAt[3], sdBtr[3];
    unpack(q, dq, c);
    relations(c, r);
    memset(out, 0, sizeof(double) * 59);

    const double al = c->alpha, phi = c->phi;
    const double k1 = pr->kappa1, k2 = pr->kappa2, k3 = pr->kappa3, cc = pr->c, ee = pr->e;
    if (pr->slicing == 1) { g_a = 2.0 / al; dg_a = -2.0 / (al * al); }
    else { g_a = 1.0; dg_a = 0.0; }
    s_on = pr->shift ? 1.0 : 0.0;

    trB = c->B[0][0] + c->B[1][1] + c->B[2][2];
    /* At^ij = gt^ik gt^jl At_kl */
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) {
            double s = 0;
            for (k = 0; k < 3; k++)
                for (l = 0; l < 3; l++) s += c->ig[i][k] * c->ig[j][l] * c->At[k][l];
            Aup[i][j] = s;
        }
    AA = 0;
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) AA += c->At[i][j] * Aup[i][j];
    /* Gt^i = gt^jk Gt^i_jk ; d_k Gt^i = -2 D_k^jl Gt^i_jl + gt^jl d_k Gt^i_jl */
    for (i = 0; i < 3; i++) {
        double s = 0;
        for (j = 0; j < 3; j++)
            for (k = 0; k < 3; k++) s += c->ig[j][k] * r->Gt[i][j][k];
        Gtv[i] = s;
    }
    for (k = 0; k < 3; k++)
        for (i = 0; i < 3; i++) {
            double s = 0;
            for (j = 0; j < 3; j++)
                for (l = 0; l < 3; l++)
                    s += -2.0 * r->Dup[k][j][l] * r->Gt[i][j][l] + c->ig[j][l] * r->dGt[k][i][j][l];
            dGtv[k][i] = s;
        }
    /* Z_i = gt_ij (Ghat^j - Gt^j)/2 ; Z^i = phi^2 (Ghat^i - Gt^i)/2 */
    for (i = 0; i < 3; i++) {
        double s = 0;
        for (j = 0; j < 3; j++) s += c->g[i][j] * (c->Ghat[j] - Gtv[j]);
        Z[i] = 0.5 * s;
        Zup[i] = 0.5 * phi * phi * (c->Ghat[i] - Gtv[i]);
    }
    /* nabla_i Z_j = D_ijl (Ghat^l - Gt^l) + gt_jl (d_i Ghat^l - d_i Gt^l)/2 - Gamma^l_ij Z_l */
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) {
            double s = 0;
            for (l = 0; l < 3; l++) {
                s += c->D[i][j][l] * (c->Ghat[l] - Gtv[l]);
                s += 0.5 * c->g[j][l] * (c->dGhat[i][l] - dGtv[i][l]);
                s -= r->Gam[l][i][j] * Z[l];
            }
            nZ[i][j] = s;
        }
    /* R + 2 nabla_k Z^k = phi^2 gt^ij (R_ij + nabla_i Z_j + nabla_j Z_i) */
    RpZ = 0;
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) RpZ += c->ig[i][j] * (r->Ric[i][j] + nZ[i][j] + nZ[j][i]);
    RpZ *= phi * phi;
    /* nabla_i nabla_j alpha = d_(i A_j) - Gamma^k_ij A_k */
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) {
            double s = 0.5 * (c->dA[i][j] + c->dA[j][i]);
            for (k = 0; k < 3; k++) s -= r->Gam[k][i][j] * c->A[k];
            DDa[i][j] = s;
        }
    /* D_k^nm At_nm and gt^nm d_k At_nm, and d_(k B_l)^l */
    for (k = 0; k < 3; k++) {
        double s = 0, t = 0, u = 0;
        for (n = 0; n < 3; n++)
            for (m = 0; m < 3; m++) {
                s += r->Dup[k][n][m] * c->At[n][m];
                t += c->ig[n][m] * c->dAt[k][n][m];
            }
        for (l = 0; l < 3; l++) u += 0.5 * (c->dB[k][l][l] + c->dB[l][k][l]);
        DA[k] = s;
        trdAt[k] = t;
        sdBtr[k] = u;
    }

    /* --- gt_ij --- */
    {
        double detg = det3(c->g);
        for (i = 0; i < 3; i++)
            for (j = i; j < 3; j++) {
                double s = 0;
                for (k = 0; k < 3; k++) {
                    s += 2.0 * c->beta[k] * c->D[k][i][j];
                    s += c->g[k][i] * c->B[j][k] + c->g[k][j] * c->B[i][k];
                }
                s += -2.0 / 3.0 * c->g[i][j] * trB;
                s += -2.0 * al * (c->At[i][j] - 1.0 / 3.0 * c->g[i][j] * r->trAt);
                s += -(1.0 / pr->tau) * (detg - 1.0) * c->g[i][j];
                out[S_G(i, j)] = s;
            }
    }
    /* --- alpha --- */
    {
        double s = 0;
        for (k = 0; k < 3; k++) s += c->beta[k] * c->A[k];
        s += -al * al * g_a * (c->K - c->K0 - 2.0 * cc * c->Theta);
        out[S_ALPHA] = s;
    }
    /* --- beta^i --- */
    for (i = 0; i < 3; i++) {
        double s = 0;
        for (k = 0; k < 3; k++) s += c->beta[k] * c->B[k][i];
        s += pr->f * c->b[i];
        out[S_BETA(i)] = s_on * s;
    }
    /* --- phi --- */
    {
        double s = 0;
        for (k = 0; k < 3; k++) s += c->beta[k] * c->P[k];
        s += 1.0 / 3.0 * phi * (al * c->K - trB);
        out[S_PHI] = s;
    }
    /* --- At_ij --- */
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) X[i][j] = -DDa[i][j] + al * (r->Ric[i][j] + nZ[i][j] + nZ[j][i]);
    trX = 0;
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) trX += c->ig[i][j] * X[i][j];
    for (i = 0; i < 3; i++)
        for (j = i; j < 3; j++) {
            double s = 0, Xs = 0.5 * (X[i][j] + X[j][i]);
            for (k = 0; k < 3; k++) s += c->beta[k] * c->dAt[k][i][j];
            s += phi * phi * (Xs - 1.0 / 3.0 * c->g[i][j] * trX);
            for (k = 0; k < 3; k++) s += c->At[k][i] * c->B[j][k] + c->At[k][j] * c->B[i][k];
            s += -2.0 / 3.0 * c->At[i][j] * trB;
            s += al * c->At[i][j] * (c->K - 2.0 * c->Theta * cc);
            for (l = 0; l < 3; l++)
                for (m = 0; m < 3; m++) s += -2.0 * al * c->At[i][l] * c->ig[l][m] * c->At[m][j];
            out[S_AT(i, j)] = s;
        }
    /* --- K --- */
    {
        double s = 0, lap = 0;
        for (k = 0; k < 3; k++) s += c->beta[k] * c->dK[k];
        for (i = 0; i < 3; i++)
            for (j = 0; j < 3; j++) lap += c->ig[i][j] * DDa[i][j];
        s += -phi * phi * lap; /* nabla^i nabla_i alpha = phi^2 gt^ij nabla_i nabla_j alpha */
        s += al * RpZ;
        s += al * c->K * (c->K - 2.0 * c->Theta * cc);
        s += -3.0 * al * k1 * (1.0 + k2) * c->Theta;
        out[S_K] = s;
    }
    /* --- Theta --- */
    {
        double s = 0;
        for (k = 0; k < 3; k++) s += c->beta[k] * c->dTheta[k];
        s += 0.5 * al * ee * ee * RpZ;
        s += 0.5 * al * ee * ee * (2.0 / 3.0 * c->K * c->K - AA);
        s += -al * c->Theta * c->K * cc;
        for (i = 0; i < 3; i++) s += -Zup[i] * c->A[i];
        s += -al * k1 * (2.0 + k2) * c->Theta;
        out[S_THETA] = s;
    }
    /* --- Ghat^i --- */
    double rhsGhat[3];
    for (i = 0; i < 3; i++) {
        double s = 0;
        for (k = 0; k < 3; k++) s += c->beta[k] * c->dGhat[k][i];
        for (k = 0; k < 3; k++) s += 2.0 * al * c->ig[k][i] * c->dTheta[k];
        for (k = 0; k < 3; k++)
            for (l = 0; l < 3; l++) s += c->ig[k][l] * 0.5 * (c->dB[k][l][i] + c->dB[l][k][i]);
        for (k = 0; k < 3; k++) s += s_on * 1.0 / 3.0 * c->ig[i][k] * sdBtr[k];
        if (!pr->formulation)
            for (k = 0; k < 3; k++) s += 2.0 * al * c->ig[i][k] * trdAt[k]; /* red */
        for (j = 0; j < 3; j++) s += -4.0 / 3.0 * al * c->ig[i][j] * c->dK[j];
        s += 2.0 / 3.0 * Gtv[i] * trB;
        for (k = 0; k < 3; k++) s += -Gtv[k] * c->B[k][i];
        {
            double t = 0;
            for (j = 0; j < 3; j++) {
                for (k = 0; k < 3; k++) t += r->Gt[i][j][k] * Aup[j][k];
                t += -3.0 * Aup[i][j] * c->P[j] / phi;
            }
            s += 2.0 * al * t;
        }
        for (k = 0; k < 3; k++)
            s += -2.0 * al * c->ig[k][i] * (c->Theta * c->A[k] / al + 2.0 / 3.0 * c->K * Z[k]);
        for (j = 0; j < 3; j++) s += -2.0 * Aup[i][j] * c->A[j];
        if (!pr->formulation)
            for (k = 0; k < 3; k++) s += -4.0 * al * c->ig[i][k] * DA[k]; /* red */
        for (j = 0; j < 3; j++) s += -2.0 * al * k1 * c->ig[i][j] * Z[j];
        {
            double t = 0;
            for (j = 0; j < 3; j++) t += 2.0 / 3.0 * c->ig[i][j] * Z[j] * trB;
            for (j = 0; j < 3; j++)
                for (k = 0; k < 3; k++) t += -c->ig[j][k] * Z[j] * c->B[k][i];
            s += 2.0 * k3 * t;
        }
        rhsGhat[i] = s;
        out[S_GHAT(i)] = s;
    }
    /* --- b^i --- */
    for (i = 0; i < 3; i++) {
        double s = 0;
        for (k = 0; k < 3; k++) s += c->beta[k] * c->db[k][i];
        s += rhsGhat[i];
        for (k = 0; k < 3; k++) s += -c->beta[k] * c->dGhat[k][i];
        s += -pr->eta * c->b[i];
        out[S_BB(i)] = s_on * s;
    }
    /* --- A_k --- */
    for (k = 0; k < 3; k++) {
        double s = 0;
        for (l = 0; l < 3; l++) s += c->beta[l] * c->dA[l][k];
        s += -al * al * g_a * (c->dK[k] - 0.0 /* d_k K_0 */ - 2.0 * cc * c->dTheta[k]);
        s += -al * g_a * trdAt[k]; /* red */
        for (l = 0; l < 3; l++) s += c->B[k][l] * c->A[l];
        s += 2.0 * al * g_a * DA[k]; /* red */
        s += -(2.0 * al * g_a + al * al * dg_a) * (c->K - c->K0 - 2.0 * cc * c->Theta) * c->A[k];
        out[S_A(k)] = s;
    }
    /* --- B_k^i --- */
    for (k = 0; k < 3; k++)
        for (i = 0; i < 3; i++) {
            double s = 0;
            for (l = 0; l < 3; l++) s += c->beta[l] * c->dB[l][k][i];
            s += pr->f * c->db[k][i];
            for (j = 0; j < 3; j++)
                s += -al * al * pr->mu * c->ig[i][j] / phi * (c->dP[k][j] - c->dP[j][k]); /* red */
            for (j = 0; j < 3; j++)
                for (n = 0; n < 3; n++)
                    for (l = 0; l < 3; l++)
                        s += al * al * pr->mu * c->ig[i][j] * c->ig[n][l] *
                             (c->dD[k][l][j][n] - c->dD[l][k][j][n]); /* red */
            for (l = 0; l < 3; l++) s += c->B[k][l] * c->B[l][i];
            out[S_B(k, i)] = s_on * s;
        }
    /* --- D_kij --- */
    for (k = 0; k < 3; k++)
        for (i = 0; i < 3; i++)
            for (j = i; j < 3; j++) {
                double s = 0, t = 0;
                for (l = 0; l < 3; l++) s += c->beta[l] * c->dD[l][k][i][j];
                for (m = 0; m < 3; m++) {
                    t += 0.5 * c->g[m][i] * 0.5 * (c->dB[k][j][m] + c->dB[j][k][m]);
                    t += 0.5 * c->g[m][j] * 0.5 * (c->dB[k][i][m] + c->dB[i][k][m]);
                }
                t += -1.0 / 3.0 * c->g[i][j] * sdBtr[k];
                s += s_on * t;
                s += -al * c->dAt[k][i][j];
                s += al / 3.0 * c->g[i][j] * trdAt[k]; /* red */
                for (l = 0; l < 3; l++)
                    s += c->B[k][l] * c->D[l][i][j] + c->B[j][l] * c->D[k][l][i] +
                         c->B[i][l] * c->D[k][l][j];
                s += -2.0 / 3.0 * trB * c->D[k][i][j];
                s += -2.0 / 3.0 * al * c->g[i][j] * DA[k]; /* red */
                s += -c->A[k] * (c->At[i][j] - 1.0 / 3.0 * c->g[i][j] * r->trAt);
                out[S_D(k, i, j)] = s;
            }
    /* --- P_k --- */
    for (k = 0; k < 3; k++) {
        double s = 0;
        for (l = 0; l < 3; l++) s += c->beta[l] * c->dP[l][k];
        s += 1.0 / 3.0 * phi * (al * c->dK[k] - sdBtr[k]);
        s += 1.0 / 3.0 * al * phi * trdAt[k]; /* red */
        for (l = 0; l < 3; l++) s += c->B[k][l] * c->P[l];
        s += 1.0 / 3.0 * (al * c->K - trB) * c->P[k];
        s += 1.0 / 3.0 * phi * c->K * c->A[k];
        s += -2.0 / 3.0 * al * phi * DA[k]; /* red */
        out[S_P(k)] = s;
    }
    /* --- K_0: constant --- */
    out[S_K0] = 0.0;
    /* second-order formulation: the auxiliaries do not evolve (they are reconstructed from
       the primaries after each update); the red terms are already off above, and the red
       terms of the auxiliary equations go with those equations */
    if (pr->formulation)
        for (i = S_A(0); i <= S_P(2); i++) out[i] = 0.0;
}

/* Hamiltonian H = R + 2/3 K^2 - At_ij At^ij with R = phi^2 gt^ij R_ij (pure Ricci, no Z terms),
   momentum M_i = gt^kl (d_k At_li - 2 Gt^m_l(i At_k)m - 3 At_ik P_l / phi) - 2/3 d_i K
   (eqs. hamilton_constraints and momentum_constraints of App. B).  hm = (H, M_x, M_y, M_z). */
void orc_constraints_point(const double *q, const double *dq, double *hm)
{
    cell_t C, *c = &C;
    rel_t R, *r = &R;
    int i, j, k, l, m;
    double Rs = 0, AA = 0;
    unpack(q, dq, c);
    relations(c, r);
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++) Rs += c->ig[i][j] * r->Ric[i][j];
    Rs *= c->phi * c->phi;
    for (i = 0; i < 3; i++)
        for (j = 0; j < 3; j++)
            for (k = 0; k < 3; k++)
                for (l = 0; l < 3; l++) AA += c->At[i][j] * c->ig[i][k] * c->ig[j][l] * c->At[k][l];
    hm[0] = Rs + 2.0 / 3.0 * c->K * c->K - AA;
    for (i = 0; i < 3; i++) {
        double s = 0;
        for (k = 0; k < 3; k++)
            for (l = 0; l < 3; l++) {
                double t = c->dAt[k][l][i];
                for (m = 0; m < 3; m++)
                    t += -2.0 * 0.5 * (r->Gt[m][l][i] * c->At[k][m] + r->Gt[m][l][k] * c->At[i][m]);
                t += -3.0 * c->At[i][k] * c->P[l] / c->phi;
                s += c->ig[k][l] * t;
            }
        s += -2.0 / 3.0 * c->dK[i];
        hm[1 + i] = s;
    }
}
