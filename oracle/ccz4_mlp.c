/*
 * ccz4_mlp.c -- oracle of the learned refinement indicator (a project addition built on the
 * paper's refinement-criterion hook, Sec. 3.6): per-patch features and a small multilayer
 * perceptron with its loss gradient and an Adam step.
 *
 * TEST INFRASTRUCTURE ONLY (see ccz4_oracle.h).  Plain loops in FP64.  With bf16 = 1 every
 * operand the GPU feeds to its BF16 matrix cores (standardised inputs, weights, hidden
 * activations, and in the backward pass the pre-activation gradients) is rounded to BF16 here
 * too, so that both sides use the same quantised operands; the backward pass treats those
 * roundings as the identity (straight-through), as the GPU does.  With bf16 = 0 the network
 * is plain FP64, which is what the finite-difference pins check.
 *
 * Parameter vector (NPARAM = 9603 entries), row-major, out x in:
 *   W1[64][81] b1[64] W2[64][64] b2[64] W3[3][64] b3[3]
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "ccz4_oracle.h"

#define NIN ORC_MLP_NIN
#define NH ORC_MLP_NH
#define NOUT ORC_MLP_NOUT
#define OW1 0
#define OB1 (OW1 + NH * NIN)
#define OW2 (OB1 + NH)
#define OB2 (OW2 + NH * NH)
#define OW3 (OB2 + NH)
#define OB3 (OW3 + NOUT * NH)

/* Round to the nearest BF16 value, ties to even, of the FP32 value nearest to x (the GPU
   rounds FP32 results).  NaN stays NaN; infinities and overflow follow IEEE rounding. */
double orc_bf16_round(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f; /* inf or nan */
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    u &= 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double rnd(double x, int bf16) { return bf16 ? orc_bf16_round(x) : x; }

/* Standardised inputs, in FP32 arithmetic exactly as the GPU forms them:
   x = (feat - mu) * inv_sigma, one rounding per operation. */
void orc_mlp_standardize(int64_t n, const float *feat, const float *norm /* mu[81], inv_sigma[81] */,
                         double *x)
{
    int64_t r;
    int i;
    for (r = 0; r < n; r++)
        for (i = 0; i < NIN; i++) {
            volatile float d = feat[r * NIN + i] - norm[i];
            volatile float s = d * norm[NIN + i];
            x[r * NIN + i] = (double)s;
        }
}

/* Per-patch features: the 9^3 interior split into 3^3 blocks of 3^3 cells, block
   b = (bz*3 + by)*3 + bx; for each block the maxima over its cells of dx |grad chi| (chi = phi^2,
   central FD4 of chi along each axis), dx |grad alpha| (FD4), and dx^2 |H| (Hamiltonian
   constraint), scaled by the patch spacing as the plain criterion scales its indicators, so that
   patches of different levels are comparable; feature 3b + q = log10(max_q + 1e-12).  Q needs
   filled halos; the spacing is isotropic (dx = dx_x). */
void orc_features(const orc_mesh *m, const double *Q, double *feat)
{
    const int64_t np = orc_mesh_npatches(m);
    double *geom = (double *)malloc(sizeof(double) * 6 * (np ? np : 1));
    double *hm = (double *)malloc(sizeof(double) * 729 * 4);
    int64_t p;
    orc_mesh_patch_geom(m, geom);
    for (p = 0; p < np; p++) {
        const double *box = Q + p * (int64_t)ORC_BOXCELLS * ORC_NV;
        const double *dx = geom + 6 * p + 3;
        double mx[27][3];
        int x, y, z, a, s, b, q;
        for (b = 0; b < 27; b++) mx[b][0] = mx[b][1] = mx[b][2] = 0.0;
        orc_constraints_box(dx, box, hm);
        for (z = 0; z < 9; z++)
            for (y = 0; y < 9; y++)
                for (x = 0; x < 9; x++) {
                    double gc = 0.0, ga = 0.0;
                    for (a = 0; a < 3; a++) {
                        double wc[5], wa[5];
                        for (s = -2; s <= 2; s++) {
                            int c[3] = {x + 3, y + 3, z + 3};
                            c[a] += s;
                            const double *cell = box + (((int64_t)c[2] * ORC_NB + c[1]) * ORC_NB + c[0]) * ORC_NV;
                            wc[s + 2] = cell[10] * cell[10];
                            wa[s + 2] = cell[6];
                        }
                        const double dc = orc_fd4(wc, dx[a]), da = orc_fd4(wa, dx[a]);
                        gc += dc * dc;
                        ga += da * da;
                    }
                    gc = dx[0] * sqrt(gc);
                    ga = dx[0] * sqrt(ga);
                    const double h = dx[0] * dx[0] * fabs(hm[4 * ((z * 9 + y) * 9 + x)]);
                    b = ((z / 3) * 3 + y / 3) * 3 + x / 3;
                    if (gc > mx[b][0]) mx[b][0] = gc;
                    if (ga > mx[b][1]) mx[b][1] = ga;
                    if (h > mx[b][2]) mx[b][2] = h;
                }
        for (b = 0; b < 27; b++)
            for (q = 0; q < 3; q++) feat[p * NIN + 3 * b + q] = log10(mx[b][q] + 1e-12);
    }
    free(hm);
    free(geom);
}

/* Forward pass on n standardised inputs x[n][81].  Outputs (any may be NULL): the hidden
   activations after ReLU and rounding, a1[n][64], a2[n][64], and the logits z3[n][3].
   z1 = W1 x + b1, a1 = relu(z1); z2 = W2 a1 + b2, a2 = relu(z2); z3 = W3 a2 + b3. */
void orc_mlp_forward(int64_t n, const double *x, const double *prm, int bf16, double *a1out, double *a2out,
                     double *z3out)
{
    int64_t r;
    int i, j;
    double xin[NIN], a1[NH], a2[NH];
    for (r = 0; r < n; r++) {
        for (i = 0; i < NIN; i++) xin[i] = rnd(x[r * NIN + i], bf16);
        for (j = 0; j < NH; j++) {
            double z = prm[OB1 + j];
            for (i = 0; i < NIN; i++) z += rnd(prm[OW1 + j * NIN + i], bf16) * xin[i];
            a1[j] = rnd(z > 0 ? z : 0.0, bf16);
        }
        for (j = 0; j < NH; j++) {
            double z = prm[OB2 + j];
            for (i = 0; i < NH; i++) z += rnd(prm[OW2 + j * NH + i], bf16) * a1[i];
            a2[j] = rnd(z > 0 ? z : 0.0, bf16);
        }
        for (j = 0; j < NOUT; j++) {
            double z = prm[OB3 + j];
            for (i = 0; i < NH; i++) z += rnd(prm[OW3 + j * NH + i], bf16) * a2[i];
            if (z3out) z3out[r * NOUT + j] = z;
        }
        if (a1out) memcpy(a1out + r * NH, a1, sizeof(a1));
        if (a2out) memcpy(a2out + r * NH, a2, sizeof(a2));
    }
}

/* Mean softmax cross-entropy of the logits against labels in {0, 1, 2} (COARSEN, KEEP,
   REFINE) and its gradient with respect to every parameter (grad[NPARAM]).  Backward:
   d3 = (softmax(z3) - onehot)/n; gW3 = d3^T a2, gb3 = sum d3; d2 = (W3^T d3) * [z2 > 0];
   gW2 = d2^T a1, gb2 = sum d2; d1 = (W2^T d2) * [z1 > 0]; gW1 = d1^T x, gb1 = sum d1.  With
   bf16 the matrix operands (weights, a1, a2, x and the d's entering a product) are the rounded
   ones; the bias gradients sum the unrounded d's. */
double orc_mlp_loss_grad(int64_t n, const double *x, const int32_t *labels, const double *prm, int bf16,
                         double *grad)
{
    int64_t r;
    int i, j;
    double loss = 0.0;
    double xin[NIN], z1[NH], a1[NH], z2[NH], a2[NH], z3[NOUT], d3[NOUT], d2[NH], d1[NH];
    memset(grad, 0, sizeof(double) * ORC_MLP_NPARAM);
    for (r = 0; r < n; r++) {
        for (i = 0; i < NIN; i++) xin[i] = rnd(x[r * NIN + i], bf16);
        for (j = 0; j < NH; j++) {
            double z = prm[OB1 + j];
            for (i = 0; i < NIN; i++) z += rnd(prm[OW1 + j * NIN + i], bf16) * xin[i];
            z1[j] = z;
            a1[j] = rnd(z > 0 ? z : 0.0, bf16);
        }
        for (j = 0; j < NH; j++) {
            double z = prm[OB2 + j];
            for (i = 0; i < NH; i++) z += rnd(prm[OW2 + j * NH + i], bf16) * a1[i];
            z2[j] = z;
            a2[j] = rnd(z > 0 ? z : 0.0, bf16);
        }
        double zmax = -HUGE_VAL, se = 0.0;
        for (j = 0; j < NOUT; j++) {
            double z = prm[OB3 + j];
            for (i = 0; i < NH; i++) z += rnd(prm[OW3 + j * NH + i], bf16) * a2[i];
            z3[j] = z;
            if (z > zmax) zmax = z;
        }
        for (j = 0; j < NOUT; j++) se += exp(z3[j] - zmax);
        loss += -(z3[labels[r]] - zmax - log(se));
        for (j = 0; j < NOUT; j++) d3[j] = (exp(z3[j] - zmax) / se - (j == labels[r] ? 1.0 : 0.0)) / (double)n;
        /* layer 3 */
        for (j = 0; j < NOUT; j++) {
            const double dj = rnd(d3[j], bf16);
            grad[OB3 + j] += d3[j];
            for (i = 0; i < NH; i++) grad[OW3 + j * NH + i] += dj * a2[i];
        }
        for (i = 0; i < NH; i++) {
            double s = 0.0;
            for (j = 0; j < NOUT; j++) s += rnd(prm[OW3 + j * NH + i], bf16) * rnd(d3[j], bf16);
            d2[i] = z2[i] > 0 ? s : 0.0;
        }
        /* layer 2 */
        for (j = 0; j < NH; j++) {
            const double dj = rnd(d2[j], bf16);
            grad[OB2 + j] += d2[j];
            for (i = 0; i < NH; i++) grad[OW2 + j * NH + i] += dj * a1[i];
        }
        for (i = 0; i < NH; i++) {
            double s = 0.0;
            for (j = 0; j < NH; j++) s += rnd(prm[OW2 + j * NH + i], bf16) * rnd(d2[j], bf16);
            d1[i] = z1[i] > 0 ? s : 0.0;
        }
        /* layer 1 */
        for (j = 0; j < NH; j++) {
            const double dj = rnd(d1[j], bf16);
            grad[OB1 + j] += d1[j];
            for (i = 0; i < NIN; i++) grad[OW1 + j * NIN + i] += dj * xin[i];
        }
    }
    return loss / (double)n;
}

/* One Adam step (Kingma & Ba, Algorithm 1) on every parameter, step t >= 1:
   m = b1 m + (1-b1) g; v = b2 v + (1-b2) g^2; p -= lr (m / (1-b1^t)) / (sqrt(v / (1-b2^t)) + eps). */
void orc_adam_step(int64_t n, double *p, double *mom, double *vel, const double *g, int t, double lr, double b1,
                   double b2, double eps)
{
    int64_t i;
    const double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (i = 0; i < n; i++) {
        mom[i] = b1 * mom[i] + (1.0 - b1) * g[i];
        vel[i] = b2 * vel[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (mom[i] / c1) / (sqrt(vel[i] / c2) + eps);
    }
}
