// Pointwise first-order CCZ4 right-hand side on the device (App. B of arXiv:2406.11626).
//
// Inputs are the 59 slots of one cell and the FD4 first derivatives of slots 11..57; the
// output is the 59-slot right-hand side before Kreiss-Oliger dissipation.  The closing
// relations are evaluated in contracted form: with gt^ml gt_jl = delta^m_j the derivative of
// the physical Christoffel symbols reduces to
//   d_k Gamma^m_ij = d_k Gt^m_ij + 2 (D_kij P^m - gt_ij D_k^ml P_l)/phi
//                    - (delta^m_j dP_(ki) + delta^m_i dP_(kj) - gt_ij gt^ml dP_(kl))/phi
//                    + (delta^m_j P_i P_k + delta^m_i P_j P_k - gt_ij P_k P^m)/phi^2,
// and the two contractions the Ricci tensor needs are formed directly:
//   R_ij = sum_m d_m Gamma^m_ij - d_j (Gamma^m_im) + Gamma^l_ij Gamma^m_lm - Gamma^l_im Gamma^m_lj,
//   d_j Gamma^m_im = -2 D_j^ml D_iml + gt^ml (d_j D_iml + d_i D_jml)/2 - 3 dP_(ij)/phi + 3 P_i P_j/phi^2.
// T is the type of the nonlinear algebra (double, or float in the mixed-precision mode);
// the inverse metric, its determinant and every factor of 1/phi are formed in double.
#pragma once
#include "ccz4_layout.hpp"

namespace ccz4 {

struct RhsParams {
    double kappa1, kappa2, kappa3, tau, e, c, mu, f, eta, ko_eps;
    int32_t slicing, shift;
    int32_t formulation;  // 0: first order (red terms on), 1: second order (red terms off, aux RHS 0)
    int32_t advection;    // 0: central FD4 advection; 1: lopsided, biased towards +x_k where beta^k > 0;
                          // 2: lopsided with the pairing as printed (towards -x_k where beta^k > 0)
    int32_t transfer;     // coarse-fine halo operators: 0 as printed in App. E; 1 injection + quadratic
};

// The lopsided fourth-order first derivatives of App. D, biased towards +x (points -1..+3) or
// towards -x (points -3..+1), written as the central difference cen plus a fifth difference:
//   right = cen + (-Q-- + 5Q- - 10Q + 10Q+ - 5Q++ + Q+++) / (12 dx),
//   left  = cen + (-Q--- + 5Q-- - 10Q- + 10Q - 5Q+ + Q++) / (12 dx),
// the second being the first mirrored; selecting the operands rather than the two results keeps
// one expression per lane (i12 = 1 / (12 dx)).
__device__ __forceinline__ double lop_from_central(double cen, bool right, double m3, double m2, double m1, double c0,
                                                   double p1, double p2, double p3, double i12)
{
    const double u3 = right ? p3 : -m3, u2 = right ? p2 : -m2, u1 = right ? p1 : -m1, u0 = right ? c0 : -c0;
    const double w1 = right ? m1 : -p1, w2 = right ? m2 : -p2;
    return cen + (u3 - 5.0 * u2 + 10.0 * u1 - 10.0 * u0 + 5.0 * w1 - w2) * i12;
}
// which of the two the advection term takes along an axis with shift component be
__device__ __forceinline__ bool lop_use_right(int32_t mode, double be) { return mode == 1 ? be > 0.0 : !(be > 0.0); }

// derivative inputs: dq[a][v - 11] = d_a (slot v) for v = 11..57
constexpr int NDIFF = 47;
constexpr int DOFF = 11;

template <typename T>
struct Sym3 {
    T v[6];
    __device__ T operator()(int i, int j) const { return v[sym(i, j)]; }
};

template <typename T>
__device__ __forceinline__ T cvt(double x) { return static_cast<T>(x); }

template <typename T>
struct Geo {
    double igd[6], detg, phid, iphid;
    T g[6], ig[6], At[6], D[3][6], B[3][3], A[3], be[3], Gh[3], bb[3], al, Kt, Th, K0;
    T Pphi[3], Puphi[3], sdPphi[6];
    T Dup[3][6], Gl[3][6], Gt[3][6], Gtv[3], Wl[3], Gam[3][6], Gc[3], U[3][3], Ric[6];
};

// Metric inverse, Christoffel symbols and the symmetric Ricci tensor of one cell.
template <typename T>
__device__ __forceinline__ void compute_geo(const double *__restrict__ q, const double (*__restrict__ dq)[NDIFF],
                                            Geo<T> &G)
{
    // ---------------- metric inverse and 1/phi factors in double
    const double g00 = q[0], g01 = q[1], g02 = q[2], g11 = q[3], g12 = q[4], g22 = q[5];
    const double c00 = g11 * g22 - g12 * g12, c01 = g02 * g12 - g01 * g22, c02 = g01 * g12 - g02 * g11;
    const double detg = g00 * c00 + g01 * c01 + g02 * c02;
    G.detg = detg;
    const double idet = 1.0 / detg;
    double (&igd)[6] = G.igd;
    igd[0] = c00 * idet;
    igd[1] = c01 * idet;
    igd[2] = c02 * idet;
    igd[3] = (g00 * g22 - g02 * g02) * idet;
    igd[4] = (g01 * g02 - g00 * g12) * idet;
    igd[5] = (g00 * g11 - g01 * g01) * idet;
    const double phid = q[SPHI];
    G.phid = phid;
    const double iphid = 1.0 / phid;
    G.iphid = iphid;
    double Pphid[3], Puphid[3];
    for (int l = 0; l < 3; ++l) Pphid[l] = q[SP + l] * iphid;
    for (int m = 0; m < 3; ++m)
        Puphid[m] = igd[sym(m, 0)] * Pphid[0] + igd[sym(m, 1)] * Pphid[1] + igd[sym(m, 2)] * Pphid[2];
    // symmetrised dP / phi (double)
    double sdPphid[6];
    for (int i = 0; i < 3; ++i)
        for (int j = i; j < 3; ++j)
            sdPphid[sym(i, j)] = 0.5 * (dq[i][SP - DOFF + j] + dq[j][SP - DOFF + i]) * iphid;

    // ---------------- demote
    T(&g)[6] = G.g; T(&ig)[6] = G.ig; T(&At)[6] = G.At; T(&D)[3][6] = G.D; T(&B)[3][3] = G.B;
    T(&A)[3] = G.A; T(&be)[3] = G.be; T(&Gh)[3] = G.Gh; T(&bb)[3] = G.bb;
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        g[s] = cvt<T>(q[SG + s]);
        ig[s] = cvt<T>(igd[s]);
        At[s] = cvt<T>(q[SAT + s]);
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) {
#pragma unroll
        for (int s = 0; s < 6; ++s) D[k][s] = cvt<T>(q[SD + 6 * k + s]);
#pragma unroll
        for (int i = 0; i < 3; ++i) B[k][i] = cvt<T>(q[SB + 3 * k + i]);
        A[k] = cvt<T>(q[SA + k]);
        be[k] = cvt<T>(q[SBETA + k]);
        Gh[k] = cvt<T>(q[SGHAT + k]);
        bb[k] = cvt<T>(q[SBB + k]);
    }
    G.al = cvt<T>(q[SALPHA]);
    G.Kt = cvt<T>(q[SK]);
    G.Th = cvt<T>(q[STHETA]);
    G.K0 = cvt<T>(q[SK0]);
    T(&Pphi)[3] = G.Pphi; T(&Puphi)[3] = G.Puphi; T(&sdPphi)[6] = G.sdPphi;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        Pphi[l] = cvt<T>(Pphid[l]);
        Puphi[l] = cvt<T>(Puphid[l]);
    }
#pragma unroll
    for (int s = 0; s < 6; ++s) sdPphi[s] = cvt<T>(sdPphid[s]);

    auto dv = [&](int a, int slot) -> T { return cvt<T>(dq[a][slot - DOFF]); };

    // ---------------- raised and contracted metric quantities
    // Dm[k][i][m] = gt^in D_knm ; Dup[k][ij] = D_k^ij
    T(&Dup)[3][6] = G.Dup;
    T trD[3];   // gt^jl D_kjl
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T Dm[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int m = 0; m < 3; ++m)
                Dm[i][m] = ig[sym(i, 0)] * D[k][sym(0, m)] + ig[sym(i, 1)] * D[k][sym(1, m)] +
                           ig[sym(i, 2)] * D[k][sym(2, m)];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j)
                Dup[k][sym(i, j)] = Dm[i][0] * ig[sym(0, j)] + Dm[i][1] * ig[sym(1, j)] + Dm[i][2] * ig[sym(2, j)];
        trD[k] = Dm[0][0] + Dm[1][1] + Dm[2][2];
    }
    // lowered conformal Christoffel Gl[l][ij] = D_ijl + D_jil - D_lij, raised Gt[k][ij]
    T(&Gl)[3][6] = G.Gl; T(&Gt)[3][6] = G.Gt;
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j)
                Gl[l][sym(i, j)] = D[i][sym(j, l)] + D[j][sym(i, l)] - D[l][sym(i, j)];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int s = 0; s < 6; ++s)
            Gt[k][s] = ig[sym(k, 0)] * Gl[0][s] + ig[sym(k, 1)] * Gl[1][s] + ig[sym(k, 2)] * Gl[2][s];
    // Gt^i = gt^jk Gt^i_jk ; W_n = gt^jk Gl[n][jk]
    T(&Gtv)[3] = G.Gtv; T(&Wl)[3] = G.Wl;
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        Gtv[i] = ig[0] * Gt[i][0] + ig[3] * Gt[i][3] + ig[5] * Gt[i][5] +
                 T(2) * (ig[1] * Gt[i][1] + ig[2] * Gt[i][2] + ig[4] * Gt[i][4]);
        Wl[i] = ig[0] * Gl[i][0] + ig[3] * Gl[i][3] + ig[5] * Gl[i][5] +
                T(2) * (ig[1] * Gl[i][1] + ig[2] * Gl[i][2] + ig[4] * Gl[i][4]);
    }
    // physical Christoffel Gamma^k_ij = Gt^k_ij - (delta^k_i P_j + delta^k_j P_i - gt_ij P^k)/phi
    T(&Gam)[3][6] = G.Gam;
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                T t = -g[sym(i, j)] * Puphi[k];
                if (k == i) t += Pphi[j];
                if (k == j) t += Pphi[i];
                Gam[k][sym(i, j)] = Gt[k][sym(i, j)] - t;
            }
    T(&Gc)[3] = G.Gc;  // Gamma^m_lm
#pragma unroll
    for (int l = 0; l < 3; ++l) Gc[l] = Gam[0][sym(l, 0)] + Gam[1][sym(l, 1)] + Gam[2][sym(l, 2)];

    // ---------------- Ricci tensor (symmetric) from the derivatives of D and P
    // V_l = D_m^ml ; PP = P_m P^m / phi^2
    T V[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) V[l] = Dup[0][sym(0, l)] + Dup[1][sym(1, l)] + Dup[2][sym(2, l)];
    const T PP = Pphi[0] * Puphi[0] + Pphi[1] * Puphi[1] + Pphi[2] * Puphi[2];
    const T VP = V[0] * Pphi[0] + V[1] * Pphi[1] + V[2] * Pphi[2];
    T trsdP = T(0);  // gt^ml dP_(ml) / phi
#pragma unroll
    for (int m = 0; m < 3; ++m)
#pragma unroll
        for (int l = 0; l < 3; ++l) trsdP += ig[sym(m, l)] * sdPphi[sym(m, l)];
    // U[a][b] = gt^ml d_a D_bml  (9 values)
    T(&U)[3][3] = G.U;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const int s0 = SD + 6 * b;
            U[a][b] = ig[0] * dv(a, s0 + 0) + ig[3] * dv(a, s0 + 3) + ig[5] * dv(a, s0 + 5) +
                      T(2) * (ig[1] * dv(a, s0 + 1) + ig[2] * dv(a, s0 + 2) + ig[4] * dv(a, s0 + 4));
        }
    T(&Ric)[6] = G.Ric;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const int ij = sym(i, j);
            // S1 = sum_m d_m Gamma^m_ij
            T s1 = T(0);
            // -2 V_l Gl[l][ij]
            s1 += T(-2) * (V[0] * Gl[0][ij] + V[1] * Gl[1][ij] + V[2] * Gl[2][ij]);
            // gt^ml (d_(m D_i)jl + d_(m D_j)il - d_(m D_l)ij)
            T e1 = T(0), e2 = T(0), e3 = T(0);
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int l = 0; l < 3; ++l) {
                    const T w = ig[sym(m, l)];
                    e1 += w * (dv(m, SD + 6 * i + sym(j, l)) + dv(i, SD + 6 * m + sym(j, l)));
                    e2 += w * (dv(m, SD + 6 * j + sym(i, l)) + dv(j, SD + 6 * m + sym(i, l)));
                    e3 += w * dv(m, SD + 6 * l + ij);
                }
            s1 += T(0.5) * (e1 + e2) - e3;
            // 2 (D_mij P^m - gt_ij V_l P_l)/phi
            s1 += T(2) * (D[0][ij] * Puphi[0] + D[1][ij] * Puphi[1] + D[2][ij] * Puphi[2] - g[ij] * VP);
            // -(dP_(ji) + dP_(ij) - gt_ij gt^ml dP_(ml))/phi
            s1 += -(T(2) * sdPphi[ij] - g[ij] * trsdP);
            // (2 P_i P_j - gt_ij P_m P^m)/phi^2
            s1 += T(2) * Pphi[i] * Pphi[j] - g[ij] * PP;
            // S2 = d_j (Gamma^m_im), symmetric
            T DD = T(0);
#pragma unroll
            for (int m = 0; m < 3; ++m)
#pragma unroll
                for (int l = 0; l < 3; ++l) DD += Dup[j][sym(m, l)] * D[i][sym(m, l)];
            T s2 = T(-2) * DD + T(0.5) * (U[j][i] + U[i][j]) - T(3) * sdPphi[ij] + T(3) * Pphi[i] * Pphi[j];
            // Gamma Gamma terms
            T gg = Gam[0][ij] * Gc[0] + Gam[1][ij] * Gc[1] + Gam[2][ij] * Gc[2];
#pragma unroll
            for (int l = 0; l < 3; ++l)
#pragma unroll
                for (int m = 0; m < 3; ++m) gg -= Gam[l][sym(i, m)] * Gam[m][sym(l, j)];
            Ric[ij] = s1 - s2 + gg;
        }

}

// First-order CCZ4 right-hand side of one cell (before Kreiss-Oliger dissipation).
template <typename T>
__device__ void ccz4_algebra(const double *__restrict__ q, const double (*__restrict__ dq)[NDIFF],
                             const RhsParams &p, double *__restrict__ out)
{
    Geo<T> G;
    compute_geo<T>(q, dq, G);
    const double detg = G.detg, phid = G.phid, iphid = G.iphid;
    const T(&g)[6] = G.g; const T(&ig)[6] = G.ig; const T(&At)[6] = G.At; const T(&D)[3][6] = G.D;
    const T(&B)[3][3] = G.B; const T(&A)[3] = G.A; const T(&be)[3] = G.be; const T(&Gh)[3] = G.Gh;
    const T(&bb)[3] = G.bb; const T al = G.al, Kt = G.Kt, Th = G.Th, K0 = G.K0;
    const T(&Pphi)[3] = G.Pphi; const T(&Dup)[3][6] = G.Dup; const T(&Gt)[3][6] = G.Gt;
    const T(&Gtv)[3] = G.Gtv; const T(&Wl)[3] = G.Wl; const T(&Gam)[3][6] = G.Gam; const T(&U)[3][3] = G.U;
    const T(&Ric)[6] = G.Ric;
    auto dv = [&](int a, int slot) -> T { return cvt<T>(dq[a][slot - DOFF]); };

    const T kap1 = cvt<T>(p.kappa1), kap2 = cvt<T>(p.kappa2), kap3 = cvt<T>(p.kappa3);
    const T cc = cvt<T>(p.c), ee2 = cvt<T>(p.e * p.e), mu = cvt<T>(p.mu), ff = cvt<T>(p.f),
            eta = cvt<T>(p.eta);
    const bool onelog = p.slicing == 1;
    const bool gdrv = p.shift == 1;
    const T ga = onelog ? T(2) / al : T(1);
    const T ga_lin = onelog ? T(2) : T(2) * al;   // 2 alpha g + alpha^2 g'
    const T trB = B[0][0] + B[1][1] + B[2][2];

    // ---------------- Z4 quantities
    // d_k Gt^i = -2 D_k^jl Gt^i_jl - 2 D_k^in W_n + gt^in F_kn,
    // F_kn = gt^jl (d_k D_jln + d_j D_kln) - (gt^jl (d_k D_njl + d_n D_kjl))/2
    T dGt[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T F[3];
#pragma unroll
        for (int n = 0; n < 3; ++n) {
            T f = T(0);
#pragma unroll
            for (int jj = 0; jj < 3; ++jj)
#pragma unroll
                for (int l = 0; l < 3; ++l)
                    f += ig[sym(jj, l)] * (dv(k, SD + 6 * jj + sym(l, n)) + dv(jj, SD + 6 * k + sym(l, n)));
            F[n] = f - T(0.5) * (U[k][n] + U[n][k]);
        }
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T t = T(0);
#pragma unroll
            for (int s = 0; s < 6; ++s) t += (s == 0 || s == 3 || s == 5 ? T(1) : T(2)) * Dup[k][s] * Gt[i][s];
            t = T(-2) * t;
            t += T(-2) * (Dup[k][sym(i, 0)] * Wl[0] + Dup[k][sym(i, 1)] * Wl[1] + Dup[k][sym(i, 2)] * Wl[2]);
            t += ig[sym(i, 0)] * F[0] + ig[sym(i, 1)] * F[1] + ig[sym(i, 2)] * F[2];
            dGt[k][i] = t;
        }
    }
    T dG[3];  // Ghat - Gt
#pragma unroll
    for (int i = 0; i < 3; ++i) dG[i] = Gh[i] - Gtv[i];
    T Zl[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) Zl[i] = T(0.5) * (g[sym(i, 0)] * dG[0] + g[sym(i, 1)] * dG[1] + g[sym(i, 2)] * dG[2]);
    const T phi = cvt<T>(phid);
    const T phi2 = cvt<T>(phid * phid);
    T Zu[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) Zu[i] = T(0.5) * phi2 * dG[i];
    // nabla_i Z_j
    T nZ[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            T t = D[i][sym(j, 0)] * dG[0] + D[i][sym(j, 1)] * dG[1] + D[i][sym(j, 2)] * dG[2];
#pragma unroll
            for (int l = 0; l < 3; ++l)
                t += T(0.5) * g[sym(j, l)] * (dv(i, SGHAT + l) - dGt[i][l]) - Gam[l][sym(i, j)] * Zl[l];
            nZ[i][j] = t;
        }
    // nabla_i nabla_j alpha
    T DDa[6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            DDa[sym(i, j)] = T(0.5) * (dv(i, SA + j) + dv(j, SA + i)) -
                             (Gam[0][sym(i, j)] * A[0] + Gam[1][sym(i, j)] * A[1] + Gam[2][sym(i, j)] * A[2]);
    // traces with the conformal metric
    auto trace = [&](const T *X) -> T {
        return ig[0] * X[0] + ig[3] * X[3] + ig[5] * X[5] + T(2) * (ig[1] * X[1] + ig[2] * X[2] + ig[4] * X[4]);
    };
    T Xs[6];  // -nabla nabla alpha + alpha (R_ij + 2 nabla_(i Z_j))
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const int ij = sym(i, j);
            Xs[ij] = -DDa[ij] + al * (Ric[ij] + nZ[i][j] + nZ[j][i]);
        }
    T RZs[6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) RZs[sym(i, j)] = Ric[sym(i, j)] + nZ[i][j] + nZ[j][i];
    const T RpZ = phi2 * trace(RZs);
    const T trX = trace(Xs);
    const T lapal = phi2 * trace(DDa);
    const T trAt = trace(At);

    // At^ij, At_ij At^ij
    T Am[3][3];  // gt^ik At_kj
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Am[i][j] = ig[sym(i, 0)] * At[sym(0, j)] + ig[sym(i, 1)] * At[sym(1, j)] + ig[sym(i, 2)] * At[sym(2, j)];
    T Aup[6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            Aup[sym(i, j)] = Am[i][0] * ig[sym(0, j)] + Am[i][1] * ig[sym(1, j)] + Am[i][2] * ig[sym(2, j)];
    T AA = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) AA += Am[i][j] * Am[j][i];

    // derivative traces: trdAt_k = gt^nm d_k At_nm ; DA_k = D_k^nm At_nm ; sdBtr_k = d_(k B_l)^l
    T trdAt[3], DA[3], sdBtr[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T dA6[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) dA6[s] = dv(k, SAT + s);
        trdAt[k] = trace(dA6);
        DA[k] = Dup[k][0] * At[0] + Dup[k][3] * At[3] + Dup[k][5] * At[5] +
                T(2) * (Dup[k][1] * At[1] + Dup[k][2] * At[2] + Dup[k][4] * At[4]);
        T t = T(0);
#pragma unroll
        for (int l = 0; l < 3; ++l) t += dv(k, SB + 3 * l + l) + dv(l, SB + 3 * k + l);
        sdBtr[k] = T(0.5) * t;
    }
    const T sfac = gdrv ? T(1) : T(0);

    // ---------------- gt_ij
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const int ij = sym(i, j);
            T t = T(2) * (be[0] * D[0][ij] + be[1] * D[1][ij] + be[2] * D[2][ij]);
#pragma unroll
            for (int k = 0; k < 3; ++k) t += g[sym(k, i)] * B[j][k] + g[sym(k, j)] * B[i][k];
            t += T(-2.0 / 3.0) * g[ij] * trB;
            t += T(-2) * al * (At[ij] - T(1.0 / 3.0) * g[ij] * trAt);
            out[SG + ij] = static_cast<double>(t) - (detg - 1.0) / p.tau * q[SG + ij];
        }
    // ---------------- alpha
    const T thetaterm = Kt - K0 - T(2) * cc * Th;
    out[SALPHA] = static_cast<double>(be[0] * A[0] + be[1] * A[1] + be[2] * A[2] - al * al * ga * thetaterm);
    // ---------------- beta^i
#pragma unroll
    for (int i = 0; i < 3; ++i)
        out[SBETA + i] = gdrv ? static_cast<double>(be[0] * B[0][i] + be[1] * B[1][i] + be[2] * B[2][i] + ff * bb[i]) : 0.0;
    // ---------------- phi (phi factor applied in double)
    out[SPHI] = q[SBETA] * q[SP] + q[SBETA + 1] * q[SP + 1] + q[SBETA + 2] * q[SP + 2] +
                phid * static_cast<double>((al * Kt - trB) * T(1.0 / 3.0));
    // ---------------- At_ij
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const int ij = sym(i, j);
            T t = be[0] * dv(0, SAT + ij) + be[1] * dv(1, SAT + ij) + be[2] * dv(2, SAT + ij);
#pragma unroll
            for (int k = 0; k < 3; ++k) t += At[sym(k, i)] * B[j][k] + At[sym(k, j)] * B[i][k];
            t += T(-2.0 / 3.0) * At[ij] * trB;
            t += al * At[ij] * (Kt - T(2) * Th * cc);
            t += T(-2) * al * (At[sym(i, 0)] * Am[0][j] + At[sym(i, 1)] * Am[1][j] + At[sym(i, 2)] * Am[2][j]);
            const T tf = Xs[ij] - T(1.0 / 3.0) * g[ij] * trX;
            out[SAT + ij] = static_cast<double>(t) + phid * phid * static_cast<double>(tf);
        }
    // ---------------- K
    out[SK] = static_cast<double>(be[0] * dv(0, SK) + be[1] * dv(1, SK) + be[2] * dv(2, SK) - lapal + al * RpZ +
                                  al * Kt * (Kt - T(2) * Th * cc) - T(3) * al * kap1 * (T(1) + kap2) * Th);
    // ---------------- Theta
    out[STHETA] = static_cast<double>(be[0] * dv(0, STHETA) + be[1] * dv(1, STHETA) + be[2] * dv(2, STHETA) +
                                      T(0.5) * al * ee2 * (RpZ + T(2.0 / 3.0) * Kt * Kt - AA) - al * Th * Kt * cc -
                                      (Zu[0] * A[0] + Zu[1] * A[1] + Zu[2] * A[2]) - al * kap1 * (T(2) + kap2) * Th);
    // ---------------- Ghat^i and b^i
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T t = be[0] * dv(0, SGHAT + i) + be[1] * dv(1, SGHAT + i) + be[2] * dv(2, SGHAT + i);
        T u = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T igik = ig[sym(i, k)];
            t += T(2) * al * igik * dv(k, STHETA);
            if (!p.formulation) t += T(2) * al * igik * (trdAt[k] - T(2) * DA[k]);  // constraint additions
            t += T(-4.0 / 3.0) * al * igik * dv(k, SK);
            t += sfac * T(1.0 / 3.0) * igik * sdBtr[k];
            t += T(-2) * igik * (Th * A[k] + T(2.0 / 3.0) * al * Kt * Zl[k]);
            t += T(-2) * al * kap1 * igik * Zl[k];
            u += igik * Zl[k];
#pragma unroll
            for (int l = 0; l < 3; ++l) t += ig[sym(k, l)] * T(0.5) * (dv(k, SB + 3 * l + i) + dv(l, SB + 3 * k + i));
        }
        t += T(2.0 / 3.0) * Gtv[i] * trB - (Gtv[0] * B[0][i] + Gtv[1] * B[1][i] + Gtv[2] * B[2][i]);
        T ga2 = Gt[i][0] * Aup[0] + Gt[i][3] * Aup[3] + Gt[i][5] * Aup[5] +
                T(2) * (Gt[i][1] * Aup[1] + Gt[i][2] * Aup[2] + Gt[i][4] * Aup[4]);
        ga2 -= T(3) * (Aup[sym(i, 0)] * Pphi[0] + Aup[sym(i, 1)] * Pphi[1] + Aup[sym(i, 2)] * Pphi[2]);
        t += T(2) * al * ga2;
        t += T(-2) * (Aup[sym(i, 0)] * A[0] + Aup[sym(i, 1)] * A[1] + Aup[sym(i, 2)] * A[2]);
        // 2 kappa3 (2/3 gt^ij Z_j trB - gt^jk Z_j B_k^i)
        T zb = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T zk = ig[sym(k, 0)] * Zl[0] + ig[sym(k, 1)] * Zl[1] + ig[sym(k, 2)] * Zl[2];
            zb += zk * B[k][i];
        }
        t += T(2) * kap3 * (T(2.0 / 3.0) * u * trB - zb);
        out[SGHAT + i] = static_cast<double>(t);
        const T bt = be[0] * (dv(0, SBB + i) - dv(0, SGHAT + i)) + be[1] * (dv(1, SBB + i) - dv(1, SGHAT + i)) +
                     be[2] * (dv(2, SBB + i) - dv(2, SGHAT + i)) - eta * bb[i];
        out[SBB + i] = gdrv ? static_cast<double>(t + bt) : 0.0;
    }
    // ---------------- A_k
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T t = be[0] * dv(0, SA + k) + be[1] * dv(1, SA + k) + be[2] * dv(2, SA + k);
        t += -al * al * ga * (dv(k, SK) - T(2) * cc * dv(k, STHETA));
        t += -al * ga * (trdAt[k] - T(2) * DA[k]);                          // constraint additions
        t += B[k][0] * A[0] + B[k][1] * A[1] + B[k][2] * A[2];
        t += -ga_lin * thetaterm * A[k];
        out[SA + k] = static_cast<double>(t);
    }
    // ---------------- B_k^i
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (!gdrv) {
                out[SB + 3 * k + i] = 0.0;
                continue;
            }
            T t = be[0] * dv(0, SB + 3 * k + i) + be[1] * dv(1, SB + 3 * k + i) + be[2] * dv(2, SB + 3 * k + i);
            t += ff * dv(k, SBB + i);
            t += B[k][0] * B[0][i] + B[k][1] * B[1][i] + B[k][2] * B[2][i];
            // curl terms: -alpha^2 mu gt^ij (d_k P_j - d_j P_k)/phi + alpha^2 mu gt^ij gt^nl (d_k D_ljn - d_l D_kjn)
            T cP = T(0), cD = T(0);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                cP += ig[sym(i, j)] * cvt<T>((dq[k][SP - DOFF + j] - dq[j][SP - DOFF + k]) * iphid);
                T s = T(0);
#pragma unroll
                for (int n = 0; n < 3; ++n)
#pragma unroll
                    for (int l = 0; l < 3; ++l)
                        s += ig[sym(n, l)] * (dv(k, SD + 6 * l + sym(j, n)) - dv(l, SD + 6 * k + sym(j, n)));
                cD += ig[sym(i, j)] * s;
            }
            t += al * al * mu * (cD - cP);
            out[SB + 3 * k + i] = static_cast<double>(t);
        }
    // ---------------- D_kij
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                const int ij = sym(i, j);
                T t = be[0] * dv(0, SD + 6 * k + ij) + be[1] * dv(1, SD + 6 * k + ij) + be[2] * dv(2, SD + 6 * k + ij);
                T sb = T(0);
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    sb += g[sym(m, i)] * (dv(k, SB + 3 * j + m) + dv(j, SB + 3 * k + m)) +
                          g[sym(m, j)] * (dv(k, SB + 3 * i + m) + dv(i, SB + 3 * k + m));
                t += sfac * (T(0.25) * sb - T(1.0 / 3.0) * g[ij] * sdBtr[k]);
                t += -al * dv(k, SAT + ij);
                t += al * T(1.0 / 3.0) * g[ij] * (trdAt[k] - T(2) * DA[k]);    // constraint additions
#pragma unroll
                for (int l = 0; l < 3; ++l)
                    t += B[k][l] * D[l][ij] + B[j][l] * D[k][sym(l, i)] + B[i][l] * D[k][sym(l, j)];
                t += T(-2.0 / 3.0) * trB * D[k][ij];
                t += -A[k] * (At[ij] - T(1.0 / 3.0) * g[ij] * trAt);
                out[SD + 6 * k + ij] = static_cast<double>(t);
            }
    // ---------------- P_k (phi factors applied in double)
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T t = be[0] * dv(0, SP + k) + be[1] * dv(1, SP + k) + be[2] * dv(2, SP + k);
        t += B[k][0] * cvt<T>(q[SP]) + B[k][1] * cvt<T>(q[SP + 1]) + B[k][2] * cvt<T>(q[SP + 2]);
        t += T(1.0 / 3.0) * (al * Kt - trB) * cvt<T>(q[SP + k]);
        const T phipart = T(1.0 / 3.0) * (al * dv(k, SK) - sdBtr[k]) + T(1.0 / 3.0) * al * (trdAt[k] - T(2) * DA[k]) +
                          T(1.0 / 3.0) * Kt * A[k];
        out[SP + k] = static_cast<double>(t) + phid * static_cast<double>(phipart);
    }
    out[SK0] = 0.0;
}

// Hamiltonian and momentum constraints of one cell (App. B):
//   H = phi^2 gt^ij R_ij + 2/3 K^2 - At_ij At^ij,
//   M_i = gt^kl d_k At_li - Am^l_m Gt^m_li - Gt^m At_im - 3 P^k At_ik / phi - 2/3 d_i K,
// with Am^l_m = gt^lk At_km (the symmetrised Christoffel term of M_i written out).
__device__ inline void constraints_algebra(const double *__restrict__ q, const double (*__restrict__ dq)[NDIFF],
                                           double *__restrict__ hm)
{
    Geo<double> G;
    compute_geo<double>(q, dq, G);
    const double(&ig)[6] = G.ig;
    const double(&At)[6] = G.At;
    double Am[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            Am[i][j] = ig[sym(i, 0)] * At[sym(0, j)] + ig[sym(i, 1)] * At[sym(1, j)] + ig[sym(i, 2)] * At[sym(2, j)];
    double AA = 0.0, trR = 0.0;
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            AA += Am[i][j] * Am[j][i];
            trR += ig[sym(i, j)] * G.Ric[sym(i, j)];
        }
    hm[0] = G.phid * G.phid * trR + (2.0 / 3.0) * G.Kt * G.Kt - AA;
    for (int i = 0; i < 3; ++i) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k)
            for (int l = 0; l < 3; ++l) s += ig[sym(k, l)] * dq[k][SAT - DOFF + sym(l, i)];
        for (int m = 0; m < 3; ++m) {
            for (int l = 0; l < 3; ++l) s -= Am[l][m] * G.Gt[m][sym(l, i)];
            s -= G.Gtv[m] * At[sym(i, m)];
        }
        for (int k = 0; k < 3; ++k) s -= 3.0 * G.Puphi[k] * At[sym(i, k)];
        s -= (2.0 / 3.0) * dq[i][SK - DOFF];
        hm[1 + i] = s;
    }
}

}  // namespace ccz4
