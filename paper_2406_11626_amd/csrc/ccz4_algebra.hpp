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
