// Register-lean evaluation of the first-order CCZ4 right-hand side of one cell.
//
// The right-hand side of App. B is produced in six phases, each of which loads the slots and
// FD4 derivatives it needs straight from the patch box, contracts every derivative into the
// few combinations the equations use as soon as it is formed, and stores its output slots
// (algebra + Kreiss-Oliger) before the next phase starts.  A compiler memory barrier between
// phases keeps the live ranges of one phase out of the next.  The derivatives of D_kij enter
// only through four contractions with the inverse conformal metric,
//   G1_ij = gt^ml d_m D_ijl,  H_ij = gt^ml d_i D_mjl,  U_ab = gt^ml d_a D_bml,  E_ij = gt^ml d_m D_lij,
// from which the Ricci tensor, d_k Gt^i and the curl term of the B equation follow (see
// ccz4_algebra.hpp for the contracted closing relations).
//
// T is the type of the nonlinear algebra: double, or float for the mixed-precision mode in
// which stencil differences, the inverse metric, its determinant and every factor of 1/phi
// are formed in double and the result is promoted back to double before the KO sum is added.
#pragma once
#include "ccz4_algebra.hpp"

namespace ccz4 {

#define CCZ4_PHASE_BARRIER() asm volatile("" ::: "memory")

// One cell of one patch: the patch base pointers are uniform over the work-group (scalar
// registers), the cell offset o is per lane.
struct CellRef {
    const double *__restrict__ qb;  // patch base, slot 0
    double *__restrict__ kb;
    int o;           // offset of the cell inside a slot box
    double i12[3];   // 1 / (12 dx_a)
    double koc[3];   // eps / (64 dx_a)
    int adv;         // advection stencil (RhsParams::advection)
};

__device__ __forceinline__ constexpr int axis_stride(int a) { return a == 0 ? 1 : (a == 1 ? YS : ZS); }

__device__ __forceinline__ double ld(const CellRef &c, int v) { return c.qb[v * CS + c.o]; }

// central fourth-order first derivative of slot v along axis a
__device__ __forceinline__ double fd(const CellRef &c, int v, int a)
{
    const double *f = c.qb + v * CS + c.o;
    const int s = axis_stride(a);
    return (8.0 * (f[s] - f[-s]) - (f[2 * s] - f[-2 * s])) * c.i12[a];
}

#ifndef CCZ4_KO_PRINTED_ORDER
#define CCZ4_KO_PRINTED_ORDER 1
#endif

__device__ __forceinline__ double ko_axis(const double *__restrict__ f, int s)
{
#if CCZ4_KO_PRINTED_ORDER
#pragma clang fp contract(off)
    return f[-3 * s] - 6.0 * f[-2 * s] + 15.0 * f[-s] - 20.0 * f[0] + 15.0 * f[s] - 6.0 * f[2 * s] + f[3 * s];
#else
    // symmetric pairs, three fused multiply-adds
    const double p3 = f[-3 * s] + f[3 * s], p2 = f[-2 * s] + f[2 * s], p1 = f[-s] + f[s];
    return fma(-20.0, f[0], fma(15.0, p1, fma(-6.0, p2, p3)));
#endif
}

// Kreiss-Oliger sum over the axes of slot v (printed stencil order, no contraction)
__device__ __forceinline__ double ko(const CellRef &c, int v)
{
    const double *f = c.qb + v * CS + c.o;
    const double kx = c.koc[0] * ko_axis(f, 1), ky = c.koc[1] * ko_axis(f, YS), kz = c.koc[2] * ko_axis(f, ZS);
    return (kx + ky) + kz;
}

// derivative of slot v along axis a for the advection term: central (LOP = 0), or lopsided
// (App. D; LOP = 1) by the sign of the shift component be with the pairing c.adv
template <int LOP>
__device__ __forceinline__ double fd_adv(const CellRef &c, int v, int a, double be)
{
    if constexpr (!LOP) {
        return fd(c, v, a);
    } else {
        const double *f = c.qb + v * CS + c.o;
        const int s = axis_stride(a);
        return lop_from_central(fd(c, v, a), lop_use_right(c.adv, be), f[-3 * s], f[-2 * s], f[-s], f[0], f[s],
                                f[2 * s], f[3 * s], c.i12[a]);
    }
}

// advection beta^k d_k of slot v
template <int LOP>
__device__ __forceinline__ double adv(const CellRef &c, int v, const double be[3])
{
    return be[0] * fd_adv<LOP>(c, v, 0, be[0]) + be[1] * fd_adv<LOP>(c, v, 1, be[1]) +
           be[2] * fd_adv<LOP>(c, v, 2, be[2]);
}

// Output sinks: the plain right-hand side writes k = algebra + KO; the fused stage folds each
// finished slot at once into the RK4 stage combine (see StageSink).
template <int L>
struct RhsSink {
    static constexpr int LOP = L;  // lopsided advection stencils in the phase functions
    int so;  // second-order formulation: the auxiliaries' right-hand sides are 0
    __device__ __forceinline__ void put(const CellRef &c, int v, double alg)
    {
        c.kb[v * CS + c.o] = (so && aux_slot(v)) ? 0.0 : alg + ko(c, v);
    }
    __device__ __forceinline__ void zero(const CellRef &c, int v) { c.kb[v * CS + c.o] = 0.0; }
    __device__ __forceinline__ void finish(const CellRef &) {}
};

__device__ __forceinline__ void metric_inverse(const double g[6], double ig[6], double &det)
{
    const double c00 = g[3] * g[5] - g[4] * g[4], c01 = g[2] * g[4] - g[1] * g[5], c02 = g[1] * g[4] - g[2] * g[3];
    det = g[0] * c00 + g[1] * c01 + g[2] * c02;
    const double id = 1.0 / det;
    ig[0] = c00 * id;
    ig[1] = c01 * id;
    ig[2] = c02 * id;
    ig[3] = (g[0] * g[5] - g[2] * g[2]) * id;
    ig[4] = (g[1] * g[2] - g[0] * g[4]) * id;
    ig[5] = (g[0] * g[3] - g[1] * g[1]) * id;
}

template <typename T>
__device__ __forceinline__ T tr6(const T ig[6], const T X[6])
{
    return ig[0] * X[0] + ig[3] * X[3] + ig[5] * X[5] + T(2) * (ig[1] * X[1] + ig[2] * X[2] + ig[4] * X[4]);
}

// D_k^ij and the lowered Christoffel symbols Gl[l][ij] = D_ijl + D_jil - D_lij
template <typename T>
__device__ __forceinline__ void raise_D(const T ig[6], const T D[3][6], T Dup[3][6])
{
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T Dm[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int m = 0; m < 3; ++m)
                Dm[i][m] = ig[sym(i, 0)] * D[k][sym(0, m)] + ig[sym(i, 1)] * D[k][sym(1, m)] + ig[sym(i, 2)] * D[k][sym(2, m)];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j)
                Dup[k][sym(i, j)] = Dm[i][0] * ig[sym(0, j)] + Dm[i][1] * ig[sym(1, j)] + Dm[i][2] * ig[sym(2, j)];
    }
}

template <typename T>
__device__ __forceinline__ void christoffel(const T ig[6], const T D[3][6], T Gl[3][6], T Gt[3][6], T Gtv[3])
{
#pragma unroll
    for (int l = 0; l < 3; ++l)
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) Gl[l][sym(i, j)] = D[i][sym(j, l)] + D[j][sym(i, l)] - D[l][sym(i, j)];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int s = 0; s < 6; ++s) Gt[k][s] = ig[sym(k, 0)] * Gl[0][s] + ig[sym(k, 1)] * Gl[1][s] + ig[sym(k, 2)] * Gl[2][s];
#pragma unroll
    for (int i = 0; i < 3; ++i) Gtv[i] = tr6(ig, Gt[i]);
}

// ---------------------------------------------------------------------------------------
// phase 1: At_ij, K, Theta (Ricci tensor, nabla nabla alpha, Z4 terms).  Returns the curl
// contraction H - G1 of d D that the B equation needs.
template <typename T, typename Sink>
__device__ __forceinline__ void phase_ricci(Sink &snk, const CellRef &c, const RhsParams &p, T CmG[3][3])
{
    double gd[6], igd[6], detg;
#pragma unroll
    for (int s = 0; s < 6; ++s) gd[s] = ld(c, SG + s);
    metric_inverse(gd, igd, detg);
    T g[6], ig[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        g[s] = cvt<T>(gd[s]);
        ig[s] = cvt<T>(igd[s]);
    }
    // contractions of d D
    T G1[3][3], H[3][3], U[3][3], E[6];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
        for (int j = 0; j < 3; ++j) G1[i][j] = H[i][j] = U[i][j] = T(0);
        E[i] = E[i + 3] = T(0);
    }
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
#pragma unroll
            for (int dd = cc; dd < 3; ++dd) {
                const int s = sym(cc, dd);
#pragma unroll
                for (int a = 0; a < 3; ++a) {
                    const T v = cvt<T>(fd(c, SD + 6 * b + s, a));
                    G1[b][cc] += ig[sym(a, dd)] * v;
                    H[a][cc] += ig[sym(b, dd)] * v;
                    if (cc != dd) {
                        G1[b][dd] += ig[sym(a, cc)] * v;
                        H[a][dd] += ig[sym(b, cc)] * v;
                        U[a][b] += T(2) * ig[s] * v;
                    } else {
                        U[a][b] += ig[s] * v;
                    }
                    E[s] += ig[sym(a, b)] * v;
                }
            }
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int j = 0; j < 3; ++j) CmG[k][j] = H[k][j] - G1[k][j];

    // conformal factor terms in double
    const double phid = ld(c, SPHI);
    const double iphid = 1.0 / phid;
    double Pphid[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) Pphid[l] = ld(c, SP + l) * iphid;
    T Pphi[3], Puphi[3], sdPphi[6];
#pragma unroll
    for (int m = 0; m < 3; ++m) {
        Pphi[m] = cvt<T>(Pphid[m]);
        Puphi[m] = cvt<T>(igd[sym(m, 0)] * Pphid[0] + igd[sym(m, 1)] * Pphid[1] + igd[sym(m, 2)] * Pphid[2]);
    }
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            sdPphi[sym(i, j)] = cvt<T>(0.5 * (fd(c, SP + j, i) + fd(c, SP + i, j)) * iphid);

    T D[3][6];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int s = 0; s < 6; ++s) D[k][s] = cvt<T>(ld(c, SD + 6 * k + s));
    T Dup[3][6], Gl[3][6], Gt[3][6], Gtv[3];
    raise_D(ig, D, Dup);
    christoffel(ig, D, Gl, Gt, Gtv);
    T V[3], Wl[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        V[l] = Dup[0][sym(0, l)] + Dup[1][sym(1, l)] + Dup[2][sym(2, l)];
        Wl[l] = tr6(ig, Gl[l]);
    }
    T Gam[3][6];
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
    T Gc[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) Gc[l] = Gam[0][sym(l, 0)] + Gam[1][sym(l, 1)] + Gam[2][sym(l, 2)];
    const T PP = Pphi[0] * Puphi[0] + Pphi[1] * Puphi[1] + Pphi[2] * Puphi[2];
    const T VP = V[0] * Pphi[0] + V[1] * Pphi[1] + V[2] * Pphi[2];
    const T trsdP = tr6(ig, sdPphi);

    // symmetric Ricci tensor
    T Ric[6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const int ij = sym(i, j);
            T s1 = T(-2) * (V[0] * Gl[0][ij] + V[1] * Gl[1][ij] + V[2] * Gl[2][ij]);
            s1 += T(0.5) * (G1[i][j] + H[i][j] + G1[j][i] + H[j][i]) - E[ij];
            s1 += T(2) * (D[0][ij] * Puphi[0] + D[1][ij] * Puphi[1] + D[2][ij] * Puphi[2] - g[ij] * VP);
            s1 += -(T(2) * sdPphi[ij] - g[ij] * trsdP);
            s1 += T(2) * Pphi[i] * Pphi[j] - g[ij] * PP;
            T DD = T(0);
#pragma unroll
            for (int s = 0; s < 6; ++s) DD += (s == 0 || s == 3 || s == 5 ? T(1) : T(2)) * Dup[j][s] * D[i][s];
            const T s2 = T(-2) * DD + T(0.5) * (U[j][i] + U[i][j]) - T(3) * sdPphi[ij] + T(3) * Pphi[i] * Pphi[j];
            T gg = Gam[0][ij] * Gc[0] + Gam[1][ij] * Gc[1] + Gam[2][ij] * Gc[2];
#pragma unroll
            for (int l = 0; l < 3; ++l)
#pragma unroll
                for (int m = 0; m < 3; ++m) gg -= Gam[l][sym(i, m)] * Gam[m][sym(l, j)];
            Ric[ij] = s1 - s2 + gg;
        }
    // d_k Gt^i = -2 D_k^jl Gt^i_jl - 2 D_k^in W_n + gt^in F_kn
    T dGt[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T F[3];
#pragma unroll
        for (int n = 0; n < 3; ++n) F[n] = H[k][n] + G1[k][n] - T(0.5) * (U[k][n] + U[n][k]);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T t = T(0);
#pragma unroll
            for (int s = 0; s < 6; ++s) t += (s == 0 || s == 3 || s == 5 ? T(1) : T(2)) * Dup[k][s] * Gt[i][s];
            t = T(-2) * t - T(2) * (Dup[k][sym(i, 0)] * Wl[0] + Dup[k][sym(i, 1)] * Wl[1] + Dup[k][sym(i, 2)] * Wl[2]);
            dGt[k][i] = t + ig[sym(i, 0)] * F[0] + ig[sym(i, 1)] * F[1] + ig[sym(i, 2)] * F[2];
        }
    }
    // Z4 terms
    T dG[3], Zl[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) dG[i] = cvt<T>(ld(c, SGHAT + i)) - Gtv[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) Zl[i] = T(0.5) * (g[sym(i, 0)] * dG[0] + g[sym(i, 1)] * dG[1] + g[sym(i, 2)] * dG[2]);
    T RZ[6];  // R_ij + nabla_i Z_j + nabla_j Z_i
    {
        T nZ[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T dGh[3];
#pragma unroll
            for (int l = 0; l < 3; ++l) dGh[l] = cvt<T>(fd(c, SGHAT + l, i)) - dGt[i][l];
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                T t = D[i][sym(j, 0)] * dG[0] + D[i][sym(j, 1)] * dG[1] + D[i][sym(j, 2)] * dG[2];
#pragma unroll
                for (int l = 0; l < 3; ++l) t += T(0.5) * g[sym(j, l)] * dGh[l] - Gam[l][sym(i, j)] * Zl[l];
                nZ[i][j] = t;
            }
        }
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) RZ[sym(i, j)] = Ric[sym(i, j)] + nZ[i][j] + nZ[j][i];
    }
    // nabla_i nabla_j alpha
    T A[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) A[k] = cvt<T>(ld(c, SA + k));
    T DDa[6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            DDa[sym(i, j)] = T(0.5) * cvt<T>(fd(c, SA + j, i) + fd(c, SA + i, j)) -
                             (Gam[0][sym(i, j)] * A[0] + Gam[1][sym(i, j)] * A[1] + Gam[2][sym(i, j)] * A[2]);

    const T al = cvt<T>(ld(c, SALPHA));
    const T Kt = cvt<T>(ld(c, SK));
    const T Th = cvt<T>(ld(c, STHETA));
    T X[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) X[s] = -DDa[s] + al * RZ[s];
    const T trX = tr6(ig, X);
    const T phi2 = cvt<T>(phid * phid);
    const T RpZ = phi2 * tr6(ig, RZ);
    const T lapal = phi2 * tr6(ig, DDa);
    T At[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) At[s] = cvt<T>(ld(c, SAT + s));
    T Am[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j)
            Am[i][j] = ig[sym(i, 0)] * At[sym(0, j)] + ig[sym(i, 1)] * At[sym(1, j)] + ig[sym(i, 2)] * At[sym(2, j)];
    T AA = T(0);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) AA += Am[i][j] * Am[j][i];
    double be[3];
    T bet[3], Bm[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        be[k] = ld(c, SBETA + k);
        bet[k] = cvt<T>(be[k]);
#pragma unroll
        for (int i = 0; i < 3; ++i) Bm[k][i] = cvt<T>(ld(c, SB + 3 * k + i));
    }
    const T trB = Bm[0][0] + Bm[1][1] + Bm[2][2];
    const T cc = cvt<T>(p.c);
    // At_ij
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const int ij = sym(i, j);
            T t = T(0);
#pragma unroll
            for (int k = 0; k < 3; ++k) t += At[sym(k, i)] * Bm[j][k] + At[sym(k, j)] * Bm[i][k];
            t += T(-2.0 / 3.0) * At[ij] * trB;
            t += al * At[ij] * (Kt - T(2) * Th * cc);
            t += T(-2) * al * (At[sym(i, 0)] * Am[0][j] + At[sym(i, 1)] * Am[1][j] + At[sym(i, 2)] * Am[2][j]);
            const T tf = X[ij] - T(1.0 / 3.0) * g[ij] * trX;
            snk.put(c, SAT + ij, adv<Sink::LOP>(c, SAT + ij, be) + static_cast<double>(t) + phid * phid * static_cast<double>(tf));
        }
    const T kap1 = cvt<T>(p.kappa1), kap2 = cvt<T>(p.kappa2);
    snk.put(c, SK, adv<Sink::LOP>(c, SK, be) + static_cast<double>(-lapal + al * RpZ + al * Kt * (Kt - T(2) * Th * cc) -
                                                        T(3) * al * kap1 * (T(1) + kap2) * Th));
    const T ee2 = cvt<T>(p.e * p.e);
    const T half_phi2 = T(0.5) * phi2;
    const T ZA = half_phi2 * (dG[0] * A[0] + dG[1] * A[1] + dG[2] * A[2]);
    snk.put(c, STHETA, adv<Sink::LOP>(c, STHETA, be) + static_cast<double>(T(0.5) * al * ee2 * (RpZ + T(2.0 / 3.0) * Kt * Kt - AA) -
                                                              al * Th * Kt * cc - ZA - al * kap1 * (T(2) + kap2) * Th));
    (void)bet;
}

// ---------------------------------------------------------------------------------------
// phase 2: B_k^i (Gamma-driver only; zero with the frozen shift)
template <typename T, typename Sink>
__device__ __forceinline__ void phase_B(Sink &snk, const CellRef &c, const RhsParams &p, const T CmG[3][3])
{
    if (p.shift == 0) {
#pragma unroll
        for (int s = 0; s < 9; ++s) snk.zero(c, SB + s);
        return;
    }
    double gd[6], igd[6], detg;
#pragma unroll
    for (int s = 0; s < 6; ++s) gd[s] = ld(c, SG + s);
    metric_inverse(gd, igd, detg);
    T ig[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) ig[s] = cvt<T>(igd[s]);
    const double iphid = 1.0 / ld(c, SPHI);
    double be[3];
    T Bm[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        be[k] = ld(c, SBETA + k);
#pragma unroll
        for (int i = 0; i < 3; ++i) Bm[k][i] = cvt<T>(ld(c, SB + 3 * k + i));
    }
    // curl of P / phi: cP[k][j] = (d_k P_j - d_j P_k)/phi
    T cP[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        cP[k][k] = T(0);
#pragma unroll
        for (int j = k + 1; j < 3; ++j) {
            const double w = (fd(c, SP + j, k) - fd(c, SP + k, j)) * iphid;
            cP[k][j] = cvt<T>(w);
            cP[j][k] = cvt<T>(-w);
        }
    }
    const T al = cvt<T>(ld(c, SALPHA));
    const T a2mu = al * al * cvt<T>(p.mu);
    const T ff = cvt<T>(p.f);
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            T t = ff * cvt<T>(fd(c, SBB + i, k));
            t += Bm[k][0] * Bm[0][i] + Bm[k][1] * Bm[1][i] + Bm[k][2] * Bm[2][i];
            T curl = T(0);
#pragma unroll
            for (int j = 0; j < 3; ++j) curl += ig[sym(i, j)] * (CmG[k][j] - cP[k][j]);
            t += a2mu * curl;
            snk.put(c, SB + 3 * k + i, adv<Sink::LOP>(c, SB + 3 * k + i, be) + static_cast<double>(t));
        }
}

// ---------------------------------------------------------------------------------------
// phase 3: Ghat^i and b^i
template <typename T, typename Sink>
__device__ __forceinline__ void phase_gamma(Sink &snk, const CellRef &c, const RhsParams &p)
{
    double gd[6], igd[6], detg;
#pragma unroll
    for (int s = 0; s < 6; ++s) gd[s] = ld(c, SG + s);
    metric_inverse(gd, igd, detg);
    T g[6], ig[6], At[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        g[s] = cvt<T>(gd[s]);
        ig[s] = cvt<T>(igd[s]);
        At[s] = cvt<T>(ld(c, SAT + s));
    }
    T D[3][6];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int s = 0; s < 6; ++s) D[k][s] = cvt<T>(ld(c, SD + 6 * k + s));
    T Dup[3][6], Gl[3][6], Gt[3][6], Gtv[3];
    raise_D(ig, D, Dup);
    christoffel(ig, D, Gl, Gt, Gtv);
    // At^ij
    T Aup[6];
    {
        T Am[3][3];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = 0; j < 3; ++j)
                Am[i][j] = ig[sym(i, 0)] * At[sym(0, j)] + ig[sym(i, 1)] * At[sym(1, j)] + ig[sym(i, 2)] * At[sym(2, j)];
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j)
                Aup[sym(i, j)] = Am[i][0] * ig[sym(0, j)] + Am[i][1] * ig[sym(1, j)] + Am[i][2] * ig[sym(2, j)];
    }
    // d_k tr(At) through the constraint additions: gt^nm d_k At_nm - 2 D_k^nm At_nm
    T dtrA[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T dA6[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) dA6[s] = cvt<T>(fd(c, SAT + s, k));
        dtrA[k] = tr6(ig, dA6) - T(2) * tr6(At, Dup[k]);
    }
    // shift derivatives: GB^i = gt^kl d_(k B_l)^i and sdBtr_k = d_(k B_l)^l
    T GB[3] = {T(0), T(0), T(0)}, sdBtr[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l)
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const T v = cvt<T>(fd(c, SB + 3 * l + i, k));  // d_k B_l^i
                GB[i] += ig[sym(k, l)] * v;
                if (i == l) sdBtr[k] += T(0.5) * v;           // d_k B_l^l
                if (i == k) sdBtr[l] += T(0.5) * v;           // d_l B_k^l with (l <-> k)
            }
    double be[3];
    T Bm[3][3], A[3], Ph[3];
    const double iphid = 1.0 / ld(c, SPHI);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        be[k] = ld(c, SBETA + k);
        A[k] = cvt<T>(ld(c, SA + k));
        Ph[k] = cvt<T>(ld(c, SP + k) * iphid);
#pragma unroll
        for (int i = 0; i < 3; ++i) Bm[k][i] = cvt<T>(ld(c, SB + 3 * k + i));
    }
    const T trB = Bm[0][0] + Bm[1][1] + Bm[2][2];
    const T al = cvt<T>(ld(c, SALPHA));
    const T Kt = cvt<T>(ld(c, SK));
    const T Th = cvt<T>(ld(c, STHETA));
    T dG[3], Zl[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) dG[i] = cvt<T>(ld(c, SGHAT + i)) - Gtv[i];
#pragma unroll
    for (int i = 0; i < 3; ++i) Zl[i] = T(0.5) * (g[sym(i, 0)] * dG[0] + g[sym(i, 1)] * dG[1] + g[sym(i, 2)] * dG[2]);
    const T kap1 = cvt<T>(p.kappa1), kap3 = cvt<T>(p.kappa3);
    const T sfac = p.shift ? T(1) : T(0);
    T dTh[3], dK[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dTh[k] = cvt<T>(fd(c, STHETA, k));
        dK[k] = cvt<T>(fd(c, SK, k));
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T t = GB[i];
        T u = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T igik = ig[sym(i, k)];
            t += T(2) * al * igik * (dTh[k] + (p.formulation ? T(0) : dtrA[k])) - T(4.0 / 3.0) * al * igik * dK[k];
            t += sfac * T(1.0 / 3.0) * igik * sdBtr[k];
            t += T(-2) * igik * (Th * A[k] + T(2.0 / 3.0) * al * Kt * Zl[k] + al * kap1 * Zl[k]);
            u += igik * Zl[k];
        }
        t += T(2.0 / 3.0) * Gtv[i] * trB - (Gtv[0] * Bm[0][i] + Gtv[1] * Bm[1][i] + Gtv[2] * Bm[2][i]);
        T ga = tr6(Aup, Gt[i]) - T(3) * (Aup[sym(i, 0)] * Ph[0] + Aup[sym(i, 1)] * Ph[1] + Aup[sym(i, 2)] * Ph[2]);
        t += T(2) * al * ga;
        t += T(-2) * (Aup[sym(i, 0)] * A[0] + Aup[sym(i, 1)] * A[1] + Aup[sym(i, 2)] * A[2]);
        T zb = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T zk = ig[sym(k, 0)] * Zl[0] + ig[sym(k, 1)] * Zl[1] + ig[sym(k, 2)] * Zl[2];
            zb += zk * Bm[k][i];
        }
        t += T(2) * kap3 * (T(2.0 / 3.0) * u * trB - zb);
        const double advG = adv<Sink::LOP>(c, SGHAT + i, be);
        const double rG = advG + static_cast<double>(t);
        snk.put(c, SGHAT + i, rG);
        if (p.shift) snk.put(c, SBB + i, rG - advG + adv<Sink::LOP>(c, SBB + i, be) - p.eta * ld(c, SBB + i));
        else snk.zero(c, SBB + i);
    }
}

// ---------------------------------------------------------------------------------------
// phase 4: A_k and P_k
template <typename T, typename Sink>
__device__ __forceinline__ void phase_AP(Sink &snk, const CellRef &c, const RhsParams &p)
{
    double gd[6], igd[6], detg;
#pragma unroll
    for (int s = 0; s < 6; ++s) gd[s] = ld(c, SG + s);
    metric_inverse(gd, igd, detg);
    T ig[6], At[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        ig[s] = cvt<T>(igd[s]);
        At[s] = cvt<T>(ld(c, SAT + s));
    }
    T dtrA[3];
    {
        T D[3][6], Dup[3][6];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int s = 0; s < 6; ++s) D[k][s] = cvt<T>(ld(c, SD + 6 * k + s));
        raise_D(ig, D, Dup);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            T dA6[6];
#pragma unroll
            for (int s = 0; s < 6; ++s) dA6[s] = cvt<T>(fd(c, SAT + s, k));
            dtrA[k] = tr6(ig, dA6) - T(2) * tr6(At, Dup[k]);
        }
    }
    T sdBtr[3] = {T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int l = 0; l < 3; ++l) sdBtr[k] += T(0.5) * cvt<T>(fd(c, SB + 3 * l + l, k) + fd(c, SB + 3 * k + l, l));
    double be[3];
    T Bm[3][3], A[3], P[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        be[k] = ld(c, SBETA + k);
        A[k] = cvt<T>(ld(c, SA + k));
        P[k] = cvt<T>(ld(c, SP + k));
#pragma unroll
        for (int i = 0; i < 3; ++i) Bm[k][i] = cvt<T>(ld(c, SB + 3 * k + i));
    }
    const T trB = Bm[0][0] + Bm[1][1] + Bm[2][2];
    const T al = cvt<T>(ld(c, SALPHA));
    const T Kt = cvt<T>(ld(c, SK));
    const T Th = cvt<T>(ld(c, STHETA));
    const T K0 = cvt<T>(ld(c, SK0));
    const double phid = ld(c, SPHI);
    const T cc = cvt<T>(p.c);
    const bool onelog = p.slicing == 1;
    const T ga = onelog ? T(2) / al : T(1);
    const T ga_lin = onelog ? T(2) : T(2) * al;  // 2 alpha g + alpha^2 g'
    const T theta_term = Kt - K0 - T(2) * cc * Th;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const T dK = cvt<T>(fd(c, SK, k)), dTh = cvt<T>(fd(c, STHETA, k));
        T t = -al * al * ga * (dK - T(2) * cc * dTh) - al * ga * dtrA[k];
        t += Bm[k][0] * A[0] + Bm[k][1] * A[1] + Bm[k][2] * A[2];
        t += -ga_lin * theta_term * A[k];
        snk.put(c, SA + k, adv<Sink::LOP>(c, SA + k, be) + static_cast<double>(t));
        T u = Bm[k][0] * P[0] + Bm[k][1] * P[1] + Bm[k][2] * P[2] + T(1.0 / 3.0) * (al * Kt - trB) * P[k];
        const T phipart = T(1.0 / 3.0) * (al * dK - sdBtr[k]) + T(1.0 / 3.0) * al * dtrA[k] + T(1.0 / 3.0) * Kt * A[k];
        snk.put(c, SP + k, adv<Sink::LOP>(c, SP + k, be) + static_cast<double>(u) + phid * static_cast<double>(phipart));
    }
}

// ---------------------------------------------------------------------------------------
// phase 5: D_kij
template <typename T, typename Sink>
__device__ __forceinline__ void phase_D(Sink &snk, const CellRef &c0, const RhsParams &p)
{
    const CellRef &c = c0;
    double gd[6], igd[6], detg;
#pragma unroll
    for (int s = 0; s < 6; ++s) gd[s] = ld(c, SG + s);
    metric_inverse(gd, igd, detg);
    T g[6], ig[6], At[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        g[s] = cvt<T>(gd[s]);
        ig[s] = cvt<T>(igd[s]);
        At[s] = cvt<T>(ld(c, SAT + s));
    }
    const T trAt = tr6(ig, At);
    const T al = cvt<T>(ld(c, SALPHA));
    double be[3];
    T Bm[3][3], A[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        be[k] = ld(c, SBETA + k);
        A[k] = cvt<T>(ld(c, SA + k));
#pragma unroll
        for (int i = 0; i < 3; ++i) Bm[k][i] = cvt<T>(ld(c, SB + 3 * k + i));
    }
    const T trB = Bm[0][0] + Bm[1][1] + Bm[2][2];
    const T sfac = p.shift ? T(1) : T(0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T D[3][6];
#pragma unroll
        for (int kk = 0; kk < 3; ++kk)
#pragma unroll
            for (int s = 0; s < 6; ++s) D[kk][s] = cvt<T>(ld(c, SD + 6 * kk + s));
        T Dupk[6];
        {
            T Dm[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int m = 0; m < 3; ++m)
                    Dm[i][m] = ig[sym(i, 0)] * D[k][sym(0, m)] + ig[sym(i, 1)] * D[k][sym(1, m)] + ig[sym(i, 2)] * D[k][sym(2, m)];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = i; j < 3; ++j)
                    Dupk[sym(i, j)] = Dm[i][0] * ig[sym(0, j)] + Dm[i][1] * ig[sym(1, j)] + Dm[i][2] * ig[sym(2, j)];
        }
        T dAk[6];
#pragma unroll
        for (int s = 0; s < 6; ++s) dAk[s] = cvt<T>(fd(c, SAT + s, k));
        const T dtrA = tr6(ig, dAk) - T(2) * tr6(At, Dupk);
        // Y[j][m] = d_k B_j^m + d_j B_k^m
        T Y[3][3];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int m = 0; m < 3; ++m) Y[j][m] = cvt<T>(fd(c, SB + 3 * j + m, k) + fd(c, SB + 3 * k + m, j));
        const T sdBtr = T(0.5) * (Y[0][0] + Y[1][1] + Y[2][2]);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
            for (int j = i; j < 3; ++j) {
                const int ij = sym(i, j);
                T sb = T(0);
#pragma unroll
                for (int m = 0; m < 3; ++m) sb += g[sym(m, i)] * Y[j][m] + g[sym(m, j)] * Y[i][m];
                T t = sfac * (T(0.25) * sb - T(1.0 / 3.0) * g[ij] * sdBtr);
                t += -al * dAk[ij] + al * T(1.0 / 3.0) * g[ij] * dtrA;
#pragma unroll
                for (int l = 0; l < 3; ++l) t += Bm[k][l] * D[l][ij] + Bm[j][l] * D[k][sym(l, i)] + Bm[i][l] * D[k][sym(l, j)];
                t += T(-2.0 / 3.0) * trB * D[k][ij];
                t += -A[k] * (At[ij] - T(1.0 / 3.0) * g[ij] * trAt);
                snk.put(c, SD + 6 * k + ij, adv<Sink::LOP>(c, SD + 6 * k + ij, be) + static_cast<double>(t));
            }
        CCZ4_PHASE_BARRIER();
    }
}

// ---------------------------------------------------------------------------------------
// phase 6: gt_ij, alpha, beta^i, phi and K_0
template <typename T, typename Sink>
__device__ __forceinline__ void phase_point(Sink &snk, const CellRef &c, const RhsParams &p)
{
    double gd[6], igd[6], detg;
#pragma unroll
    for (int s = 0; s < 6; ++s) gd[s] = ld(c, SG + s);
    metric_inverse(gd, igd, detg);
    T g[6], ig[6], At[6];
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        g[s] = cvt<T>(gd[s]);
        ig[s] = cvt<T>(igd[s]);
        At[s] = cvt<T>(ld(c, SAT + s));
    }
    double be[3];
    T bet[3], Bm[3][3], A[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        be[k] = ld(c, SBETA + k);
        bet[k] = cvt<T>(be[k]);
        A[k] = cvt<T>(ld(c, SA + k));
#pragma unroll
        for (int i = 0; i < 3; ++i) Bm[k][i] = cvt<T>(ld(c, SB + 3 * k + i));
    }
    const T trB = Bm[0][0] + Bm[1][1] + Bm[2][2];
    const T trAt = tr6(ig, At);
    const T al = cvt<T>(ld(c, SALPHA));
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const int ij = sym(i, j);
            T t = T(2) * (bet[0] * cvt<T>(ld(c, SD + ij)) + bet[1] * cvt<T>(ld(c, SD + 6 + ij)) +
                          bet[2] * cvt<T>(ld(c, SD + 12 + ij)));
#pragma unroll
            for (int k = 0; k < 3; ++k) t += g[sym(k, i)] * Bm[j][k] + g[sym(k, j)] * Bm[i][k];
            t += T(-2.0 / 3.0) * g[ij] * trB;
            t += T(-2) * al * (At[ij] - T(1.0 / 3.0) * g[ij] * trAt);
            snk.put(c, SG + ij, static_cast<double>(t) - (detg - 1.0) / p.tau * gd[ij]);
        }
    const T Kt = cvt<T>(ld(c, SK)), K0 = cvt<T>(ld(c, SK0)), Th = cvt<T>(ld(c, STHETA));
    const T ga = p.slicing == 1 ? T(2) / al : T(1);
    snk.put(c, SALPHA, static_cast<double>(bet[0] * A[0] + bet[1] * A[1] + bet[2] * A[2] -
                                         al * al * ga * (Kt - K0 - T(2) * cvt<T>(p.c) * Th)));
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (p.shift)
            snk.put(c, SBETA + i, static_cast<double>(bet[0] * Bm[0][i] + bet[1] * Bm[1][i] + bet[2] * Bm[2][i] +
                                                    cvt<T>(p.f) * cvt<T>(ld(c, SBB + i))));
        else
            snk.zero(c, SBETA + i);
    }
    const double phid = ld(c, SPHI);
    snk.put(c, SPHI, be[0] * ld(c, SP) + be[1] * ld(c, SP + 1) + be[2] * ld(c, SP + 2) +
                       phid * static_cast<double>((al * Kt - trB) * T(1.0 / 3.0)));
    snk.zero(c, SK0);
}

// Pass the cell offset through an opaque register move so that the compiler can neither
// reuse loads of an earlier phase nor hoist the loads of a later one above this point.
__device__ __forceinline__ CellRef fresh(const CellRef &c)
{
    CellRef r = c;
    int o = c.o;
    asm volatile("" : "+v"(o));
    r.o = o;
    return r;
}

template <typename T, typename Sink>
__device__ __forceinline__ void rhs_cell_phased(const CellRef &c0, const RhsParams &p, Sink &snk)
{
    T CmG[3][3];
    phase_ricci<T>(snk, fresh(c0), p, CmG);
    phase_B<T>(snk, fresh(c0), p, CmG);
    phase_gamma<T>(snk, fresh(c0), p);
    phase_AP<T>(snk, fresh(c0), p);
    phase_D<T>(snk, fresh(c0), p);
    phase_point<T>(snk, fresh(c0), p);
    snk.finish(fresh(c0));
}

}  // namespace ccz4
