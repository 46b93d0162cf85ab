// LDS-staged evaluation of the first-order CCZ4 right-hand side for one z-slab of a patch
// (3 x 9 x 9 = 243 cells, one work-group of 256 threads).
//
// Every evolved slot is copied once per evaluation from the patch box into LDS with gfx950's
// direct global->LDS loads (16 bytes per lane, no registers involved), at most 15 slots per
// round.  A slot occupies, in LDS, the slab's three planes in box layout (3 x 15 x 16 doubles,
// carrying the x and y halos) followed by the interior rows of the three planes below and the
// three planes above the slab (6 x 9 rows x 10 doubles, columns x = 2..11).  Each y or z face
// halo is read either from the patch's own halo or straight from the interior of the same-level
// neighbour across that face (HaloSrc).  Every FD4
// derivative and Kreiss-Oliger sum is then read from LDS; a per-lane table maps the seven
// z-neighbours of a cell into the own planes or the halo rows.
//
// The order of the equations is chosen so that each slot is staged exactly once:
//   round 1: At, B      -> d tr(At), the shift-derivative contractions, the non-advective part of
//                          the D equations, advection + KO of At and B (kept in registers)
//   round 2: D (15)     -> contractions G1, H, U, E of d D; outputs of those D slots
//   round 3: D (3), P, A, Ghat, K, Theta
//                       -> last contractions and D outputs; Ricci tensor, nabla nabla alpha and
//                          the Z terms; outputs At, K, Theta, Ghat, A, P; B and b without d b
//   round 4: b, gt, alpha, beta, phi
//                       -> outputs B, b, gt, alpha, beta, phi and K_0 = 0
// The algebra is the one of ccz4_rhs_phased.hpp, term for term (App. B); T is double, or float
// for the mixed-precision mode with the same split between FP64 and FP32 parts.
#pragma once
#include "ccz4_rhs_phased.hpp"

namespace ccz4 {

// Row pitch of the staged own planes in LDS (doubles): 18 (default), whose odd pair count spreads
// the rows of a wave's reads over the LDS banks (the extra pair is a repeat copy), or the box row
// (16), whose rows all fall on the same banks.
#ifndef CCZ4_LDS_ROW
#define CCZ4_LDS_ROW 18
#endif
constexpr int LROW = CCZ4_LDS_ROW;
static_assert(LROW == 16 || LROW == 18, "LDS row pitch: 16 or 18 doubles");
constexpr int LPAIRS = LROW / 2;                  // 16-byte copies per staged row
constexpr int LPLANE = NBX * LROW;                // one staged plane, 15 rows
constexpr int LDS_OWN = 3 * LPLANE;               // the slab's planes
constexpr int LDS_OWN_PAIRS = 3 * NBX * LPAIRS;   // 360 or 405 copies
constexpr int LDS_OWN_CHUNKS = (LDS_OWN_PAIRS + 63) / 64;
constexpr int LDS_HROW = 10;                      // halo row: x = 2..11 (16-byte aligned pairs)
constexpr int LDS_HALO = 6 * 9 * LDS_HROW;        // 540 doubles
constexpr int LDS_SLOT = LDS_OWN + LDS_HALO;      // 1260 (1350) doubles
constexpr int LDS_NBUF = 15;
constexpr int LDS_DOUBLES = LDS_NBUF * LDS_SLOT;  // 151200 bytes

typedef __attribute__((address_space(3))) void lds_void_t;

// cache-policy bits of the staging copies (0: the default policy)
#ifndef CCZ4_STAGE_CPOL
#define CCZ4_STAGE_CPOL 0
#endif

// Where the y and z face halos of a patch are read from: d[2 (a - 1) + (side > 0)] (a = 1, 2) is
// added to the element index of a halo cell of the face of axis a on that side.  0 reads the
// patch's own halo (filled beforehand); for a same-level neighbour n it is (n - p) PS -+ 9 stride_a,
// which reads the neighbour's interior cell at the same position directly, so that those halos
// need no copy.  The x halos always come from the patch's own halo: x-face sources would split a
// 16-byte pair (x = 2 from the neighbour, x = 3 from the patch) and need 4-byte copies, which cost
// more than the x-face copies themselves (the x neighbours are mostly resident in the same L2).
struct HaloSrc {
    int64_t d[4];
};

// Issue the direct global->LDS copies of slot v of slab sl into buffer b (does not wait).
// Own planes: 45 rows of LPAIRS pairs in 64-lane chunks (with an 18-double pitch the ninth pair of
// a row repeats its eighth), the rows y <= 2 and y >= 12 from the y faces'
// sources; halo rows: 270 pairs in five chunks, pair e being plane e / 45 (0..2 below, 3..5
// above), row (e / 5) % 9, columns 2 + 2 (e % 5), planes outside the patch from the z faces'
// sources.
__device__ __forceinline__ void lds_stage_slot(const double *__restrict__ qp, double *lds, int sl, int v, int b,
                                               int w, int lane, const HaloSrc &hs)
{
    const double *box = qp + v * CS;
    double *dst = lds + b * LDS_SLOT;
    const double *own = box + (3 + 3 * sl) * ZS;
    const int w0 = (w + b) & 3;
    for (int ch = w0; ch < LDS_OWN_CHUNKS; ch += 4)
        if (ch * 64 + lane < LDS_OWN_PAIRS) {
            const int q = ch * 64 + lane, r = q / LPAIRS, j = q % LPAIRS, y = r % 15;
            const int e = r * XS + 2 * (j < 8 ? j : 7);
            // selects, not an index into hs.d: a lane-dependent index would put the array in memory
            const int64_t d = y <= 2 ? hs.d[0] : (y >= 12 ? hs.d[1] : 0);
            __builtin_amdgcn_global_load_lds((const void *)(own + e + d), (lds_void_t *)(dst + ch * 128), 16, 0, CCZ4_STAGE_CPOL);
        }
    const int w1 = (w + b + 2) & 3;
    for (int ch = w1; ch < 5; ch += 4) {
        const int e = ch * 64 + lane;
        if (e < 270) {
            const int hp = e / 45, row = (e / 5) % 9, pr = e % 5;
            const int z = hp < 3 ? 3 * sl + hp : 3 * sl + 3 + hp;
            const int64_t zd = z <= 2 ? hs.d[2] : (z >= 12 ? hs.d[3] : 0);
            __builtin_amdgcn_global_load_lds((const void *)(box + (z * ZS + (row + 3) * YS + 2 + 2 * pr) + zd),
                                             (lds_void_t *)(dst + LDS_OWN + ch * 128), 16, 0, CCZ4_STAGE_CPOL);
        }
    }
}

// Issue the copies of a round's N slots into buffers 0..N-1 once every wave is done with the
// previous round's buffers; returns without waiting for them.
template <int N>
__device__ __forceinline__ void lds_issue(const double *__restrict__ qp, double *lds, int sl, const int (&slots)[N],
                                          int w, int lane, const HaloSrc &hs)
{
    __syncthreads();
#pragma unroll
    for (int j = 0; j < N; ++j) lds_stage_slot(qp, lds, sl, slots[j], j, w, lane, hs);
}

// Wait for every outstanding memory operation of the lane and make the staged slots visible to
// the work-group.
__device__ __forceinline__ void lds_wait()
{
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
}

// Stage the N slots of a round and wait for them.
template <int N>
__device__ __forceinline__ void lds_round(const double *__restrict__ qp, double *lds, int sl, const int (&slots)[N],
                                          int w, int lane, const HaloSrc &hs)
{
    lds_issue(qp, lds, sl, slots, w, lane, hs);
    lds_wait();
}

// One cell's view of the staged slab.
struct LdsCell {
    const double *s;  // LDS base
    int c;            // index of the cell in the own planes: zl * 240 + y * 16 + x
    int zo[7];        // index of the z-neighbour at offset k - 3
    double i12[3];    // 1 / (12 dx_a)
    double koc[3];    // eps / (64 dx_a)
};

__device__ __forceinline__ double lv(const LdsCell &c, int b, int a, int k)
{
    const double *f = c.s + b * LDS_SLOT;
    return a == 0 ? f[c.c + k] : (a == 1 ? f[c.c + k * LROW] : f[c.zo[k + 3]]);
}

// The LDS offsets of cell (x, y) (box indices) in plane zl (0..2) of the staged slab: its own
// index and those of its seven z-neighbours (own planes, or the halo rows below and above).
__device__ __forceinline__ void lds_cell_offsets(LdsCell &C, int x, int y, int zl)
{
    C.c = zl * LPLANE + y * LROW + x;
#pragma unroll
    for (int k = -3; k <= 3; ++k) {
        const int z2 = zl + k;
        C.zo[k + 3] = (z2 >= 0 && z2 <= 2) ? z2 * LPLANE + y * LROW + x
                                            : LDS_OWN + (z2 < 0 ? z2 + 3 : z2) * 90 + (y - 3) * LDS_HROW + (x - 2);
    }
}

__device__ __forceinline__ double fd(const LdsCell &c, int b, int a)
{
    return (8.0 * (lv(c, b, a, 1) - lv(c, b, a, -1)) - (lv(c, b, a, 2) - lv(c, b, a, -2))) * c.i12[a];
}

__device__ __forceinline__ double ko_axis_lds(const LdsCell &c, int b, int a)
{
#if CCZ4_KO_PRINTED_ORDER
#pragma clang fp contract(off)
    return lv(c, b, a, -3) - 6.0 * lv(c, b, a, -2) + 15.0 * lv(c, b, a, -1) - 20.0 * lv(c, b, a, 0) +
           15.0 * lv(c, b, a, 1) - 6.0 * lv(c, b, a, 2) + lv(c, b, a, 3);
#else
    const double p3 = lv(c, b, a, -3) + lv(c, b, a, 3), p2 = lv(c, b, a, -2) + lv(c, b, a, 2),
                 p1 = lv(c, b, a, -1) + lv(c, b, a, 1);
    return fma(-20.0, lv(c, b, a, 0), fma(15.0, p1, fma(-6.0, p2, p3)));
#endif
}

__device__ __forceinline__ double ko(const LdsCell &c, int b)
{
    const double kx = c.koc[0] * ko_axis_lds(c, b, 0), ky = c.koc[1] * ko_axis_lds(c, b, 1),
                 kz = c.koc[2] * ko_axis_lds(c, b, 2);
    return (kx + ky) + kz;
}

__device__ __forceinline__ double adv(const LdsCell &c, int b, const double be[3])
{
    return be[0] * fd(c, b, 0) + be[1] * fd(c, b, 1) + be[2] * fd(c, b, 2);
}

// Output sinks of the slab evaluation: put(v, r) receives the complete right-hand side of slot v
// (algebra, advection and KO) of the lane's cell, at offset o of the patch box.
struct LdsRhsSink {
    double *__restrict__ kb;
    int o;
    int so;  // second-order formulation: the auxiliaries' right-hand sides are 0
    // K is written once and not read again in this launch, and no other work-group writes the
    // same lines: nontemporal stores keep the staged lines in L2 (2% per launch).
    __device__ __forceinline__ void put(int v, double r) { __builtin_nontemporal_store(r, kb + v * CS + o); }
    __device__ __forceinline__ void finish() {}
    // A round's outputs in two halves (see flush below): the RHS alone reads nothing.
    template <int N>
    __device__ __forceinline__ void load(const int (&)[N], double (&)[N], double (&)[N]) {}
    template <int N>
    __device__ __forceinline__ void store(const int (&slots)[N], const double (&r)[N], const double (&)[N],
                                          const double (&)[N])
    {
#pragma unroll
        for (int j = 0; j < N; ++j) put(slots[j], (so && aux_slot(slots[j])) ? 0.0 : r[j]);
    }
};

// (s, d) of the symmetric index s = sym(cc, dd), cc <= dd
__device__ __forceinline__ constexpr int sym_first(int s) { return s < 3 ? 0 : (s < 5 ? 1 : 2); }
__device__ __forceinline__ constexpr int sym_second(int s) { return s < 3 ? s : (s < 5 ? s - 2 : 2); }

template <typename T>
__device__ __forceinline__ void dD_accumulate(const double d[3], int j, const T ig[6], T G1[3][3], T H[3][3],
                                              T U[3][3], T E[6])
{
    const int b = j / 6, s = j % 6;  // D_b,s with s = sym(cc, dd)
    const int cc = sym_first(s), dd = sym_second(s);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const T v = cvt<T>(d[a]);
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

// An opaque copy of the cell's offsets, so that loads of one block of the algebra are neither
// merged with nor hoisted above those of another (this bounds the registers each block holds).
__device__ __forceinline__ LdsCell fresh(const LdsCell &c)
{
    LdsCell r = c;
    asm volatile("" : "+v"(r.c));
#pragma unroll
    for (int k = 0; k < 7; ++k) asm volatile("" : "+v"(r.zo[k]));
    return r;
}

__device__ __forceinline__ int fresh(int o)
{
    asm volatile("" : "+v"(o));
    return o;
}

// The pointwise metric of the cell, its slots read by ld(v): g, its inverse and its determinant.
template <typename T, typename Ld>
__device__ __forceinline__ void load_metric_with(Ld ld, double gd[6], double igd[6], double &detg, T g[6], T ig[6])
{
#pragma unroll
    for (int s = 0; s < 6; ++s) gd[s] = ld(SG + s);
    metric_inverse(gd, igd, detg);
#pragma unroll
    for (int s = 0; s < 6; ++s) {
        g[s] = cvt<T>(gd[s]);
        ig[s] = cvt<T>(igd[s]);
    }
}

// ... of the cell at offset o of the patch box
template <typename T>
__device__ __forceinline__ void load_metric(const double *__restrict__ qp, int o, double gd[6], double igd[6],
                                            double &detg, T g[6], T ig[6])
{
    load_metric_with<T>([&](int v) -> double { return qp[v * CS + o]; }, gd, igd, detg, g, ig);
}

// The LDS buffer that holds slot v during round r of rhs_slab_lds, or -1 (see the round lists).
__device__ __forceinline__ constexpr int round_buffer(int r, int v)
{
    if (r == 1) return (v >= SAT && v < SAT + 6) ? v - SAT : ((v >= SB && v < SB + 9) ? 6 + v - SB : -1);
    if (r == 3)
        return (v >= SD + 15 && v < SD + 18) ? v - SD - 15
               : (v >= SP && v < SP + 3)     ? 3 + v - SP
               : (v >= SA && v < SA + 3)     ? 6 + v - SA
               : (v >= SGHAT && v < SGHAT + 3) ? 9 + v - SGHAT
               : v == SK                     ? 12
               : v == STHETA                 ? 13
                                             : -1;
    if (r == 4)
        return (v >= SBB && v < SBB + 3)     ? v - SBB
               : (v >= SG && v < SG + 6)     ? 3 + v - SG
               : v == SALPHA                 ? 9
               : (v >= SBETA && v < SBETA + 3) ? 10 + v - SBETA
               : v == SPHI                   ? 13
                                             : -1;
    return -1;
}

// Pointwise value of slot v at the lane's cell during round R: from the staged copy in LDS when
// the round stages v (the same double), else from the patch box at offset o.
#ifndef CCZ4_PW_LDS
#define CCZ4_PW_LDS 1
#endif
template <int R>
__device__ __forceinline__ double pw(const double *__restrict__ qp, int o, const LdsCell &C, int v)
{
    if (CCZ4_PW_LDS) {
        const int b = round_buffer(R, v);
        if (b >= 0) return C.s[b * LDS_SLOT + C.c];
    }
    return qp[v * CS + o];
}

// The three FD4 derivatives and the Kreiss-Oliger sum of staged buffer b at the lane's cell,
// from the 19 distinct stencil points; the compiler barrier after the reads keeps the LDS
// loads of one slot from being hoisted above those of the previous one.
struct SlotDeriv {
    double d[3];
    double k;
    double a;  // advection beta^k d_k (central or lopsided), with the 4-argument form only
};

__device__ __forceinline__ SlotDeriv stencils(const LdsCell &c, int b)
{
    SlotDeriv r;
#pragma unroll
    for (int a = 0; a < 3; ++a) r.d[a] = fd(c, b, a);
    r.k = ko(c, b);
    r.a = 0.0;
    CCZ4_PHASE_BARRIER();
    return r;
}

// ... and the advection term with shift be: the central derivatives (LOP = 0), or the lopsided
// stencils of App. D (LOP = 1, pairing `mode` as RhsParams::advection) from the same staged
// points.  LOP is a template parameter so that the central kernel carries no lopsided code.
template <int LOP>
__device__ __forceinline__ SlotDeriv stencils(const LdsCell &c, int b, const double be[3], int32_t mode)
{
    SlotDeriv r;
#pragma unroll
    for (int a = 0; a < 3; ++a) r.d[a] = fd(c, b, a);
    r.k = ko(c, b);
    if constexpr (!LOP) {
        r.a = be[0] * r.d[0] + be[1] * r.d[1] + be[2] * r.d[2];
    } else {
        double s[3];
#pragma unroll
        for (int a = 0; a < 3; ++a)
            s[a] = lop_from_central(r.d[a], lop_use_right(mode, be[a]), lv(c, b, a, -3), lv(c, b, a, -2),
                                    lv(c, b, a, -1), lv(c, b, a, 0), lv(c, b, a, 1), lv(c, b, a, 2), lv(c, b, a, 3),
                                    c.i12[a]);
        r.a = be[0] * s[0] + be[1] * s[1] + be[2] * s[2];
    }
    CCZ4_PHASE_BARRIER();
    return r;
}

__device__ __forceinline__ double dot3(const double be[3], const double d[3])
{
    return be[0] * d[0] + be[1] * d[1] + be[2] * d[2];
}

// r = v, materialised here: the opaque move keeps the computation of v inside its block of
// the algebra instead of letting it drift towards the round's output loop.
__device__ __forceinline__ void keep(double &r, double v)
{
    r = v;
    asm volatile("" : "+v"(r));
}

// Round 3's Ghat^i sector: its right-hand side (ro3[11..13]), the part of b^i's right-hand side it
// shares (rGb) and the pointwise part of the gt_ij equation (pwG), from the cell's metric, D, At,
// B, A, P / phi, the Christoffel symbols and Z, and the contractions carried from rounds 1 and 2.
template <typename T, int LOP>
__device__ __forceinline__ void ghat_sector(const LdsCell &C, const RhsParams &p, const double be[3], const T g[6],
                                            const T ig[6], const double gd[6], double detg, const T (&D)[3][6],
                                            const T (&Gt)[3][6], const T Gtv[3], const T At[6], const T (&Am)[3][3],
                                            const T (&Bm)[3][3], const T A[3], const T Ph[3], T trB, T al, T Kt, T Th,
                                            const T Zl[3], const T GB[3], const T sdBtr[3], const T dtrA[3], T red,
                                            T sfac, double (&ro3)[20], double (&rGb)[3], double (&pwG)[6])
{
    T Aup[6];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j)
            Aup[sym(i, j)] = Am[i][0] * ig[sym(0, j)] + Am[i][1] * ig[sym(1, j)] + Am[i][2] * ig[sym(2, j)];
    const T kap1 = cvt<T>(p.kappa1), kap3 = cvt<T>(p.kappa3);
    T dTh[3], dK[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dTh[k] = cvt<T>(fd(C, 13, k));
        dK[k] = cvt<T>(fd(C, 12, k));
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        T t = GB[i];
        T u = T(0);
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const T igik = ig[sym(i, k)];
            t += T(2) * al * igik * (dTh[k] + red * dtrA[k]) - T(4.0 / 3.0) * al * igik * dK[k];
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
        const SlotDeriv sG = stencils<LOP>(C, 9 + i, be, p.advection);
        const double advG = sG.a;
        const double rG = advG + static_cast<double>(t);
        keep(ro3[11 + i], rG + sG.k);
        rGb[i] = rG - advG;
    }
    // gt_ij: 2 beta^k D_kij + gt_ki B_j^k + gt_kj B_i^k - 2/3 gt_ij tr B - 2 alpha (At_ij - gt_ij tr At / 3)
    // - (det gt - 1) gt_ij / tau
    T bet[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) bet[k] = cvt<T>(be[k]);
    const T trAt = tr6(ig, At);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j) {
            const int ij = sym(i, j);
            T t = T(2) * (bet[0] * D[0][ij] + bet[1] * D[1][ij] + bet[2] * D[2][ij]);
#pragma unroll
            for (int k = 0; k < 3; ++k) t += g[sym(k, i)] * Bm[j][k] + g[sym(k, j)] * Bm[i][k];
            t += T(-2.0 / 3.0) * g[ij] * trB;
            t += T(-2) * al * (At[ij] - T(1.0 / 3.0) * g[ij] * trAt);
            keep(pwG[ij], static_cast<double>(t) - (detg - 1.0) / p.tau * gd[ij]);
        }
}

// Output slots of rounds 2, 3 and 4, in the order of the round's output buffer.
__device__ constexpr int R2_OUT[15] = {SD, SD + 1, SD + 2, SD + 3, SD + 4, SD + 5, SD + 6, SD + 7,
                                       SD + 8, SD + 9, SD + 10, SD + 11, SD + 12, SD + 13, SD + 14};
__device__ constexpr int R3_OUT[20] = {SD + 15, SD + 16, SD + 17, SAT, SAT + 1, SAT + 2, SAT + 3,
                                       SAT + 4, SAT + 5, SK, STHETA, SGHAT, SGHAT + 1, SGHAT + 2,
                                       SA, SA + 1, SA + 2, SP, SP + 1, SP + 2};
__device__ constexpr int R4_OUT[24] = {SB, SB + 1, SB + 2, SB + 3, SB + 4, SB + 5, SB + 6, SB + 7,
                                       SB + 8, SBB, SBB + 1, SBB + 2, SG, SG + 1, SG + 2, SG + 3,
                                       SG + 4, SG + 5, SALPHA, SBETA, SBETA + 1, SBETA + 2, SPHI, SK0};

// A round's outputs go to the sink in two halves: its global loads (the RK4 combine reads Q^n
// and the accumulator), issued together, and its stores.  Between the two the caller issues the
// staging of the following round, so that those copies and the sink's loads are in flight
// together, and waits for both; the stores are then left in flight over the next barrier.
// Right-hand side of the lane's cell of slab sl of the patch at qp.  Every lane of the
// work-group must call this (staging and barriers); only lanes with act = true compute.
template <typename T, int LOP, typename Sink>
__device__ __forceinline__ void rhs_slab_lds(const double *__restrict__ qp, double *lds, int sl, bool act, int o0,
                                             const LdsCell &C0, const RhsParams &p, Sink &snk, const HaloSrc &hs)
{
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const bool gdrv = p.shift != 0;
    const T sfac = gdrv ? T(1) : T(0);
    const T cc = cvt<T>(p.c);
    // the red terms of the Ghat equation (2 alpha gt^ik d_k tr At, with d_k gt^nm = -2 D_k^nm)
    // belong to the first-order formulation only
    const T red = p.formulation ? T(0) : T(1);
    // Round 3's Ghat sector shares the Ricci sector's loads and Christoffel symbols when the algebra is
    // FP32 (room in the register file); with FP64 algebra it reloads them in a block of its own, which
    // keeps the register peak of the Ricci sector below spilling.
    constexpr bool GHAT_IN_RICCI = sizeof(T) == 4;

    // carried between rounds
    T dtrA[3], sdBtr[3], GB[3], partD[3][6];
    double advkoAt[6], advkoB[9];
    T G1[3][3], H[3][3], U[3][3], E[6];
    T BB[3][3], curl[3][3];
    double rGb[3];
    // the pointwise parts of the gt, alpha, beta and phi equations, formed in round 3 where their
    // inputs are at hand (round 4 adds the Kreiss-Oliger sums and f b^i)
    double pwG[6], pwA, pwPhi;
    T bB[3];
    double ro2[15], ro3[20], ro4[24];  // each round's outputs, handed to the sink after the round

    // ------------------------------------------------------------ round 1: At, B
    {
        const int r1[15] = {SAT, SAT + 1, SAT + 2, SAT + 3, SAT + 4, SAT + 5, SB, SB + 1, SB + 2,
                            SB + 3, SB + 4, SB + 5, SB + 6, SB + 7, SB + 8};
        lds_round(qp, lds, sl, r1, w, lane, hs);
    }
    if (act) {
        {  // B: advection + KO, GB^i = gt^kl d_(k B_l)^i, sdBtr_k = d_(k B_l)^l, and the shift
           // terms of the D equations
            const LdsCell C = fresh(C0);
            const int o = fresh(o0);
            double be[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) be[k] = qp[(SBETA + k) * CS + o];
            double gd[6], igd[6], detg;
            T g[6], ig[6];
            load_metric<T>(qp, o, gd, igd, detg, g, ig);
            double dB[3][3][3];  // dB[l][i][k] = d_k B_l^i
#pragma unroll
            for (int i = 0; i < 3; ++i) GB[i] = sdBtr[i] = T(0);
#pragma unroll
            for (int l = 0; l < 3; ++l)
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    const SlotDeriv sd = stencils<LOP>(C, 6 + 3 * l + i, be, p.advection);
                    advkoB[3 * l + i] = gdrv ? sd.a + sd.k : 0.0;
#pragma unroll
                    for (int k = 0; k < 3; ++k) dB[l][i][k] = sd.d[k];
                }
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int l = 0; l < 3; ++l)
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        const T v = cvt<T>(dB[l][i][k]);
                        GB[i] += ig[sym(k, l)] * v;
                        if (i == l) sdBtr[k] += T(0.5) * v;
                        if (i == k) sdBtr[l] += T(0.5) * v;
                    }
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                T Y[3][3];  // d_k B_j^m + d_j B_k^m
#pragma unroll
                for (int j = 0; j < 3; ++j)
#pragma unroll
                    for (int m = 0; m < 3; ++m) Y[j][m] = cvt<T>(dB[j][m][k] + dB[k][m][j]);
                const T sdB = T(0.5) * (Y[0][0] + Y[1][1] + Y[2][2]);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = i; j < 3; ++j) {
                        const int ij = sym(i, j);
                        T sb = T(0);
#pragma unroll
                        for (int m = 0; m < 3; ++m) sb += g[sym(m, i)] * Y[j][m] + g[sym(m, j)] * Y[i][m];
                        partD[k][ij] = sfac * (T(0.25) * sb - T(1.0 / 3.0) * g[ij] * sdB);
                    }
            }
        }
        CCZ4_PHASE_BARRIER();
        {  // At: advection + KO, d_k tr(At), and the rest of the D equations
            const LdsCell C = fresh(C0);
            const int o = fresh(o0);
            auto q = [&](int v) -> double { return pw<1>(qp, o, C, v); };
            double be[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) be[k] = q(SBETA + k);
            double dA[6][3];
#pragma unroll
            for (int s = 0; s < 6; ++s) {
                const SlotDeriv sd = stencils<LOP>(C, s, be, p.advection);
                advkoAt[s] = sd.a + sd.k;
#pragma unroll
                for (int k = 0; k < 3; ++k) dA[s][k] = sd.d[k];
            }
            double gd[6], igd[6], detg;
            T g[6], ig[6];
            load_metric<T>(qp, o, gd, igd, detg, g, ig);
            T At[6], D[3][6], Bm[3][3], A[3];
#pragma unroll
            for (int s = 0; s < 6; ++s) At[s] = cvt<T>(q(SAT + s));
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                A[k] = cvt<T>(q(SA + k));
#pragma unroll
                for (int s = 0; s < 6; ++s) D[k][s] = cvt<T>(q(SD + 6 * k + s));
#pragma unroll
                for (int i = 0; i < 3; ++i) Bm[k][i] = cvt<T>(q(SB + 3 * k + i));
            }
            const T trB = Bm[0][0] + Bm[1][1] + Bm[2][2];
            const T trAt = tr6(ig, At);
            const T al = cvt<T>(q(SALPHA));
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                T Dupk[6];
                {
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
                            Dupk[sym(i, j)] = Dm[i][0] * ig[sym(0, j)] + Dm[i][1] * ig[sym(1, j)] + Dm[i][2] * ig[sym(2, j)];
                }
                T dAk[6];
#pragma unroll
                for (int s = 0; s < 6; ++s) dAk[s] = cvt<T>(dA[s][k]);
                dtrA[k] = tr6(ig, dAk) - T(2) * tr6(At, Dupk);
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = i; j < 3; ++j) {
                        const int ij = sym(i, j);
                        T t = partD[k][ij];
                        t += -al * dAk[ij] + al * T(1.0 / 3.0) * g[ij] * dtrA[k];
#pragma unroll
                        for (int l = 0; l < 3; ++l)
                            t += Bm[k][l] * D[l][ij] + Bm[j][l] * D[k][sym(l, i)] + Bm[i][l] * D[k][sym(l, j)];
                        t += T(-2.0 / 3.0) * trB * D[k][ij];
                        t += -A[k] * (At[ij] - T(1.0 / 3.0) * g[ij] * trAt);
                        partD[k][ij] = t;
                    }
            }
        }
    }

    // ------------------------------------------------------------ round 2: D_x.., D_y.., D_zxx..D_zxz
    {
        const int r2[15] = {SD, SD + 1, SD + 2, SD + 3, SD + 4, SD + 5, SD + 6, SD + 7,
                            SD + 8, SD + 9, SD + 10, SD + 11, SD + 12, SD + 13, SD + 14};
        lds_round(qp, lds, sl, r2, w, lane, hs);
    }
    if (act) {
        const LdsCell C = fresh(C0);
        const int o = fresh(o0);
        double gd[6], igd[6], detg;
        T g[6], ig[6];
        load_metric<T>(qp, o, gd, igd, detg, g, ig);
        double be[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) be[k] = qp[(SBETA + k) * CS + o];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
#pragma unroll
            for (int j = 0; j < 3; ++j) G1[i][j] = H[i][j] = U[i][j] = T(0);
            E[i] = E[i + 3] = T(0);
        }
#pragma unroll
        for (int j = 0; j < 15; ++j) {
            const SlotDeriv sd = stencils<LOP>(C, j, be, p.advection);
            dD_accumulate<T>(sd.d, j, ig, G1, H, U, E);
            keep(ro2[j], sd.a + static_cast<double>(partD[j / 6][j % 6]) + sd.k);
        }
    }

    {
        const int r3[14] = {SD + 15, SD + 16, SD + 17, SP, SP + 1, SP + 2, SA, SA + 1, SA + 2,
                            SGHAT, SGHAT + 1, SGHAT + 2, SK, STHETA};
        double qa[15], qb[15];
        if (act) snk.load(R2_OUT, qa, qb);
        lds_issue(qp, lds, sl, r3, w, lane, hs);
        __builtin_amdgcn_s_waitcnt(0);  // the sink's loads and this wave's copies have landed
        if (act) snk.store(R2_OUT, ro2, qa, qb);
    }
    __syncthreads();  // every wave's copies have landed; the stores may still be in flight

    // ------------------------------------------------------------ round 3
    // buffers: 0..2 D_zyy, D_zyz, D_zzz; 3..5 P; 6..8 A; 9..11 Ghat; 12 K; 13 Theta
    if (act) {
        const LdsCell C = fresh(C0);
        const int o = fresh(o0);
        auto q = [&](int v) -> double { return pw<3>(qp, o, C, v); };
        double be[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) be[k] = q(SBETA + k);
        {
            double gd[6], igd[6], detg;
            T g[6], ig[6];
            load_metric<T>(qp, o, gd, igd, detg, g, ig);
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                const SlotDeriv sd = stencils<LOP>(C, j, be, p.advection);
                dD_accumulate<T>(sd.d, 15 + j, ig, G1, H, U, E);
                keep(ro3[j], sd.a + static_cast<double>(partD[2][3 + j]) + sd.k);
            }
        }
        {  // ---- Ricci sector: At, K, Theta; the curl term of B
            const int o1 = fresh(o);
            auto q1 = [&](int v) -> double { return pw<3>(qp, o1, C, v); };
            double gd[6], igd[6], detg;
            T g[6], ig[6];
            load_metric<T>(qp, o1, gd, igd, detg, g, ig);
            const double phid = q1(SPHI), iphid = 1.0 / phid;
            double Pphid[3];
#pragma unroll
            for (int l = 0; l < 3; ++l) Pphid[l] = q1(SP + l) * iphid;
            T Pphi[3], Puphi[3], sdPphi[6];
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                Pphi[m] = cvt<T>(Pphid[m]);
                Puphi[m] = cvt<T>(igd[sym(m, 0)] * Pphid[0] + igd[sym(m, 1)] * Pphid[1] + igd[sym(m, 2)] * Pphid[2]);
            }
            {
                double dP[3][3];  // dP[j][i] = d_i P_j
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const SlotDeriv sd = stencils(C, 3 + j);
#pragma unroll
                    for (int i = 0; i < 3; ++i) dP[j][i] = sd.d[i];
                }
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = i; j < 3; ++j) sdPphi[sym(i, j)] = cvt<T>(0.5 * (dP[j][i] + dP[i][j]) * iphid);
            }
            T D[3][6];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int s = 0; s < 6; ++s) D[k][s] = cvt<T>(q1(SD + 6 * k + s));
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
                    const T s2 =
                        T(-2) * DD + T(0.5) * (U[j][i] + U[i][j]) - T(3) * sdPphi[ij] + T(3) * Pphi[i] * Pphi[j];
                    T gg = Gam[0][ij] * Gc[0] + Gam[1][ij] * Gc[1] + Gam[2][ij] * Gc[2];
#pragma unroll
                    for (int l = 0; l < 3; ++l)
#pragma unroll
                        for (int m = 0; m < 3; ++m) gg -= Gam[l][sym(i, m)] * Gam[m][sym(l, j)];
                    Ric[ij] = s1 - s2 + gg;
                }
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
                    t = T(-2) * t -
                        T(2) * (Dup[k][sym(i, 0)] * Wl[0] + Dup[k][sym(i, 1)] * Wl[1] + Dup[k][sym(i, 2)] * Wl[2]);
                    dGt[k][i] = t + ig[sym(i, 0)] * F[0] + ig[sym(i, 1)] * F[1] + ig[sym(i, 2)] * F[2];
                }
            }
            T dG[3], Zl[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) dG[i] = cvt<T>(q1(SGHAT + i)) - Gtv[i];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                Zl[i] = T(0.5) * (g[sym(i, 0)] * dG[0] + g[sym(i, 1)] * dG[1] + g[sym(i, 2)] * dG[2]);
            T RZ[6];
            {
                T nZ[3][3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    T dGh[3];
#pragma unroll
                    for (int l = 0; l < 3; ++l) dGh[l] = cvt<T>(fd(C, 9 + l, i)) - dGt[i][l];
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
            T A[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) A[k] = cvt<T>(q1(SA + k));
            T DDa[6];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = i; j < 3; ++j)
                    DDa[sym(i, j)] = T(0.5) * cvt<T>(fd(C, 6 + j, i) + fd(C, 6 + i, j)) -
                                     (Gam[0][sym(i, j)] * A[0] + Gam[1][sym(i, j)] * A[1] + Gam[2][sym(i, j)] * A[2]);
            const T al = cvt<T>(q1(SALPHA)), Kt = cvt<T>(q1(SK)), Th = cvt<T>(q1(STHETA));
            T X[6];
#pragma unroll
            for (int s = 0; s < 6; ++s) X[s] = -DDa[s] + al * RZ[s];
            const T trX = tr6(ig, X);
            const T phi2 = cvt<T>(phid * phid);
            const T RpZ = phi2 * tr6(ig, RZ);
            const T lapal = phi2 * tr6(ig, DDa);
            T At[6];
#pragma unroll
            for (int s = 0; s < 6; ++s) At[s] = cvt<T>(q1(SAT + s));
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
            T Bm[3][3];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int i = 0; i < 3; ++i) Bm[k][i] = cvt<T>(q1(SB + 3 * k + i));
            const T trB = Bm[0][0] + Bm[1][1] + Bm[2][2];
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
                    keep(ro3[3 + ij], advkoAt[ij] + static_cast<double>(t) + phid * phid * static_cast<double>(tf));
                }
            const T kap1 = cvt<T>(p.kappa1), kap2 = cvt<T>(p.kappa2);
            CCZ4_PHASE_BARRIER();
            const SlotDeriv sK = stencils<LOP>(C, 12, be, p.advection);
            keep(ro3[9], (sK.a + static_cast<double>(-lapal + al * RpZ + al * Kt * (Kt - T(2) * Th * cc) -
                                                             T(3) * al * kap1 * (T(1) + kap2) * Th) +
                      sK.k));
            const T ee2 = cvt<T>(p.e * p.e);
            const T ZA = T(0.5) * phi2 * (dG[0] * A[0] + dG[1] * A[1] + dG[2] * A[2]);
            const SlotDeriv sTh = stencils<LOP>(C, 13, be, p.advection);
            keep(ro3[10], (sTh.a +
                                static_cast<double>(T(0.5) * al * ee2 * (RpZ + T(2.0 / 3.0) * Kt * Kt - AA) -
                                                    al * Th * Kt * cc - ZA - al * kap1 * (T(2) + kap2) * Th) +
                      sTh.k));
            // B without f d_k b^i (completed in round 4): B_k^l B_l^i and alpha^2 mu gt^ij (curl D - curl P)
            if (gdrv) {
                T cP[3][3];
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    cP[k][k] = T(0);
#pragma unroll
                    for (int j = k + 1; j < 3; ++j) {
                        const double wv = (fd(C, 3 + j, k) - fd(C, 3 + k, j)) * iphid;
                        cP[k][j] = cvt<T>(wv);
                        cP[j][k] = cvt<T>(-wv);
                    }
                }
                const T a2mu = al * al * cvt<T>(p.mu);
#pragma unroll
                for (int k = 0; k < 3; ++k)
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        BB[k][i] = Bm[k][0] * Bm[0][i] + Bm[k][1] * Bm[1][i] + Bm[k][2] * Bm[2][i];
                        T cu = T(0);
#pragma unroll
                        for (int j = 0; j < 3; ++j) cu += ig[sym(i, j)] * ((H[k][j] - G1[k][j]) - cP[k][j]);
                        curl[k][i] = a2mu * cu;
                    }
            }
            if constexpr (GHAT_IN_RICCI)  // the same metric, D, At, B, A, P / phi and Christoffel symbols
                ghat_sector<T, LOP>(C, p, be, g, ig, gd, detg, D, Gt, Gtv, At, Am, Bm, A, Pphi, trB, al, Kt, Th, Zl, GB,
                                    sdBtr, dtrA, red, sfac, ro3, rGb, pwG);
        }
        CCZ4_PHASE_BARRIER();
        if constexpr (!GHAT_IN_RICCI) {  // ---- Ghat^i, and the part of b^i it shares
            const int o1 = fresh(o);
            auto q1 = [&](int v) -> double { return pw<3>(qp, o1, C, v); };
            double gd[6], igd[6], detg;
            T g[6], ig[6];
            load_metric<T>(qp, o1, gd, igd, detg, g, ig);
            T D[3][6], At[6];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int s = 0; s < 6; ++s) D[k][s] = cvt<T>(q1(SD + 6 * k + s));
#pragma unroll
            for (int s = 0; s < 6; ++s) At[s] = cvt<T>(q1(SAT + s));
            T Dup[3][6], Gl[3][6], Gt[3][6], Gtv[3];
            raise_D(ig, D, Dup);
            christoffel(ig, D, Gl, Gt, Gtv);
            T Am[3][3];
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Am[i][j] = ig[sym(i, 0)] * At[sym(0, j)] + ig[sym(i, 1)] * At[sym(1, j)] + ig[sym(i, 2)] * At[sym(2, j)];
            T Bm[3][3], A[3], Ph[3];
            const double iphid = 1.0 / q1(SPHI);
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                A[k] = cvt<T>(q1(SA + k));
                Ph[k] = cvt<T>(q1(SP + k) * iphid);
#pragma unroll
                for (int i = 0; i < 3; ++i) Bm[k][i] = cvt<T>(q1(SB + 3 * k + i));
            }
            const T trB = Bm[0][0] + Bm[1][1] + Bm[2][2];
            const T al = cvt<T>(q1(SALPHA)), Kt = cvt<T>(q1(SK)), Th = cvt<T>(q1(STHETA));
            T dG[3], Zl[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) dG[i] = cvt<T>(q1(SGHAT + i)) - Gtv[i];
#pragma unroll
            for (int i = 0; i < 3; ++i)
                Zl[i] = T(0.5) * (g[sym(i, 0)] * dG[0] + g[sym(i, 1)] * dG[1] + g[sym(i, 2)] * dG[2]);
            ghat_sector<T, LOP>(C, p, be, g, ig, gd, detg, D, Gt, Gtv, At, Am, Bm, A, Ph, trB, al, Kt, Th, Zl, GB, sdBtr,
                                dtrA, red, sfac, ro3, rGb, pwG);
        }
        CCZ4_PHASE_BARRIER();
        {  // ---- A_k and P_k
            const int o1 = fresh(o);
            auto q1 = [&](int v) -> double { return pw<3>(qp, o1, C, v); };
            T Bm[3][3], A[3], P[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                A[k] = cvt<T>(q1(SA + k));
                P[k] = cvt<T>(q1(SP + k));
#pragma unroll
                for (int i = 0; i < 3; ++i) Bm[k][i] = cvt<T>(q1(SB + 3 * k + i));
            }
            const T trB = Bm[0][0] + Bm[1][1] + Bm[2][2];
            const T al = cvt<T>(q1(SALPHA)), Kt = cvt<T>(q1(SK)), Th = cvt<T>(q1(STHETA)), K0 = cvt<T>(q1(SK0));
            const double phid = q1(SPHI);
            const bool onelog = p.slicing == 1;
            const T ga = onelog ? T(2) / al : T(1);
            const T ga_lin = onelog ? T(2) : T(2) * al;  // 2 alpha g + alpha^2 g'
            const T theta_term = Kt - K0 - T(2) * cc * Th;
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const T dK = cvt<T>(fd(C, 12, k)), dTh = cvt<T>(fd(C, 13, k));
                T t = -al * al * ga * (dK - T(2) * cc * dTh) - al * ga * dtrA[k];
                t += Bm[k][0] * A[0] + Bm[k][1] * A[1] + Bm[k][2] * A[2];
                t += -ga_lin * theta_term * A[k];
                const SlotDeriv sA = stencils<LOP>(C, 6 + k, be, p.advection);
                keep(ro3[14 + k], sA.a + static_cast<double>(t) + sA.k);
                const T u = Bm[k][0] * P[0] + Bm[k][1] * P[1] + Bm[k][2] * P[2] + T(1.0 / 3.0) * (al * Kt - trB) * P[k];
                const T phipart =
                    T(1.0 / 3.0) * (al * dK - sdBtr[k]) + T(1.0 / 3.0) * al * dtrA[k] + T(1.0 / 3.0) * Kt * A[k];
                const SlotDeriv sP = stencils<LOP>(C, 3 + k, be, p.advection);
                keep(ro3[17 + k], sP.a + static_cast<double>(u) + phid * static_cast<double>(phipart) + sP.k);
            }
            // alpha: beta^k A_k - alpha^2 g (K - K_0 - 2 c Theta); beta^i: beta^k B_k^i (+ f b^i in round 4);
            // phi: beta^k P_k + phi (alpha K - tr B) / 3
            T bet[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) bet[k] = cvt<T>(be[k]);
            keep(pwA, static_cast<double>(bet[0] * A[0] + bet[1] * A[1] + bet[2] * A[2] -
                                          al * al * ga * (Kt - K0 - T(2) * cc * Th)));
#pragma unroll
            for (int i = 0; i < 3; ++i) bB[i] = bet[0] * Bm[0][i] + bet[1] * Bm[1][i] + bet[2] * Bm[2][i];
            keep(pwPhi, be[0] * q1(SP) + be[1] * q1(SP + 1) + be[2] * q1(SP + 2) +
                            phid * static_cast<double>((al * Kt - trB) * T(1.0 / 3.0)));
        }
    }

    {
        const int r4[14] = {SBB, SBB + 1, SBB + 2, SG, SG + 1, SG + 2, SG + 3, SG + 4, SG + 5,
                            SALPHA, SBETA, SBETA + 1, SBETA + 2, SPHI};
        double qa[20], qb[20];
        if (act) snk.load(R3_OUT, qa, qb);
        lds_issue(qp, lds, sl, r4, w, lane, hs);
        __builtin_amdgcn_s_waitcnt(0);  // the sink's loads and this wave's copies have landed
        if (act) snk.store(R3_OUT, ro3, qa, qb);
    }
    __syncthreads();  // every wave's copies have landed; the stores may still be in flight

    // ------------------------------------------------------------ round 4
    // buffers: 0..2 b; 3..8 gt; 9 alpha; 10..12 beta; 13 phi
    if (act) {
        const LdsCell C = fresh(C0);
        const int o = fresh(o0);
        auto q = [&](int v) -> double { return pw<4>(qp, o, C, v); };
        double be[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) be[k] = q(SBETA + k);
        // B_k^i and b^i
        if (gdrv) {
            const T ff = cvt<T>(p.f);
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const SlotDeriv sb = stencils<LOP>(C, i, be, p.advection);
#pragma unroll
                for (int k = 0; k < 3; ++k) {
                    T t = ff * cvt<T>(sb.d[k]);
                    t += BB[k][i];
                    t += curl[k][i];
                    keep(ro4[3 * k + i], advkoB[3 * k + i] + static_cast<double>(t));
                }
                keep(ro4[9 + i], rGb[i] + sb.a - p.eta * q(SBB + i) + sb.k);
            }
        } else {
#pragma unroll
            for (int s = 0; s < 9; ++s) keep(ro4[s], 0.0);
#pragma unroll
            for (int i = 0; i < 3; ++i) keep(ro4[9 + i], 0.0);
        }
        // gt_ij, alpha, beta^i, phi: the pointwise parts from round 3 and the KO sums; K_0: 0
#pragma unroll
        for (int s = 0; s < 6; ++s) keep(ro4[12 + s], pwG[s] + stencils(C, 3 + s).k);
        keep(ro4[18], pwA + stencils(C, 9).k);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (gdrv)
                keep(ro4[19 + i], (static_cast<double>(bB[i] + cvt<T>(p.f) * cvt<T>(q(SBB + i))) +
                                   stencils(C, 10 + i).k));
            else
                keep(ro4[19 + i], 0.0);
        }
        keep(ro4[22], pwPhi + stencils(C, 13).k);
        keep(ro4[23], 0.0);
    }
    {
        double qa[24], qb[24];
        if (act) {
            snk.load(R4_OUT, qa, qb);
            snk.store(R4_OUT, ro4, qa, qb);
        }
    }
    if (act) snk.finish();
}

}  // namespace ccz4
