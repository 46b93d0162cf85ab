// HIP kernels of the CCZ4 FD4 hot path for gfx950 (MI355X).
//
// State layout: per leaf patch, slot-major boxes of 15 x 15 x 16 doubles (see ccz4.h).
// Every kernel maps one thread to one cell (or one halo cell) so that consecutive lanes walk
// the contiguous x rows of a box.
#include <hip/hip_runtime.h>

#include <algorithm>

#include "ccz4_algebra.hpp"
#include "ccz4_kernels.hpp"
#include "ccz4_rhs_lds.hpp"
#include "ccz4_rhs_phased.hpp"

namespace ccz4 {

// ------------------------------------------------------------------ initial data
// Closed forms of the three scenarios at a point; the first-order auxiliaries are the
// analytic derivatives (A = d alpha, B = d beta, D = d gt / 2, P = d phi).
__device__ void init_point(int scen, const double *sp, double x, double y, double z, double *q)
{
    for (int v = 0; v < NV; ++v) q[v] = 0.0;
    if (scen == 0) {
        const double A = sp[0], kk = sp[1];
        const double w = kk * M_PI;
        const double Hh = 1.0 - A * sin(w * x);
        const double dH = -A * w * cos(w * x);
        const double sq = sqrt(Hh);
        const double Kxx = dH / (2.0 * sq);
        const double Hm13 = pow(Hh, -1.0 / 3.0);
        q[SG + 0] = Hh * Hm13;
        q[SG + 3] = Hm13;
        q[SG + 5] = Hm13;
        q[SALPHA] = sq;
        q[SPHI] = pow(Hh, -1.0 / 6.0);
        q[SAT + 0] = (2.0 / 3.0) * Hm13 * Kxx;
        q[SAT + 3] = -(1.0 / 3.0) * Hm13 / Hh * Kxx;
        q[SAT + 5] = q[SAT + 3];
        q[SK] = Kxx / Hh;
        q[SGHAT + 0] = (2.0 / 3.0) * Hm13 * Hm13 / Hh * dH;
        q[SA + 0] = Kxx;
        q[SD + 0] = (1.0 / 3.0) * Hm13 * dH;
        q[SD + 3] = -(1.0 / 6.0) * Hm13 / Hh * dH;
        q[SD + 5] = q[SD + 3];
        q[SP + 0] = -(1.0 / 6.0) * q[SPHI] / Hh * dH;
        return;
    }
    q[SG + 0] = q[SG + 3] = q[SG + 5] = 1.0;
    if (scen == 1) {
        const double M = sp[0];
        const double rx = x - sp[1], ry = y - sp[2], rz = z - sp[3];
        const double r = sqrt(rx * rx + ry * ry + rz * rz);
        const double psi = 1.0 + 0.5 * M / r;
        const double ipsi = 1.0 / psi;
        const double f = 0.5 * M / (r * r * r);  // -d_k psi = f x_k
        const double phi = ipsi * ipsi;
        q[SPHI] = phi;
        const double pk = 2.0 * phi * ipsi * f;  // d_k phi = -2 psi^-3 d_k psi
        q[SP + 0] = pk * rx;
        q[SP + 1] = pk * ry;
        q[SP + 2] = pk * rz;
        const int lapse = (int)sp[4];
        if (lapse == 0) {
            q[SALPHA] = phi;
            q[SA + 0] = q[SP + 0];
            q[SA + 1] = q[SP + 1];
            q[SA + 2] = q[SP + 2];
        } else {
            const double as = (2.0 - psi) * ipsi;   // (1 - M/2r)/(1 + M/2r)
            const double wgt = lapse == 1 ? 0.5 : 1.0;
            q[SALPHA] = lapse == 1 ? 0.5 * (as + 1.0) : as;
            const double ak = wgt * 2.0 * phi * f;  // d_k alpha_s = -2 psi^-2 d_k psi
            q[SA + 0] = ak * rx;
            q[SA + 1] = ak * ry;
            q[SA + 2] = ak * rz;
        }
        return;
    }
    // two Brill-Lindquist holes with Bowen-York curvature
    double psi = 1.0, dpsi[3] = {0.0, 0.0, 0.0}, Ah[6] = {0, 0, 0, 0, 0, 0};
    for (int h = 0; h < 2; ++h) {
        const double *s = sp + 7 * h;
        const double d[3] = {x - s[1], y - s[2], z - s[3]};
        const double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
        const double r = sqrt(r2);
        const double n[3] = {d[0] / r, d[1] / r, d[2] / r};
        psi += 0.5 * s[0] / r;
        for (int i = 0; i < 3; ++i) dpsi[i] -= 0.5 * s[0] * d[i] / (r2 * r);
        const double Pn = s[4] * n[0] + s[5] * n[1] + s[6] * n[2];
        const double c = 1.5 / r2;
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j)
                Ah[sym(i, j)] += c * (s[4 + i] * n[j] + s[4 + j] * n[i] - ((i == j) - n[i] * n[j]) * Pn);
    }
    const double ipsi = 1.0 / psi;
    const double phi = ipsi * ipsi;
    const double ip6 = phi * phi * phi;
    q[SPHI] = phi;
    q[SALPHA] = phi;
    for (int i = 0; i < 3; ++i) {
        q[SP + i] = -2.0 * phi * ipsi * dpsi[i];
        q[SA + i] = q[SP + i];
    }
    for (int s = 0; s < 6; ++s) q[SAT + s] = ip6 * Ah[s];
}

// det gt = 1 by rescaling, then remove the trace of At with the rescaled metric
__device__ void project_cell(double *q)
{
    const double det = q[0] * (q[3] * q[5] - q[4] * q[4]) - q[1] * (q[1] * q[5] - q[4] * q[2]) +
                       q[2] * (q[1] * q[4] - q[3] * q[2]);
    const double s = 1.0 / cbrt(det);
    double g[6];
    for (int v = 0; v < 6; ++v) g[v] = q[v] * s;
    const double c00 = g[3] * g[5] - g[4] * g[4], c01 = g[2] * g[4] - g[1] * g[5], c02 = g[1] * g[4] - g[2] * g[3];
    const double c11 = g[0] * g[5] - g[2] * g[2], c12 = g[1] * g[2] - g[0] * g[4], c22 = g[0] * g[3] - g[1] * g[1];
    const double dn = g[0] * c00 + g[1] * c01 + g[2] * c02;
    const double tr = (c00 * q[11] + c11 * q[14] + c22 * q[16] + 2.0 * (c01 * q[12] + c02 * q[13] + c12 * q[15])) / dn;
    for (int v = 0; v < 6; ++v) {
        q[v] = g[v];
        q[11 + v] -= g[v] * tr * (1.0 / 3.0);
    }
}

__global__ void k_init(double *__restrict__ Q, const PatchGeom *__restrict__ geom,
                       const uint8_t *__restrict__ bmask, int32_t npatch, int32_t scen, InitArgs a)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)npatch * 3375) return;
    const int p = (int)(t / 3375);
    const int c = (int)(t % 3375);
    const int x = c % 15, y = (c / 15) % 15, z = c / 225;
    const int inx = (x >= 3 && x < 12), iny = (y >= 3 && y < 12), inz = (z >= 3 && z < 12);
    const int nin = inx + iny + inz;
    bool active = nin == 3;
    if (nin == 2) {
        // face-slab ghost: which face?  bmask bit (2*axis + (side>0)) marks Sommerfeld faces
        const int axis = !inx ? 0 : (!iny ? 1 : 2);
        const int cc = axis == 0 ? x : (axis == 1 ? y : z);
        const int bit = 2 * axis + (cc >= 12 ? 1 : 0);
        active = (bmask[p] >> bit) & 1;
    }
    if (!active) return;
    const PatchGeom g = geom[p];
    double q[NV];
    init_point(scen, a.sp, g.org[0] + (x - 2.5) * g.dx[0], g.org[1] + (y - 2.5) * g.dx[1],
               g.org[2] + (z - 2.5) * g.dx[2], q);
    if (nin == 3) project_cell(q);
    double *Qp = Q + (int64_t)p * PS + boff(x, y, z);
    for (int v = 0; v < NV; ++v) Qp[(int64_t)v * CS] = q[v];
}

// ------------------------------------------------------------------ halo fill
// One block per face task, one thread per halo cell of the 3 x 9 x 9 slab, loop over slots.
// Axis a face: ghost layer L (1..3) sits at box coordinate 11 + L (side +1) or 3 - L (side -1);
// interior depth d (1..3) from the face at 12 - d (side +1) or 2 + d (side -1).
__device__ __forceinline__ int ghost_c(int side, int L) { return side > 0 ? 11 + L : 3 - L; }
__device__ __forceinline__ int depth_c(int side, int d) { return side > 0 ? 12 - d : 2 + d; }

// slab thread -> (layer L in 1..3, tangential t1, t2 in 0..8) with the lowest box axis fastest
__device__ __forceinline__ void slab_coords(int axis, int idx, int &L, int &t1, int &t2)
{
    if (axis == 0) {  // layer index is the contiguous x
        L = idx % 3 + 1;
        t1 = (idx / 3) % 9;   // y
        t2 = idx / 27;        // z
    } else {
        t1 = idx % 9;         // x
        t2 = (idx / 9) % 9;   // z (axis 1) or y (axis 2)
        L = idx / 81 + 1;
    }
}

__device__ __forceinline__ int slab_off(int axis, int coordA, int t1, int t2)
{
    // t1/t2 are the tangential axes in increasing order: axis0 -> (y, z); axis1 -> (x, z); axis2 -> (x, y)
    if (axis == 0) return boff(coordA, t1 + 3, t2 + 3);
    if (axis == 1) return boff(t1 + 3, coordA, t2 + 3);
    return boff(t1 + 3, t2 + 3, coordA);
}

// P_parallel row F (0..26) -> (first coarse index, weights w0, w1)
__device__ __forceinline__ void ppar(int F, int &l, double &w0, double &w1)
{
    // u = (F + 1/2)/3 - 1/2 = (2F - 2)/6 ; l = clamp(floor(u), 0, 7)
    const int num = F - 1;  // u = num / 3
    int lf = num >= 0 ? num / 3 : -1;
    l = lf < 0 ? 0 : (lf > 7 ? 7 : lf);
    const double u = (double)num / 3.0;
    w1 = u - l;
    w0 = 1.0 - w1;
}

// One block per (face task, batch of eight slots), one thread per slab cell; a copy issues all
// loads of its batch before its stores, since source and destination share the state array.
constexpr int SB8 = 8;

__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_fill(
    double *__restrict__ Q, const FaceTask *__restrict__ tasks, int32_t ntask, int32_t transfer)
{
    const int ti = blockIdx.x;
    const int idx = threadIdx.x;
    if (ti >= ntask || idx >= NFACE) return;
    // blockIdx.y picks a batch of eight slots, so that a task's slots are filled in parallel
    const int v_lo = (int)blockIdx.y * SB8, v_hi = v_lo + SB8 < NV ? v_lo + SB8 : NV;
    const FaceTask tk = tasks[ti];
    int L, t1, t2;
    slab_coords(tk.axis, idx, L, t1, t2);
    double *dst = Q + (int64_t)tk.patch * PS + slab_off(tk.axis, ghost_c(tk.side, L), t1, t2);
    const bool inject = tk.kind == FK_RESTRICT && transfer == 1;
    if (tk.kind == FK_COPY || tk.kind == FK_NEUMANN || inject) {
        // copies; with the higher-order operators the restriction is one too: coarse ghost c_{2+L}
        // takes the fine cell with the same centre, tangentially the middle of the three fine
        // cells under it, along the normal the fine interior depth 3L - 1
        const int F1 = 3 * t1 + 1, F2 = 3 * t2 + 1;
        const double *src =
            tk.kind == FK_COPY ? Q + (int64_t)tk.src[0] * PS + slab_off(tk.axis, depth_c(-tk.side, L), t1, t2)
            : inject ? Q + (int64_t)tk.src[(F2 / 9) * 3 + F1 / 9] * PS +
                           slab_off(tk.axis, depth_c(-tk.side, 3 * L - 1), F1 % 9, F2 % 9)
                     : Q + (int64_t)tk.patch * PS + slab_off(tk.axis, depth_c(tk.side, 1), t1, t2);
        {
            double r[SB8];
#pragma unroll
            for (int j = 0; j < SB8; ++j) r[j] = (v_lo + j < v_hi) ? src[(v_lo + j) * CS] : 0.0;
#pragma unroll
            for (int j = 0; j < SB8; ++j)
                if (v_lo + j < v_hi) dst[(v_lo + j) * CS] = r[j];
        }
    } else if (tk.kind == FK_RESTRICT) {
        // coarse ghost c_{2+L}; fine interior layers f3..f5 = depth 1..3 from the kid's face -side;
        // R_perp rows (1/3,1/3,1/3), (0,-2,3), (0,-5,6) over (f3,f4,f5); R_avg over 3x3 fine cells
        double wf[3];
        if (L == 1) { wf[0] = wf[1] = wf[2] = 1.0 / 3.0; }
        else if (L == 2) { wf[0] = 0.0; wf[1] = -2.0; wf[2] = 3.0; }
        else { wf[0] = 0.0; wf[1] = -5.0; wf[2] = 6.0; }
        const int k1 = (3 * t1) / 9, k2 = (3 * t2) / 9;
        const double *kid = Q + (int64_t)tk.src[k2 * 3 + k1] * PS;
        const int f1 = (3 * t1) % 9, f2 = (3 * t2) % 9;
        int off[3][9];
        for (int m = 0; m < 3; ++m)
            for (int b2 = 0; b2 < 3; ++b2)
                for (int b1 = 0; b1 < 3; ++b1)
                    off[m][b2 * 3 + b1] = slab_off(tk.axis, depth_c(-tk.side, m + 1), f1 + b1, f2 + b2);
        for (int v = v_lo; v < v_hi; ++v) {
            double acc = 0.0;
            for (int m = 0; m < 3; ++m) {
                if (wf[m] == 0.0) continue;
                double sum = 0.0;
#pragma unroll
                for (int n = 0; n < 9; ++n) sum += kid[v * CS + off[m][n]];
                acc += wf[m] * (sum * (1.0 / 9.0));
            }
            dst[v * CS] = acc;
        }
    } else if (transfer == 1) {  // FK_PROLONG, higher order
        // three-point Lagrange quadratics along every axis.  Tangentially fine cell F sits at
        // coarse coordinate u = (F + 1/2)/3 - 1/2, taken from the coarse centres l-1, l, l+1 with
        // l the nearest one kept in 1..7; along the normal fine ghost L sits s = 1/2 - (L - 1/2)/3
        // coarse cells from c2 towards the face, taken from c1, c2 and the restricted c3.
        const double *cp = Q + (int64_t)tk.src[0] * PS;
        const double sn = 0.5 - (L - 0.5) / 3.0;
        const double wn[3] = {sn * (sn - 1.0) / 2.0, 1.0 - sn * sn, sn * (sn + 1.0) / 2.0};
        const int cn[3] = {depth_c(-tk.side, 2), depth_c(-tk.side, 1), ghost_c(-tk.side, 1)};
        int j[2];
        double w[2][3];
        const int F[2] = {9 * tk.o1 + t1, 9 * tk.o2 + t2};
#pragma unroll
        for (int d = 0; d < 2; ++d) {
            const double u = (F[d] + 0.5) / 3.0 - 0.5;
            int l = (int)floor(u + 0.5);
            l = l < 1 ? 1 : (l > 7 ? 7 : l);
            const double s = u - l;
            j[d] = l;
            w[d][0] = s * (s - 1.0) / 2.0;
            w[d][1] = 1.0 - s * s;
            w[d][2] = s * (s + 1.0) / 2.0;
        }
        for (int v = v_lo; v < v_hi; ++v) {
            const double *c = cp + v * CS;
            double acc = 0.0;
#pragma unroll
            for (int kn = 0; kn < 3; ++kn)
#pragma unroll
                for (int k2 = 0; k2 < 3; ++k2)
#pragma unroll
                    for (int k1 = 0; k1 < 3; ++k1)
                        acc += wn[kn] * w[1][k2] * w[0][k1] * c[slab_off(tk.axis, cn[kn], j[0] - 1 + k1, j[1] - 1 + k2)];
            dst[v * CS] = acc;
        }
    } else {  // FK_PROLONG
        // fine ghost L -> f_{3-L}; P_perp rows over coarse (c0..c5): f0 = c1/3 + 2c2/3, f1 = c2,
        // f2 = 2c2/3 + c3/3; c0..c2 coarse interior depth 3..1 from the coarse face -side, c3..c5
        // its ghosts 1..3
        const double *cp = Q + (int64_t)tk.src[0] * PS;
        int cA[2];
        double wA[2];
        if (L == 3) { cA[0] = depth_c(-tk.side, 2); wA[0] = 1.0 / 3.0; cA[1] = depth_c(-tk.side, 1); wA[1] = 2.0 / 3.0; }
        else if (L == 2) { cA[0] = depth_c(-tk.side, 1); wA[0] = 1.0; cA[1] = cA[0]; wA[1] = 0.0; }
        else { cA[0] = depth_c(-tk.side, 1); wA[0] = 2.0 / 3.0; cA[1] = ghost_c(-tk.side, 1); wA[1] = 1.0 / 3.0; }
        int l1, l2;
        double a0, a1, b0, b1;
        ppar(9 * tk.o1 + t1, l1, a0, a1);
        ppar(9 * tk.o2 + t2, l2, b0, b1);
        int off[2][4];
        for (int m = 0; m < 2; ++m) {
            off[m][0] = slab_off(tk.axis, cA[m], l1, l2);
            off[m][1] = slab_off(tk.axis, cA[m], l1 + 1, l2);
            off[m][2] = slab_off(tk.axis, cA[m], l1, l2 + 1);
            off[m][3] = slab_off(tk.axis, cA[m], l1 + 1, l2 + 1);
        }
        for (int v = v_lo; v < v_hi; ++v) {
            const double *c = cp + v * CS;
            double acc = 0.0;
            for (int m = 0; m < 2; ++m) {
                if (wA[m] == 0.0) continue;
                const double r0 = a0 * c[off[m][0]] + a1 * c[off[m][1]];
                const double r1 = a0 * c[off[m][2]] + a1 * c[off[m][3]];
                acc += wA[m] * (b0 * r0 + b1 * r1);
            }
            dst[v * CS] = acc;
        }
    }
}

// ------------------------------------------------------------------ right-hand side
__device__ __forceinline__ bool frozen_slot(int v)
{
    return (v >= SBETA && v < SBETA + 3) || (v >= SBB && v < SBB + 3) || (v >= SB && v < SB + 9);
}

// Work-group -> (patch, z-slab of 3 planes) with the three slabs of a patch on one XCD:
// consecutive block ids are dealt to the 8 XCDs in turn, so logical block L runs at physical
// id (L % per) * 8 + L / per with per = grid / 8 (the grid is padded to a multiple of 8).
__device__ __forceinline__ int64_t xcd_logical_block(int64_t b, int64_t nblk)
{
    const int64_t per = nblk / 8;
    return (b % 8) * per + b / 8;
}

#ifndef CCZ4_RHS_WPE
#define CCZ4_RHS_WPE 1
#endif

template <typename T, int LOP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CCZ4_RHS_WPE))) void k_rhs(const double *__restrict__ Q, double *__restrict__ K,
                                             const PatchGeom *__restrict__ geom, int32_t npatch,
                                             RhsParams prm, int32_t linear, const int32_t *__restrict__ order)
{
    const int64_t lb = linear ? (int64_t)blockIdx.x : xcd_logical_block(blockIdx.x, gridDim.x);
    if (lb / 3 >= npatch || threadIdx.x >= 243) return;
    const int p = order[lb / 3];
    const int c = (int)(lb % 3) * 243 + threadIdx.x;
    const PatchGeom g = geom[p];
    CellRef cr;
    cr.qb = Q + (int64_t)p * PS;
    cr.kb = K + (int64_t)p * PS;
    cr.o = boff(c % 9 + 3, (c / 9) % 9 + 3, c / 81 + 3);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cr.i12[a] = 1.0 / (12.0 * g.dx[a]);
        cr.koc[a] = prm.ko_eps / (64.0 * g.dx[a]);
    }
    cr.adv = prm.advection;
    RhsSink<LOP> snk;
    snk.so = prm.formulation;
    rhs_cell_phased<T>(cr, prm, snk);
}

// Fused stage: the right-hand side of Qs folded slot by slot into stage s of RK4 (two-register
// form) on the interior cells, with the projection of Q^{n+1} at s = 3.  Qs is read through the
// stencils, Qn and acc pointwise; Qnext must differ from Qs (other cells still read Qs).
template <int L>
struct StageSink {
    static constexpr int LOP = L;  // lopsided advection stencils in the phase functions
    const double *__restrict__ qn;
    double *__restrict__ acc;
    double *__restrict__ qx;
    int s;
    int so;  // second-order formulation: the auxiliaries are left alone (reconstructed afterwards)
    double dt;
    double carry[12];  // s = 3: gt_ij and At_ij of Q^{n+1}, projected in finish()
    int oc;            // the cell's index in a slot of the accumulator (acc_cell)
    int64_t pd[3];     // offsets (doubles, from this cell) of its copies in same-level neighbours'
                       // face halos of Q_next along each axis, 0 for none

    // Q_next at element e, and its copies in the neighbours' halos
    // The copies into the y and z face halos (made only when a step ends) are streamed past the
    // caches: no stage reads them (the next stage gathers those halos from the neighbours'
    // interiors) and their rows are partial lines that nothing else writes, so cached they only
    // wait in L2 as dirty lines for the next launch to evict (2-3 ms per step on 24^3 patches).
    // The x-face copies stay cached: they complete lines of the neighbour's own rows in L2.
    __device__ __forceinline__ void out(int64_t e, double val)
    {
        qx[e] = val;
        if (pd[0] != 0) qx[e + pd[0]] = val;
#pragma unroll
        for (int a = 1; a < 3; ++a)
            if (pd[a] != 0) __builtin_nontemporal_store(val, qx + e + pd[a]);
    }

    __device__ __forceinline__ void combine_at(int o, int v, double r)
    {
        if (so && aux_slot(v)) return;
        const int e = v * CS + o;
        if (s == 0) {
            const double q0 = qn[e];
            acc[v * CS + oc] = q0 + (1.0 / 6.0) * dt * r;
            out(e, q0 + 0.5 * dt * r);
        } else if (s < 3) {
            acc[v * CS + oc] = acc[v * CS + oc] + (1.0 / 3.0) * dt * r;
            out(e, qn[e] + (s == 1 ? 0.5 : 1.0) * dt * r);
        } else {
            const double val = acc[v * CS + oc] + (1.0 / 6.0) * dt * r;
            if (v < 6) carry[v] = val;
            else if (v >= SAT && v < SAT + 6) carry[v - SAT + 6] = val;
            else out(e, val);
        }
    }
    __device__ __forceinline__ void put(const CellRef &c, int v, double alg) { combine_at(c.o, v, alg + ko(c, v)); }
    __device__ __forceinline__ void zero(const CellRef &c, int v) { combine_at(c.o, v, 0.0); }
    __device__ __forceinline__ void finish(const CellRef &c) { finish_at(c.o); }
    __device__ __forceinline__ void finish_at(int o)
    {
        if (s != 3) return;
        double q[SAT + 6];
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            q[v] = carry[v];
            q[SAT + v] = carry[6 + v];
        }
        project_cell(q);
#pragma unroll
        for (int v = 0; v < 6; ++v) {
            out(v * CS + o, q[v]);
            out((SAT + v) * CS + o, q[SAT + v]);
        }
    }
};

// Offsets (in doubles, relative to the cell's own element) of the copies of interior cell
// (x, y, z) of patch p in the face halos of its same-level neighbours: a cell within three layers
// of a face whose neighbour nbr[6p + 2a + (side > 0)] is a leaf of the same level appears in that
// neighbour's ghost layer at box coordinate c_a - 9 (side +1) or c_a + 9 (side -1).  0: no copy.
__device__ __forceinline__ void push_offsets(const int32_t *__restrict__ nbr, int p, int x, int y, int z, int o,
                                             int64_t pd[3], int axes = 7)
{
    const int c[3] = {x, y, z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        pd[a] = 0;
        if (!nbr || !((axes >> a) & 1)) continue;
        const int side = c[a] >= 9 ? 1 : (c[a] <= 5 ? -1 : 0);
        if (side == 0) continue;
        const int np = nbr[p * 6 + 2 * a + (side > 0 ? 1 : 0)];
        if (np < 0) continue;
        int m[3] = {x, y, z};
        m[a] = side > 0 ? c[a] - 9 : c[a] + 9;
        pd[a] = (int64_t)(np - p) * PS + (boff(m[0], m[1], m[2]) - o);
    }
}

// Fused stage on the Sommerfeld ghosts of boundary face fi: G_L of Qs combined at once into
// stage s (one thread per ghost cell, all slots).
__device__ __forceinline__ void stage_ghost_face(int fi, int idx, int32_t s, double dt, const double *__restrict__ Qs,
                                                 const double *__restrict__ Qn, double *__restrict__ acc,
                                                 double *__restrict__ Qx, const PatchGeom *__restrict__ geom,
                                                 const BoundaryFace *__restrict__ bf, const double *__restrict__ bg,
                                                 int32_t frozen)
{
    if (idx >= NFACE) return;
    const BoundaryFace f = bf[fi];
    int L, t1, t2;
    slab_coords(f.axis, idx, L, t1, t2);
    const int cg = ghost_c(f.side, L);
    const int og = slab_off(f.axis, cg, t1, t2);
    const int ci = L == 1 ? depth_c(f.side, 1) : ghost_c(f.side, L - 1);
    const int oi = slab_off(f.axis, ci, t1, t2);
    const PatchGeom g = geom[f.patch];
    int cx, cy, cz;
    if (f.axis == 0) { cx = cg; cy = t1 + 3; cz = t2 + 3; }
    else if (f.axis == 1) { cx = t1 + 3; cy = cg; cz = t2 + 3; }
    else { cx = t1 + 3; cy = t2 + 3; cz = cg; }
    const double X = g.org[0] + (cx - 2.5) * g.dx[0];
    const double Y = g.org[1] + (cy - 2.5) * g.dx[1];
    const double Z = g.org[2] + (cz - 2.5) * g.dx[2];
    const double rr = sqrt(X * X + Y * Y + Z * Z);
    const double xn = f.axis == 0 ? X : (f.axis == 1 ? Y : Z);
    const double cadv = rr / (fabs(xn) * g.dx[f.axis]), cdmp = 1.0 / rr;
    const int64_t base = (int64_t)f.patch * PS;
    const double *B = bg + (int64_t)f.bg * NV * NFACE + idx;
    const int oa = acc_ghost(f.axis, f.side, idx);
    // the slots in batches of eight, every load of a batch issued before its arithmetic and stores
    // (this work-group holds a whole CU's LDS while it runs, so it must not wait slot by slot)
    for (int v0 = 0; v0 < NV; v0 += SB8) {
        double qL[SB8], qI[SB8], qB[SB8], q0[SB8], a0[SB8];
#pragma unroll
        for (int j = 0; j < SB8; ++j) {
            const int v = v0 + j;
            if (v >= NV) break;
            qL[j] = Qs[base + v * CS + og];
            qI[j] = Qs[base + v * CS + oi];
            qB[j] = B[v * NFACE];
            q0[j] = s < 3 ? Qn[base + v * CS + og] : 0.0;
            a0[j] = s > 0 ? acc[base + v * CS + oa] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < SB8; ++j) {
            const int v = v0 + j;
            if (v >= NV) break;
            const double r = (v != SK0 && !(frozen && frozen_slot(v)))
                                 ? -cadv * (qL[j] - qI[j]) - cdmp * (qL[j] - qB[j]) : 0.0;
            const int64_t e = base + v * CS + og;
            const int64_t ea = base + v * CS + oa;
            if (s == 0) {
                acc[ea] = q0[j] + (1.0 / 6.0) * dt * r;
                Qx[e] = q0[j] + 0.5 * dt * r;
            } else if (s < 3) {
                acc[ea] = a0[j] + (1.0 / 3.0) * dt * r;
                Qx[e] = q0[j] + (s == 1 ? 0.5 : 1.0) * dt * r;
            } else {
                Qx[e] = a0[j] + (1.0 / 6.0) * dt * r;
            }
        }
    }
}


// The Sommerfeld ghost cells beside z-slab sl of patch p, handled by that slab's work-group after
// its interior: of each boundary face of the patch, the ghost cells next to the slab's three planes
// (81 for an x or y face; the whole face slab of 243 for the z face below slab 0 or above slab 2).
// Those rows were just fetched and written by the same work-group, so the ghost update finds them
// in the L2 instead of touching a line of HBM for every 3 ghost cells of an x face.  cell(fi, idx)
// is called once for every such ghost cell (face fi of the boundary-face list, index idx in its slab).
template <typename Cell>
__device__ __forceinline__ void ghost_slab_cells(int p, int sl, const int32_t *__restrict__ pface, Cell &&cell)
{
#pragma unroll
    for (int f = 0; f < 6; ++f) {
        const int fi = pface[p * 6 + f];
        const int axis = f >> 1;
        const int n = fi < 0 ? 0 : (axis < 2 ? 81 : ((f & 1) ? (sl == 2 ? NFACE : 0) : (sl == 0 ? NFACE : 0)));
        for (int r = (int)threadIdx.x; r < n; r += (int)blockDim.x) {
            // slab_coords order: x face idx = (L - 1) + 3 y + 27 z; y face idx = x + 9 z + 81 (L - 1)
            const int idx = axis == 0 ? 81 * sl + r : (axis == 1 ? 81 * (r / 27) + 27 * sl + r % 27 : r);
            cell(fi, idx);
        }
    }
}

// Right-hand side G_L of all slots at ghost cell idx of boundary face fi (what k_rhs_sommerfeld
// computes one thread per slot), the slots in batches of eight with every load of a batch first.
__device__ __forceinline__ void rhs_ghost_cell(int fi, int idx, const double *__restrict__ Q, double *__restrict__ K,
                                               const PatchGeom *__restrict__ geom,
                                               const BoundaryFace *__restrict__ bf, const double *__restrict__ bg,
                                               int32_t frozen)
{
    if (idx >= NFACE) return;
    const BoundaryFace f = bf[fi];
    int L, t1, t2;
    slab_coords(f.axis, idx, L, t1, t2);
    const int cg = ghost_c(f.side, L);
    const int og = slab_off(f.axis, cg, t1, t2);
    const int ci = L == 1 ? depth_c(f.side, 1) : ghost_c(f.side, L - 1);
    const int oi = slab_off(f.axis, ci, t1, t2);
    const PatchGeom g = geom[f.patch];
    int cx, cy, cz;
    if (f.axis == 0) { cx = cg; cy = t1 + 3; cz = t2 + 3; }
    else if (f.axis == 1) { cx = t1 + 3; cy = cg; cz = t2 + 3; }
    else { cx = t1 + 3; cy = t2 + 3; cz = cg; }
    const double X = g.org[0] + (cx - 2.5) * g.dx[0];
    const double Y = g.org[1] + (cy - 2.5) * g.dx[1];
    const double Z = g.org[2] + (cz - 2.5) * g.dx[2];
    const double rr = sqrt(X * X + Y * Y + Z * Z);
    const double xn = f.axis == 0 ? X : (f.axis == 1 ? Y : Z);
    const double *Qp = Q + (int64_t)f.patch * PS;
    double *Kp = K + (int64_t)f.patch * PS;
    const double *B = bg + (int64_t)f.bg * NV * NFACE + idx;
    for (int v0 = 0; v0 < NV; v0 += SB8) {
        double qL[SB8], qI[SB8], qB[SB8];
#pragma unroll
        for (int j = 0; j < SB8; ++j) {
            const int v = v0 + j;
            if (v >= NV) break;
            qL[j] = Qp[v * CS + og];
            qI[j] = Qp[v * CS + oi];
            qB[j] = B[v * NFACE];
        }
#pragma unroll
        for (int j = 0; j < SB8; ++j) {
            const int v = v0 + j;
            if (v >= NV) break;
            Kp[v * CS + og] = (v == SK0 || (frozen && frozen_slot(v)))
                                  ? 0.0
                                  : -(rr / (fabs(xn) * g.dx[f.axis])) * (qL[j] - qI[j]) - (1.0 / rr) * (qL[j] - qB[j]);
        }
    }
}

template <typename T, int LOP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(CCZ4_RHS_WPE))) void k_stage(
    const double *__restrict__ Qs, const double *__restrict__ Qn, double *__restrict__ acc, double *__restrict__ Qx,
    const PatchGeom *__restrict__ geom, int32_t npatch, int32_t nb_slab, RhsParams prm, int32_t s, double dt,
    const BoundaryFace *__restrict__ bf, const double *__restrict__ bg, const int32_t *__restrict__ nbr,
    int32_t paxes, int32_t linear, const int32_t *__restrict__ order)
{
    if ((int32_t)blockIdx.x >= nb_slab) {
        stage_ghost_face((int)blockIdx.x - nb_slab, threadIdx.x, s, dt, Qs, Qn, acc, Qx, geom, bf, bg, prm.shift == 0);
        return;
    }
    const int64_t lb = linear ? (int64_t)blockIdx.x : xcd_logical_block(blockIdx.x, nb_slab);
    if (lb / 3 >= npatch || threadIdx.x >= 243) return;
    const int p = order[lb / 3];
    const int c = (int)(lb % 3) * 243 + threadIdx.x;
    const PatchGeom g = geom[p];
    CellRef cr;
    cr.qb = Qs + (int64_t)p * PS;
    cr.kb = nullptr;
    cr.o = boff(c % 9 + 3, (c / 9) % 9 + 3, c / 81 + 3);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        cr.i12[a] = 1.0 / (12.0 * g.dx[a]);
        cr.koc[a] = prm.ko_eps / (64.0 * g.dx[a]);
    }
    cr.adv = prm.advection;
    StageSink<LOP> snk;
    snk.qn = Qn + (int64_t)p * PS;
    snk.acc = acc + (int64_t)p * PS;
    snk.qx = Qx + (int64_t)p * PS;
    snk.s = s;
    snk.so = prm.formulation;
    snk.dt = dt;
    snk.oc = acc_cell((int)(lb % 3), (int)threadIdx.x);
    push_offsets(nbr, p, c % 9 + 3, (c / 9) % 9 + 3, c / 81 + 3, cr.o, snk.pd, paxes);
    rhs_cell_phased<T>(cr, prm, snk);
}

// LDS-staged variants: one work-group per (patch, z-slab), every lane takes part in staging;
// the 151 KB of LDS leave one work-group per CU, so the waves may use the whole register file.
__device__ __forceinline__ void lds_cell_setup(double *lds, int sl, const PatchGeom &g, const RhsParams &prm,
                                               LdsCell &C, int &o, bool &act)
{
    const int tid = threadIdx.x;
    act = tid < 243;
    const int cc = act ? tid : 242;
    const int x = cc % 9 + 3, y = (cc / 9) % 9 + 3, zl = cc / 81;
    C.s = lds;
    lds_cell_offsets(C, x, y, zl);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C.i12[a] = 1.0 / (12.0 * g.dx[a]);
        C.koc[a] = prm.ko_eps / (64.0 * g.dx[a]);
    }
    o = boff(x, y, zl + 3 + 3 * sl);
}

template <typename T, int LOP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_rhs_lds(
    const double *__restrict__ Q, double *__restrict__ K, const PatchGeom *__restrict__ geom, int32_t npatch,
    RhsParams prm, const BoundaryFace *__restrict__ bf, const double *__restrict__ bg,
    const int32_t *__restrict__ pface, int32_t linear, const int32_t *__restrict__ order)
{
    __shared__ double lds[LDS_DOUBLES];
    const int64_t lb = linear ? (int64_t)blockIdx.x : xcd_logical_block(blockIdx.x, gridDim.x);
    if (lb / 3 >= npatch) return;  // uniform over the work-group
    const int p = order[lb / 3];
    const int sl = (int)(lb % 3);
    const PatchGeom g = geom[p];
    LdsCell C;
    int o;
    bool act;
    lds_cell_setup(lds, sl, g, prm, C, o, act);
    LdsRhsSink snk;
    snk.kb = K + (int64_t)p * PS;
    snk.o = o;
    snk.so = prm.formulation;
    const HaloSrc hs{{0, 0, 0, 0}};
    rhs_slab_lds<T, LOP>(Q + (int64_t)p * PS, lds, sl, act, o, C, prm, snk, hs);
    if (pface) {
        const int32_t frozen = prm.shift == 0;
        ghost_slab_cells(p, sl, pface, [&](int fi, int idx) { rhs_ghost_cell(fi, idx, Q, K, geom, bf, bg, frozen); });
    }
}

struct LdsStageSink {
    StageSink<0> *st;
    int o;
    __device__ __forceinline__ void put(int v, double r) { st->combine_at(o, v, r); }
    __device__ __forceinline__ void finish() { st->finish_at(o); }
    // A round's outputs in two halves: every load of Q^n and acc first, so that they are in
    // flight together (the compiler cannot move them past the stores itself, not knowing that
    // acc, Q^n and Q_next do not overlap), then the combines and stores.  The acc stream, and
    // Q^n at s > 0, are touched once per launch, so they go through the caches as nontemporal:
    // the lines the slab staging shares between work-groups stay in L2 longer (2-3% per stage).
    // At s = 0, Q^n is Q_s and its loads hit the lines just staged, which must stay.  Q_next
    // keeps ordinary stores: its rows are partial lines that merge in L2 with the copies the
    // neighbours push into the same lines.
    template <int N>
    __device__ __forceinline__ void load(const int (&slots)[N], double (&a)[N], double (&b)[N])
    {
        const int s = st->s;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            if (st->so && aux_slot(slots[j])) continue;
            const int e = slots[j] * CS + o;
            a[j] = s == 0 ? st->qn[e] : (s < 3 ? __builtin_nontemporal_load(st->qn + e) : 0.0);
            b[j] = s > 0 ? __builtin_nontemporal_load(st->acc + slots[j] * CS + st->oc) : 0.0;
        }
    }
    template <int N>
    __device__ __forceinline__ void store(const int (&slots)[N], const double (&r)[N], const double (&a)[N],
                                          const double (&b)[N])
    {
        const int s = st->s;
        const double dt = st->dt;
#pragma unroll
        for (int j = 0; j < N; ++j) {
            const int v = slots[j];
            if (st->so && aux_slot(v)) continue;
            const int e = v * CS + o;
            if (s == 0) {
                __builtin_nontemporal_store(a[j] + (1.0 / 6.0) * dt * r[j], st->acc + v * CS + st->oc);
                st->out(e, a[j] + 0.5 * dt * r[j]);
            } else if (s < 3) {
                __builtin_nontemporal_store(b[j] + (1.0 / 3.0) * dt * r[j], st->acc + v * CS + st->oc);
                st->out(e, a[j] + (s == 1 ? 0.5 : 1.0) * dt * r[j]);
            } else {
                const double val = b[j] + (1.0 / 6.0) * dt * r[j];
                if (v < 6) st->carry[v] = val;
                else if (v >= SAT && v < SAT + 6) st->carry[v - SAT + 6] = val;
                else st->out(e, val);
            }
        }
    }
};

template <typename T, int LOP>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_stage_lds(
    const double *__restrict__ Qs, const double *__restrict__ Qn, double *__restrict__ acc, double *__restrict__ Qx,
    const PatchGeom *__restrict__ geom, int32_t npatch, int32_t nb_slab, RhsParams prm, int32_t s, double dt,
    const BoundaryFace *__restrict__ bf, const double *__restrict__ bg, const int32_t *__restrict__ pface,
    const int32_t *__restrict__ nbr, int32_t paxes, const int32_t *__restrict__ gnbr, int32_t linear,
    const int32_t *__restrict__ order)
{
    __shared__ double lds[LDS_DOUBLES];
    const int64_t lb = linear ? (int64_t)blockIdx.x : xcd_logical_block(blockIdx.x, nb_slab);
    if (lb / 3 >= npatch) return;  // uniform over the work-group
    const int p = order[lb / 3];
    const int sl = (int)(lb % 3);
    const PatchGeom g = geom[p];
    LdsCell C;
    int o;
    bool act;
    lds_cell_setup(lds, sl, g, prm, C, o, act);
    StageSink<0> ss;
    ss.qn = Qn + (int64_t)p * PS;
    ss.acc = acc + (int64_t)p * PS;
    ss.qx = Qx + (int64_t)p * PS;
    ss.s = s;
    ss.so = prm.formulation;
    ss.dt = dt;
    ss.oc = acc_cell(sl, act ? (int)threadIdx.x : 242);
    {
        const int cc = act ? (int)threadIdx.x : 242;
        push_offsets(nbr, p, cc % 9 + 3, (cc / 9) % 9 + 3, cc / 81 + 3 + 3 * sl, o, ss.pd, paxes);
    }
    LdsStageSink snk{&ss, o};
    HaloSrc hs;
#pragma unroll
    for (int f = 0; f < 4; ++f) {  // faces y-, y+, z-, z+
        const int n = gnbr ? gnbr[p * 6 + 2 + f] : -1;
        hs.d[f] = n >= 0 ? (int64_t)(n - p) * PS + ((f & 1) ? -9 : 9) * (f < 2 ? YS : ZS) : 0;
    }
    rhs_slab_lds<T, LOP>(Qs + (int64_t)p * PS, lds, sl, act, o, C, prm, snk, hs);
    if (pface) {
        const int32_t frozen = prm.shift == 0;
        ghost_slab_cells(p, sl, pface, [&](int fi, int idx) {
            stage_ghost_face(fi, idx, s, dt, Qs, Qn, acc, Qx, geom, bf, bg, frozen);
        });
    }
}

// Sommerfeld ghosts: one thread per (boundary face, slot, ghost cell)
__global__ __launch_bounds__(256) void k_rhs_sommerfeld(const double *__restrict__ Q, double *__restrict__ K,
                                                        const PatchGeom *__restrict__ geom,
                                                        const BoundaryFace *__restrict__ bf,
                                                        const double *__restrict__ bg, int32_t nbf, int32_t frozen)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nbf * NV * NFACE) return;
    const int fi = (int)(t / (NV * NFACE));
    const int r = (int)(t % (NV * NFACE));
    const int v = r / NFACE;
    const int idx = r % NFACE;
    const BoundaryFace f = bf[fi];
    int L, t1, t2;
    slab_coords(f.axis, idx, L, t1, t2);
    const int cg = ghost_c(f.side, L);
    const int og = slab_off(f.axis, cg, t1, t2);
    double *Kp = K + (int64_t)f.patch * PS + v * CS + og;
    if (v == SK0 || (frozen && frozen_slot(v))) {
        *Kp = 0.0;
        return;
    }
    const int ci = L == 1 ? depth_c(f.side, 1) : ghost_c(f.side, L - 1);
    const int oi = slab_off(f.axis, ci, t1, t2);
    const PatchGeom g = geom[f.patch];
    int cx, cy, cz;
    if (f.axis == 0) { cx = cg; cy = t1 + 3; cz = t2 + 3; }
    else if (f.axis == 1) { cx = t1 + 3; cy = cg; cz = t2 + 3; }
    else { cx = t1 + 3; cy = t2 + 3; cz = cg; }
    const double X = g.org[0] + (cx - 2.5) * g.dx[0];
    const double Y = g.org[1] + (cy - 2.5) * g.dx[1];
    const double Z = g.org[2] + (cz - 2.5) * g.dx[2];
    const double rr = sqrt(X * X + Y * Y + Z * Z);
    const double xn = f.axis == 0 ? X : (f.axis == 1 ? Y : Z);
    const double *Qp = Q + (int64_t)f.patch * PS + v * CS;
    const double qL = Qp[og];
    *Kp = -(rr / (fabs(xn) * g.dx[f.axis])) * (qL - Qp[oi]) - (1.0 / rr) * (qL - bg[(int64_t)f.bg * NV * NFACE + v * NFACE + idx]);
}

__global__ void k_capture_bg(const double *__restrict__ Q, const BoundaryFace *__restrict__ bf,
                             double *__restrict__ bg, int32_t nbf)
{
    const int fi = blockIdx.x;
    if (fi >= nbf) return;
    const int idx = threadIdx.x;
    if (idx >= NFACE) return;
    const BoundaryFace f = bf[fi];
    int L, t1, t2;
    slab_coords(f.axis, idx, L, t1, t2);
    const int og = slab_off(f.axis, ghost_c(f.side, L), t1, t2);
    const double *Qp = Q + (int64_t)f.patch * PS;
    for (int v = 0; v < NV; ++v) bg[(int64_t)f.bg * NV * NFACE + v * NFACE + idx] = Qp[v * CS + og];
}

// ------------------------------------------------------------------ RK4 stage
// classical RK4 in two-register form: weights of acc (b) and of the stage state (a)
__device__ __forceinline__ void rk_one(int s, double dt, const double *__restrict__ qn, const double *__restrict__ kk,
                                       double *__restrict__ acc, double *__restrict__ qx, int64_t e)
{
    const double kv = kk[e];
    if (s == 0) {
        const double q0 = qn[e];
        acc[e] = q0 + (1.0 / 6.0) * dt * kv;
        qx[e] = q0 + 0.5 * dt * kv;
    } else if (s == 1) {
        acc[e] = acc[e] + (1.0 / 3.0) * dt * kv;
        qx[e] = qn[e] + 0.5 * dt * kv;
    } else if (s == 2) {
        acc[e] = acc[e] + (1.0 / 3.0) * dt * kv;
        qx[e] = qn[e] + dt * kv;
    } else {
        qx[e] = acc[e] + (1.0 / 6.0) * dt * kv;
    }
}

// one thread per interior cell; slots in batches of eight; at s = 3 the cell is projected
__global__ __launch_bounds__(256) void k_rk4(int32_t s, double dt, const double *__restrict__ Qn,
                                             const double *__restrict__ Kk, double *__restrict__ acc,
                                             double *__restrict__ Qx, int32_t npatch)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)npatch * NCELL) return;
    const int p = (int)(t / NCELL);
    const int c = (int)(t % NCELL);
    const int64_t base = (int64_t)p * PS + boff(c % 9 + 3, (c / 9) % 9 + 3, c / 81 + 3);
    if (s < 3) {
        for (int v0 = 0; v0 < NV; v0 += SB8) {
#pragma unroll
            for (int j = 0; j < SB8; ++j)
                if (v0 + j < NV) rk_one(s, dt, Qn, Kk, acc, Qx, base + (int64_t)(v0 + j) * CS);
        }
        return;
    }
    double q[NV];
    for (int v0 = 0; v0 < NV; v0 += SB8) {
#pragma unroll
        for (int j = 0; j < SB8; ++j)
            if (v0 + j < NV) {
                const int64_t e = base + (int64_t)(v0 + j) * CS;
                q[v0 + j] = acc[e] + (1.0 / 6.0) * dt * Kk[e];
            }
    }
    project_cell(q);
    for (int v = 0; v < NV; ++v) Qx[base + (int64_t)v * CS] = q[v];
}

// Sommerfeld ghosts: one thread per (boundary face, slot, ghost cell); no projection
__global__ __launch_bounds__(256) void k_rk4_ghost(int32_t s, double dt, const double *__restrict__ Qn,
                                                   const double *__restrict__ Kk, double *__restrict__ acc,
                                                   double *__restrict__ Qx, const BoundaryFace *__restrict__ bf,
                                                   int32_t nbf)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)nbf * NV * NFACE) return;
    const int fi = (int)(t / (NV * NFACE));
    const int r = (int)(t % (NV * NFACE));
    const int v = r / NFACE;
    const int idx = r % NFACE;
    const BoundaryFace f = bf[fi];
    int L, t1, t2;
    slab_coords(f.axis, idx, L, t1, t2);
    const int64_t e = (int64_t)f.patch * PS + v * CS + slab_off(f.axis, ghost_c(f.side, L), t1, t2);
    rk_one(s, dt, Qn, Kk, acc, Qx, e);
}

// ------------------------------------------------------------------ constraints
// H = R + 2/3 K^2 - At_ij At^ij with R = phi^2 gt^ij R_ij;
// M_i = gt^kl (d_k At_li - Gt^m_li At_km - Gt^m_lk At_im - 3 At_ik P_l/phi) - 2/3 d_i K.
// Only the first derivatives of D (Ricci tensor from the relations), P (Ricci tensor), At and K
// (momentum constraint) enter: 28 slots.  One work-group per z-slab of a leaf stages them into LDS
// in two rounds of 14 (the stage kernel's slab staging, own halos), forms each cell's FD4
// differences from LDS, and takes the pointwise values of the staged slots from LDS too; the
// other slots are read from the state, their loads in flight with the second round's copies.  Per-block partial sums (H^2, |M|^2, counted cells,
// non-finite cells) in a fixed order for k_reduce_parts.
constexpr int CONS_NB = 14;
__global__ __launch_bounds__(256) void k_constraints_lds(const double *__restrict__ Q, double *__restrict__ HM,
                                                         const PatchGeom *__restrict__ geom, int32_t npatch,
                                                         double r_excise, double *__restrict__ part)
{
    __shared__ double lds[CONS_NB * LDS_SLOT];
    __shared__ double red[4][256];
    const int64_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int p = (int)(lb / 3);
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    double h2 = 0.0, m2 = 0.0, cnt = 0.0, bad = 0.0;
    if (p < npatch) {  // uniform over the work-group
        const int sl = (int)(lb % 3);
        const PatchGeom g = geom[p];
        const bool act = tid < 243;
        const int cc = act ? tid : 242;
        const int x = cc % 9 + 3, y = (cc / 9) % 9 + 3, zl = cc / 81;
        LdsCell C;
        C.s = lds;
        lds_cell_offsets(C, x, y, zl);
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            C.i12[a] = 1.0 / (12.0 * g.dx[a]);
            C.koc[a] = 0.0;
        }
        const HaloSrc hs{{0, 0, 0, 0}};
        const double *qb = Q + (int64_t)p * PS;
        const int z = zl + 3 + 3 * sl;
        const int o = boff(x, y, z);
        double q[NV], dq[3][NDIFF];
        const int ra[CONS_NB] = {SD, SD + 1, SD + 2, SD + 3, SD + 4, SD + 5, SD + 6, SD + 7,
                                 SD + 8, SD + 9, SD + 10, SD + 11, SD + 12, SD + 13};
        lds_round(qb, lds, sl, ra, w, lane, hs);
        if (act)
#pragma unroll
            for (int j = 0; j < CONS_NB; ++j) {
                q[ra[j]] = lv(C, j, 0, 0);
#pragma unroll
                for (int a = 0; a < 3; ++a) dq[a][ra[j] - DOFF] = fd(C, j, a);
            }
        const int rb[CONS_NB] = {SD + 14, SD + 15, SD + 16, SD + 17, SP, SP + 1, SP + 2,
                                 SAT, SAT + 1, SAT + 2, SAT + 3, SAT + 4, SAT + 5, SK};
        lds_issue(qb, lds, sl, rb, w, lane, hs);
        // the remaining slots pointwise (every slot takes part in the finiteness count), in
        // flight together with the second round's copies; an idle lane reads cell 242's values
#pragma unroll
        for (int v = 0; v < SAT; ++v) q[v] = qb[v * CS + o];
#pragma unroll
        for (int v = STHETA; v < SD; ++v) q[v] = qb[v * CS + o];
        q[SK0] = qb[SK0 * CS + o];
        lds_wait();
        if (act) {
#pragma unroll
            for (int j = 0; j < CONS_NB; ++j) {
                q[rb[j]] = lv(C, j, 0, 0);
#pragma unroll
                for (int a = 0; a < 3; ++a) dq[a][rb[j] - DOFF] = fd(C, j, a);
            }
            bool fin = true;
#pragma unroll
            for (int v = 0; v < NV; ++v) fin = fin && isfinite(q[v]);
            double hm[4];
            constraints_algebra(q, dq, hm);
#pragma unroll
            for (int j = 0; j < 4; ++j) fin = fin && isfinite(hm[j]);
            const int c = sl * NFACE + tid;
            if (HM)
#pragma unroll
                for (int j = 0; j < 4; ++j) HM[((int64_t)p * 4 + j) * NCELL + c] = hm[j];
            const double X = g.org[0] + (x - 2.5) * g.dx[0], Y = g.org[1] + (y - 2.5) * g.dx[1],
                         Z = g.org[2] + (z - 2.5) * g.dx[2];
            const double r = sqrt(X * X + Y * Y + Z * Z);
            if (!fin) bad = 1.0;
            else if (r >= r_excise) {
                h2 = hm[0] * hm[0];
                m2 = hm[1] * hm[1] + hm[2] * hm[2] + hm[3] * hm[3];
                cnt = 1.0;
            }
        }
    }
    // block reduction (deterministic order)
    red[0][tid] = h2;
    red[1][tid] = m2;
    red[2][tid] = cnt;
    red[3][tid] = bad;
    __syncthreads();
    for (int s = 128; s > 0; s >>= 1) {
        if (tid < s)
            for (int j = 0; j < 4; ++j) red[j][tid] += red[j][tid + s];
        __syncthreads();
    }
    if (tid == 0)
        for (int j = 0; j < 4; ++j) part[(int64_t)blockIdx.x * 4 + j] = red[j][0];
}

__global__ void k_reduce_parts(const double *__restrict__ part, int64_t nblk, double *__restrict__ out)
{
    // one block of 256 threads: strided partial sums, then a tree
    __shared__ double red[4][256];
    double s[4] = {0, 0, 0, 0};
    for (int64_t b = threadIdx.x; b < nblk; b += 256)
        for (int j = 0; j < 4; ++j) s[j] += part[b * 4 + j];
    for (int j = 0; j < 4; ++j) red[j][threadIdx.x] = s[j];
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int j = 0; j < 4; ++j) red[j][threadIdx.x] += red[j][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double n = red[2][0];
        out[0] = n > 0 ? sqrt(red[0][0] / n) : 0.0;
        out[1] = n > 0 ? sqrt(red[1][0] / n) : 0.0;
        out[2] = red[3][0];
    }
}

// ------------------------------------------------------------------ refinement tags
// one block (256 threads) per leaf; HM must hold this leaf's H
__global__ void k_tag_indicator(const double *__restrict__ Q, const double *__restrict__ HM,
                                const PatchGeom *__restrict__ geom, double *__restrict__ ind)
{
    const int p = blockIdx.x;
    const double *Qp = Q + (int64_t)p * PS;
    double gc = 0.0, ga = 0.0, hm = 0.0;
    for (int c = threadIdx.x; c < NCELL; c += blockDim.x) {
        const int x = c % 9 + 3, y = (c / 9) % 9 + 3, z = c / 81 + 3;
        const int o = boff(x, y, z);
        const double ph = Qp[SPHI * CS + o], al = Qp[SALPHA * CS + o];
        const double chi = ph * ph;
        const int st[3] = {1, YS, ZS};
        const int cc[3] = {x, y, z};
        for (int a = 0; a < 3; ++a) {
            if (cc[a] + 1 >= 12) continue;
            const double ph2 = Qp[SPHI * CS + o + st[a]];
            gc = fmax(gc, fabs(ph2 * ph2 - chi));
            ga = fmax(ga, fabs(Qp[SALPHA * CS + o + st[a]] - al));
        }
        hm = fmax(hm, fabs(HM[(int64_t)p * 4 * NCELL + c]));
    }
    __shared__ double red[3][256];
    red[0][threadIdx.x] = gc;
    red[1][threadIdx.x] = ga;
    red[2][threadIdx.x] = hm;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
            for (int j = 0; j < 3; ++j) red[j][threadIdx.x] = fmax(red[j][threadIdx.x], red[j][threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const double dx = geom[p].dx[0];
        ind[3 * p] = red[0][0];
        ind[3 * p + 1] = red[1][0];
        ind[3 * p + 2] = dx * dx * red[2][0];
    }
}

// sib[p*27 + n]: the 27 sibling leaves of leaf p (-1 if a sibling is not a leaf); level-0 leaves
// have no siblings (sib[p*27] = -2)
__global__ void k_tag_decide(const double *__restrict__ ind, const int32_t *__restrict__ sib,
                             const PatchGeom *__restrict__ geom, int32_t npatch, double theta_r,
                             double theta_c, int32_t max_level, int8_t *__restrict__ tags)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npatch) return;
    auto e_of = [&](int q) { return fmax(fmax(ind[3 * q], ind[3 * q + 1]), ind[3 * q + 2]); };
    const double e = e_of(p);
    const int lev = geom[p].level;
    int8_t tg = 0;
    if (e >= theta_r) tg = lev < max_level ? 1 : 0;
    else if (lev > 0 && e < theta_c) {
        bool ok = true;
        for (int n = 0; n < 27 && ok; ++n) {
            const int s = sib[(int64_t)p * 27 + n];
            if (s < 0 || !(e_of(s) < theta_c)) ok = false;
        }
        tg = ok ? -1 : 0;
    }
    tags[p] = tg;
}

// ------------------------------------------------------------------ regrid transfer
// One work-group per leaf of the new mesh.  COPY: the whole box.  PROLONG: at each fine cell
// centre the tensor product over the axes of linear interpolation on the parent's interior
// (fine index f = 9 o + x across the parent, u = (f + 1/2)/3 - 1/2, l = clamp(floor(u), 0, 7),
// weights 1 - (u - l), u - l), summed in the order dz, dy, dx.  RESTRICT: the mean of the 3^3
// fine cells.  No contraction, so that the sums round exactly as written.
__global__ __launch_bounds__(256) void k_regrid(const double *__restrict__ Qo, double *__restrict__ Qn,
                                                const RegridTask *__restrict__ tasks, int32_t n)
{
#pragma clang fp contract(off)
    const int p = blockIdx.x;
    if (p >= n) return;
    const RegridTask tk = tasks[p];
    double *dst = Qn + (int64_t)p * PS;
    if (tk.kind == RG_COPY) {
        const double *src = Qo + (int64_t)tk.src * PS;
        for (int e = threadIdx.x; e < PS; e += blockDim.x) dst[e] = src[e];
        return;
    }
    for (int e = threadIdx.x; e < NCELL * NV; e += blockDim.x) {
        const int v = e / NCELL, c = e % NCELL;
        const int x = c % 9, y = (c / 9) % 9, z = c / 81;
        double s = 0.0;
        if (tk.kind == RG_PROLONG) {
            const double *src = Qo + (int64_t)tk.src * PS + (int64_t)v * CS;
            const int fc[3] = {x, y, z};
            int l[3];
            double wt[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const int f = 9 * tk.o[a] + fc[a];
                const double uu = (f + 0.5) / 3.0 - 0.5;
                int ll = (int)floor(uu);
                ll = ll < 0 ? 0 : (ll > PN - 2 ? PN - 2 : ll);
                l[a] = ll;
                wt[a] = uu - ll;
            }
            for (int dz = 0; dz < 2; ++dz)
                for (int dy = 0; dy < 2; ++dy)
                    for (int dx = 0; dx < 2; ++dx) {
                        const double wgt = (dz ? wt[2] : 1.0 - wt[2]) * (dy ? wt[1] : 1.0 - wt[1]) *
                                           (dx ? wt[0] : 1.0 - wt[0]);
                        s += wgt * src[boff(l[0] + dx + 3, l[1] + dy + 3, l[2] + dz + 3)];
                    }
        } else {
            const int kid = tk.kid[(z / 3) * 9 + (y / 3) * 3 + x / 3];
            const double *src = Qo + (int64_t)kid * PS + (int64_t)v * CS;
            for (int dz = 0; dz < 3; ++dz)
                for (int dy = 0; dy < 3; ++dy)
                    for (int dx = 0; dx < 3; ++dx)
                        s += src[boff(3 * (x % 3) + dx + 3, 3 * (y % 3) + dy + 3, 3 * (z % 3) + dz + 3)];
            s = s / 27.0;
        }
        dst[(int64_t)v * CS + boff(x + 3, y + 3, z + 3)] = s;
    }
}

// Differences of primaries V0..V1-1, staged in LDS buffers 0.., into the auxiliaries of the cell.
template <int V0, int V1>
__device__ __forceinline__ void reconstruct_from_lds(const LdsCell &C, double *__restrict__ qb, int o,
                                                     const int64_t (&pd)[3])
{
#pragma unroll
    for (int v = V0; v < V1; ++v)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double d = fd(C, v - V0, a);
            // D_a(ij) = d_a gt_ij / 2, A_a = d_a alpha, B_a^i = d_a beta^i, P_a = d_a phi
            const int dst = v < SALPHA ? SD + 6 * a + v
                          : v == SALPHA ? SA + a
                          : v < SPHI ? SB + 3 * a + (v - SBETA)
                                     : SP + a;
            const double u = v < SALPHA ? 0.5 * d : d;
            const int64_t e = (int64_t)dst * CS + o;
            qb[e] = u;
            if (pd[0] != 0) qb[e + pd[0]] = u;
#pragma unroll
            for (int k = 1; k < 3; ++k)  // streamed, as the stage sink's y and z copies
                if (pd[k] != 0) __builtin_nontemporal_store(u, qb + e + pd[k]);
        }
}

// Second-order formulation (Sec. 3.2, explicit gradient reconstruction; Algorithm 2): the
// auxiliaries from central FD4 differences of the primaries by their definitions,
// A_k = d_k alpha, B_k^i = d_k beta^i, D_kij = d_k gt_ij / 2, P_k = d_k phi, on the interior
// cells of every leaf.  One work-group per z-slab copies the slab's 11 primaries into LDS exactly as
// the stage kernel stages a slot (the slab's planes with their x and y halos, the interior rows of
// the three planes below and above), then every lane forms its cell's 33 differences from LDS
// (110 KB: one work-group per CU; two rounds of six primaries in 60 KB, two work-groups per CU, ran
// 5% slower; one thread per cell reading its stencils through the caches ran 30% slower).  The
// primaries' halos must be filled, except, with gnbr, the y and z face halos shared with a
// same-level leaf, which are then read from that leaf's interior.  With nbr, every value within
// three layers of a face shared with a same-level leaf and normal to an axis of paxes is also
// written into that leaf's face halo (as the stage push does).
__global__ __launch_bounds__(256) void k_reconstruct_lds(double *__restrict__ Q, const PatchGeom *__restrict__ geom,
                                                         int32_t npatch, const int32_t *__restrict__ nbr,
                                                         int32_t paxes, const int32_t *__restrict__ gnbr)
{
    __shared__ double lds[(SPHI + 1) * LDS_SLOT];
    const int64_t lb = xcd_logical_block(blockIdx.x, gridDim.x);
    const int p = (int)(lb / 3);
    if (p >= npatch) return;  // uniform over the work-group
    const int sl = (int)(lb % 3);
    const PatchGeom g = geom[p];
    const int tid = threadIdx.x, w = tid >> 6, lane = tid & 63;
    const bool act = tid < 243;
    const int cc = act ? tid : 242;
    const int x = cc % 9 + 3, y = (cc / 9) % 9 + 3, zl = cc / 81;
    LdsCell C;
    C.s = lds;
    lds_cell_offsets(C, x, y, zl);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        C.i12[a] = 1.0 / (12.0 * g.dx[a]);
        C.koc[a] = 0.0;
    }
    HaloSrc hs;
#pragma unroll
    for (int f = 0; f < 4; ++f) {  // faces y-, y+, z-, z+
        const int n = gnbr ? gnbr[p * 6 + 2 + f] : -1;
        hs.d[f] = n >= 0 ? (int64_t)(n - p) * PS + ((f & 1) ? -9 : 9) * (f < 2 ? YS : ZS) : 0;
    }
    double *qb = Q + (int64_t)p * PS;
    const int z = zl + 3 + 3 * sl;
    const int o = boff(x, y, z);
    int64_t pd[3];
    push_offsets(nbr, p, x, y, z, o, pd, paxes);
    const int slots[SPHI + 1] = {0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10};
    lds_round(qb, lds, sl, slots, w, lane, hs);
    if (act) reconstruct_from_lds<0, SPHI + 1>(C, qb, o, pd);
}


hipError_t launch_reconstruct(double *Q, const PatchGeom *geom, int32_t npatch, const int32_t *nbr, int32_t paxes,
                              const int32_t *gnbr, hipStream_t st)
{
    if (npatch <= 0) return hipSuccess;
    const int64_t nb = ((int64_t)npatch * 3 + 7) / 8 * 8;  // a multiple of 8 for the XCD block order
    hipLaunchKernelGGL(k_reconstruct_lds, dim3((unsigned)nb), dim3(256), 0, st, Q, geom, npatch, nbr, paxes, gnbr);
    return hipGetLastError();
}

// The cube index of coordinate v at the finest level, and whether leaf g (level l, lower corner
// org + i * edge_l) holds that index: i * 3^(top - l) <= K < (i + 1) * 3^(top - l).  One rounded
// index serves every level, so the leaves tile the domain without gaps or overlaps even for points
// within rounding of a face.
__device__ __forceinline__ double fine_index(const LeafLookup &lk, int a, double v)
{
    return floor((v - lk.org[a]) / lk.fine[a]);
}
__device__ __forceinline__ bool leaf_holds(const LeafLookup &lk, const PatchGeom &g, const double K[3])
{
    double s = 1.0;
    for (int l = g.level; l < lk.top; ++l) s *= 3.0;
    bool in = true;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double i = rint((g.org[a] - lk.org[a]) / (lk.fine[a] * s));
        in = in && K[a] >= i * s && K[a] < (i + 1.0) * s;
    }
    return in;
}

// Tracers (Sec. 3.8): one work-group per point.  The lanes test a strided share of the leaves for
// the one holding the point (leaf_holds); the trilinear weights come from the 2^3 cell centres
// around the point at that leaf's spacing.  A cell inside the leaf's interior is read there; a
// cell outside it is read from the interior of the leaf of the same level that holds its centre
// (a second strided search), so that no value comes from an edge or corner region of a halo,
// which no fill writes; a cell whose centre is outside the domain or in a leaf of another level is
// read from the leaf's own box (its face halo, filled by the boundary or coarse-fine fill).  Each
// requested slot is then interpolated by one lane.  advance: the point moves by dt * (-beta)
// (puncture tracker, explicit Euler).  A point outside every leaf samples NaN and stays.
__global__ __launch_bounds__(256) void k_tracers(const double *__restrict__ Q, const PatchGeom *__restrict__ geom,
                                                 int32_t npatch, double *__restrict__ pos, TracerSlots sl,
                                                 LeafLookup lk, double *__restrict__ out, double dt,
                                                 int32_t advance)
{
    __shared__ int leaf;
    __shared__ int owner[8];
    __shared__ double beta[3];
    const int64_t i = blockIdx.x;
    if (threadIdx.x == 0) leaf = -1;
    if (threadIdx.x < 8) owner[threadIdx.x] = -1;
    __syncthreads();
    const double x[3] = {pos[3 * i], pos[3 * i + 1], pos[3 * i + 2]};
    const double K[3] = {fine_index(lk, 0, x[0]), fine_index(lk, 1, x[1]), fine_index(lk, 2, x[2])};
    for (int p = (int)threadIdx.x; p < npatch; p += (int)blockDim.x)
        if (leaf_holds(lk, geom[p], K)) leaf = p;  // one leaf holds a point: one lane at most
    __syncthreads();
    const int p = leaf;  // uniform over the work-group
    int i0[3] = {3, 3, 3};
    double w[3] = {0.0, 0.0, 0.0};
    PatchGeom gp{};
    if (p >= 0) {
        gp = geom[p];
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double u = (x[a] - gp.org[a]) / gp.dx[a] - 0.5;
            const double f = floor(u);
            i0[a] = (int)f + 3;  // box index of the lower centre: 2..11
            w[a] = u - f;
        }
        // owners of the cells outside the leaf's interior (one leaf holds a centre: one lane each)
        for (int q = (int)threadIdx.x; q < npatch; q += (int)blockDim.x) {
            const PatchGeom g = geom[q];
            if (q == p || g.level != gp.level) continue;
            for (int c = 0; c < 8; ++c) {
                const int b[3] = {i0[0] + (c & 1), i0[1] + ((c >> 1) & 1), i0[2] + ((c >> 2) & 1)};
                if (b[0] >= 3 && b[0] <= 11 && b[1] >= 3 && b[1] <= 11 && b[2] >= 3 && b[2] <= 11) continue;
                double Kc[3];
#pragma unroll
                for (int a = 0; a < 3; ++a)
                    Kc[a] = fine_index(lk, a, gp.org[a] + ((double)(b[a] - 3) + 0.5) * gp.dx[a]);
                if (leaf_holds(lk, g, Kc)) owner[c] = q;
            }
        }
    }
    __syncthreads();
    const int nout = advance ? 3 : sl.n;
    const int t = (int)threadIdx.x;
    if (t < nout) {
        const int v = advance ? SBETA + t : sl.v[t];
        double val = __builtin_nan("");
        if (p >= 0) {
            val = 0.0;
#pragma unroll
            for (int c = 0; c < 8; ++c) {
                const int cx = c & 1, cy = (c >> 1) & 1, cz = (c >> 2) & 1;
                int b[3] = {i0[0] + cx, i0[1] + cy, i0[2] + cz};
                int q = owner[c];
                if (q >= 0) {
                    const PatchGeom g = geom[q];
#pragma unroll
                    for (int a = 0; a < 3; ++a) {
                        const double xc = gp.org[a] + ((double)(b[a] - 3) + 0.5) * gp.dx[a];
                        b[a] = min(11, max(3, (int)floor((xc - g.org[a]) / g.dx[a]) + 3));
                    }
                } else {
                    q = p;
                }
                const double wt = (cx ? w[0] : 1.0 - w[0]) * (cy ? w[1] : 1.0 - w[1]) * (cz ? w[2] : 1.0 - w[2]);
                val += wt * Q[(int64_t)q * PS + v * CS + boff(b[0], b[1], b[2])];
            }
        }
        if (advance) beta[t] = val;
        else out[i * sl.n + t] = val;
    }
    if (advance) {
        __syncthreads();
        if (t == 0 && p >= 0)
#pragma unroll
            for (int a = 0; a < 3; ++a) pos[3 * i + a] = x[a] + dt * (-beta[a]);
    }
}

hipError_t launch_tracers(const double *Q, const PatchGeom *geom, int32_t npatch, int64_t n, double *pos,
                          const TracerSlots &sl, const LeafLookup &lk, double *out, double dt, int32_t advance, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tracers, dim3((unsigned)n), dim3(256), 0, st, Q, geom, npatch, pos, sl, lk, out, dt, advance);
    return hipGetLastError();
}

// Tracker-based refinement (refinement by coordinates): REFINE a leaf of level l < min(max_level,
// radii.n) whose closed cube lies within r[l] of a tracer; COARSEN a leaf of level >= 1 whose parent
// cube lies farther than r[l - 1] from every tracer; KEEP otherwise.  One lane per leaf.
__device__ __forceinline__ double cube_distance(const double lo[3], const double L[3], int64_t n,
                                                const double *__restrict__ pos)
{
    double best = __builtin_huge_val();
    for (int64_t i = 0; i < n; ++i) {
        double d2 = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const double x = pos[3 * i + a];
            const double c = x < lo[a] ? lo[a] : (x > lo[a] + L[a] ? lo[a] + L[a] : x);
            d2 += (c - x) * (c - x);
        }
        best = fmin(best, sqrt(d2));
    }
    return best;
}

__global__ __launch_bounds__(256) void k_tag_tracers(const TrackBox *__restrict__ box, int32_t npatch, int64_t n,
                                                     const double *__restrict__ pos, TrackRadii R, int32_t max_level,
                                                     int8_t *__restrict__ tags)
{
    const int p = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (p >= npatch) return;
    const TrackBox b = box[p];
    int8_t t = 0;
    if (b.level < max_level && b.level < R.n && cube_distance(b.lo, b.L, n, pos) <= R.r[b.level])
        t = 1;
    else if (b.level >= 1 && (b.level - 1 >= R.n || cube_distance(b.plo, b.pL, n, pos) > R.r[b.level - 1]))
        t = -1;
    tags[p] = t;
}

hipError_t launch_tag_tracers(const TrackBox *box, int32_t npatch, int64_t n, const double *pos, const TrackRadii &R,
                              int32_t max_level, int8_t *tags, hipStream_t st)
{
    if (npatch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tag_tracers, dim3((unsigned)((npatch + 255) / 256)), dim3(256), 0, st, box, npatch, n, pos, R,
                       max_level, tags);
    return hipGetLastError();
}

hipError_t launch_regrid(const double *Qo, double *Qn, const RegridTask *tasks, int32_t n, hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_regrid, dim3(n), dim3(256), 0, st, Qo, Qn, tasks, n);
    return hipGetLastError();
}

// ------------------------------------------------------------------ launchers
hipError_t launch_init(double *Q, const PatchGeom *geom, const uint8_t *bmask, int32_t npatch, int32_t scen,
                       const InitArgs &a, hipStream_t st)
{
    const int64_t n = (int64_t)npatch * 3375;
    hipLaunchKernelGGL(k_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Q, geom, bmask, npatch, scen, a);
    return hipGetLastError();
}

hipError_t launch_fill(double *Q, const FaceTask *tasks, int32_t ntask, int32_t transfer, hipStream_t st)
{
    if (ntask <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill, dim3(ntask, (NV + SB8 - 1) / SB8), dim3(256), 0, st, Q, tasks, ntask, transfer);
    return hipGetLastError();
}

hipError_t launch_rhs(const double *Q, double *K, const PatchGeom *geom, int32_t npatch, const RhsParams &p,
                      int32_t precision, int32_t variant, const int32_t *order, const BoundaryFace *bf,
                      const double *bg, int32_t nbf, const int32_t *pface, hipStream_t st)
{
    // the LDS kernel computes the Sommerfeld ghosts' right-hand side inside the slab work-groups;
    // the phased kernel leaves it to k_rhs_sommerfeld
    const int32_t *slab_ghosts = nbf > 0 ? pface : nullptr;
    const int64_t nb = ((int64_t)npatch * 3 + 7) / 8 * 8;
    const int32_t lin = (variant & KV_LINEAR) ? 1 : 0;
    if (variant & KV_LDS) {
        const dim3 g((unsigned)nb), b(256);
        if (p.advection) {
            if (precision == 1)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rhs_lds<float, 1>), g, b, 0, st, Q, K, geom, npatch, p, bf, bg,
                                   slab_ghosts, lin, order);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rhs_lds<double, 1>), g, b, 0, st, Q, K, geom, npatch, p, bf, bg,
                                   slab_ghosts, lin, order);
        } else {
            if (precision == 1)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rhs_lds<float, 0>), g, b, 0, st, Q, K, geom, npatch, p, bf, bg,
                                   slab_ghosts, lin, order);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rhs_lds<double, 0>), g, b, 0, st, Q, K, geom, npatch, p, bf, bg,
                                   slab_ghosts, lin, order);
        }
    } else {
        const dim3 g((unsigned)nb), b(256);
        if (p.advection) {
            if (precision == 1)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rhs<float, 1>), g, b, 0, st, Q, K, geom, npatch, p, lin, order);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rhs<double, 1>), g, b, 0, st, Q, K, geom, npatch, p, lin, order);
        } else {
            if (precision == 1)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rhs<float, 0>), g, b, 0, st, Q, K, geom, npatch, p, lin, order);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_rhs<double, 0>), g, b, 0, st, Q, K, geom, npatch, p, lin, order);
        }
        if (nbf > 0) {
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            return launch_rhs_sommerfeld(Q, K, geom, bf, bg, nbf, p.shift == 0 ? 1 : 0, st);
        }
    }
    return hipGetLastError();
}

// 3 work-groups per patch (grid padded to a multiple of 8 for the XCD mapping).  The Sommerfeld
// ghost faces get one more work-group each in the same launch with the phased kernel; with the
// LDS kernel each slab work-group updates the ghost cells beside its own planes.
hipError_t launch_stage(int32_t s, double dt, const double *Qs, const double *Qn, double *acc, double *Qx,
                        const PatchGeom *geom, int32_t npatch, const RhsParams &p, int32_t precision,
                        int32_t variant, const int32_t *order, const BoundaryFace *bf, const double *bg, int32_t nbf,
                        const int32_t *pface, const int32_t *nbr, int32_t paxes, const int32_t *gnbr,
                        hipStream_t st)
{
    // the LDS kernel updates the Sommerfeld ghosts inside the slab work-groups (per-leaf face table)
    const int32_t *slab_ghosts = nbf > 0 ? pface : nullptr;
    const int64_t nb_slab = ((int64_t)npatch * 3 + 7) / 8 * 8;
    const int64_t nb = nb_slab + (nbf > 0 ? nbf : 0);
    const int32_t ns = (int32_t)nb_slab;
    const int32_t lin = (variant & KV_LINEAR) ? 1 : 0;
    if (variant & KV_LDS) {
        const dim3 g((unsigned)nb_slab), b(256);
        if (p.advection) {
            if (precision == 1)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_stage_lds<float, 1>), g, b, 0, st, Qs, Qn, acc, Qx, geom, npatch,
                                   ns, p, s, dt, bf, bg, slab_ghosts, nbr, paxes, gnbr, lin, order);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_stage_lds<double, 1>), g, b, 0, st, Qs, Qn, acc, Qx, geom, npatch,
                                   ns, p, s, dt, bf, bg, slab_ghosts, nbr, paxes, gnbr, lin, order);
        } else {
            if (precision == 1)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_stage_lds<float, 0>), g, b, 0, st, Qs, Qn, acc, Qx, geom, npatch,
                                   ns, p, s, dt, bf, bg, slab_ghosts, nbr, paxes, gnbr, lin, order);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_stage_lds<double, 0>), g, b, 0, st, Qs, Qn, acc, Qx, geom, npatch,
                                   ns, p, s, dt, bf, bg, slab_ghosts, nbr, paxes, gnbr, lin, order);
        }
    } else {
        const dim3 g((unsigned)nb), b(256);
        if (p.advection) {
            if (precision == 1)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_stage<float, 1>), g, b, 0, st, Qs, Qn, acc, Qx, geom, npatch, ns,
                                   p, s, dt, bf, bg, nbr, paxes, lin, order);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_stage<double, 1>), g, b, 0, st, Qs, Qn, acc, Qx, geom, npatch, ns,
                                   p, s, dt, bf, bg, nbr, paxes, lin, order);
        } else {
            if (precision == 1)
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_stage<float, 0>), g, b, 0, st, Qs, Qn, acc, Qx, geom, npatch, ns,
                                   p, s, dt, bf, bg, nbr, paxes, lin, order);
            else
                hipLaunchKernelGGL(HIP_KERNEL_NAME(k_stage<double, 0>), g, b, 0, st, Qs, Qn, acc, Qx, geom, npatch, ns,
                                   p, s, dt, bf, bg, nbr, paxes, lin, order);
        }
    }
    return hipGetLastError();
}

hipError_t launch_rhs_sommerfeld(const double *Q, double *K, const PatchGeom *geom, const BoundaryFace *bf,
                                 const double *bg, int32_t nbf, int32_t frozen, hipStream_t st)
{
    if (nbf <= 0) return hipSuccess;
    const int64_t n = (int64_t)nbf * NV * NFACE;
    hipLaunchKernelGGL(k_rhs_sommerfeld, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, Q, K, geom, bf, bg,
                       nbf, frozen);
    return hipGetLastError();
}

hipError_t launch_capture_bg(const double *Q, const BoundaryFace *bf, double *bg, int32_t nbf, hipStream_t st)
{
    if (nbf <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_capture_bg, dim3(nbf), dim3(256), 0, st, Q, bf, bg, nbf);
    return hipGetLastError();
}

hipError_t launch_rk4(int32_t s, double dt, const double *Qn, const double *K, double *acc, double *Qx,
                      int32_t npatch, const BoundaryFace *bf, int32_t nbf, hipStream_t st)
{
    const int64_t n = (int64_t)npatch * NCELL;
    hipLaunchKernelGGL(k_rk4, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s, dt, Qn, K, acc, Qx, npatch);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (nbf <= 0) return hipSuccess;
    const int64_t ng = (int64_t)nbf * NV * NFACE;
    hipLaunchKernelGGL(k_rk4_ghost, dim3((unsigned)((ng + 255) / 256)), dim3(256), 0, st, s, dt, Qn, K, acc, Qx, bf,
                       nbf);
    return hipGetLastError();
}

// one work-group per z-slab, a multiple of 8 for the XCD block order (at least 8)
int64_t constraints_blocks(int32_t npatch) { return std::max<int64_t>(8, ((int64_t)npatch * 3 + 7) / 8 * 8); }

hipError_t launch_constraints(const double *Q, double *HM, const PatchGeom *geom, int32_t npatch,
                              double r_excise, double *part, double *out3, hipStream_t st)
{
    const int64_t nb = constraints_blocks(npatch);
    hipLaunchKernelGGL(k_constraints_lds, dim3((unsigned)nb), dim3(256), 0, st, Q, HM, geom, npatch, r_excise, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_reduce_parts, dim3(1), dim3(256), 0, st, part, nb, out3);
    return hipGetLastError();
}

hipError_t launch_tags(const double *Q, const double *HM, const PatchGeom *geom, const int32_t *sib,
                       int32_t npatch, double theta_r, double theta_c, int32_t max_level, int8_t *tags,
                       double *ind, hipStream_t st)
{
    hipLaunchKernelGGL(k_tag_indicator, dim3(npatch), dim3(256), 0, st, Q, HM, geom, ind);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tag_decide, dim3((npatch + 127) / 128), dim3(128), 0, st, ind, sib, geom, npatch,
                       theta_r, theta_c, max_level, tags);
    return hipGetLastError();
}

}  // namespace ccz4
