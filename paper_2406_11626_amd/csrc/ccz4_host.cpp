// Host side of the C ABI (include/ccz4.h): leaf forest, face-task plan of the halo fill,
// Sommerfeld boundary faces, sibling table of the refinement criterion, and the calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <new>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <unordered_set>
#include <vector>

#include "../../include/ccz4.h"
#include "ccz4_kernels.hpp"
#include "ccz4_mlp.hpp"

using namespace ccz4;

namespace {

thread_local std::string g_err;

ccz4_status fail(ccz4_status s, const std::string &msg)
{
    g_err = msg;
    return s;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return fail(CCZ4_EHIP, std::string(#expr) + ": " + hipGetErrorString(e_));         \
    } while (0)

inline uint64_t key(int lev, int i, int j, int k)
{
    return ((uint64_t)lev << 48) | ((uint64_t)(uint16_t)k << 32) | ((uint64_t)(uint16_t)j << 16) | (uint16_t)i;
}

template <typename T>
struct DevBuf {
    T *p = nullptr;
    size_t n = 0;
    hipError_t upload(const std::vector<T> &v)
    {
        release();
        n = v.size();
        if (!n) return hipSuccess;
        hipError_t e = hipMalloc((void **)&p, n * sizeof(T));
        if (e != hipSuccess) { p = nullptr; return e; }
        return hipMemcpy(p, v.data(), n * sizeof(T), hipMemcpyHostToDevice);
    }
    hipError_t alloc(size_t cnt)
    {
        release();
        n = cnt;
        if (!n) return hipSuccess;
        hipError_t e = hipMalloc((void **)&p, n * sizeof(T));
        if (e != hipSuccess) p = nullptr;
        return e;
    }
    void release()
    {
        if (p) (void)hipFree(p);
        p = nullptr;
        n = 0;
    }
};

}  // namespace

struct ccz4_ctx {
    int device = 0;
    int n0[3];
    double origin[3], extent[3];
    int bc;
    RhsParams prm;
    std::vector<std::array<int, 4>> leaf;     // lev, i, j, k
    std::vector<std::array<int, 4>> refined;  // refined cubes of the forest (lev, i, j, k)
    std::unordered_map<uint64_t, int> index;  // leaf key -> leaf index
    std::vector<PatchGeom> geom;
    std::vector<TrackBox> tbox;           // cubes of the leaves and of their parents
    DevBuf<TrackBox> d_tbox;
    std::vector<FaceTask> ph_copy, ph_neu, ph_res, ph_pro;  // fill tasks by kind (restrict before prolong)
    std::vector<int32_t> nbr;                 // [leaf][6] same-level face neighbour or -1
    std::vector<BoundaryFace> bface;
    std::vector<int32_t> pface;               // per leaf and face 2 axis + (side > 0): index into bface or -1
    std::vector<uint8_t> bmask;
    std::vector<int32_t> sib;
    DevBuf<PatchGeom> d_geom;
    DevBuf<FaceTask> d_phc, d_phn, d_phr, d_php;
    DevBuf<int32_t> d_nbr;
    DevBuf<int32_t> d_order;                  // KV_ORDERS leaf permutations, npatch each
    DevBuf<BoundaryFace> d_bf;
    DevBuf<int32_t> d_pface;
    DevBuf<uint8_t> d_bmask;
    DevBuf<int32_t> d_sib;
    DevBuf<double> d_bg, d_part, d_out3, d_hm;
    DevBuf<int8_t> d_pre;                     // learned tags, first pass
    double *h_out3 = nullptr;  // pinned
    bool bg_valid = false;
    int32_t kernel[2] = {KV_LDS, KV_LDS};  // per precision
};

namespace {

int level_n(const ccz4_ctx *c, int lev, int a)
{
    int n = c->n0[a];
    for (int l = 0; l < lev; ++l) n *= 3;
    return n;
}

ccz4_status build_plan(ccz4_ctx *c, const ccz4_grid_desc *g)
{
    std::unordered_set<uint64_t> refined;
    int maxlev = 0;
    for (int r = 0; r < g->n_refined; ++r) {
        const int32_t *e = g->refined + 4 * r;
        if (e[0] < 0 || e[0] > 12 || e[1] < 0 || e[2] < 0 || e[3] < 0)
            return fail(CCZ4_EINVAL, "refined entry out of range");
        refined.insert(key(e[0], e[1], e[2], e[3]));
        maxlev = std::max(maxlev, e[0] + 1);
    }
    auto is_ref = [&](int l, int i, int j, int k) { return refined.count(key(l, i, j, k)) > 0; };
    // leaves: level-0 cubes and the children of refined cubes whose ancestors are refined
    std::vector<std::array<int, 4>> cubes;
    for (int k = 0; k < c->n0[2]; ++k)
        for (int j = 0; j < c->n0[1]; ++j)
            for (int i = 0; i < c->n0[0]; ++i) cubes.push_back({0, i, j, k});
    std::vector<std::array<int, 4>> leaves;
    size_t head = 0;
    while (head < cubes.size()) {
        const auto cu = cubes[head++];
        if (!is_ref(cu[0], cu[1], cu[2], cu[3])) {
            leaves.push_back(cu);
            continue;
        }
        c->refined.push_back(cu);
        for (int w = 0; w < 3; ++w)
            for (int v = 0; v < 3; ++v)
                for (int u = 0; u < 3; ++u) cubes.push_back({cu[0] + 1, 3 * cu[1] + u, 3 * cu[2] + v, 3 * cu[3] + w});
    }
    std::sort(leaves.begin(), leaves.end(), [](const std::array<int, 4> &a, const std::array<int, 4> &b) {
        if (a[0] != b[0]) return a[0] < b[0];
        if (a[3] != b[3]) return a[3] < b[3];
        if (a[2] != b[2]) return a[2] < b[2];
        return a[1] < b[1];
    });
    if (leaves.size() > (size_t)INT32_MAX / 4) return fail(CCZ4_EINVAL, "too many leaves");
    c->leaf = leaves;
    std::unordered_map<uint64_t, int> &index = c->index;
    index.clear();
    for (size_t p = 0; p < leaves.size(); ++p)
        index[key(leaves[p][0], leaves[p][1], leaves[p][2], leaves[p][3])] = (int)p;
    auto find = [&](int l, int i, int j, int k) -> int {
        auto it = index.find(key(l, i, j, k));
        return it == index.end() ? -1 : it->second;
    };
    // geometry
    c->geom.resize(leaves.size());
    for (size_t p = 0; p < leaves.size(); ++p) {
        PatchGeom &pg = c->geom[p];
        pg.level = leaves[p][0];
        pg.pad = 0;
        for (int a = 0; a < 3; ++a) {
            const double L = c->extent[a] / level_n(c, pg.level, a);
            pg.org[a] = c->origin[a] + L * leaves[p][1 + a];
            pg.dx[a] = L / PN;
        }
    }
    c->tbox.resize(leaves.size());
    for (size_t p = 0; p < leaves.size(); ++p) {
        TrackBox &b = c->tbox[p];
        const int lev = leaves[p][0];
        b.level = lev;
        b.pad = 0;
        for (int a = 0; a < 3; ++a) {
            b.L[a] = c->extent[a] / level_n(c, lev, a);
            b.lo[a] = c->origin[a] + b.L[a] * leaves[p][1 + a];
            b.pL[a] = lev > 0 ? c->extent[a] / level_n(c, lev - 1, a) : 0.0;
            b.plo[a] = lev > 0 ? c->origin[a] + b.pL[a] * (leaves[p][1 + a] / 3) : 0.0;
        }
    }
    // face tasks
    c->ph_copy.clear();
    c->ph_neu.clear();
    c->ph_res.clear();
    c->ph_pro.clear();
    c->bface.clear();
    c->nbr.assign(leaves.size() * 6, -1);
    c->bmask.assign(leaves.size(), 0);
    for (size_t p = 0; p < leaves.size(); ++p) {
        const int lev = leaves[p][0];
        for (int a = 0; a < 3; ++a)
            for (int side = -1; side <= 1; side += 2) {
                int n[3] = {leaves[p][1], leaves[p][2], leaves[p][3]};
                n[a] += side;
                const int na = level_n(c, lev, a);
                FaceTask t{};
                t.patch = (int)p;
                t.axis = a;
                t.side = side;
                for (int s = 0; s < 9; ++s) t.src[s] = -1;
                if (n[a] < 0 || n[a] >= na) {
                    if (c->bc == CCZ4_BC_PERIODIC) {
                        n[a] = (n[a] + na) % na;
                    } else if (c->bc == CCZ4_BC_NEUMANN) {
                        t.kind = FK_NEUMANN;
                        c->ph_neu.push_back(t);
                        continue;
                    } else {
                        BoundaryFace b{(int)p, a, side, (int)c->bface.size()};
                        c->bface.push_back(b);
                        c->bmask[p] |= (uint8_t)(1u << (2 * a + (side > 0 ? 1 : 0)));
                        continue;
                    }
                }
                const int nb = find(lev, n[0], n[1], n[2]);
                if (nb >= 0) {
                    t.kind = FK_COPY;
                    t.src[0] = nb;
                    c->ph_copy.push_back(t);
                    c->nbr[p * 6 + 2 * a + (side > 0 ? 1 : 0)] = nb;
                    continue;
                }
                // tangential axes in increasing order
                const int b1 = a == 0 ? 1 : 0, b2 = a == 2 ? 1 : 2;
                bool nbexists = lev == 0 || is_ref(lev - 1, n[0] / 3, n[1] / 3, n[2] / 3);
                if (nbexists && is_ref(lev, n[0], n[1], n[2])) {
                    t.kind = FK_RESTRICT;
                    for (int u2 = 0; u2 < 3; ++u2)
                        for (int u1 = 0; u1 < 3; ++u1) {
                            int ci[3];
                            ci[a] = 3 * n[a] + (side > 0 ? 0 : 2);
                            ci[b1] = 3 * n[b1] + u1;
                            ci[b2] = 3 * n[b2] + u2;
                            const int kid = find(lev + 1, ci[0], ci[1], ci[2]);
                            if (kid < 0)
                                return fail(CCZ4_ELAYOUT, "level jump of more than one across a face");
                            t.src[u2 * 3 + u1] = kid;
                        }
                    c->ph_res.push_back(t);
                    continue;
                }
                if (lev == 0) return fail(CCZ4_ELAYOUT, "face neighbour missing at level 0");
                const int cp = find(lev - 1, n[0] / 3, n[1] / 3, n[2] / 3);
                if (cp < 0) return fail(CCZ4_ELAYOUT, "level jump of more than one across a face");
                t.kind = FK_PROLONG;
                t.src[0] = cp;
                t.o1 = n[b1] - 3 * (n[b1] / 3);
                t.o2 = n[b2] - 3 * (n[b2] / 3);
                c->ph_pro.push_back(t);
            }
    }
    // siblings
    c->sib.assign(leaves.size() * 27, -1);
    for (size_t p = 0; p < leaves.size(); ++p) {
        const int lev = leaves[p][0];
        if (lev == 0) {
            c->sib[p * 27] = -2;
            continue;
        }
        const int pi = leaves[p][1] / 3, pj = leaves[p][2] / 3, pk = leaves[p][3] / 3;
        for (int w = 0; w < 3; ++w)
            for (int v = 0; v < 3; ++v)
                for (int u = 0; u < 3; ++u)
                    c->sib[p * 27 + (w * 3 + v) * 3 + u] = find(lev, 3 * pi + u, 3 * pj + v, 3 * pk + w);
    }
    (void)maxlev;
    return CCZ4_OK;
}

RhsParams to_rhs(const ccz4_params *p)
{
    RhsParams r;
    r.kappa1 = p->kappa1;
    r.kappa2 = p->kappa2;
    r.kappa3 = p->kappa3;
    r.tau = p->tau;
    r.e = p->e;
    r.c = p->c;
    r.mu = p->mu;
    r.f = p->f;
    r.eta = p->eta;
    r.ko_eps = p->ko_eps;
    r.slicing = p->slicing;
    r.shift = p->shift;
    r.formulation = p->formulation;
    r.advection = p->advection;
    r.transfer = p->transfer;
    return r;
}

ccz4_status check_params(const ccz4_params *p)
{
    if (!p) return fail(CCZ4_EINVAL, "params is NULL");
    if (p->slicing != 0 && p->slicing != 1) return fail(CCZ4_EINVAL, "slicing must be 0 or 1");
    if (p->shift != 0 && p->shift != 1) return fail(CCZ4_EINVAL, "shift must be 0 or 1");
    if (p->formulation != CCZ4_FORMULATION_FIRST_ORDER && p->formulation != CCZ4_FORMULATION_SECOND_ORDER)
        return fail(CCZ4_EINVAL, "formulation must be 0 (first order) or 1 (second order)");
    if (p->advection < CCZ4_ADVECTION_CENTRAL || p->advection > CCZ4_ADVECTION_LOPSIDED_PRINTED)
        return fail(CCZ4_EINVAL, "advection must be 0 (central), 1 (lopsided, upwind) or 2 (lopsided, as printed)");
    if (p->transfer != CCZ4_TRANSFER_APP_E && p->transfer != CCZ4_TRANSFER_HIGHER_ORDER)
        return fail(CCZ4_EINVAL, "transfer must be 0 (App. E operators) or 1 (higher order)");
    if (!(p->tau > 0)) return fail(CCZ4_EINVAL, "tau must be > 0");
    return CCZ4_OK;
}

inline hipStream_t S(void *s) { return (hipStream_t)s; }

ccz4_status check_ptr(const void *p, const char *name)
{
    if (!p) return fail(CCZ4_EINVAL, std::string(name) + " is NULL");
    if (((uintptr_t)p) % 8) return fail(CCZ4_EINVAL, std::string(name) + " is not 8-byte aligned");
    return CCZ4_OK;
}

}  // namespace

extern "C" {

const char *ccz4_last_error(void) { return g_err.c_str(); }

// The orders in which a right-hand-side or stage launch may walk the leaves (levels in turn, each
// level by its cube index (i, j, k)): 0 canonical (i fastest), 1 z-pencils (k fastest, then j, then
// i), 2 bricks of 4^3 cubes (canonical inside a brick and between bricks), 3 Morton (bits of i, j,
// k interleaved, i lowest).  The launch's logical patch q takes leaf order[q]; the leaves a stage
// reads besides its own (the y and z face neighbours) are then processed closer in time.
static std::vector<int32_t> leaf_orders(const std::vector<std::array<int, 4>> &leaf)
{
    const size_t n = leaf.size();
    std::vector<int32_t> out(KV_ORDERS * n);
    auto morton = [](uint32_t i, uint32_t j, uint32_t k) {
        uint64_t m = 0;
        for (int b = 0; b < 20; ++b)
            m |= (uint64_t)((i >> b) & 1) << (3 * b) | (uint64_t)((j >> b) & 1) << (3 * b + 1) |
                 (uint64_t)((k >> b) & 1) << (3 * b + 2);
        return m;
    };
    for (int o = 0; o < KV_ORDERS; ++o) {
        std::vector<std::pair<std::array<uint64_t, 3>, int32_t>> key(n);
        for (size_t p = 0; p < n; ++p) {
            const uint64_t l = (uint64_t)leaf[p][0], i = (uint64_t)leaf[p][1], j = (uint64_t)leaf[p][2],
                           k = (uint64_t)leaf[p][3];
            std::array<uint64_t, 3> kk{l, 0, 0};
            if (o == 0) kk[1] = (k << 40) | (j << 20) | i;
            else if (o == 1) kk[1] = (i << 40) | (j << 20) | k;
            else if (o == 2) {
                kk[1] = ((k >> 2) << 40) | ((j >> 2) << 20) | (i >> 2);
                kk[2] = ((k & 3) << 4) | ((j & 3) << 2) | (i & 3);
            } else kk[1] = morton((uint32_t)i, (uint32_t)j, (uint32_t)k);
            key[p] = {kk, (int32_t)p};
        }
        std::sort(key.begin(), key.end());
        for (size_t q = 0; q < n; ++q) out[o * n + q] = key[q].second;
    }
    return out;
}

ccz4_status ccz4_create(ccz4_ctx **out, const ccz4_grid_desc *g, const ccz4_params *prm)
{
    if (!out) return fail(CCZ4_EINVAL, "out is NULL");
    *out = nullptr;
    if (!g) return fail(CCZ4_EINVAL, "grid is NULL");
    ccz4_status st = check_params(prm);
    if (st) return st;
    for (int a = 0; a < 3; ++a) {
        if (g->n0[a] <= 0 || g->n0[a] > 4096) return fail(CCZ4_EINVAL, "n0 out of range");
        if (!(g->extent[a] > 0)) return fail(CCZ4_EINVAL, "extent must be > 0");
    }
    if (g->bc < 0 || g->bc > 2) return fail(CCZ4_EINVAL, "bc must be 0, 1 or 2");
    if (g->n_refined < 0 || (g->n_refined > 0 && !g->refined)) return fail(CCZ4_EINVAL, "bad refined list");
    ccz4_ctx *c = new (std::nothrow) ccz4_ctx();
    if (!c) return fail(CCZ4_ENOMEM, "context allocation failed");
    for (int a = 0; a < 3; ++a) {
        c->n0[a] = g->n0[a];
        c->origin[a] = g->origin[a];
        c->extent[a] = g->extent[a];
    }
    c->bc = g->bc;
    c->prm = to_rhs(prm);
    hipError_t he = hipGetDevice(&c->device);
    if (he != hipSuccess) {
        delete c;
        return fail(CCZ4_EHIP, std::string("hipGetDevice: ") + hipGetErrorString(he));
    }
    st = build_plan(c, g);
    if (st) {
        delete c;
        return st;
    }
    const size_t nbf = c->bface.size();
    const int64_t nblk = constraints_blocks((int32_t)c->leaf.size());
    hipError_t e = hipSuccess;
    if (e == hipSuccess) e = c->d_geom.upload(c->geom);
    if (e == hipSuccess) e = c->d_tbox.upload(c->tbox);
    if (e == hipSuccess) e = c->d_phc.upload(c->ph_copy);
    if (e == hipSuccess) e = c->d_phn.upload(c->ph_neu);
    if (e == hipSuccess) e = c->d_phr.upload(c->ph_res);
    if (e == hipSuccess) e = c->d_php.upload(c->ph_pro);
    if (e == hipSuccess) e = c->d_nbr.upload(c->nbr);
    if (e == hipSuccess) e = c->d_order.upload(leaf_orders(c->leaf));
    if (e == hipSuccess) e = c->d_pre.alloc(c->leaf.size());
    if (e == hipSuccess) e = c->d_bf.upload(c->bface);
    c->pface.assign(c->leaf.size() * 6, -1);
    for (size_t i = 0; i < c->bface.size(); ++i) {
        const BoundaryFace &b = c->bface[i];
        c->pface[(size_t)b.patch * 6 + 2 * b.axis + (b.side > 0 ? 1 : 0)] = (int32_t)i;
    }
    if (e == hipSuccess && !c->pface.empty()) e = c->d_pface.upload(c->pface);
    if (e == hipSuccess) e = c->d_bmask.upload(c->bmask);
    if (e == hipSuccess) e = c->d_sib.upload(c->sib);
    if (e == hipSuccess) e = c->d_bg.alloc(nbf * NV * NFACE);
    if (e == hipSuccess) e = c->d_part.alloc((size_t)nblk * 4);
    if (e == hipSuccess) e = c->d_out3.alloc(4);
    if (e == hipSuccess) e = hipHostMalloc((void **)&c->h_out3, 4 * sizeof(double), hipHostMallocDefault);
    if (e != hipSuccess) {
        ccz4_destroy(c);
        return fail(e == hipErrorOutOfMemory ? CCZ4_ENOMEM : CCZ4_EHIP,
                    std::string("device tables: ") + hipGetErrorString(e));
    }
    *out = c;
    return CCZ4_OK;
}

void ccz4_destroy(ccz4_ctx *c)
{
    if (!c) return;
    (void)hipDeviceSynchronize();
    c->d_geom.release();
    c->d_tbox.release();
    c->d_phc.release();
    c->d_phn.release();
    c->d_phr.release();
    c->d_php.release();
    c->d_nbr.release();
    c->d_order.release();
    c->d_pre.release();
    c->d_bf.release();
    c->d_pface.release();
    c->d_bmask.release();
    c->d_sib.release();
    c->d_bg.release();
    c->d_part.release();
    c->d_out3.release();
    c->d_hm.release();
    if (c->h_out3) (void)hipHostFree(c->h_out3);
    delete c;
}

ccz4_status ccz4_set_params(ccz4_ctx *c, const ccz4_params *prm)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    ccz4_status st = check_params(prm);
    if (st) return st;
    c->prm = to_rhs(prm);
    return CCZ4_OK;
}

ccz4_status ccz4_layout(const ccz4_ctx *c, int64_t *n_patches, int64_t *patch_doubles, int64_t *bytes)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    if (n_patches) *n_patches = (int64_t)c->leaf.size();
    if (patch_doubles) *patch_doubles = PS;
    if (bytes) *bytes = (int64_t)c->leaf.size() * PS * (int64_t)sizeof(double);
    return CCZ4_OK;
}

ccz4_status ccz4_patch_table(const ccz4_ctx *c, int32_t *ids, double *geom)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    for (size_t p = 0; p < c->leaf.size(); ++p) {
        if (ids)
            for (int j = 0; j < 4; ++j) ids[4 * p + j] = c->leaf[p][j];
        if (geom)
            for (int a = 0; a < 3; ++a) {
                geom[6 * p + a] = c->geom[p].org[a];
                geom[6 * p + 3 + a] = c->geom[p].dx[a];
            }
    }
    return CCZ4_OK;
}

ccz4_status ccz4_init_patches(ccz4_ctx *c, double *Q, int32_t scen, const double *sp, int32_t nsp, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    ccz4_status st = check_ptr(Q, "Q");
    if (st) return st;
    const int need = scen == CCZ4_SCEN_GAUGE_WAVE ? 2 : (scen == CCZ4_SCEN_PUNCTURE ? 5 : (scen == CCZ4_SCEN_BL_BY ? 14 : -1));
    if (need < 0) return fail(CCZ4_EINVAL, "unknown scenario");
    if (nsp < need || !sp) return fail(CCZ4_EINVAL, "too few scenario parameters");
    InitArgs a{};
    for (int i = 0; i < need; ++i) a.sp[i] = sp[i];
    HIP_TRY(launch_init(Q, c->d_geom.p, c->d_bmask.p, (int32_t)c->leaf.size(), scen, a, S(stream)));
    HIP_TRY(launch_capture_bg(Q, c->d_bf.p, c->d_bg.p, (int32_t)c->bface.size(), S(stream)));
    c->bg_valid = true;
    return CCZ4_OK;
}

ccz4_status ccz4_set_background(ccz4_ctx *c, const double *Q, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    ccz4_status st = check_ptr(Q, "Q");
    if (st) return st;
    HIP_TRY(launch_capture_bg(Q, c->d_bf.p, c->d_bg.p, (int32_t)c->bface.size(), S(stream)));
    c->bg_valid = true;
    return CCZ4_OK;
}

ccz4_status ccz4_fill_halos(ccz4_ctx *c, double *Q, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    ccz4_status st = check_ptr(Q, "Q");
    if (st) return st;
    return ccz4_fill_halos_kinds(c, Q, CCZ4_FILL_ALL, stream);
}

ccz4_status ccz4_fill_halos_kinds(ccz4_ctx *c, double *Q, int32_t kinds, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    ccz4_status st = check_ptr(Q, "Q");
    if (st) return st;
    if (kinds & ~CCZ4_FILL_ALL) return fail(CCZ4_EINVAL, "unknown fill kinds");
    if (kinds & CCZ4_FILL_SAME_LEVEL) HIP_TRY(launch_fill(Q, c->d_phc.p, (int32_t)c->ph_copy.size(), c->prm.transfer, S(stream)));
    if (kinds & CCZ4_FILL_NEUMANN) HIP_TRY(launch_fill(Q, c->d_phn.p, (int32_t)c->ph_neu.size(), c->prm.transfer, S(stream)));
    if (kinds & CCZ4_FILL_LEVELS) {
        HIP_TRY(launch_fill(Q, c->d_phr.p, (int32_t)c->ph_res.size(), c->prm.transfer, S(stream)));
        HIP_TRY(launch_fill(Q, c->d_php.p, (int32_t)c->ph_pro.size(), c->prm.transfer, S(stream)));
    }
    return CCZ4_OK;
}

ccz4_status ccz4_plan_counts(const ccz4_ctx *c, int64_t *counts)
{
    if (!c || !counts) return fail(CCZ4_EINVAL, "ctx or counts is NULL");
    counts[0] = (int64_t)c->ph_copy.size();
    counts[1] = (int64_t)c->ph_neu.size();
    counts[2] = (int64_t)c->ph_res.size();
    counts[3] = (int64_t)c->ph_pro.size();
    counts[4] = (int64_t)c->bface.size();
    return CCZ4_OK;
}

// The leaf permutation of launch configuration v.
static const int32_t *order_of(const ccz4_ctx *c, int32_t v)
{
    return c->d_order.p + (size_t)((v >> KV_ORDER_SHIFT) & (KV_ORDERS - 1)) * c->leaf.size();
}

ccz4_status ccz4_rhs(ccz4_ctx *c, const double *Q, double *k, int32_t precision, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    ccz4_status st = check_ptr(Q, "Q");
    if (!st) st = check_ptr(k, "k");
    if (st) return st;
    if (Q == k) return fail(CCZ4_EINVAL, "Q and k must not alias");
    if (precision != CCZ4_PREC_FP64 && precision != CCZ4_PREC_MIXED) return fail(CCZ4_EINVAL, "bad precision");
    if (!c->bface.empty() && !c->bg_valid)
        return fail(CCZ4_ESTATE, "Sommerfeld background not set (call ccz4_init_patches or ccz4_set_background)");
    HIP_TRY(launch_rhs(Q, k, c->d_geom.p, (int32_t)c->leaf.size(), c->prm, precision, c->kernel[precision],
                       order_of(c, c->kernel[precision]), c->d_bf.p, c->d_bg.p, (int32_t)c->bface.size(),
                       c->d_pface.p, S(stream)));
    return CCZ4_OK;
}

ccz4_status ccz4_rk4_stage(ccz4_ctx *c, int32_t s, double dt, const double *Qn, const double *k, double *acc,
                           double *Qnext, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    if (s < 0 || s > 3) return fail(CCZ4_EINVAL, "stage must be 0..3");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(CCZ4_EINVAL, "dt must be finite and > 0");
    ccz4_status st = check_ptr(Qn, "Qn");
    if (!st) st = check_ptr(k, "k");
    if (!st) st = check_ptr(acc, "acc");
    if (!st) st = check_ptr(Qnext, "Qnext");
    if (st) return st;
    if (s < 3 && Qnext == Qn) return fail(CCZ4_EINVAL, "Qnext may alias Qn only at s = 3");
    HIP_TRY(launch_rk4(s, dt, Qn, k, acc, Qnext, (int32_t)c->leaf.size(), c->d_bf.p, (int32_t)c->bface.size(),
                       S(stream)));
    return CCZ4_OK;
}

// Halo handling of stage s of a fused step with kernel variant v (and of the reconstruction that
// follows it in the second-order formulation).  The LDS kernel and the reconstruction read the
// same-level y and z face halos of their input straight from the neighbours, so stages 0..2 copy
// only the x-face halos, and stage 3 copies all of them, leaving Q^{n+1} with complete halos.
// The phased kernel reads its own halos: with it every face is copied after every stage.
static int32_t step_stage_flags(const ccz4_ctx *, int32_t v, int32_t s)
{
    if (!(v & KV_LDS)) return CCZ4_STAGE_FILL_SAME_LEVEL;
    return CCZ4_STAGE_GATHER_SAME_LEVEL | (s == 3 ? CCZ4_STAGE_FILL_SAME_LEVEL : CCZ4_STAGE_FILL_SAME_LEVEL_X);
}

static hipError_t launch_reconstruct_flags(const ccz4_ctx *c, double *Q, int32_t flags, hipStream_t st)
{
    const bool push = flags & (CCZ4_STAGE_FILL_SAME_LEVEL | CCZ4_STAGE_FILL_SAME_LEVEL_X);
    return launch_reconstruct(Q, c->d_geom.p, (int32_t)c->leaf.size(), push ? c->d_nbr.p : nullptr,
                              (flags & CCZ4_STAGE_FILL_SAME_LEVEL) ? 7 : 1,
                              (flags & CCZ4_STAGE_GATHER_SAME_LEVEL) ? c->d_nbr.p : nullptr, st);
}

// One fused stage launch with the halo handling of `flags` (validated by the caller).
static hipError_t launch_stage_flags(const ccz4_ctx *c, int32_t s, double dt, const double *Qs, const double *Qn,
                                     double *acc, double *Qx, int32_t precision, int32_t variant, int32_t flags,
                                     hipStream_t st)
{
    const bool push = flags & (CCZ4_STAGE_FILL_SAME_LEVEL | CCZ4_STAGE_FILL_SAME_LEVEL_X);
    const int32_t axes = (flags & CCZ4_STAGE_FILL_SAME_LEVEL) ? 7 : 1;
    return launch_stage(s, dt, Qs, Qn, acc, Qx, c->d_geom.p, (int32_t)c->leaf.size(), c->prm, precision, variant,
                        order_of(c, variant), c->d_bf.p, c->d_bg.p, (int32_t)c->bface.size(), c->d_pface.p,
                        push ? c->d_nbr.p : nullptr, axes,
                        (flags & CCZ4_STAGE_GATHER_SAME_LEVEL) ? c->d_nbr.p : nullptr, st);
}

ccz4_status ccz4_step_stage_flags(ccz4_ctx *c, int32_t precision, int32_t s, int32_t *flags)
{
    if (!c || !flags) return fail(CCZ4_EINVAL, "ctx or flags is NULL");
    if (precision != CCZ4_PREC_FP64 && precision != CCZ4_PREC_MIXED) return fail(CCZ4_EINVAL, "bad precision");
    if (s < 0 || s > 3) return fail(CCZ4_EINVAL, "stage must be 0..3");
    *flags = step_stage_flags(c, c->kernel[precision], s);
    return CCZ4_OK;
}

ccz4_status ccz4_rhs_rk4_stage(ccz4_ctx *c, int32_t s, double dt, const double *Qs, const double *Qn, double *acc,
                               double *Qnext, int32_t precision, int32_t flags, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    if (s < 0 || s > 3) return fail(CCZ4_EINVAL, "stage must be 0..3");
    if (!(dt > 0) || !std::isfinite(dt)) return fail(CCZ4_EINVAL, "dt must be finite and > 0");
    ccz4_status st = check_ptr(Qs, "Qs");
    if (!st) st = check_ptr(Qn, "Qn");
    if (!st) st = check_ptr(acc, "acc");
    if (!st) st = check_ptr(Qnext, "Qnext");
    if (st) return st;
    if (precision != CCZ4_PREC_FP64 && precision != CCZ4_PREC_MIXED) return fail(CCZ4_EINVAL, "bad precision");
    if (flags & ~(CCZ4_STAGE_FILL_SAME_LEVEL | CCZ4_STAGE_GATHER_SAME_LEVEL | CCZ4_STAGE_FILL_SAME_LEVEL_X))
        return fail(CCZ4_EINVAL, "unknown stage flags");
    if ((flags & CCZ4_STAGE_GATHER_SAME_LEVEL) && !(c->kernel[precision] & KV_LDS))
        return fail(CCZ4_EINVAL, "CCZ4_STAGE_GATHER_SAME_LEVEL needs the LDS kernel");
    if (Qnext == Qs) return fail(CCZ4_EINVAL, "Qnext must not alias Qs");
    if (s < 3 && Qnext == Qn) return fail(CCZ4_EINVAL, "Qnext may alias Qn only at s = 3");
    if (acc == Qs || acc == Qn || acc == Qnext) return fail(CCZ4_EINVAL, "acc must not alias the states");
    if (!c->bface.empty() && !c->bg_valid)
        return fail(CCZ4_ESTATE, "Sommerfeld background not set (call ccz4_init_patches or ccz4_set_background)");
    HIP_TRY(launch_stage_flags(c, s, dt, Qs, Qn, acc, Qnext, precision, c->kernel[precision], flags, S(stream)));
    return CCZ4_OK;
}

ccz4_status ccz4_reconstruct_aux(ccz4_ctx *c, double *Q, int32_t flags, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    ccz4_status st = check_ptr(Q, "Q");
    if (st) return st;
    if (flags & ~(CCZ4_STAGE_FILL_SAME_LEVEL | CCZ4_STAGE_GATHER_SAME_LEVEL | CCZ4_STAGE_FILL_SAME_LEVEL_X))
        return fail(CCZ4_EINVAL, "unknown reconstruction flags");
    HIP_TRY(launch_reconstruct_flags(c, Q, flags, S(stream)));
    return CCZ4_OK;
}

// The point lookup of the tracer kernel: the domain corner and the cube edge of the finest level
// of the mesh (the edge as extent / (n0 * 3^top), the same rounded quotient as the leaf geometry's).
static LeafLookup leaf_lookup(const ccz4_ctx *c)
{
    LeafLookup lk{};
    for (const auto &l : c->leaf) lk.top = std::max(lk.top, (int32_t)l[0]);
    int32_t f = 1;
    for (int32_t l = 0; l < lk.top; ++l) f *= 3;
    for (int a = 0; a < 3; ++a) {
        lk.org[a] = c->origin[a];
        lk.fine[a] = c->extent[a] / (double)(c->n0[a] * f);
    }
    return lk;
}

ccz4_status ccz4_tracers_sample(ccz4_ctx *c, const double *Q, int64_t n, const double *pos, int32_t nslots,
                                const int32_t *slots, double *out, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    if (n < 0 || n > INT32_MAX) return fail(CCZ4_EINVAL, "bad number of tracers");
    if (n == 0) return CCZ4_OK;
    ccz4_status st = check_ptr(Q, "Q");
    if (st) return st;
    if (!pos || !out || !slots) return fail(CCZ4_EINVAL, "pos, slots or out is NULL");
    if (nslots < 1 || nslots > NV) return fail(CCZ4_EINVAL, "nslots must be 1..59");
    TracerSlots sl;
    sl.n = nslots;
    for (int s = 0; s < nslots; ++s) {
        if (slots[s] < 0 || slots[s] >= NV) return fail(CCZ4_EINVAL, "slot out of range");
        sl.v[s] = slots[s];
    }
    HIP_TRY(launch_tracers(Q, c->d_geom.p, (int32_t)c->leaf.size(), n, const_cast<double *>(pos), sl, leaf_lookup(c),
                           out, 0.0, 0, S(stream)));
    return CCZ4_OK;
}

ccz4_status ccz4_tracers_advance(ccz4_ctx *c, const double *Q, int64_t n, double *pos, double dt, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    if (n < 0 || n > INT32_MAX) return fail(CCZ4_EINVAL, "bad number of tracers");
    if (!std::isfinite(dt)) return fail(CCZ4_EINVAL, "dt must be finite");
    if (n == 0) return CCZ4_OK;
    ccz4_status st = check_ptr(Q, "Q");
    if (st) return st;
    if (!pos) return fail(CCZ4_EINVAL, "pos is NULL");
    TracerSlots sl;
    sl.n = 0;
    HIP_TRY(launch_tracers(Q, c->d_geom.p, (int32_t)c->leaf.size(), n, pos, sl, leaf_lookup(c), nullptr, dt, 1,
                           S(stream)));
    return CCZ4_OK;
}

ccz4_status ccz4_tag_tracers(ccz4_ctx *c, int64_t n, const double *pos, int32_t nradii, const double *radii,
                             int32_t max_level, int8_t *tags, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    if (n < 0) return fail(CCZ4_EINVAL, "bad number of tracers");
    if (!tags || (n > 0 && !pos)) return fail(CCZ4_EINVAL, "pos or tags is NULL");
    if (nradii < 0 || nradii > MAX_TRACK_LEVELS || (nradii > 0 && !radii))
        return fail(CCZ4_EINVAL, "nradii must be 0..16 with radii given");
    TrackRadii R;
    R.n = nradii;
    for (int l = 0; l < MAX_TRACK_LEVELS; ++l) R.r[l] = l < nradii ? radii[l] : 0.0;
    HIP_TRY(launch_tag_tracers(c->d_tbox.p, (int32_t)c->leaf.size(), n, pos, R, max_level, tags, S(stream)));
    return CCZ4_OK;
}

ccz4_status ccz4_set_kernel(ccz4_ctx *c, int32_t precision, int32_t kernel)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    if (precision != CCZ4_PREC_FP64 && precision != CCZ4_PREC_MIXED) return fail(CCZ4_EINVAL, "bad precision");
    if (kernel < 0 || kernel >= KV_COUNT) return fail(CCZ4_EINVAL, "unknown kernel");
    c->kernel[precision] = kernel;  // the ABI codes are the launch configurations
    return CCZ4_OK;
}

ccz4_status ccz4_get_kernel(const ccz4_ctx *c, int32_t precision, int32_t *kernel)
{
    if (!c || !kernel) return fail(CCZ4_EINVAL, "ctx or kernel is NULL");
    if (precision != CCZ4_PREC_FP64 && precision != CCZ4_PREC_MIXED) return fail(CCZ4_EINVAL, "bad precision");
    *kernel = c->kernel[precision];
    return CCZ4_OK;
}

ccz4_status ccz4_autotune(ccz4_ctx *c, const double *Q, double *acc, double *Qx, int32_t precision, int32_t reps,
                          double *ms, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    ccz4_status st = check_ptr(Q, "Q");
    if (!st) st = check_ptr(acc, "acc");
    if (!st) st = check_ptr(Qx, "Qx");
    if (st) return st;
    if (precision != CCZ4_PREC_FP64 && precision != CCZ4_PREC_MIXED) return fail(CCZ4_EINVAL, "bad precision");
    if (reps < 1) return fail(CCZ4_EINVAL, "reps must be >= 1");
    if (Q == acc || Q == Qx || acc == Qx) return fail(CCZ4_EINVAL, "Q, acc and Qx must be distinct");
    if (!c->bface.empty() && !c->bg_valid)
        return fail(CCZ4_ESTATE, "Sommerfeld background not set (call ccz4_init_patches or ccz4_set_background)");
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    hipError_t he = hipEventCreate(&e1);
    if (he != hipSuccess) {
        (void)hipEventDestroy(e0);
        return fail(CCZ4_EHIP, std::string("hipEventCreate: ") + hipGetErrorString(he));
    }
    double best = 0.0;
    int32_t pick = c->kernel[precision];
    const double dt = 1e-3;
    for (int32_t v = 0; v < KV_COUNT && he == hipSuccess; ++v) {
        // the middle stage of a step as the step graph runs it with this variant
        const int32_t fl = step_stage_flags(c, v, 1);
        auto stage = [&]() { return launch_stage_flags(c, 1, dt, Q, Q, acc, Qx, precision, v, fl, S(stream)); };
        he = stage();  // warm-up
        if (he == hipSuccess) he = hipEventRecord(e0, S(stream));
        for (int r = 0; r < reps && he == hipSuccess; ++r) he = stage();
        if (he == hipSuccess) he = hipEventRecord(e1, S(stream));
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float t = 0.f;
        if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
        const double per = (double)t / reps;
        if (ms) ms[v] = per;
        if (he == hipSuccess && (v == 0 || per < best)) {
            best = per;
            pick = v;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (he != hipSuccess) return fail(CCZ4_EHIP, std::string("autotune: ") + hipGetErrorString(he));
    c->kernel[precision] = pick;
    return CCZ4_OK;
}

// A captured fused RK4 step: four stages with same-level halo push and the Neumann / coarse-fine
// fill between them, replayed as one graph launch.
struct ccz4_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

ccz4_status ccz4_step_graph_create(ccz4_ctx *c, double *Qn, double *Q1, double *Q2, double *acc, double dt,
                                   int32_t precision, ccz4_graph **out)
{
    if (!c || !out) return fail(CCZ4_EINVAL, "ctx or out is NULL");
    *out = nullptr;
    ccz4_status st = check_ptr(Qn, "Qn");
    if (!st) st = check_ptr(Q1, "Q1");
    if (!st) st = check_ptr(Q2, "Q2");
    if (!st) st = check_ptr(acc, "acc");
    if (st) return st;
    if (!(dt > 0) || !std::isfinite(dt)) return fail(CCZ4_EINVAL, "dt must be finite and > 0");
    if (precision != CCZ4_PREC_FP64 && precision != CCZ4_PREC_MIXED) return fail(CCZ4_EINVAL, "bad precision");
    const double *bufs[4] = {Qn, Q1, Q2, acc};
    for (int i = 0; i < 4; ++i)
        for (int j = i + 1; j < 4; ++j)
            if (bufs[i] == bufs[j]) return fail(CCZ4_EINVAL, "Qn, Q1, Q2 and acc must be distinct");
    if (!c->bface.empty() && !c->bg_valid)
        return fail(CCZ4_ESTATE, "Sommerfeld background not set (call ccz4_init_patches or ccz4_set_background)");
    hipStream_t cs = nullptr;
    HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    ccz4_graph *g = new (std::nothrow) ccz4_graph;
    if (!g) {
        (void)hipStreamDestroy(cs);
        return fail(CCZ4_ENOMEM, "graph");
    }
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    double *src[4] = {Qn, Q1, Q2, Q1}, *dst[4] = {Q1, Q2, Q1, Qn};
    for (int s = 0; s < 4 && e == hipSuccess; ++s) {
        const int32_t fl = step_stage_flags(c, c->kernel[precision], s);
        e = launch_stage_flags(c, s, dt, src[s], Qn, acc, dst[s], precision, c->kernel[precision], fl, cs);
        if (e == hipSuccess) e = launch_fill(dst[s], c->d_phn.p, (int32_t)c->ph_neu.size(), c->prm.transfer, cs);
        if (e == hipSuccess) e = launch_fill(dst[s], c->d_phr.p, (int32_t)c->ph_res.size(), c->prm.transfer, cs);
        if (e == hipSuccess) e = launch_fill(dst[s], c->d_php.p, (int32_t)c->ph_pro.size(), c->prm.transfer, cs);
        if (c->prm.formulation == CCZ4_FORMULATION_SECOND_ORDER) {
            // Algorithm 2: the auxiliaries of the new state from its primaries, then their halos
            if (e == hipSuccess) e = launch_reconstruct_flags(c, dst[s], fl, cs);
            if (e == hipSuccess) e = launch_fill(dst[s], c->d_phn.p, (int32_t)c->ph_neu.size(), c->prm.transfer, cs);
            if (e == hipSuccess) e = launch_fill(dst[s], c->d_phr.p, (int32_t)c->ph_res.size(), c->prm.transfer, cs);
            if (e == hipSuccess) e = launch_fill(dst[s], c->d_php.p, (int32_t)c->ph_pro.size(), c->prm.transfer, cs);
        }
    }
    hipError_t e2 = hipStreamEndCapture(cs, &g->graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0);
    (void)hipStreamDestroy(cs);
    if (e != hipSuccess) {
        ccz4_step_graph_destroy(g);
        return fail(CCZ4_EHIP, std::string("step graph: ") + hipGetErrorString(e));
    }
    *out = g;
    return CCZ4_OK;
}

ccz4_status ccz4_step_graph_launch(ccz4_graph *g, void *stream)
{
    if (!g || !g->exec) return fail(CCZ4_EINVAL, "graph is NULL");
    HIP_TRY(hipGraphLaunch(g->exec, S(stream)));
    return CCZ4_OK;
}

void ccz4_step_graph_destroy(ccz4_graph *g)
{
    if (!g) return;
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

namespace {

// face neighbour of cube (l, c) along axis a, side sd (periodic wrap); false if outside
bool face_nb(const ccz4_ctx *c, int l, const int cu[3], int a, int sd, int nb[3])
{
    const int na = level_n(c, l, a);
    nb[0] = cu[0];
    nb[1] = cu[1];
    nb[2] = cu[2];
    nb[a] += sd;
    if (nb[a] < 0 || nb[a] >= na) {
        if (c->bc != CCZ4_BC_PERIODIC) return false;
        nb[a] = (nb[a] + na) % na;
    }
    return true;
}

}  // namespace

ccz4_status ccz4_regrid_plan(const ccz4_ctx *c, const int8_t *tags, int32_t max_level, int32_t *refined_out,
                             int64_t cap, int64_t *n_out)
{
    if (!c || !tags || !n_out) return fail(CCZ4_EINVAL, "ctx, tags or n_out is NULL");
    if (max_level < 0 || max_level > 12) return fail(CCZ4_EINVAL, "max_level out of range");
    std::unordered_set<uint64_t> R;
    for (const auto &cu : c->refined) R.insert(key(cu[0], cu[1], cu[2], cu[3]));
    auto has = [&](int l, int i, int j, int k) { return R.count(key(l, i, j, k)) > 0; };
    std::vector<std::array<int, 4>> cubes(c->refined);
    auto add = [&](int l, int i, int j, int k) {
        if (R.insert(key(l, i, j, k)).second) cubes.push_back({l, i, j, k});
    };
    auto leaf_of = [&](int l, int i, int j, int k) -> int {
        auto it = c->index.find(key(l, i, j, k));
        return it == c->index.end() ? -1 : it->second;
    };
    const size_t np = c->leaf.size();
    for (size_t p = 0; p < np; ++p)
        if (tags[p] == 1 && c->leaf[p][0] < max_level) add(c->leaf[p][0], c->leaf[p][1], c->leaf[p][2], c->leaf[p][3]);
    // coarsening of families whose 27 leaves all ask for it, unless a neighbour stays refined
    for (const auto &P : c->refined) {
        const int L = P[0] + 1;
        bool all = true;
        for (int w = 0; w < 3 && all; ++w)
            for (int v = 0; v < 3 && all; ++v)
                for (int u = 0; u < 3 && all; ++u) {
                    const int q = leaf_of(L, 3 * P[1] + u, 3 * P[2] + v, 3 * P[3] + w);
                    if (q < 0 || tags[q] != -1) all = false;
                }
        for (int w = 0; w < 3 && all; ++w)
            for (int v = 0; v < 3 && all; ++v)
                for (int u = 0; u < 3 && all; ++u) {
                    const int ch[3] = {3 * P[1] + u, 3 * P[2] + v, 3 * P[3] + w};
                    for (int a = 0; a < 3 && all; ++a)
                        for (int sd = -1; sd <= 1 && all; sd += 2) {
                            int nb[3];
                            if (!face_nb(c, L, ch, a, sd, nb)) continue;
                            if (nb[0] / 3 == P[1] && nb[1] / 3 == P[2] && nb[2] / 3 == P[3]) continue;
                            if (has(L, nb[0], nb[1], nb[2])) all = false;
                        }
                }
        if (all) R.erase(key(P[0], P[1], P[2], P[3]));
    }
    // balance: the face neighbours of a refined cube of level L >= 1 have refined parents
    bool changed = true;
    while (changed) {
        changed = false;
        for (size_t r = 0; r < cubes.size(); ++r) {
            const auto cu = cubes[r];
            if (!has(cu[0], cu[1], cu[2], cu[3]) || cu[0] == 0) continue;
            const int ci[3] = {cu[1], cu[2], cu[3]};
            for (int a = 0; a < 3; ++a)
                for (int sd = -1; sd <= 1; sd += 2) {
                    int nb[3];
                    if (!face_nb(c, cu[0], ci, a, sd, nb)) continue;
                    if (!has(cu[0] - 1, nb[0] / 3, nb[1] / 3, nb[2] / 3)) {
                        add(cu[0] - 1, nb[0] / 3, nb[1] / 3, nb[2] / 3);
                        changed = true;
                    }
                }
        }
    }
    std::vector<std::array<int, 4>> outv;
    for (const auto &cu : cubes)
        if (has(cu[0], cu[1], cu[2], cu[3])) outv.push_back(cu);
    std::sort(outv.begin(), outv.end());
    outv.erase(std::unique(outv.begin(), outv.end()), outv.end());
    std::sort(outv.begin(), outv.end(), [](const std::array<int, 4> &x, const std::array<int, 4> &y) {
        if (x[0] != y[0]) return x[0] < y[0];
        if (x[3] != y[3]) return x[3] < y[3];
        if (x[2] != y[2]) return x[2] < y[2];
        return x[1] < y[1];
    });
    *n_out = (int64_t)outv.size();
    if ((int64_t)outv.size() > cap) return fail(CCZ4_EINVAL, "refined_out too small (see n_out)");
    if (!refined_out && !outv.empty()) return fail(CCZ4_EINVAL, "refined_out is NULL");
    for (size_t r = 0; r < outv.size(); ++r)
        for (int q = 0; q < 4; ++q) refined_out[4 * r + q] = outv[r][q];
    return CCZ4_OK;
}

ccz4_status ccz4_regrid_transfer(const ccz4_ctx *co, const double *Qo, const ccz4_ctx *cn, double *Qn, void *stream)
{
    if (!co || !cn) return fail(CCZ4_EINVAL, "ctx is NULL");
    ccz4_status st = check_ptr(Qo, "Qold");
    if (!st) st = check_ptr(Qn, "Qnew");
    if (st) return st;
    if (Qo == Qn) return fail(CCZ4_EINVAL, "Qold and Qnew must differ");
    for (int a = 0; a < 3; ++a)
        if (co->n0[a] != cn->n0[a] || co->origin[a] != cn->origin[a] || co->extent[a] != cn->extent[a])
            return fail(CCZ4_EINVAL, "meshes of different domains");
    auto leaf_of = [&](int l, int i, int j, int k) -> int {
        auto it = co->index.find(key(l, i, j, k));
        return it == co->index.end() ? -1 : it->second;
    };
    std::vector<RegridTask> tasks(cn->leaf.size());
    for (size_t p = 0; p < cn->leaf.size(); ++p) {
        const auto &lf = cn->leaf[p];
        RegridTask &t = tasks[p];
        std::memset(&t, 0, sizeof(t));
        const int same = leaf_of(lf[0], lf[1], lf[2], lf[3]);
        if (same >= 0) {
            t.kind = RG_COPY;
            t.src = same;
            continue;
        }
        const int par = lf[0] > 0 ? leaf_of(lf[0] - 1, lf[1] / 3, lf[2] / 3, lf[3] / 3) : -1;
        if (par >= 0) {
            t.kind = RG_PROLONG;
            t.src = par;
            for (int a = 0; a < 3; ++a) t.o[a] = lf[1 + a] % 3;
            continue;
        }
        t.kind = RG_RESTRICT;
        for (int w = 0; w < 3; ++w)
            for (int v = 0; v < 3; ++v)
                for (int u = 0; u < 3; ++u) {
                    const int kid = leaf_of(lf[0] + 1, 3 * lf[1] + u, 3 * lf[2] + v, 3 * lf[3] + w);
                    if (kid < 0) return fail(CCZ4_ELAYOUT, "new leaf neither kept, inside an old leaf, nor covering 27");
                    t.kid[w * 9 + v * 3 + u] = kid;
                }
    }
    DevBuf<RegridTask> d;
    HIP_TRY(d.upload(tasks));
    HIP_TRY(launch_regrid(Qo, Qn, d.p, (int32_t)tasks.size(), S(stream)));
    HIP_TRY(hipStreamSynchronize(S(stream)));  // the task table is released on return
    return CCZ4_OK;
}

ccz4_status ccz4_features(ccz4_ctx *c, const double *Q, const double *HM, float *feat, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    ccz4_status st = check_ptr(Q, "Q");
    if (!st) st = check_ptr(HM, "HM");
    if (!st) st = check_ptr(feat, "feat");
    if (st) return st;
    HIP_TRY(launch_features(Q, HM, c->d_geom.p, (int32_t)c->leaf.size(), feat, S(stream)));
    return CCZ4_OK;
}

ccz4_status ccz4_mlp_forward(const float *params, const float *norm, const float *feat, int64_t n, float *logits,
                             void *stream)
{
    if (!params || !norm || !logits || (n > 0 && !feat)) return fail(CCZ4_EINVAL, "NULL buffer");
    if (n < 0) return fail(CCZ4_EINVAL, "n < 0");
    HIP_TRY(launch_mlp_forward(params, norm, feat, n, logits, S(stream)));
    return CCZ4_OK;
}

ccz4_status ccz4_mlp_workspace(int64_t n, int64_t *floats)
{
    if (!floats || n < 0) return fail(CCZ4_EINVAL, "bad arguments");
    *floats = (int64_t)(n > 0 ? mlp_tiles(n) : 0) * (MLP_NPARAM + 1);
    return CCZ4_OK;
}

ccz4_status ccz4_mlp_grad(const float *params, const float *norm, const float *feat, const int8_t *tags, int64_t n,
                          float *work, int64_t work_floats, float *grad, float *loss, void *stream)
{
    if (!params || !norm || !feat || !tags || !work || !grad) return fail(CCZ4_EINVAL, "NULL buffer");
    if (n <= 0) return fail(CCZ4_EINVAL, "n must be > 0");
    const int64_t base = (int64_t)mlp_tiles(n) * (MLP_NPARAM + 1);
    if (work_floats < base) return fail(CCZ4_EINVAL, "workspace too small");
    float *trace = work_floats >= base + (int64_t)MLP_TRACE * n ? work + base : nullptr;
    HIP_TRY(launch_mlp_grad(params, norm, feat, tags, n, work, trace, grad, loss, S(stream)));
    return CCZ4_OK;
}

ccz4_status ccz4_mlp_grad_noalloc(const float *params, const float *norm, const float *feat, const int8_t *tags,
                                  int64_t n, float *grad, float *loss, void *stream)
{
    if (!params || !norm || !feat || !tags || !grad) return fail(CCZ4_EINVAL, "NULL buffer");
    if (n <= 0) return fail(CCZ4_EINVAL, "n must be > 0");
    if (n > (int64_t)MLP_SCRATCH_TILES * 64)
        return fail(CCZ4_EINVAL, "n exceeds CCZ4_MLP_NOALLOC_MAX_ROWS (" + std::to_string(MLP_SCRATCH_TILES * 64) +
                                     "): use ccz4_mlp_grad with a workspace");
    float *work = nullptr;
    HIP_TRY(mlp_scratch(&work));
    HIP_TRY(launch_mlp_grad(params, norm, feat, tags, n, work, nullptr, grad, loss, S(stream)));
    return CCZ4_OK;
}

ccz4_status ccz4_mlp_adam(float *params, float *m, float *v, const float *grad, int32_t step, float lr, float beta1,
                          float beta2, float eps, void *stream)
{
    if (!params || !m || !v || !grad) return fail(CCZ4_EINVAL, "NULL buffer");
    if (step < 1 || !(lr > 0) || !(beta1 >= 0 && beta1 < 1) || !(beta2 >= 0 && beta2 < 1) || !(eps > 0))
        return fail(CCZ4_EINVAL, "bad Adam hyper-parameters");
    const double c1 = 1.0 - std::pow((double)beta1, step), c2 = 1.0 - std::pow((double)beta2, step);
    HIP_TRY(launch_mlp_adam(params, m, v, grad, lr, beta1, beta2, eps, (float)c1, (float)c2, S(stream)));
    return CCZ4_OK;
}

ccz4_status ccz4_tag_learned(ccz4_ctx *c, const float *logits, const int8_t *plain_tags, float conf, int32_t max_level,
                             int8_t *tags, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    if (!logits || !plain_tags || !tags) return fail(CCZ4_EINVAL, "NULL buffer");
    if (!(conf >= 0 && conf <= 1)) return fail(CCZ4_EINVAL, "conf must lie in [0, 1]");
    HIP_TRY(launch_tag_learned(logits, plain_tags, c->d_geom.p, c->d_sib.p, (int32_t)c->leaf.size(), conf, max_level,
                               c->d_pre.p, tags, S(stream)));
    return CCZ4_OK;
}

ccz4_status ccz4_constraints(ccz4_ctx *c, const double *Q, double *HM, double r_excise, double *norms, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    ccz4_status st = check_ptr(Q, "Q");
    if (st) return st;
    HIP_TRY(launch_constraints(Q, HM, c->d_geom.p, (int32_t)c->leaf.size(), r_excise, c->d_part.p, c->d_out3.p,
                               S(stream)));
    if (!norms) return CCZ4_OK;
    HIP_TRY(hipMemcpyAsync(c->h_out3, c->d_out3.p, 3 * sizeof(double), hipMemcpyDeviceToHost, S(stream)));
    HIP_TRY(hipStreamSynchronize(S(stream)));
    for (int j = 0; j < 3; ++j) norms[j] = c->h_out3[j];
    if (norms[2] > 0) return fail(CCZ4_ENONFINITE, "non-finite values in the state or the constraints");
    return CCZ4_OK;
}

ccz4_status ccz4_tag_refine(ccz4_ctx *c, const double *Q, double theta_r, double theta_c, int32_t max_level,
                            int8_t *tags, double *indicator, void *stream)
{
    if (!c) return fail(CCZ4_EINVAL, "ctx is NULL");
    ccz4_status st = check_ptr(Q, "Q");
    if (st) return st;
    if (!tags) return fail(CCZ4_EINVAL, "tags is NULL");
    const size_t np = c->leaf.size();
    if (c->d_hm.n < np * 4 * NCELL) HIP_TRY(c->d_hm.alloc(np * 4 * NCELL));
    double *ind = indicator;
    DevBuf<double> tmp;
    if (!ind) {
        HIP_TRY(tmp.alloc(np * 3));
        ind = tmp.p;
    }
    HIP_TRY(launch_constraints(Q, c->d_hm.p, c->d_geom.p, (int32_t)np, 0.0, c->d_part.p, c->d_out3.p, S(stream)));
    HIP_TRY(launch_tags(Q, c->d_hm.p, c->d_geom.p, c->d_sib.p, (int32_t)np, theta_r, theta_c, max_level, tags, ind,
                        S(stream)));
    if (tmp.p) {
        HIP_TRY(hipStreamSynchronize(S(stream)));
        tmp.release();
    }
    return CCZ4_OK;
}

}  // extern "C"
