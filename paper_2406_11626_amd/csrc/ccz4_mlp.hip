// Learned refinement indicator on gfx950: per-patch features, a 81 -> 64 -> 64 -> 3 perceptron
// on BF16 matrix cores (v_mfma_f32_16x16x16_bf16, FP32 accumulation) with its loss gradient,
// an Adam step on FP32 master weights, and the combination with the plain criterion.
//
// Parameter vector (NPARAM = 9603 floats), row-major, out x in:
//   W1[64][81] b1[64] W2[64][64] b2[64] W3[3][64] b3[3]
// The inputs are standardised in FP32, x = (feat - mu) * inv_sigma, then rounded to BF16 with
// the weights; hidden activations are rounded to BF16 after the ReLU; in the backward pass the
// pre-activation gradients entering a product are rounded to BF16 and the roundings are taken
// as the identity (straight-through).  The bias gradients sum the FP32 gradients.
#include <hip/hip_runtime.h>

#include <mutex>

#include "ccz4_kernels.hpp"
#include "ccz4_mlp.hpp"

namespace ccz4 {

namespace {

constexpr int NIN = MLP_NIN, NINP = 96, NH = MLP_NH, NOUT = MLP_NOUT, NOUTP = 16;
constexpr int OW1 = 0, OB1 = OW1 + NH * NIN, OW2 = OB1 + NH, OB2 = OW2 + NH * NH, OW3 = OB2 + NH,
              OB3 = OW3 + NOUT * NH;
static_assert(OB3 + NOUT == MLP_NPARAM, "parameter layout");
constexpr int TILE = 64;  // rows (patches) per work-group, 16 per wave

typedef short bf4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// FP32 -> BF16, round to nearest, ties to even (NaN -> quiet NaN)
__device__ __forceinline__ float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

__device__ __forceinline__ uint16_t f2bf(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u & 0x007fffffu) ? (uint16_t)0x7fc0 : (uint16_t)(u >> 16);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// One 16 x 16 output tile of C = A B over K (a multiple of 16) on the matrix cores.  A(i, k) and
// B(k, j) return BF16 bits; lane l supplies A rows l % 16 and B columns l % 16 at the four k of
// its group l / 16; the result element r of lane l is C(4 (l / 16) + r, l % 16).
template <typename FA, typename FB>
__device__ __forceinline__ f4_t mma_tile(FA A, FB B, int K)
{
    const int l = threadIdx.x & 63, li = l & 15, lk = (l >> 4) * 4;
    f4_t acc = {0.f, 0.f, 0.f, 0.f};
    for (int k0 = 0; k0 < K; k0 += 16) {
        bf4_t a, b;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            a[r] = (short)A(li, k0 + lk + r);
            b[r] = (short)B(k0 + lk + r, li);
        }
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, acc, 0, 0, 0);
    }
    return acc;
}

struct MlpShared {
    uint16_t w1[NH][NINP];    // W1, inputs padded to 96
    uint16_t w2[NH][NH];
    uint16_t w3[NOUTP][NH];   // W3, outputs padded to 16
    uint16_t x[TILE][NINP];   // standardised inputs
    uint16_t a1[TILE][NH];    // BF16 hidden activations
    uint16_t a2[TILE][NH];
    float z1[TILE][NH];       // FP32 pre-activations (ReLU masks of the backward pass)
    float z2[TILE][NH];
    float z3[TILE][NOUTP];
    uint16_t db[TILE][NH];    // BF16 pre-activation gradient of the current layer
    float part[TILE];         // per-row loss
};

// forward pass of one tile of rows [r0, r0 + TILE); returns with z3 (logits) in LDS
__device__ void mlp_forward_tile(MlpShared &S, const float *__restrict__ prm, const float *__restrict__ norm,
                                 const float *__restrict__ feat, int64_t n, int64_t r0)
{
    const int t = threadIdx.x, w = t >> 6, l = t & 63, li = l & 15, lk = (l >> 4) * 4;
    for (int e = t; e < NH * NINP; e += blockDim.x) {
        const int j = e / NINP, i = e % NINP;
        S.w1[j][i] = i < NIN ? f2bf(prm[OW1 + j * NIN + i]) : (uint16_t)0;
    }
    for (int e = t; e < NH * NH; e += blockDim.x) S.w2[e / NH][e % NH] = f2bf(prm[OW2 + e]);
    for (int e = t; e < NOUTP * NH; e += blockDim.x) {
        const int j = e / NH, i = e % NH;
        S.w3[j][i] = j < NOUT ? f2bf(prm[OW3 + j * NH + i]) : (uint16_t)0;
    }
    for (int e = t; e < TILE * NINP; e += blockDim.x) {
        const int r = e / NINP, i = e % NINP;
        uint16_t v = 0;
        if (i < NIN && r0 + r < n) {
#pragma clang fp contract(off)
            const float d = feat[(r0 + r) * NIN + i] - norm[i];
            v = f2bf(d * norm[NIN + i]);
        }
        S.x[r][i] = v;
    }
    __syncthreads();
    // layer 1: rows 16 w .. 16 w + 15 of the tile, four column tiles of 16 hidden units
    for (int jb = 0; jb < 4; ++jb) {
        const f4_t c = mma_tile([&](int i, int k) { return S.x[16 * w + i][k]; },
                                [&](int k, int j) { return S.w1[16 * jb + j][k]; }, NINP);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * w + lk + r, col = 16 * jb + li;
            const float z = c[r] + prm[OB1 + col];
            S.z1[row][col] = z;
            S.a1[row][col] = f2bf(z > 0.f ? z : 0.f);
        }
    }
    __syncthreads();
    for (int jb = 0; jb < 4; ++jb) {
        const f4_t c = mma_tile([&](int i, int k) { return S.a1[16 * w + i][k]; },
                                [&](int k, int j) { return S.w2[16 * jb + j][k]; }, NH);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * w + lk + r, col = 16 * jb + li;
            const float z = c[r] + prm[OB2 + col];
            S.z2[row][col] = z;
            S.a2[row][col] = f2bf(z > 0.f ? z : 0.f);
        }
    }
    __syncthreads();
    {
        const f4_t c = mma_tile([&](int i, int k) { return S.a2[16 * w + i][k]; },
                                [&](int k, int j) { return S.w3[j][k]; }, NH);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * w + lk + r, col = li;
            S.z3[row][col] = col < NOUT ? c[r] + prm[OB3 + col] : 0.f;
        }
    }
    __syncthreads();
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ prm, const float *__restrict__ norm,
                                                     const float *__restrict__ feat, int64_t n,
                                                     float *__restrict__ logits)
{
    __shared__ MlpShared S;
    const int64_t r0 = (int64_t)blockIdx.x * TILE;
    mlp_forward_tile(S, prm, norm, feat, n, r0);
    for (int e = threadIdx.x; e < TILE * NOUT; e += blockDim.x) {
        const int r = e / NOUT, j = e % NOUT;
        if (r0 + r < n) logits[(r0 + r) * NOUT + j] = S.z3[r][j];
    }
}

// Loss and gradient partials of one tile: part[blk][0 .. NPARAM-1] gradient, [NPARAM] loss sum.
// With trace != nullptr, each row also leaves the operands of its matrix products there (as FP32
// values, MLP_TRACE per row): the BF16 standardised input, the BF16 activations a1 and a2, and the
// FP32 pre-activation gradients d3, d2 and d1 before their BF16 rounding.
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ prm, const float *__restrict__ norm,
                                                  const float *__restrict__ feat, const int8_t *__restrict__ tags,
                                                  int64_t n, float *__restrict__ part, float *__restrict__ trace)
{
    __shared__ MlpShared S;
    __shared__ float d3[TILE][NOUTP];
    __shared__ float dsum[NH];
    const int64_t r0 = (int64_t)blockIdx.x * TILE;
    const int t = threadIdx.x, w = t >> 6, l = t & 63, li = l & 15, lk = (l >> 4) * 4;
    float *out = part + (int64_t)blockIdx.x * (MLP_NPARAM + 1);
    mlp_forward_tile(S, prm, norm, feat, n, r0);
    if (trace) {
        for (int e = t; e < TILE * (NIN + 2 * NH); e += blockDim.x) {
            const int r = e / (NIN + 2 * NH), i = e % (NIN + 2 * NH);
            if (r0 + r >= n) continue;
            const uint16_t b = i < NIN ? S.x[r][i] : (i < NIN + NH ? S.a1[r][i - NIN] : S.a2[r][i - NIN - NH]);
            trace[(r0 + r) * MLP_TRACE + i] = bf2f(b);
        }
    }
    const float inv_n = 1.0f / (float)n;
    // softmax cross-entropy per row
    if (t < TILE) {
        float lossr = 0.f;
        float d[NOUT] = {0.f, 0.f, 0.f};
        if (r0 + t < n) {
            const int lab = (int)tags[r0 + t] + 1;  // COARSEN, KEEP, REFINE -> 0, 1, 2
            const float zm = fmaxf(fmaxf(S.z3[t][0], S.z3[t][1]), S.z3[t][2]);
            float e[NOUT], se = 0.f;
#pragma unroll
            for (int j = 0; j < NOUT; ++j) {
                e[j] = expf(S.z3[t][j] - zm);
                se += e[j];
            }
            lossr = -(S.z3[t][lab] - zm - logf(se));
#pragma unroll
            for (int j = 0; j < NOUT; ++j) d[j] = (e[j] / se - (j == lab ? 1.f : 0.f)) * inv_n;
        }
        S.part[t] = lossr;
#pragma unroll
        for (int j = 0; j < NOUTP; ++j) {
            d3[t][j] = j < NOUT ? d[j] : 0.f;
            S.db[t][j] = j < NOUT ? f2bf(d[j]) : (uint16_t)0;
        }
        if (trace && r0 + t < n)
#pragma unroll
            for (int j = 0; j < NOUT; ++j) trace[(r0 + t) * MLP_TRACE + NIN + 2 * NH + j] = d[j];
    }
    __syncthreads();
    if (t == 0) {
        float s = 0.f;
        for (int r = 0; r < TILE; ++r) s += S.part[r];
        out[MLP_NPARAM] = s;
    }
    if (t < NOUT) {
        float s = 0.f;
        for (int r = 0; r < TILE; ++r) s += d3[r][t];
        out[OB3 + t] = s;
    }
    // gW3[j][h] = sum_rows d3b[row][j] a2[row][h]: wave w takes hidden units 16 w .. 16 w + 15
    {
        const f4_t c = mma_tile([&](int i, int k) { return S.db[k][i]; },
                                [&](int k, int j) { return S.a2[k][16 * w + j]; }, TILE);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int j = lk + r, h = 16 * w + li;
            if (j < NOUT) out[OW3 + j * NH + h] = c[r];
        }
    }
    // d2 = (d3b W3) * [z2 > 0]
    float d2v[4][4];
    for (int hb = 0; hb < 4; ++hb) {
        const f4_t c = mma_tile([&](int i, int k) { return S.db[16 * w + i][k]; },
                                [&](int k, int j) { return S.w3[k][16 * hb + j]; }, NOUTP);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * w + lk + r, h = 16 * hb + li;
            d2v[hb][r] = S.z2[row][h] > 0.f ? c[r] : 0.f;
        }
    }
    __syncthreads();  // every wave is done reading d3b
    for (int hb = 0; hb < 4; ++hb)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * w + lk + r, h = 16 * hb + li;
            S.z2[row][h] = d2v[hb][r];  // z2 is no longer needed: keep the FP32 d2 there
            S.db[row][h] = f2bf(d2v[hb][r]);
        }
    __syncthreads();
    if (t < NH) {
        float s = 0.f;
        for (int r = 0; r < TILE; ++r) s += S.z2[r][t];
        dsum[t] = s;
    }
    if (trace)
        for (int e = t; e < TILE * NH; e += blockDim.x) {
            const int r = e / NH, h = e % NH;
            if (r0 + r < n) trace[(r0 + r) * MLP_TRACE + NIN + 2 * NH + NOUT + h] = S.z2[r][h];
        }
    // gW2[o][i] = sum_rows d2b[row][o] a1[row][i]: 16 tiles, four per wave
    for (int q = 0; q < 4; ++q) {
        const int ob = w, ib = q;
        const f4_t c = mma_tile([&](int i, int k) { return S.db[k][16 * ob + i]; },
                                [&](int k, int j) { return S.a1[k][16 * ib + j]; }, TILE);
#pragma unroll
        for (int r = 0; r < 4; ++r) out[OW2 + (16 * ob + lk + r) * NH + 16 * ib + li] = c[r];
    }
    __syncthreads();
    if (t < NH) out[OB2 + t] = dsum[t];
    // d1 = (d2b W2) * [z1 > 0]
    float d1v[4][4];
    for (int ib = 0; ib < 4; ++ib) {
        const f4_t c = mma_tile([&](int i, int k) { return S.db[16 * w + i][k]; },
                                [&](int k, int j) { return S.w2[k][16 * ib + j]; }, NH);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * w + lk + r, h = 16 * ib + li;
            d1v[ib][r] = S.z1[row][h] > 0.f ? c[r] : 0.f;
        }
    }
    __syncthreads();
    for (int ib = 0; ib < 4; ++ib)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int row = 16 * w + lk + r, h = 16 * ib + li;
            S.z1[row][h] = d1v[ib][r];
            S.db[row][h] = f2bf(d1v[ib][r]);
        }
    __syncthreads();
    if (t < NH) {
        float s = 0.f;
        for (int r = 0; r < TILE; ++r) s += S.z1[r][t];
        out[OB1 + t] = s;
    }
    if (trace)
        for (int e = t; e < TILE * NH; e += blockDim.x) {
            const int r = e / NH, h = e % NH;
            if (r0 + r < n) trace[(r0 + r) * MLP_TRACE + NIN + 3 * NH + NOUT + h] = S.z1[r][h];
        }
    // gW1[o][i] = sum_rows d1b[row][o] x[row][i]: 4 x 6 tiles, six per wave
    for (int q = 0; q < 6; ++q) {
        const int ob = w, ib = q;
        const f4_t c = mma_tile([&](int i, int k) { return S.db[k][16 * ob + i]; },
                                [&](int k, int j) { return S.x[k][16 * ib + j]; }, TILE);
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = 16 * ib + li;
            if (i < NIN) out[OW1 + (16 * ob + lk + r) * NIN + i] = c[r];
        }
    }
}

// The per-tile partials are summed in two levels, each in a fixed order (deterministic): first the
// tiles of each chunk of MLP_RCHUNK consecutive tiles, in place into the chunk's first row (every
// column of a chunk's rows is read and written by one thread only), then the chunks' rows.  One
// sequential sum over all tiles ran on a few dozen work-groups and took 0.9 ms for 3771 tiles.
constexpr int MLP_RCHUNK = 64;

__global__ void k_mlp_reduce_chunks(float *__restrict__ part, int32_t ntile)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q > MLP_NPARAM) return;
    const int32_t b0 = blockIdx.y * MLP_RCHUNK;
    const int32_t b1 = min(b0 + MLP_RCHUNK, ntile);
    float s = 0.f;
    for (int32_t b = b0; b < b1; ++b) s += part[(int64_t)b * (MLP_NPARAM + 1) + q];
    part[(int64_t)b0 * (MLP_NPARAM + 1) + q] = s;
}

// grad[q] = the sum of the chunks' rows of column q (q = NPARAM: the loss, divided by n)
__global__ void k_mlp_reduce(const float *__restrict__ part, int32_t ntile, int64_t n, float *__restrict__ grad,
                             float *__restrict__ loss)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q > MLP_NPARAM) return;
    float s = 0.f;
    for (int32_t b = 0; b < ntile; b += MLP_RCHUNK) s += part[(int64_t)b * (MLP_NPARAM + 1) + q];
    if (q < MLP_NPARAM) grad[q] = s;
    else if (loss) *loss = s / (float)n;
}

__global__ void k_mlp_adam(float *__restrict__ p, float *__restrict__ m, float *__restrict__ v,
                           const float *__restrict__ g, float lr, float b1, float b2, float eps, float c1, float c2)
{
    const int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= MLP_NPARAM) return;
    const float gq = g[q];
    const float mq = b1 * m[q] + (1.f - b1) * gq;
    const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
    m[q] = mq;
    v[q] = vq;
    p[q] -= lr * (mq / c1) / (sqrtf(vq / c2) + eps);
}

// Features: one work-group per patch, one thread per interior cell; the indicators are scaled
// by the patch spacing (dx |grad chi|, dx |grad alpha|, dx^2 |H|) like the plain criterion's.
__global__ __launch_bounds__(256) void k_features(const double *__restrict__ Q, const double *__restrict__ HM,
                                                  const PatchGeom *__restrict__ geom, float *__restrict__ feat)
{
    __shared__ double cellv[NCELL * 3];  // per interior cell: |grad chi|, |grad alpha|, |H|
    const int p = blockIdx.x, t = threadIdx.x;
    const PatchGeom g = geom[p];
    const double *qp = Q + (int64_t)p * PS;
    __shared__ double mx[27][3];
    if (t < 81) mx[t / 3][t % 3] = 0.0;
    for (int c = t; c < NCELL; c += blockDim.x) {
        const int x = c % 9 + 3, y = (c / 9) % 9 + 3, z = c / 81 + 3;
        const int o = boff(x, y, z);
        double gc = 0.0, ga = 0.0;
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const int s = a == 0 ? 1 : (a == 1 ? YS : ZS);
            double wc[5], wa[5];
#pragma unroll
            for (int k = -2; k <= 2; ++k) {
                const double ph = qp[SPHI * CS + o + k * s];
                wc[k + 2] = ph * ph;
                wa[k + 2] = qp[SALPHA * CS + o + k * s];
            }
            const double i12 = 1.0 / (12.0 * g.dx[a]);
            const double dc = (8.0 * (wc[3] - wc[1]) - (wc[4] - wc[0])) * i12;
            const double da = (8.0 * (wa[3] - wa[1]) - (wa[4] - wa[0])) * i12;
            gc += dc * dc;
            ga += da * da;
        }
        cellv[3 * c + 0] = g.dx[0] * sqrt(gc);
        cellv[3 * c + 1] = g.dx[0] * sqrt(ga);
        cellv[3 * c + 2] = g.dx[0] * g.dx[0] * fabs(HM[((int64_t)p * 4 + 0) * NCELL + c]);
    }
    __syncthreads();
    if (t < 81) {
        const int b = t / 3, q = t % 3;
        const int bx = b % 3, by = (b / 3) % 3, bz = b / 9;
        double m = 0.0;
        for (int dz = 0; dz < 3; ++dz)
            for (int dy = 0; dy < 3; ++dy)
                for (int dx = 0; dx < 3; ++dx) {
                    const int c = ((3 * bz + dz) * 9 + 3 * by + dy) * 9 + 3 * bx + dx;
                    m = fmax(m, cellv[3 * c + q]);
                }
        feat[(int64_t)p * NIN + 3 * b + q] = (float)log10(m + 1e-12);
    }
}

// Learned tags, first pass: plain REFINE is kept; a confident learned REFINE is added (below
// max_level); a plain COARSEN survives unless the network is confident that the patch is not
// to be coarsened (pre = -1 marks the surviving candidates).
__global__ void k_tag_learned_pre(const float *__restrict__ logits, const int8_t *__restrict__ plain,
                                  const PatchGeom *__restrict__ geom, int32_t npatch, float conf, int32_t max_level,
                                  int8_t *__restrict__ pre)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npatch) return;
    const float z0 = logits[3 * p], z1 = logits[3 * p + 1], z2 = logits[3 * p + 2];
    const float zm = fmaxf(fmaxf(z0, z1), z2);
    const float e0 = expf(z0 - zm), e1 = expf(z1 - zm), e2 = expf(z2 - zm);
    const float pm = 1.0f / (e0 + e1 + e2);  // probability of the arg-max class (its e is 1)
    const int cls = z2 >= zm ? 1 : (z1 >= zm ? 0 : -1);  // ties go to the higher class
    const bool sure = pm >= conf;
    int8_t tg = 0;
    if (plain[p] == 1) tg = 1;
    else if (sure && cls == 1 && geom[p].level < max_level) tg = 1;
    else if (plain[p] == -1 && !(sure && cls != -1)) tg = -1;
    pre[p] = tg;
}

// second pass: a family coarsens only if all 27 of its leaves are coarsening candidates
__global__ void k_tag_learned_family(const int8_t *__restrict__ pre, const int32_t *__restrict__ sib,
                                     int32_t npatch, int8_t *__restrict__ tags)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npatch) return;
    int8_t tg = pre[p];
    if (tg == -1) {
        for (int n = 0; n < 27; ++n) {
            const int s = sib[(int64_t)p * 27 + n];
            if (s < 0 || pre[s] != -1) {
                tg = 0;
                break;
            }
        }
    }
    tags[p] = tg;
}

}  // namespace

int32_t mlp_tiles(int64_t n) { return (int32_t)((n + TILE - 1) / TILE); }

// Per-tile partial sums of the loss gradient for callers that cannot allocate a workspace: a
// file-scope device array, one copy per GPU, held until the process ends.  Its device address is
// taken once per device with hipGetSymbolAddress (the array's name is not a device address in
// host code) and kept; kernels receive that address.  Every grad call on a GPU shares the array.
__device__ __align__(256) float scratch[MLP_SCRATCH_TILES * (MLP_NPARAM + 1)];

hipError_t mlp_scratch(float **out)
{
    constexpr int MAXDEV = 64;
    static std::mutex mu;
    static float *addr[MAXDEV] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= MAXDEV) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = static_cast<float *>(ptr);
    }
    *out = addr[dev];
    return hipSuccess;
}

hipError_t launch_features(const double *Q, const double *HM, const PatchGeom *geom, int32_t npatch, float *feat,
                           hipStream_t st)
{
    if (npatch <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3(npatch), dim3(256), 0, st, Q, HM, geom, feat);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *prm, const float *norm, const float *feat, int64_t n, float *logits,
                              hipStream_t st)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3(mlp_tiles(n)), dim3(256), 0, st, prm, norm, feat, n, logits);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *prm, const float *norm, const float *feat, const int8_t *tags, int64_t n,
                           float *work, float *trace, float *grad, float *loss, hipStream_t st)
{
    const int32_t nt = mlp_tiles(n);
    if ((nt + MLP_RCHUNK - 1) / MLP_RCHUNK > 65535) return hipErrorInvalidConfiguration;  // grid y of the reduction
    hipLaunchKernelGGL(k_mlp_grad, dim3(nt), dim3(256), 0, st, prm, norm, feat, tags, n, work, trace);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const unsigned qb = (MLP_NPARAM + 1 + 255) / 256;
    hipLaunchKernelGGL(k_mlp_reduce_chunks, dim3(qb, (unsigned)((nt + MLP_RCHUNK - 1) / MLP_RCHUNK)), dim3(256), 0, st,
                       work, nt);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_mlp_reduce, dim3(qb), dim3(256), 0, st, work, nt, n, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *prm, float *m, float *v, const float *grad, float lr, float b1, float b2, float eps,
                           float c1, float c2, hipStream_t st)
{
    hipLaunchKernelGGL(k_mlp_adam, dim3((MLP_NPARAM + 255) / 256), dim3(256), 0, st, prm, m, v, grad, lr, b1, b2, eps,
                       c1, c2);
    return hipGetLastError();
}

hipError_t launch_tag_learned(const float *logits, const int8_t *plain, const PatchGeom *geom, const int32_t *sib,
                              int32_t npatch, float conf, int32_t max_level, int8_t *pre, int8_t *tags,
                              hipStream_t st)
{
    if (npatch <= 0) return hipSuccess;
    const unsigned nb = (unsigned)((npatch + 127) / 128);
    hipLaunchKernelGGL(k_tag_learned_pre, dim3(nb), dim3(128), 0, st, logits, plain, geom, npatch, conf, max_level,
                       pre);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_tag_learned_family, dim3(nb), dim3(128), 0, st, pre, sib, npatch, tags);
    return hipGetLastError();
}

}  // namespace ccz4
