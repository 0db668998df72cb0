// Total variation of the coefficient grid (the L_TV term of Sec. 3.2, Eq. 8, Plenoxels'
// regulariser) and its gradient, in one pass over the grid.
//
// For vertex v and stored coefficient channel c, Delta_a(v, c) = C(v + e_a, c) - C(v, c)
// along each axis a (0 where v + e_a is outside the grid) and s(v, c) = |Delta(v, c)|;
// TV = (1 / |V|) sum over v, c of s(v, c).  The gradient at u collects +Delta_a / s from the
// backward neighbours u - e_a and -Delta_a / s from u itself (0 where s = 0).
//
// 2D: one thread per coefficient word, walking the grid by rows along x: a workgroup takes
// rows y in turn and its threads the row's res_x * C contiguous words, so each of the 7
// neighbour reads (u, u + e_a, u - e_a, u - e_a + e_b) is a coalesced wave access at a
// constant offset, served mostly by L1/L2; HBM sees the coefficients about once and the
// gradient once.
// 3D: one thread per coefficient word of a z plane, marching through ZS consecutive planes.
// The 13 reads a word needs come from 7 columns of the lattice (u's own and its x, y and xy
// neighbours); each column is loaded once per plane it is needed on, so ZS words take
// 7 ZS + 6 loads instead of 13 ZS, all issued before the first word is evaluated.  A
// workgroup covers 256 consecutive words of a plane (rows are contiguous), so every load is a
// coalesced wave access.
// Norms use the hardware reciprocal square root (|Delta| / s = Delta rsq(s^2)).
#include "tg_internal.hpp"

namespace tg {

constexpr int kTvThreads = 256;
// Squared norms below the smallest normal float count as 0 (the reciprocal square root is
// not taken of a denormal): only differences under 1e-19 in magnitude are affected.
constexpr float kTvMinNorm2 = 1.17549435e-38f;

// Word-level TV terms of one vertex word u: s(u) (returned) and the gradient at u, from u's
// value, its forward neighbours fn[a] = C(u + e_a), backward neighbours bn[a] = C(u - e_a)
// and the diagonal ones dn[a][b] = C(u - e_a + e_b) (each 0-offset where it leaves the grid).
template <int DIM>
__device__ __forceinline__ float tv_word(float cu, const float* fn, const float* bn, const float (*dn)[3], float& gsum)
{
    float du[DIM], su2 = 0.0f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        du[a] = fn[a] - cu;
        su2 = fmaf(du[a], du[a], su2);
    }
    const float inv = su2 >= kTvMinNorm2 ? __builtin_amdgcn_rsqf(su2) : 0.0f;
    gsum = 0.0f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) gsum = fmaf(-du[a], inv, gsum);
    // the backward neighbours p = u - e_a, whose difference along a ends at u (for u on the
    // first layer p = u and that difference is 0: no term)
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const float cp = bn[a];
        const float da = cu - cp;
        float sp2 = da * da;
#pragma unroll
        for (int b = 0; b < DIM; ++b) {
            if (b == a) continue;
            const float db = dn[a][b] - cp;
            sp2 = fmaf(db, db, sp2);
        }
        const float ip = sp2 >= kTvMinNorm2 ? __builtin_amdgcn_rsqf(sp2) : 0.0f;
        gsum = fmaf(da, ip, gsum);
    }
    return su2 * inv;
}

// 2D: rows along x, a workgroup per row in turn.
template <int C>
__global__ __launch_bounds__(kTvThreads) void k_tv2(Geom g, const float* __restrict__ master,
                                                    float* __restrict__ grad, int accumulate, float scale,
                                                    double* __restrict__ partials)
{
    const int rx = g.res[0], ry = g.res[1];
    const int64_t sa[2] = {(int64_t)C, (int64_t)rx * C};  // word stride of e_a
    const int roww = rx * C;
    double acc = 0.0;
    for (int64_t y = blockIdx.x; y < ry; y += gridDim.x) {
        const int64_t base = y * roww;
        for (int w = threadIdx.x; w < roww; w += kTvThreads) {
            const int x = w / C;
            const int u[2] = {x, (int)y};
            const int64_t gi = base + w;
            // Neighbour offsets, 0 where the neighbour is outside the grid: the difference is
            // then exactly 0, as the definition has it, and every load is unconditional.
            int64_t of[2], ob[2];  // to u + e_a, u - e_a
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                of[a] = u[a] + 1 < g.res[a] ? sa[a] : 0;
                ob[a] = u[a] >= 1 ? sa[a] : 0;
            }
            const float cu = master[gi];
            float fn[3], bn[3], dn[3][3];  // C(u + e_a), C(u - e_a), C(u - e_a + e_b)
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                fn[a] = master[gi + of[a]];
                bn[a] = master[gi - ob[a]];
            }
            dn[0][1] = master[gi - ob[0] + of[1]];  // p + e_b in the grid iff u + e_b is
            dn[1][0] = master[gi - ob[1] + of[0]];
            float gsum;
            acc += (double)tv_word<2>(cu, fn, bn, dn, gsum);
            const float v = gsum * scale;
            grad[gi] = accumulate ? grad[gi] + v : v;
        }
    }
    const double tot = block_sum_f64<kTvThreads>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// 3D: z planes marched by each thread (see the file comment).
constexpr int kTvPlanes = 8;  // z planes a thread of the 3D kernel marches through

template <int C>
__global__ __launch_bounds__(kTvThreads) void k_tv3(Geom g, const float* __restrict__ master,
                                                    float* __restrict__ grad, int accumulate, float scale,
                                                    double* __restrict__ partials)
{
    constexpr int ZS = kTvPlanes;
    const int rx = g.res[0], ry = g.res[1], rz = g.res[2];
    const int64_t roww = (int64_t)rx * C, planew = roww * ry;
    const int64_t nchunk = (planew + kTvThreads - 1) / kTvThreads;
    const int64_t ntiles = nchunk * ((rz + ZS - 1) / ZS);
    // XCD-aware tiles: workgroups are dealt round-robin to the 8 XCDs, so with a grid that is a
    // multiple of 8, XCD x (blockIdx % 8) takes the contiguous band x of the tiles; the rows
    // y +- 1 a tile reads are then mostly read by the same XCD.
    int64_t t0 = blockIdx.x, t1 = ntiles, tstep = gridDim.x;
    if (gridDim.x % 8 == 0) {
        const int64_t band = (ntiles + 7) / 8;
        t0 = (blockIdx.x % 8) * band + blockIdx.x / 8;
        t1 = min(ntiles, (int64_t)(blockIdx.x % 8 + 1) * band);
        tstep = gridDim.x / 8;
    }
    double acc = 0.0;
    for (int64_t t = t0; t < t1; t += tstep) {
        const int64_t seg = t / nchunk, i = (t - seg * nchunk) * kTvThreads + threadIdx.x;
        const bool active = i < planew;
        const int64_t ic = active ? i : planew - 1;  // inactive lanes load in-bounds words
        const int y = (int)(ic / roww);
        const int x = (int)((ic - (int64_t)y * roww) / C);
        // neighbour offsets in words, 0 where the neighbour is outside the grid (the
        // difference is then exactly 0, as the definition has it)
        const int64_t ofx = x + 1 < rx ? C : 0, obx = x >= 1 ? C : 0;
        const int64_t ofy = y + 1 < ry ? roww : 0, oby = y >= 1 ? roww : 0;
        const int z0 = (int)seg * ZS;
        // plane p's word (clamped to the grid: at z = 0 the plane below is z itself, at the
        // top the plane above is z itself, which is the 0 offset of the definition)
        auto at = [&](int p) { return (int64_t)min(max(p, 0), rz - 1) * planew + ic; };
        float A[ZS + 2], Xp[ZS + 1], Yp[ZS + 1];  // planes z0 - 1 ...
        float Xm[ZS + 1], Ym[ZS + 1], XmYp[ZS], XpYm[ZS];  // planes z0 ...
#pragma unroll
        for (int j = 0; j < ZS + 2; ++j) A[j] = master[at(z0 - 1 + j)];
#pragma unroll
        for (int j = 0; j < ZS + 1; ++j) {
            Xp[j] = master[at(z0 - 1 + j) + ofx];
            Yp[j] = master[at(z0 - 1 + j) + ofy];
            Xm[j] = master[at(z0 + j) - obx];
            Ym[j] = master[at(z0 + j) - oby];
        }
#pragma unroll
        for (int j = 0; j < ZS; ++j) {
            XmYp[j] = master[at(z0 + j) - obx + ofy];
            XpYm[j] = master[at(z0 + j) + ofx - oby];
        }
#pragma unroll
        for (int k = 0; k < ZS; ++k) {
            const int z = z0 + k;
            if (!active || z >= rz) continue;
            const float fn[3] = {Xp[k + 1], Yp[k + 1], A[k + 2]};  // u + e_x, u + e_y, u + e_z
            const float bn[3] = {Xm[k], Ym[k], A[k]};              // u - e_x, u - e_y, u - e_z
            float dn[3][3];                                        // u - e_a + e_b
            dn[0][1] = XmYp[k];
            dn[0][2] = Xm[k + 1];
            dn[1][0] = XpYm[k];
            dn[1][2] = Ym[k + 1];
            dn[2][0] = Xp[k];
            dn[2][1] = Yp[k];
            float gsum;
            acc += (double)tv_word<3>(A[k + 1], fn, bn, dn, gsum);
            const float v = gsum * scale;
            const int64_t gi = (int64_t)z * planew + ic;
            grad[gi] = accumulate ? grad[gi] + v : v;
        }
    }
    const double tot = block_sum_f64<kTvThreads>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

hipError_t launch_tv(const tg_grid* g, float weight, double* tv_out, float* grad, bool accumulate,
                     double* partials, hipStream_t s)
{
    const int dim = g->desc.dim;
    int64_t want;  // workgroups with work
    if (dim == 3) {
        const int64_t planew = (int64_t)g->desc.res[0] * g->desc.res[1] * g->C;
        want = (planew + kTvThreads - 1) / kTvThreads * ((g->desc.res[2] + kTvPlanes - 1) / kTvPlanes);
    } else {
        want = g->desc.res[1];
    }
    const unsigned nb = (unsigned)std::min<int64_t>(want, kMaxReduceBlocks);
    const float scale = (float)((double)weight / (double)g->nvert);
    const int acc = accumulate ? 1 : 0;
#define TG_TV3(CC)                                                                                         \
    if (dim == 3 && g->C == CC) {                                                                          \
        hipLaunchKernelGGL((k_tv3<CC>), dim3(nb), dim3(kTvThreads), 0, s, g->geom, g->bufs.master, grad,     \
                           acc, scale, partials);                                                          \
    } else
#define TG_TV2(CC)                                                                                         \
    if (dim == 2 && g->C == CC) {                                                                          \
        hipLaunchKernelGGL((k_tv2<CC>), dim3(nb), dim3(kTvThreads), 0, s, g->geom, g->bufs.master, grad,     \
                           acc, scale, partials);                                                          \
    } else
    TG_TV3(10) TG_TV3(4) TG_TV3(1) TG_TV3(13) TG_TV3(12) TG_TV2(6) TG_TV2(3) TG_TV2(1) TG_TV2(7) TG_TV2(9)
    {
        return hipErrorInvalidValue;
    }
#undef TG_TV3
#undef TG_TV2
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // *tv_out = (sum of the partials) / |V|: the scale is applied by a one-block finish
    return launch_sum_finish_scaled(partials, nb, 1.0 / (double)g->nvert, tv_out, s);
}

}  // namespace tg
