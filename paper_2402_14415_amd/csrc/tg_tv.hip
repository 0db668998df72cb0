// Total variation of the coefficient grid (the L_TV term of Sec. 3.2, Eq. 8, Plenoxels'
// regulariser) and its gradient, in one pass over the grid.
//
// For vertex v and stored coefficient channel c, Delta_a(v, c) = C(v + e_a, c) - C(v, c)
// along each axis a (0 where v + e_a is outside the grid) and s(v, c) = |Delta(v, c)|;
// TV = (1 / |V|) sum over v, c of s(v, c).  The gradient at u collects +Delta_a / s from the
// backward neighbours u - e_a and -Delta_a / s from u itself (0 where s = 0).
//
// One thread per coefficient word, walking the grid by rows along x: a workgroup takes rows
// (y, z) in turn and its threads the row's res_x * C contiguous words, so each of the up to
// 13 neighbour reads (u, u + e_a, u - e_a, u - e_a + e_b) is a coalesced wave access at a
// constant offset, served mostly by L1/L2; HBM sees the coefficients about once and the
// gradient once.  Norms use the hardware reciprocal square root (|Delta| / s = Delta rsq(s^2)).
#include "tg_internal.hpp"

namespace tg {

constexpr int kTvThreads = 256;
// Squared norms below the smallest normal float count as 0 (the reciprocal square root is
// not taken of a denormal): only differences under 1e-19 in magnitude are affected.
constexpr float kTvMinNorm2 = 1.17549435e-38f;

template <int DIM, int C>
__global__ __launch_bounds__(kTvThreads) void k_tv(Geom g, const float* __restrict__ master,
                                                   float* __restrict__ grad, int accumulate, float scale,
                                                   double* __restrict__ partials)
{
    const int rx = g.res[0], ry = g.res[1], rz = DIM == 3 ? g.res[2] : 1;
    const int64_t sa[3] = {(int64_t)C, (int64_t)rx * C, (int64_t)rx * ry * C};  // word stride of e_a
    const int64_t rows = (int64_t)ry * rz;
    const int roww = rx * C;
    double acc = 0.0;
    // XCD-aware rows: workgroups are dealt round-robin to the 8 XCDs, so with a grid that is a
    // multiple of 8, XCD x (blockIdx % 8) takes the contiguous band x of the rows and its
    // workgroups stride through that band together; the neighbour rows a row reads (y +- 1,
    // z +- 1) are then mostly in the same XCD's L2.
    int64_t r0 = blockIdx.x, r1 = rows, rstep = gridDim.x;
    if (gridDim.x % 8 == 0) {
        const int64_t band = (rows + 7) / 8;
        r0 = (blockIdx.x % 8) * band + blockIdx.x / 8;
        r1 = min(rows, (int64_t)(blockIdx.x % 8 + 1) * band);
        rstep = gridDim.x / 8;
    }
    for (int64_t r = r0; r < r1; r += rstep) {
        const int y = (int)(r % ry), z = (int)(r / ry);
        const int64_t base = r * roww;
        for (int w = threadIdx.x; w < roww; w += kTvThreads) {
            const int x = w / C;
            const int u[3] = {x, y, z};
            const int64_t gi = base + w;
            // Neighbour offsets, 0 where the neighbour is outside the grid: the difference is
            // then exactly 0, as the definition has it, and every load is unconditional.
            int64_t of[3], ob[3];  // to u + e_a, u - e_a
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                of[a] = u[a] + 1 < g.res[a] ? sa[a] : 0;
                ob[a] = u[a] >= 1 ? sa[a] : 0;
            }
            const float cu = master[gi];
            float fn[DIM], bn[DIM], dn[DIM][DIM];  // C(u + e_a), C(u - e_a), C(u - e_a + e_b)
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                fn[a] = master[gi + of[a]];
                bn[a] = master[gi - ob[a]];
#pragma unroll
                for (int b = 0; b < DIM; ++b)
                    if (b != a) dn[a][b] = master[gi - ob[a] + of[b]];  // p + e_b in the grid iff u + e_b is
            }
            float du[DIM], su2 = 0.0f;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                du[a] = fn[a] - cu;
                su2 = fmaf(du[a], du[a], su2);
            }
            const float inv = su2 >= kTvMinNorm2 ? __builtin_amdgcn_rsqf(su2) : 0.0f;
            acc += (double)(su2 * inv);  // s(u)
            float gsum = 0.0f;
#pragma unroll
            for (int a = 0; a < DIM; ++a) gsum = fmaf(-du[a], inv, gsum);
            // the backward neighbours p = u - e_a, whose difference along a ends at u (for
            // u on the first layer p = u and that difference is 0: no term)
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
            const float v = gsum * scale;
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
    const int64_t rows = (int64_t)g->desc.res[1] * (dim == 3 ? g->desc.res[2] : 1);
    const unsigned nb = (unsigned)std::min<int64_t>(rows, kMaxReduceBlocks);
    const float scale = (float)((double)weight / (double)g->nvert);
    const int acc = accumulate ? 1 : 0;
#define TG_TV_CASE(D, CC)                                                                                  \
    if (dim == D && g->C == CC) {                                                                          \
        hipLaunchKernelGGL((k_tv<D, CC>), dim3(nb), dim3(kTvThreads), 0, s, g->geom, g->bufs.master, grad,   \
                           acc, scale, partials);                                                          \
    } else
    TG_TV_CASE(3, 10) TG_TV_CASE(3, 4) TG_TV_CASE(3, 1) TG_TV_CASE(2, 6) TG_TV_CASE(2, 3) TG_TV_CASE(2, 1)
    TG_TV_CASE(3, 13) TG_TV_CASE(2, 7) TG_TV_CASE(3, 12) TG_TV_CASE(2, 9)
    {
        return hipErrorInvalidValue;
    }
#undef TG_TV_CASE
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    // *tv_out = (sum of the partials) / |V|: the scale is applied by a one-block finish
    return launch_sum_finish_scaled(partials, nb, 1.0 / (double)g->nvert, tv_out, s);
}

}  // namespace tg
