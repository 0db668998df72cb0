// Total variation of the coefficient grid (the L_TV term of Sec. 3.2, Eq. 8, Plenoxels'
// regulariser) and its gradient, in one pass over the grid.
//
// For vertex v and stored coefficient channel c, Delta_a(v, c) = C(v + e_a, c) - C(v, c)
// along each axis a (0 where v + e_a is outside the grid) and s(v, c) = |Delta(v, c)|;
// TV = (1 / |V|) sum over v, c of s(v, c).  The gradient at u collects +Delta_a / s from the
// backward neighbours u - e_a and -Delta_a / s from u itself (0 where s = 0).
//
// A workgroup owns a tile of T^dim vertices.  It stages the tile and a one-vertex halo on
// every side ((T+2)^dim vertex blocks, rows copied contiguously from the [vertex][C] layout)
// into LDS, computes every owned vertex's gradient from LDS only, stages the results in LDS
// and writes them row by row.  HBM sees the coefficients once (the halo comes mostly from
// L2) and the gradient once.
#include "tg_internal.hpp"

namespace tg {

template <int DIM> struct TvShape {
    static constexpr int T = DIM == 3 ? 8 : 16;          // tile edge in vertices
    static constexpr int NT = DIM == 3 ? T * T * T : T * T;  // threads = owned vertices
    static constexpr int E = T + 2;                        // staged edge (with the halo)
    static constexpr int NROWS = DIM == 3 ? E * E : E;     // staged rows along x
};

template <int DIM, int C>
__global__ __launch_bounds__(TvShape<DIM>::NT) void k_tv(Geom g, const float* __restrict__ master,
                                                        float* __restrict__ grad, int accumulate, float scale,
                                                        double* __restrict__ partials)
{
    using S = TvShape<DIM>;
    constexpr int T = S::T, E = S::E, NT = S::NT;
    constexpr int ROWW = E * C;  // words of one staged row
    __shared__ float reg[S::NROWS * ROWW];
    __shared__ float out[NT * C];

    int nt[3] = {1, 1, 1};
#pragma unroll
    for (int a = 0; a < DIM; ++a) nt[a] = (g.res[a] + T - 1) / T;
    const int64_t ntiles = (int64_t)nt[0] * nt[1] * nt[2];
    const int tx = threadIdx.x % T, ty = (threadIdx.x / T) % T, tz = DIM == 3 ? threadIdx.x / (T * T) : 0;
    double acc = 0.0;

    for (int64_t tile = blockIdx.x; tile < ntiles; tile += gridDim.x) {
        int v0[3] = {0, 0, 0};
        v0[0] = (int)(tile % nt[0]) * T;
        v0[1] = (int)((tile / nt[0]) % nt[1]) * T;
        if constexpr (DIM == 3) v0[2] = (int)(tile / ((int64_t)nt[0] * nt[1])) * T;

        // stage vertices [v0 - 1, v0 + T] on every axis; words outside the grid are not read
        for (int e = threadIdx.x; e < S::NROWS * ROWW; e += NT) {
            const int row = e / ROWW, off = e - row * ROWW;
            const int gy = v0[1] - 1 + (DIM == 3 ? row % E : row);
            const int gz = DIM == 3 ? v0[2] - 1 + row / E : 0;
            const int gx = v0[0] - 1 + off / C;
            bool ok = gx >= 0 && gx < g.res[0] && gy >= 0 && gy < g.res[1];
            if constexpr (DIM == 3) ok = ok && gz >= 0 && gz < g.res[2];
            if (ok) {
                int64_t vtx = (int64_t)gx + (int64_t)gy * g.stride[1];
                if constexpr (DIM == 3) vtx += (int64_t)gz * g.stride[2];
                reg[e] = master[vtx * C + (off - (off / C) * C)];
            }
        }
        __syncthreads();

        const int u[3] = {v0[0] + tx, v0[1] + ty, v0[2] + tz};
        bool own = u[0] < g.res[0] && u[1] < g.res[1];
        if constexpr (DIM == 3) own = own && u[2] < g.res[2];
        if (own) {
            // staged index of the vertex at local offset (x, y, z) from the tile origin
            auto at = [&](int x, int y, int z) -> int {
                return DIM == 3 ? (((z + 1) * E + (y + 1)) * E + (x + 1)) * C : ((y + 1) * E + (x + 1)) * C;
            };
            const int l[3] = {tx, ty, tz};
            bool fwd[3], bwd[3];  // u + e_a, u - e_a inside the grid
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                fwd[a] = u[a] + 1 < g.res[a];
                bwd[a] = u[a] >= 1;
            }
#pragma unroll
            for (int c = 0; c < C; ++c) {
                const float cu = reg[at(l[0], l[1], l[2]) + c];
                // s(u) and the forward differences at u
                float du[3] = {0.0f, 0.0f, 0.0f};
                float su2 = 0.0f;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    if (fwd[a]) {
                        const int n = at(l[0] + (a == 0), l[1] + (a == 1), l[2] + (a == 2)) + c;
                        du[a] = reg[n] - cu;
                    }
                    su2 = fmaf(du[a], du[a], su2);
                }
                const float su = sqrtf(su2);
                acc += (double)su;
                float gsum = 0.0f;
                if (su > 0.0f) {
                    const float inv = 1.0f / su;
#pragma unroll
                    for (int a = 0; a < DIM; ++a) gsum -= du[a] * inv;
                }
                // the backward neighbours p = u - e_a, whose difference along a ends at u
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    if (!bwd[a]) continue;
                    const int p[3] = {l[0] - (a == 0), l[1] - (a == 1), l[2] - (a == 2)};
                    const float cp = reg[at(p[0], p[1], p[2]) + c];
                    float sp2 = 0.0f, da = 0.0f;
#pragma unroll
                    for (int b = 0; b < DIM; ++b) {
                        float db;
                        if (b == a) {
                            db = cu - cp;  // u is inside the grid
                            da = db;
                        } else {
                            // p + e_b is inside the grid when u + e_b is (same index on b)
                            db = fwd[b] ? reg[at(p[0] + (b == 0), p[1] + (b == 1), p[2] + (b == 2)) + c] - cp : 0.0f;
                        }
                        sp2 = fmaf(db, db, sp2);
                    }
                    if (sp2 > 0.0f) gsum += da / sqrtf(sp2);
                }
                out[threadIdx.x * C + c] = gsum * scale;
            }
        }
        __syncthreads();

        // write the owned vertices' gradients row by row (T C contiguous words per row)
        constexpr int OROWS = DIM == 3 ? T * T : T;
        const int nx = min(T, g.res[0] - v0[0]);
        for (int e = threadIdx.x; e < OROWS * T * C; e += NT) {
            const int row = e / (T * C), off = e - row * (T * C);
            const int y = row % T, z = DIM == 3 ? row / T : 0;
            bool ok = off < nx * C && v0[1] + y < g.res[1];
            if constexpr (DIM == 3) ok = ok && v0[2] + z < g.res[2];
            if (!ok) continue;
            int64_t vrow = (int64_t)v0[0] + (int64_t)(v0[1] + y) * g.stride[1];
            if constexpr (DIM == 3) vrow += (int64_t)(v0[2] + z) * g.stride[2];
            const int64_t gi = vrow * C + off;
            // out is [owned vertex][C] with vertex = x + T (y + T z): the same row order
            const float v = out[row * T * C + off];
            grad[gi] = accumulate ? grad[gi] + v : v;
        }
        __syncthreads();  // reg and out are rewritten by the next tile
    }
    const double tot = block_sum_f64<NT>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

hipError_t launch_tv(const tg_grid* g, float weight, double* tv_out, float* grad, bool accumulate,
                     double* partials, hipStream_t s)
{
    const int dim = g->desc.dim;
    const int T = dim == 3 ? TvShape<3>::T : TvShape<2>::T;
    int64_t ntiles = 1;
    for (int a = 0; a < dim; ++a) ntiles *= (g->desc.res[a] + T - 1) / T;
    const unsigned nb = (unsigned)std::min<int64_t>(ntiles, kMaxReduceBlocks);
    const float scale = (float)((double)weight / (double)g->nvert);
    const int acc = accumulate ? 1 : 0;
#define TG_TV_CASE(D, CC)                                                                                  \
    if (dim == D && g->C == CC) {                                                                          \
        hipLaunchKernelGGL((k_tv<D, CC>), dim3(nb), dim3(TvShape<D>::NT), 0, s, g->geom, g->bufs.master, grad, \
                           acc, scale, partials);                                                          \
    } else
    TG_TV_CASE(3, 10) TG_TV_CASE(3, 4) TG_TV_CASE(3, 1) TG_TV_CASE(2, 6) TG_TV_CASE(2, 3) TG_TV_CASE(2, 1)
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
