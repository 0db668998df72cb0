// TaylorGrid adjoint with respect to the coefficients, owner-computes per vertex brick.
//
// The field and its gradient are linear in the coefficients; for upstream gradients
// (g_f, g_grad) a query contributes to coefficient alpha of corner vertex v_b
//   m_alpha(d_b) s_b + sum_a u_a dm_alpha/dd_a(d_b),   s_b = g_f w_b + g_grad . grad w_b,
//   u = w_b g_grad,  m_alpha(d) = d^alpha / alpha!  (the Taylor monomials of Sec. 3.1, Eq. 1).
//
// Gather formulation: a workgroup owns a brick of B^dim vertices and one thread owns one
// vertex, accumulating its C coefficients in registers.  The brick's records (the queries
// whose cells touch its vertices: the primary and secondary buckets of the vertex brick,
// see tg_sort.hip) are staged in LDS in chunks, counting-sorted by cell (LDS integer
// atomics); each thread then walks the records of the 2^dim cells around its vertex, as
// one flattened loop over (corner, record) so that a lane's trip count is its total record
// count.  No floating-point atomics, no races, and every vertex is written exactly once.
// Crowded bricks are split into several work items whose partial sums a merge kernel adds.
#include "tg_internal.hpp"

namespace tg {

template <int DIM> __device__ __forceinline__ void vbrick_coords(const Geom& g, int32_t brick, int32_t* bc)
{
    bc[0] = brick % g.nvb[0];
    if constexpr (DIM == 3) {
        const int32_t r = brick / g.nvb[0];
        bc[1] = r % g.nvb[1];
        bc[2] = r / g.nvb[1];
    } else {
        bc[1] = brick / g.nvb[0];
    }
}

template <int DIM> struct BwdShape {
    static constexpr int B = BrickEdge<DIM>::value;
    static constexpr int NOWN = DIM == 3 ? B * B * B : B * B;  // vertices = threads
    static constexpr int NC1 = B + 1;                           // cells -1..B-1 per axis
    static constexpr int NCELL = DIM == 3 ? NC1 * NC1 * NC1 : NC1 * NC1;
    static constexpr int CHUNK = 512;                           // records staged at a time
};

// Writes (or adds) one vertex's C coefficients.
template <int C>
__device__ __forceinline__ void store_vertex(float* __restrict__ dst, const float* v, int accumulate)
{
    if constexpr (C % 2 == 0) {
        float2* o = reinterpret_cast<float2*>(dst);
#pragma unroll
        for (int k = 0; k < C / 2; ++k) {
            float2 x = make_float2(v[2 * k], v[2 * k + 1]);
            if (accumulate) {
                const float2 old = o[k];
                x.x += old.x;
                x.y += old.y;
            }
            o[k] = x;
        }
    } else {
#pragma unroll
        for (int k = 0; k < C; ++k) dst[k] = accumulate ? dst[k] + v[k] : v[k];
    }
}

template <int DIM, int K>
__global__ __launch_bounds__(BwdShape<DIM>::NOWN) void k_backward(Geom g, const int4* __restrict__ items,
                                                                 const int32_t* __restrict__ meta, int64_t max_items,
                                                                 float* __restrict__ parts,
                                                                 const float4* __restrict__ rec,
                                                                 const int32_t* __restrict__ offs,
                                                                 const float* __restrict__ gf,
                                                                 const float* __restrict__ gg,
                                                                 float* __restrict__ grad, int accumulate)
{
    using S = BwdShape<DIM>;
    constexpr int B = S::B, NOWN = S::NOWN, NC1 = S::NC1, NCELL = S::NCELL, CHUNK = S::CHUNK;
    constexpr int C = NumCoeffs<DIM, K>::value;
    constexpr int PER = CHUNK / NOWN;
    __shared__ float4 ent[2 * CHUNK];  // cell-sorted (t, g_f) and (g_grad, -) per record
    __shared__ uint32_t cstart[NCELL + 1];
    __shared__ uint32_t ccount[NCELL];
    __shared__ int32_t wsum[NOWN / 64];

    // Split bricks' items come first (longest first), whole bricks from the array's end.
    const int32_t nsplit = meta[META_BSPLIT], nwhole = meta[META_BWHOLE];
    const int32_t bid = blockIdx.x;
    int32_t item;
    if (bid < nsplit) item = bid;
    else if (bid < nsplit + nwhole) item = (int32_t)(max_items - 1 - (bid - nsplit));
    else return;
    const int4 wi = items[item];
    const int32_t brick = wi.x, chunk = wi.y, nchunk = wi.z;
    const int32_t beg = offs[2 * brick] + chunk * kBwdItem;
    const int32_t end = min(offs[2 * brick + 2], beg + kBwdItem);
    if (accumulate && nchunk == 1 && beg >= end) return;

    int32_t bc[3];
    vbrick_coords<DIM>(g, brick, bc);
    int32_t base[3], nown[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        base[a] = bc[a] * B;
        nown[a] = min(B, g.res[a] - base[a]);
    }
    // this thread's vertex, relative to the brick
    int v[3];
    {
        int r = threadIdx.x;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            v[a] = r % B;
            r /= B;
        }
    }
    bool mine = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) mine = mine && v[a] < nown[a];

    float acc[C];
#pragma unroll
    for (int k = 0; k < C; ++k) acc[k] = 0.0f;

    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int32_t cbeg = beg; cbeg < end; cbeg += CHUNK) {
        const int m = min(CHUNK, end - cbeg);
        for (int e = threadIdx.x; e < NCELL; e += NOWN) ccount[e] = 0u;
        __syncthreads();

        // Stage: decode records, rank them within their cell.
        int my_cell[PER];
        uint32_t my_rank[PER];
        float4 my_e0[PER], my_e1[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * NOWN;
            my_cell[u] = -1;
            if (i < m) {
                const float4 r = rec[cbeg + i];
                const float q[3] = {r.x, r.y, r.z};
                const int32_t idx = __float_as_int(r.w);
                AxisLoc L[DIM];
                locate<DIM>(g, q, L);
                float sg[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int a = 0; a < DIM; ++a) sg[a] = (gg && !L[a].clamped) ? gg[(int64_t)idx * DIM + a] : 0.0f;
                int cell = 0;
#pragma unroll
                for (int a = DIM - 1; a >= 0; --a) cell = cell * NC1 + min(max(L[a].cell - base[a] + 1, 0), B);
                my_cell[u] = cell;
                my_e0[u] = make_float4(L[0].t, L[1].t, DIM == 3 ? L[DIM - 1].t : 0.0f, gf ? gf[idx] : 0.0f);
                my_e1[u] = make_float4(sg[0], sg[1], sg[2], 0.0f);
                my_rank[u] = atomicAdd(&ccount[cell], 1u);
            }
        }
        __syncthreads();
        // exclusive scan of the cell counts
        {
            constexpr int CPT = (NCELL + NOWN - 1) / NOWN;
            uint32_t c[CPT];
            uint32_t s = 0;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int idx = threadIdx.x * CPT + k;
                c[k] = idx < NCELL ? ccount[idx] : 0u;
                s += c[k];
            }
            uint32_t incl = s;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t o = __shfl_up(incl, d, 64);
                if (lane >= d) incl += o;
            }
            if (lane == 63) wsum[wave] = (int32_t)incl;
            __syncthreads();
            uint32_t before = 0;
            for (int w = 0; w < wave; ++w) before += (uint32_t)wsum[w];
            uint32_t run = before + incl - s;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int idx = threadIdx.x * CPT + k;
                if (idx < NCELL) cstart[idx] = run;
                run += c[k];
            }
            if (threadIdx.x == NOWN - 1) cstart[NCELL] = run;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            if (my_cell[u] < 0) continue;
            const uint32_t pos = cstart[my_cell[u]] + my_rank[u];
            ent[2 * pos] = my_e0[u];
            ent[2 * pos + 1] = my_e1[u];
        }
        __syncthreads();

        // Gather: every (corner, record) pair of this thread's vertex, one flattened loop.
        // The record ranges of the 2^dim cells around the vertex are read up front (they do
        // not depend on each other); the loop then picks the corner with register selects.
        if (mine) {
            constexpr int NB = 1 << DIM;
            uint32_t cs[NB], pre[NB + 1];
            pre[0] = 0u;
#pragma unroll
            for (int b = 0; b < NB; ++b) {
                int cell = 0;
#pragma unroll
                for (int a = DIM - 1; a >= 0; --a) cell = cell * NC1 + (v[a] - ((b >> a) & 1) + 1);
                cs[b] = cstart[cell];
                pre[b + 1] = cstart[cell + 1];
            }
#pragma unroll
            for (int b = 0; b < NB; ++b) pre[b + 1] = pre[b] + (pre[b + 1] - cs[b]);
            const uint32_t total = pre[NB];
            for (uint32_t k = 0; k < total; ++k) {
                int b = 0;
                uint32_t e = cs[0] + k;
#pragma unroll
                for (int bb = 1; bb < NB; ++bb)
                    if (k >= pre[bb]) {
                        b = bb;
                        e = cs[bb] + (k - pre[bb]);
                    }
                const float4 e0 = ent[2 * e], e1 = ent[2 * e + 1];
                const float t[3] = {e0.x, e0.y, e0.z};
                const float sg[3] = {e1.x, e1.y, e1.z};
                // weight of this corner and its gradient, and the offset from this vertex
                float w = 1.0f, d[DIM], fa[DIM], da[DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    const bool ba = (b >> a) & 1;
                    fa[a] = ba ? t[a] : 1.0f - t[a];
                    da[a] = ba ? g.inv_h[a] : -g.inv_h[a];
                    d[a] = (ba ? t[a] - 1.0f : t[a]) * g.h[a];
                    w *= fa[a];
                }
                float dw[DIM];
                if constexpr (DIM == 3) {
                    dw[0] = da[0] * fa[1] * fa[2];
                    dw[1] = fa[0] * da[1] * fa[2];
                    dw[2] = fa[0] * fa[1] * da[2];
                } else {
                    dw[0] = da[0] * fa[1];
                    dw[1] = fa[0] * da[1];
                }
                float s = e0.w * w;
                float uu[DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    s = fmaf(sg[a], dw[a], s);
                    uu[a] = w * sg[a];
                }
                float out[C];
                corner_adjoint<DIM, K>(d, s, uu, out);
#pragma unroll
                for (int k2 = 0; k2 < C; ++k2) acc[k2] += out[k2];
            }
        }
        __syncthreads();
    }

    int64_t vert = (int64_t)(base[0] + v[0]) + (int64_t)(base[1] + v[1]) * g.stride[1];
    if constexpr (DIM == 3) vert += (int64_t)(base[2] + v[2]) * g.stride[2];
    if (nchunk > 1) {
        // partial sums of a split brick: slot = item index, laid out [vertex][C] per brick
        if (mine) {
            float* slot = parts + (int64_t)item * (NOWN * C) + threadIdx.x * C;
#pragma unroll
            for (int k = 0; k < C; ++k) slot[k] = acc[k];
        }
        return;
    }
    if (mine) store_vertex<C>(grad + vert * C, acc, accumulate);
}

// Adds the partial sums of every split brick, in slot order, and writes the brick.
template <int DIM, int K>
__global__ __launch_bounds__(BwdShape<DIM>::NOWN) void k_backward_merge(Geom g, const int4* __restrict__ items,
                                                                       const int32_t* __restrict__ split_first,
                                                                       const int32_t* __restrict__ meta,
                                                                       const float* __restrict__ parts,
                                                                       float* __restrict__ grad, int accumulate)
{
    using S = BwdShape<DIM>;
    constexpr int B = S::B, NOWN = S::NOWN;
    constexpr int C = NumCoeffs<DIM, K>::value;
    if ((int32_t)blockIdx.x >= meta[META_NSPLITB]) return;
    const int4 wi = items[split_first[blockIdx.x]];
    const int32_t brick = wi.x, nchunk = wi.z, first = wi.w;
    int32_t bc[3];
    vbrick_coords<DIM>(g, brick, bc);
    int v[3];
    {
        int r = threadIdx.x;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            v[a] = r % B;
            r /= B;
        }
    }
    bool mine = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a) mine = mine && v[a] < min(B, g.res[a] - bc[a] * B);
    if (!mine) return;
    float acc[C];
#pragma unroll
    for (int k = 0; k < C; ++k) acc[k] = 0.0f;
    for (int j = 0; j < nchunk; ++j) {
        const float* slot = parts + (int64_t)(first + j) * (NOWN * C) + threadIdx.x * C;
#pragma unroll
        for (int k = 0; k < C; ++k) acc[k] += slot[k];
    }
    int64_t vert = (int64_t)(bc[0] * B + v[0]) + (int64_t)(bc[1] * B + v[1]) * g.stride[1];
    if constexpr (DIM == 3) vert += (int64_t)(bc[2] * B + v[2]) * g.stride[2];
    store_vertex<C>(grad + vert * C, acc, accumulate);
}

hipError_t launch_backward(const tg_grid* g, int64_t n, const char* ws, const WsLayout& L, const float* g_f,
                           const float* g_grad, bool accumulate, hipStream_t s)
{
    (void)n;
    const float4* rec = reinterpret_cast<const float4*>(ws + L.rec_off);
    const int32_t* offs = reinterpret_cast<const int32_t*>(ws + L.offs_off);
    const int4* items = reinterpret_cast<const int4*>(ws + L.bitems_off);
    const int32_t* meta = reinterpret_cast<const int32_t*>(ws + L.meta_off);
    float* parts = reinterpret_cast<float*>(const_cast<char*>(ws) + L.parts_off);
    const int32_t* split_first = reinterpret_cast<const int32_t*>(ws + L.splitb_off);
    const dim3 grid((unsigned)L.max_bitems);
    const int dim = g->desc.dim, K = g->desc.order;
    float* gr = g->bufs.grad;
    const int acc = accumulate ? 1 : 0;
#define TG_BWD_CASE(D, KK)                                                                                   \
    if (dim == D && K == KK) {                                                                               \
        const dim3 block(BwdShape<D>::NOWN);                                                                 \
        hipLaunchKernelGGL((k_backward<D, KK>), grid, block, 0, s, g->geom, items, meta, L.max_bitems, parts, rec, \
                           offs, g_f, g_grad, gr, acc);                                                      \
        hipLaunchKernelGGL((k_backward_merge<D, KK>), dim3((unsigned)g->nbricks), block, 0, s, g->geom, items, \
                           split_first, meta, parts, gr, acc);                                               \
        return hipGetLastError();                                                                            \
    }
    TG_BWD_CASE(3, 2) TG_BWD_CASE(3, 1) TG_BWD_CASE(3, 0) TG_BWD_CASE(2, 2) TG_BWD_CASE(2, 1) TG_BWD_CASE(2, 0)
#undef TG_BWD_CASE
    return hipErrorInvalidValue;
}

}  // namespace tg
