// TaylorGrid adjoint with respect to the coefficients, owner-computes per vertex brick.
//
// The field and its gradient are linear in the coefficients; for upstream gradients
// (g_f, g_grad) a query contributes to coefficient alpha of corner vertex v_b
//   m_alpha(d_b) s_b + sum_a u_a dm_alpha/dd_a(d_b),   s_b = g_f w_b + g_grad . grad w_b,
//   u = w_b g_grad,  m_alpha(d) = d^alpha / alpha!  (the Taylor monomials of Sec. 3.1, Eq. 1).
//
// Gather formulation: a workgroup owns a brick of B^dim vertices and, in each pass over the
// brick's records, one thread owns one vertex, accumulating its C coefficients in registers
// (vertices go to lanes by their pair count in the pass; the sums move with them through
// LDS between passes).  The brick's records (the queries
// whose cells touch its vertices: the primary and secondary buckets of the vertex brick,
// see tg_sort.hip) are staged in LDS in chunks, counting-sorted by cell (LDS integer
// atomics); each thread then walks the records of the 2^dim cells around its vertex, as
// one flattened loop over (corner, record) so that a lane's trip count is its total record
// count.  No floating-point atomics, no races, and every vertex is written exactly once.
// Crowded bricks are split into several work items whose partial sums a merge kernel adds.
// With Adam in the epilogue there is no merge launch: the first item of a split brick stages
// all of the brick's records (in more passes) when they number at most kBwdWholeMax, and the
// items of a larger brick store their partial sums, the one that finishes last (found with a
// device-scope count per brick) adding them in item order.
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
    static constexpr int NRUN = 1 << (DIM - 1);                 // runs of 2 x-adjacent cells per vertex
    static constexpr int PER = kBwdItem / NOWN;                 // records staged per thread and pass
    static constexpr int NBIN = 256;                            // trip-count bins
};
static_assert(kBwdItem % BwdShape<3>::NOWN == 0 && kBwdItem % BwdShape<2>::NOWN == 0,
              "a backward item must split evenly over the threads");

// Adds one (corner, query) pair's contribution to a vertex's coefficient adjoint:
//   acc_alpha += m_alpha(d) s + sum_a u_a dm_alpha/dd_a(d)
// with the monomials m of Sec. 3.1 Eq. 1 (1, d_a, d_a^2 / 2, d_a d_c), written as FMAs.
template <int DIM, int K>
__device__ __forceinline__ void accumulate_corner(const float* d, float s, const float* u, float* acc)
{
    acc[0] += s;
    if constexpr (K >= 1) {
        float q[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            q[a] = fmaf(s, d[a], u[a]);  // s d_a + u_a
            acc[1 + a] += q[a];
        }
        if constexpr (K == kOrderFull) {
            // H_ab (row-major): d(T)/dH_ab = d_a d_b / 2, d(grad_c T)/dH_ab = (delta_ca d_b + delta_cb d_a) / 2
            const float hs = 0.5f * s;
#pragma unroll
            for (int a = 0; a < DIM; ++a)
#pragma unroll
                for (int b2 = 0; b2 < DIM; ++b2)
                    acc[1 + DIM + a * DIM + b2] =
                        fmaf(0.5f * u[b2], d[a], fmaf(0.5f * u[a], d[b2], fmaf(hs * d[a], d[b2], acc[1 + DIM + a * DIM + b2])));
        } else if constexpr (K == 2) {
            const float hs = 0.5f * s;
            if constexpr (DIM == 3) {
                acc[4] = fmaf(fmaf(hs, d[0], u[0]), d[0], acc[4]);     // xx: d_x (s d_x / 2 + u_x)
                acc[5] = fmaf(u[1], d[0], fmaf(q[0], d[1], acc[5]));   // xy: d_y (s d_x + u_x) + u_y d_x
                acc[6] = fmaf(u[2], d[0], fmaf(q[0], d[2], acc[6]));   // xz
                acc[7] = fmaf(fmaf(hs, d[1], u[1]), d[1], acc[7]);     // yy
                acc[8] = fmaf(u[2], d[1], fmaf(q[1], d[2], acc[8]));   // yz
                acc[9] = fmaf(fmaf(hs, d[2], u[2]), d[2], acc[9]);     // zz
            } else {
                acc[3] = fmaf(fmaf(hs, d[0], u[0]), d[0], acc[3]);     // xx
                acc[4] = fmaf(u[1], d[0], fmaf(q[0], d[1], acc[4]));   // xy
                acc[5] = fmaf(fmaf(hs, d[1], u[1]), d[1], acc[5]);     // yy
            }
        }
    }
}

// Linear index of a cell relative to the brick: cell coordinates -1..B-1 map to 0..B.
template <int DIM>
__device__ __forceinline__ int rel_cell(const int* c)
{
    constexpr int NC1 = BwdShape<DIM>::NC1;
    return DIM == 3 ? (c[2] * NC1 + c[1]) * NC1 + c[0] : c[1] * NC1 + c[0];
}

// Optimizer state for the adjoint kernels that apply Adam in the same pass (AD >= 0: the
// storage type of the coefficient copy).  partials receives one FP64 sum(dC^2) per block.
struct AdamBuf {
    AdamArgs A;
    float* master;
    float* m;
    float* v;
    void* coeffs;
    double* partials;
    const float* extra;  // gradient added to the adjoint before the update (NULL: none)
};

// Element of the brick's [vertex][C] block list that register k of this thread holds in the
// epilogue: with an even C, pairs of neighbouring elements (never split by a row of B*C), so
// that global memory is accessed in 8-byte words.
template <int DIM, int C>
__device__ __forceinline__ int epi_elem(int k)
{
    constexpr int NOWN = BwdShape<DIM>::NOWN;
    if constexpr (C % 2 == 0) return 2 * ((int)threadIdx.x + (k >> 1) * NOWN) + (k & 1);
    else return (int)threadIdx.x + k * NOWN;
}

// Writes the brick's coefficient adjoint to grad (AD < 0: =, or += when accumulating), or
// applies Adam to it (AD >= 0), walking the brick row by row so that consecutive threads
// touch consecutive words.  vk[k] is the value of element epi_elem(k) of the brick's
// [vertex][C] block list (vertex = x + B (y + B z)); a row of B vertices along x is B * C
// contiguous words in memory.  Returns this thread's share of sum(value^2).
template <int DIM, int C, int AD>
__device__ __forceinline__ double brick_epilogue(const Geom& g, const int32_t* base, const int32_t* nown,
                                                 const float* vk, float* __restrict__ grad, int accumulate,
                                                 const AdamBuf& AB)
{
    using S = BwdShape<DIM>;
    constexpr int B = S::B, RL = B * C;
    constexpr int W = C % 2 == 0 ? 2 : 1;  // elements per access
    double ss = 0.0;
#pragma unroll
    for (int k = 0; k < C; k += W) {
        const int e = epi_elem<DIM, C>(k);
        const int r = e / RL, p = e - r * RL;
        const int y = r % B, z = r / B;
        bool ok = p < nown[0] * C && y < nown[1];
        if constexpr (DIM == 3) ok = ok && z < nown[2];
        if (!ok) continue;
        int64_t vrow = (int64_t)base[0] + (int64_t)(base[1] + y) * g.stride[1];
        if constexpr (DIM == 3) vrow += (int64_t)(base[2] + z) * g.stride[2];
        const int64_t gi = vrow * C + p;
        if constexpr (W == 2) {
            // 8-byte aligned: C and p are even
            if constexpr (AD >= 0) {
                float2 th = *reinterpret_cast<const float2*>(AB.master + gi);
                float2 m = *reinterpret_cast<const float2*>(AB.m + gi);
                float2 v = *reinterpret_cast<const float2*>(AB.v + gi);
                float2 gk = make_float2(vk[k], vk[k + 1]);
                if (AB.extra) {
                    const float2 x = *reinterpret_cast<const float2*>(AB.extra + gi);
                    gk.x += x.x;
                    gk.y += x.y;
                }
                ss += (double)gk.x * (double)gk.x + (double)gk.y * (double)gk.y;
                adam_elem(AB.A, gk.x, th.x, m.x, v.x);
                adam_elem(AB.A, gk.y, th.y, m.y, v.y);
                *reinterpret_cast<float2*>(AB.master + gi) = th;
                *reinterpret_cast<float2*>(AB.m + gi) = m;
                *reinterpret_cast<float2*>(AB.v + gi) = v;
                if constexpr (AD == ST_BF16)
                    *reinterpret_cast<uint32_t*>(static_cast<uint16_t*>(AB.coeffs) + gi) =
                        (uint32_t)float_to_bf16_rne(th.x) | ((uint32_t)float_to_bf16_rne(th.y) << 16);
                else if constexpr (AD == ST_F16)
                    *reinterpret_cast<uint32_t*>(static_cast<uint16_t*>(AB.coeffs) + gi) =
                        (uint32_t)float_to_f16_rne_sat(th.x) | ((uint32_t)float_to_f16_rne_sat(th.y) << 16);
            } else {
                float2 o = make_float2(vk[k], vk[k + 1]);
                if (accumulate) {
                    const float2 old = *reinterpret_cast<const float2*>(grad + gi);
                    o.x += old.x;
                    o.y += old.y;
                }
                *reinterpret_cast<float2*>(grad + gi) = o;
            }
        } else {
            float val = vk[k];
            if constexpr (AD >= 0) {
                if (AB.extra) val += AB.extra[gi];
                float th = AB.master[gi], m = AB.m[gi], v = AB.v[gi];
                ss += (double)val * (double)val;
                adam_elem(AB.A, val, th, m, v);
                AB.master[gi] = th;
                AB.m[gi] = m;
                AB.v[gi] = v;
                store_copy<AD>(AB.coeffs, gi, th);
            } else {
                grad[gi] = accumulate ? grad[gi] + val : val;
            }
        }
    }
    return ss;
}

template <int DIM, int K, int AD>
__global__ __launch_bounds__(BwdShape<DIM>::NOWN) __attribute__((amdgpu_waves_per_eu(DIM == 3 ? 6 : 4))) void k_backward(Geom g, const int4* __restrict__ items,
                                                                 const int32_t* __restrict__ meta, int64_t max_items,
                                                                 float* __restrict__ parts,
                                                                 int2* __restrict__ split,
                                                                 const float4* __restrict__ rec,
                                                                 const float* __restrict__ gf,
                                                                 const float* __restrict__ gg,
                                                                 const float4* __restrict__ urec,
                                                                 float* __restrict__ grad, int accumulate, AdamBuf AB,
                                                                 int64_t nq, int packed)
{
    using S = BwdShape<DIM>;
    constexpr int B = S::B, NOWN = S::NOWN, NCELL = S::NCELL, NRUN = S::NRUN, PER = S::PER, NBIN = S::NBIN;
    constexpr int C = NumCoeffs<DIM, K>::value;
    // Per staged record, in cell order: (g_f, g_grad), then per axis the corner factors of
    // both sides, (1 - t, t h) for the corner below and (t, (t - 1) h) for the corner above
    // (weight factor, offset from the vertex in world units), so that a visit reads 16 B plus
    // the one 8 B pair per axis that its corner needs, chosen by address.
    // In 3D, records are 5 float4 apart (80 B, one unused): at 64 B, the lanes of a wave,
    // which read different records, all hit the same two groups of 4 LDS banks; at 80 B,
    // 8 consecutive records start on 8 different groups.  (2D keeps 64 B: its 4 workgroups
    // per CU would not fit in the LDS at 80 B.)
    constexpr int kEntStride = DIM == 3 ? 5 : 4;
    __shared__ float4 ent[kEntStride * kBwdItem];
    __shared__ uint32_t cstart[NCELL + 1];
    __shared__ uint32_t ccount[NCELL];
    __shared__ uint32_t bins[NBIN];
    __shared__ uint16_t perm[NOWN];
    __shared__ int32_t wsum[NOWN / 64];

    // Items of bricks with more than one pass of records come first (the longest work
    // starts first), the others from the array's end; in XCD-aware order.
    const int32_t nfront = meta[META_BFRONT], nback = meta[META_BBACK];
    const int32_t bid = blockIdx.x, lb = xcd_grouped<kXcdGroup>(bid, nfront + nback);
    int32_t item;
    if (lb < nfront) {
        item = lb;
    } else if (lb < nfront + nback) {
        item = (int32_t)(max_items - 1 - (lb - nfront));
    } else {
        if constexpr (AD >= 0) {
            if (threadIdx.x == 0) AB.partials[bid] = 0.0;
        }
        return;
    }
    const int4 wi = items[item];
    const int32_t brick = wi.x, beg = wi.y;
    int32_t end = wi.z, nchunk = wi.w;
    if (accumulate && nchunk == 1 && end <= beg) return;
    int32_t first_item = item;
    if constexpr (AD >= 0) {
        if (nchunk > 1) {
            // a split brick: its items are consecutive from first_item
            first_item = split[brick].y;
            const int32_t brick_end = items[first_item + nchunk - 1].z;
            if (brick_end - items[first_item].y <= kBwdWholeMax) {
                if (item != first_item) {  // the first item takes the whole brick
                    if (threadIdx.x == 0) AB.partials[bid] = 0.0;
                    return;
                }
                end = brick_end;
                nchunk = 1;
            }
        }
    }

    int32_t bc[3];
    vbrick_coords<DIM>(g, brick, bc);
    int32_t base[3], nown[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        base[a] = bc[a] * B;
        nown[a] = min(B, g.res[a] - base[a]);
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;

    // The records of the 2^dim cells around vertex v form NRUN runs: for every choice of
    // the y (and z) corner bits, the two x-adjacent cells (v_x - 1, v_x) are neighbours in
    // cell order.  A record in the run's first cell sees v as its x-high corner.
    auto vertex_runs = [&](int vid, int* v, bool& owned, uint32_t* off, uint32_t* mid, uint32_t* pre) {
        int r = vid;
        owned = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            v[a] = r % B;
            r /= B;
            owned = owned && v[a] < nown[a];
        }
        pre[0] = 0u;
#pragma unroll
        for (int j = 0; j < NRUN; ++j) {
            int c[3] = {v[0], v[1] - (j & 1) + 1, DIM == 3 ? v[2] - (j >> 1) + 1 : 0};
            const int lo = rel_cell<DIM>(c);
            const uint32_t s0 = cstart[lo], s1 = cstart[lo + 1], s2 = cstart[lo + 2];
            mid[j] = s1;
            pre[j + 1] = pre[j] + (owned ? s2 - s0 : 0u);
            off[j] = s0 - pre[j];  // record index = off[j] + k for k in [pre[j], pre[j + 1])
        }
    };

    float acc[C];
#pragma unroll
    for (int k = 0; k < C; ++k) acc[k] = 0.0f;
    int vid = threadIdx.x;  // this thread's vertex (x + B (y + B z) within the brick)

    // The record table's space holds the accumulators between passes ([vertex][C]).
    float* vals = reinterpret_cast<float*>(ent);

    // One pass per kBwdItem records: stage them in LDS sorted by cell, then every thread
    // adds the pairs of its vertex.  Lanes are assigned to vertices anew in every pass, by
    // that pass's pair counts (the records of a crowded brick's passes differ: its secondary
    // records touch only the vertices of its lower faces); a vertex's sums move to its new
    // lane through LDS.
    for (int32_t cbeg = beg; cbeg < end; cbeg += kBwdItem) {
        const int m = min(kBwdItem, end - cbeg);
        const bool first_pass = cbeg == beg;
        if (!first_pass) {
            __syncthreads();  // the previous pass is done with the record table
#pragma unroll
            for (int k = 0; k < C; ++k) vals[vid * C + k] = acc[k];
        }
        for (int e = threadIdx.x; e < NCELL; e += NOWN) ccount[e] = 0u;
        for (int e = threadIdx.x; e < NBIN; e += NOWN) bins[e] = 0u;
        __syncthreads();

        // Stage: decode this thread's records and rank each within its cell.
        int my_cell[PER];
        uint32_t my_rank[PER];
        float4 my_t[PER], my_g[PER];  // (t, g_f) and (g_grad, -): the rest is derived at placement
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * NOWN;
            my_cell[u] = -1;
            if (i < m) {
                const float4 r = rec[cbeg + i];
                const float q[3] = {r.x, r.y, r.z};
                const int32_t tag = __float_as_int(r.w);
                // upstream gradients of the record's query: in record order (found through the
                // primary copy), or in query order (the query index is the primary's tag), as
                // separate arrays or packed (g_f, g_grad) in one 16-byte row of gf
                float ugf = 0.0f, ugg[3] = {0.0f, 0.0f, 0.0f};
                const int32_t prim = (tag & kRecSecondary) ? (tag & ~kRecSecondary) : cbeg + i;
                if (urec) {
                    const float4 uv = urec[prim];
                    ugf = uv.x;
                    ugg[0] = uv.y;
                    ugg[1] = uv.z;
                    ugg[2] = uv.w;
                } else {
                    const int32_t idx = (tag & kRecSecondary) ? __float_as_int(rec[prim].w) : tag;
                    if (packed) {
                        const float4 uv = reinterpret_cast<const float4*>(gf)[idx];
                        ugf = uv.x;
                        ugg[0] = uv.y;
                        ugg[1] = uv.z;
                        ugg[2] = uv.w;
                    } else {
                        if (gf) ugf = gf[idx];
                        if (gg) {
#pragma unroll
                            for (int a = 0; a < DIM; ++a) ugg[a] = gg[(int64_t)idx * DIM + a];
                        }
                    }
                }
                AxisLoc L[DIM];
                locate<DIM>(g, q, L);
                float sg[3] = {0.0f, 0.0f, 0.0f}, t[3] = {0.0f, 0.0f, 0.0f};
                int c[3] = {0, 0, 0};
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    sg[a] = L[a].clamped ? 0.0f : ugg[a];
                    t[a] = L[a].t;
                    c[a] = min(max(L[a].cell - base[a] + 1, 0), B);
                }
                if constexpr (K == kOrderRGB1) {
                    // three channels' upstream values (g_f is [3][nq]); no gradient terms: the
                    // slots of the gradient upstream carry channels 1 and 2
                    const int32_t idx = (tag & kRecSecondary) ? __float_as_int(rec[prim].w) : tag;
                    ugf = gf[idx];
                    sg[0] = gf[nq + idx];
                    sg[1] = gf[2 * nq + idx];
                    sg[2] = 0.0f;
                }
                my_cell[u] = rel_cell<DIM>(c);
                my_t[u] = make_float4(t[0], t[1], t[2], ugf);
                my_g[u] = make_float4(sg[0], sg[1], sg[2], 0.0f);
                my_rank[u] = atomicAdd(&ccount[my_cell[u]], 1u);
            }
        }
        __syncthreads();
        // exclusive scan of the cell counts
        {
            constexpr int CPT = (NCELL + NOWN - 1) / NOWN;
            uint32_t c[CPT];
            uint32_t sum = 0;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int idx = threadIdx.x * CPT + k;
                c[k] = idx < NCELL ? ccount[idx] : 0u;
                sum += c[k];
            }
            uint32_t incl = sum;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t o = __shfl_up(incl, d, 64);
                if (lane >= d) incl += o;
            }
            if (lane == 63) wsum[wave] = (int32_t)incl;
            __syncthreads();
            uint32_t before = 0;
            for (int w = 0; w < wave; ++w) before += (uint32_t)wsum[w];
            uint32_t run = before + incl - sum;
#pragma unroll
            for (int k = 0; k < CPT; ++k) {
                const int idx = threadIdx.x * CPT + k;
                if (idx < NCELL) cstart[idx] = run;
                run += c[k];
            }
            if (threadIdx.x == NOWN - 1) cstart[NCELL] = run;
        }
        __syncthreads();

        // Lane assignment: threads take vertices in decreasing order of their record count in
        // this pass, so the lanes of a wave have similar trip counts (the gather loop runs as
        // long as its longest lane).
        int v[3];
        bool owned;
        uint32_t off[NRUN], mid[NRUN], pre[NRUN + 1];
        {
            vertex_runs(threadIdx.x, v, owned, off, mid, pre);
            const uint32_t key = NBIN - 1 - min(pre[NRUN], (uint32_t)(NBIN - 1));
            const uint32_t brank = atomicAdd(&bins[key], 1u);
            __syncthreads();
            if (wave == 0) {
                constexpr int BPL = NBIN / 64;
                uint32_t c[BPL], sum = 0;
#pragma unroll
                for (int k = 0; k < BPL; ++k) {
                    c[k] = bins[lane * BPL + k];
                    sum += c[k];
                }
                uint32_t incl = sum;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t o = __shfl_up(incl, d, 64);
                    if (lane >= d) incl += o;
                }
                uint32_t run = incl - sum;
#pragma unroll
                for (int k = 0; k < BPL; ++k) {
                    bins[lane * BPL + k] = run;
                    run += c[k];
                }
            }
            __syncthreads();
            perm[bins[key] + brank] = (uint16_t)threadIdx.x;
            __syncthreads();
            vid = perm[threadIdx.x];
        }
        if (!first_pass) {
#pragma unroll
            for (int k = 0; k < C; ++k) acc[k] = vals[vid * C + k];
            __syncthreads();  // every sum is read before the records overwrite the table
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            if (my_cell[u] < 0) continue;
            const uint32_t pos = cstart[my_cell[u]] + my_rank[u];
            const float4 t = my_t[u], sg = my_g[u];
            const float ta[3] = {t.x, t.y, t.z};
            ent[kEntStride * pos] = make_float4(t.w, sg.x, sg.y, sg.z);
#pragma unroll
            for (int a = 0; a < DIM; ++a)
                ent[kEntStride * pos + 1 + a] =
                    make_float4(1.0f - ta[a], ta[a] * g.h[a], ta[a], (ta[a] - 1.0f) * g.h[a]);
        }

        __syncthreads();  // records placed
        vertex_runs(vid, v, owned, off, mid, pre);

        const uint32_t total = pre[NRUN];
        for (uint32_t k = 0; k < total; ++k) {
            uint32_t e = off[0] + k, md = mid[0];
            int j = 0;
#pragma unroll
            for (int jj = 1; jj < NRUN; ++jj)
                if (k >= pre[jj]) {
                    e = off[jj] + k;
                    md = mid[jj];
                    j = jj;
                }
            // b[a]: the record lies in the cell below the vertex on axis a, so the vertex is
            // that cell's upper corner
            const bool b[3] = {e < md, (j & 1) != 0, (j >> 1) != 0};
            // e < kBwdItem: the 24-bit multiply is full rate (a 32-bit one takes 4 passes)
            const float* er = reinterpret_cast<const float*>(reinterpret_cast<const char*>(ent) +
                                                             __umul24(e, (uint32_t)sizeof(float4) * kEntStride));
            const float4 E0 = *reinterpret_cast<const float4*>(er);
            const float sg[3] = {E0.y, E0.z, E0.w};
            float fa[DIM], d[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const float2 P = *reinterpret_cast<const float2*>(er + 4 * (1 + a) + (b[a] ? 2 : 0));
                fa[a] = P.x;  // this corner's weight factor on axis a
                d[a] = P.y;   // offset from the vertex, world units
            }
            float w, fo[DIM];  // fo[a]: product of the other axes' factors
            if constexpr (DIM == 3) {
                fo[0] = fa[1] * fa[2];
                fo[1] = fa[0] * fa[2];
                fo[2] = fa[0] * fa[1];
                w = fa[0] * fo[0];
            } else {
                fo[0] = fa[1];
                fo[1] = fa[0];
                w = fa[0] * fa[1];
            }
            float dw[DIM];  // d w / d x_a: +-(1/h_a) fo[a], + for the upper corner
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const float p = g.inv_h[a] * fo[a];
                dw[a] = b[a] ? p : -p;
            }
            if constexpr (K == kOrderRGB1) {
                // each channel is an order-1 series with upstream value only
                const float up[kRGB] = {E0.x, sg[0], sg[1]};
                const float zero[DIM] = {};
#pragma unroll
                for (int ch = 0; ch < kRGB; ++ch) accumulate_corner<DIM, 1>(d, up[ch] * w, zero, acc + ch * (1 + DIM));
            } else {
                float s = E0.x * w;
                float uu[DIM];
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    s = fmaf(sg[a], dw[a], s);
                    uu[a] = w * sg[a];
                }
                accumulate_corner<DIM, K>(d, s, uu, acc);
            }
        }
    }

    // Hand the sums over through LDS in [vertex][C] order (the record table is free now),
    // then write them row by row.
    __syncthreads();
#pragma unroll
    for (int k = 0; k < C; ++k) vals[vid * C + k] = acc[k];
    __syncthreads();
    float vk[C];
#pragma unroll
    for (int k = 0; k < C; ++k) vk[k] = vals[epi_elem<DIM, C>(k)];
    if (nchunk > 1) {
        // partial sums of a split brick: slot = item index, laid out [vertex][C]
        float* slot = parts + (int64_t)item * (NOWN * C);
#pragma unroll
        for (int k = 0; k < C; ++k) slot[epi_elem<DIM, C>(k)] = vk[k];
        if constexpr (AD < 0) {
            return;  // the merge launch adds the slots
        } else {
            // The item that finishes last adds the brick's slots in item order (the same sums
            // whichever item it is).  The release fence makes this slot visible to every XCD
            // before the count moves; the acquire fence drops this XCD's stale copies of the
            // other slots.  Only bricks above kBwdWholeMax records come here.
            __shared__ int32_t last_item;
            __threadfence();
            __syncthreads();
            if (threadIdx.x == 0) last_item = atomicAdd(&split[brick].x, 1) == nchunk - 1;
            __syncthreads();
            if (!last_item) {
                if (threadIdx.x == 0) AB.partials[bid] = 0.0;  // the last item counts the brick
                return;
            }
            __threadfence();
            if (threadIdx.x == 0) split[brick].x = 0;  // ready for the next call on this sort
#pragma unroll
            for (int k = 0; k < C; ++k) vk[k] = 0.0f;
            for (int32_t j = 0; j < nchunk; ++j) {
                const float* sl = parts + (int64_t)(first_item + j) * (NOWN * C);
#pragma unroll
                for (int k = 0; k < C; ++k) vk[k] += sl[epi_elem<DIM, C>(k)];
            }
        }
    }
    if constexpr (AD >= 0) {
        const double tot = block_sum_f64<NOWN>(brick_epilogue<DIM, C, AD>(g, base, nown, vk, grad, 0, AB));
        if (threadIdx.x == 0) AB.partials[bid] = tot;
    } else {
        brick_epilogue<DIM, C, AD>(g, base, nown, vk, grad, accumulate, AB);
    }
}

// The adjoint without Adam: adds the partial sums of every split brick, in slot order, and
// writes (or accumulates) the brick's gradient.  Block b takes split bricks b, b + G, ... (G
// blocks).
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
    const int32_t nsplit = meta[META_NSPLITB];
    for (int32_t sb = blockIdx.x; sb < nsplit; sb += gridDim.x) {
        const int32_t first = split_first[sb];
        const int4 wi = items[first];
        const int32_t brick = wi.x, nchunk = wi.w;
        int32_t bc[3], base[3], nown[3];
        vbrick_coords<DIM>(g, brick, bc);
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            base[a] = bc[a] * B;
            nown[a] = min(B, g.res[a] - base[a]);
        }
        float vk[C];
#pragma unroll
        for (int k = 0; k < C; ++k) vk[k] = 0.0f;
        for (int j = 0; j < nchunk; ++j) {
            const float* slot = parts + (int64_t)(first + j) * (NOWN * C);
#pragma unroll
            for (int k = 0; k < C; ++k) vk[k] += slot[epi_elem<DIM, C>(k)];
        }
        brick_epilogue<DIM, C, -1>(g, base, nown, vk, grad, accumulate, AdamBuf{});
    }
}

template <int AD>
static hipError_t launch_backward_impl(const tg_grid* g, const char* ws, const WsLayout& L, const float* g_f,
                                       const float* g_grad, const float4* urec, bool accumulate, const AdamBuf& AB,
                                       hipStream_t s, int64_t nq, bool packed)
{
    const float4* rec = reinterpret_cast<const float4*>(ws + L.rec_off);
    const int4* items = reinterpret_cast<const int4*>(ws + L.bitems_off);
    const int32_t* meta = reinterpret_cast<const int32_t*>(ws + L.meta_off);
    float* parts = reinterpret_cast<float*>(const_cast<char*>(ws) + L.parts_off);
    const int32_t* split_first = reinterpret_cast<const int32_t*>(ws + L.splitb_off);
    int2* split = reinterpret_cast<int2*>(const_cast<char*>(ws) + L.split_off);
    const dim3 grid((unsigned)L.max_bitems);
    const int dim = g->desc.dim, K = g->kord;
    float* gr = g->bufs.grad;
    const int acc = accumulate ? 1 : 0;
#define TG_BWD_CASE(D, KK)                                                                                   \
    if (dim == D && K == KK) {                                                                               \
        const dim3 block(BwdShape<D>::NOWN);                                                                 \
        hipLaunchKernelGGL((k_backward<D, KK, AD>), grid, block, 0, s, g->geom, items, meta, L.max_bitems, parts, \
                           split, rec, g_f, packed ? nullptr : g_grad, urec, gr, acc, AB, nq, packed ? 1 : 0); \
        if (AD < 0)                                                                                           \
            hipLaunchKernelGGL((k_backward_merge<D, KK>), dim3((unsigned)L.merge_blocks), block, 0, s, g->geom, \
                               items, split_first, meta, parts, gr, acc);                                   \
        return hipGetLastError();                                                                            \
    }
    TG_BWD_CASE(3, 2) TG_BWD_CASE(3, 1) TG_BWD_CASE(3, 0) TG_BWD_CASE(2, 2) TG_BWD_CASE(2, 1) TG_BWD_CASE(2, 0)
    TG_BWD_CASE(3, kOrderFull) TG_BWD_CASE(2, kOrderFull) TG_BWD_CASE(3, kOrderRGB1) TG_BWD_CASE(2, kOrderRGB1)
#undef TG_BWD_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_backward(const tg_grid* g, int64_t n, const char* ws, const WsLayout& L, const float* g_f,
                           const float* g_grad, bool accumulate, hipStream_t s, bool packed)
{
    return launch_backward_impl<-1>(g, ws, L, g_f, g_grad, nullptr, accumulate, AdamBuf{}, s, n, packed);
}

hipError_t launch_backward_adam(const tg_grid* g, int64_t n, const char* ws, const WsLayout& L, const float* g_f,
                                const float* g_grad, const tg_adam_params& p, double* grad_norm_sq, hipStream_t s,
                                bool record_order, const float* extra_grad, bool packed)
{
    const float4* urec = record_order ? reinterpret_cast<const float4*>(ws + L.urec_off) : nullptr;
    AdamBuf AB;
    AB.A = make_adam_args(p);
    AB.master = g->bufs.master;
    AB.m = g->bufs.adam_m;
    AB.v = g->bufs.adam_v;
    AB.coeffs = g->bufs.coeffs;
    AB.partials = reinterpret_cast<double*>(const_cast<char*>(ws) + L.bpart_off);
    AB.extra = extra_grad;
    hipError_t e;
    switch (g->desc.storage) {
    case ST_F32: e = launch_backward_impl<ST_F32>(g, ws, L, g_f, g_grad, urec, false, AB, s, n, packed); break;
    case ST_BF16: e = launch_backward_impl<ST_BF16>(g, ws, L, g_f, g_grad, urec, false, AB, s, n, packed); break;
    default: e = launch_backward_impl<ST_F16>(g, ws, L, g_f, g_grad, urec, false, AB, s, n, packed); break;
    }
    if (e != hipSuccess || !grad_norm_sq) return e;
    return launch_sum_finish(AB.partials, L.max_bitems, grad_norm_sq, s);
}

}  // namespace tg
