// TaylorGrid adjoint with respect to the coefficients, owner-computes per vertex brick.
//
// The field and its gradient are linear in the coefficients; for upstream gradients
// (g_f, g_grad) a query contributes to coefficient alpha of corner vertex v_b
//   m_alpha(d_b) s_b + sum_a u_a dm_alpha/dd_a(d_b),   s_b = g_f w_b + g_grad . grad w_b,
//   u = w_b g_grad,  m_alpha(d) = d^alpha / alpha!  (the Taylor monomials of Sec. 3.1, Eq. 1).
// One workgroup owns a brick of B^dim vertices and accumulates, in LDS, the contributions
// of every query whose cell touches one of its vertices (the primary and secondary buckets
// of that vertex brick, see tg_sort.hip); the brick is then written to HBM once with
// coalesced row stores.  No global atomics, and every vertex is written exactly once.
//
// LDS accumulation: LDS floating-point atomics are an order of magnitude slower than LDS
// integer atomics on this GPU, so each vertex's accumulator is updated with a plain
// vectorised read-add-write (float4) under a per-vertex claim taken with an integer LDS
// compare-and-swap.  Two lanes only contend when their queries share a vertex, which is
// rare in the bucket's arbitrary order; a lane that loses the claim retries.
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

// Accumulator row stride: C rounded up to a multiple of 4 (one float4 per 4 coefficients).
template <int C> struct AccPad { static constexpr int value = (C + 3) / 4 * 4; };

template <int C, int CP>
__device__ __forceinline__ void add_row(float* row, const float* v)
{
    float4* p = reinterpret_cast<float4*>(row);
#pragma unroll
    for (int k = 0; k < CP / 4; ++k) {
        float4 a = p[k];
        a.x += v[4 * k + 0];
        if (4 * k + 1 < C) a.y += v[4 * k + 1];
        if (4 * k + 2 < C) a.z += v[4 * k + 2];
        if (4 * k + 3 < C) a.w += v[4 * k + 3];
        p[k] = a;
    }
}

// Blocks are visited in an order that gives each XCD (blocks are dealt round-robin to the
// 8 XCDs) a contiguous range of bricks, so neighbouring bricks share an L2.
__device__ __forceinline__ int32_t xcd_brick(int64_t nbricks)
{
    const int32_t per = (int32_t)((nbricks + 7) / 8);
    return (int32_t)(blockIdx.x % 8) * per + (int32_t)(blockIdx.x / 8);
}

template <int DIM, int K>
__global__ __launch_bounds__(kThreads) void k_backward(Geom g, int64_t nbricks, const float4* __restrict__ rec,
                                                      const int32_t* __restrict__ offs,
                                                      const float* __restrict__ gf, const float* __restrict__ gg,
                                                      float* __restrict__ grad, int accumulate)
{
    constexpr int B = BrickEdge<DIM>::value;
    constexpr int C = NumCoeffs<DIM, K>::value;
    constexpr int CP = AccPad<C>::value;
    constexpr int NOWN = DIM == 3 ? B * B * B : B * B;
    __shared__ __align__(16) float acc[NOWN * CP];
    __shared__ uint32_t claim[NOWN];

    const int32_t brick = xcd_brick(nbricks);
    if (brick >= nbricks) return;
    const int32_t beg = offs[2 * brick];
    const int32_t end = offs[2 * brick + 2];
    if (accumulate && beg == end) return;

    int32_t bc[3];
    vbrick_coords<DIM>(g, brick, bc);
    int32_t base[3], nown[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        base[a] = bc[a] * B;
        nown[a] = min(B, g.res[a] - base[a]);
    }

    for (int e = threadIdx.x; e < NOWN * CP / 4; e += kThreads)
        reinterpret_cast<float4*>(acc)[e] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    for (int e = threadIdx.x; e < NOWN; e += kThreads) claim[e] = 0u;
    __syncthreads();

    for (int32_t j = beg + threadIdx.x; j < end; j += kThreads) {
        const float4 r = rec[j];
        const float q[3] = {r.x, r.y, r.z};
        const int32_t idx = __float_as_int(r.w);
        AxisLoc L[DIM];
        locate<DIM>(g, q, L);
        const AxisFactors<DIM> F = axis_factors<DIM>(g, L);
        const float sf = gf ? gf[idx] : 0.0f;
        float sg[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) sg[a] = (gg && !L[a].clamped) ? gg[(int64_t)idx * DIM + a] : 0.0f;
        int rel[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) rel[a] = L[a].cell - base[a];  // in [-1, B - 1]

#pragma unroll
        for (int b = 0; b < (1 << DIM); ++b) {
            int lv[DIM];
            bool owned = true;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                lv[a] = rel[a] + ((b >> a) & 1);
                owned = owned && lv[a] >= 0 && lv[a] < nown[a];
            }
            if (!owned) continue;
            float w, dw[DIM];
            corner_weight<DIM>(F, b, w, dw);
            float d[DIM];
            corner_offset<DIM>(F, b, d);
            float s = sf * w;
            float u[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                s = fmaf(sg[a], dw[a], s);
                u[a] = w * sg[a];
            }
            float out[CP];
            corner_adjoint<DIM, K>(d, s, u, out);
#pragma unroll
            for (int k = C; k < CP; ++k) out[k] = 0.0f;
            int l = lv[0] + B * lv[1];
            if constexpr (DIM == 3) l += B * B * lv[2];
            // Claim-protected update, in wave-uniform rounds: in each round every lane that
            // still has to update tries to claim its vertex; a winner updates and releases
            // within the same round (the compiler barrier keeps the update and the release
            // inside the round), so a lane that lost waits at most for holders that are
            // already inside their bounded update.  Every claim starts at 0.
            bool done = false;
            do {
                bool mine = false;
                if (!done) {
                    uint32_t expect = 0u;
                    mine = __hip_atomic_compare_exchange_strong(&claim[l], &expect, 1u, __ATOMIC_ACQUIRE,
                                                                __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
                }
                if (mine) {
                    add_row<C, CP>(acc + l * CP, out);
                    __hip_atomic_store(&claim[l], 0u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_WORKGROUP);
                    done = true;
                }
                asm volatile("" ::: "memory");
            } while (__any(!done));
        }
    }
    __syncthreads();

    // Write the owned vertices: each row of nown[0] vertices is C * nown[0] contiguous floats.
    constexpr int ROWLEN = B * C;
    for (int e = threadIdx.x; e < NOWN * C; e += kThreads) {
        const int row = e / ROWLEN;
        const int rem = e - row * ROWLEN;
        const int vx = rem / C;
        const int cc = rem - vx * C;
        const int ry = DIM == 3 ? row % B : row;
        const int rz = DIM == 3 ? row / B : 0;
        bool ok = vx < nown[0] && ry < nown[1];
        if constexpr (DIM == 3) ok = ok && rz < nown[2];
        if (!ok) continue;
        int64_t vert = (int64_t)(base[0] + vx) + (int64_t)(base[1] + ry) * g.stride[1];
        if constexpr (DIM == 3) vert += (int64_t)(base[2] + rz) * g.stride[2];
        float* p = grad + vert * C + cc;
        const float v = acc[(row * B + vx) * CP + cc];
        if (accumulate) *p += v;
        else *p = v;
    }
}

hipError_t launch_backward(const tg_grid* g, int64_t n, const char* ws, const WsLayout& L, const float* g_f,
                           const float* g_grad, bool accumulate, hipStream_t s)
{
    (void)n;
    const float4* rec = reinterpret_cast<const float4*>(ws + L.rec_off);
    const int32_t* offs = reinterpret_cast<const int32_t*>(ws + L.offs_off);
    const dim3 grid((unsigned)(8 * ((g->nbricks + 7) / 8))), block(kThreads);
    const int dim = g->desc.dim, K = g->desc.order;
    float* gr = g->bufs.grad;
    const int acc = accumulate ? 1 : 0;
#define TG_BWD_CASE(D, KK)                                                                                    \
    if (dim == D && K == KK) {                                                                                \
        hipLaunchKernelGGL((k_backward<D, KK>), grid, block, 0, s, g->geom, g->nbricks, rec, offs, g_f, g_grad, gr, \
                           acc);                                                                              \
        return hipGetLastError();                                                                             \
    }
    TG_BWD_CASE(3, 2) TG_BWD_CASE(3, 1) TG_BWD_CASE(3, 0) TG_BWD_CASE(2, 2) TG_BWD_CASE(2, 1) TG_BWD_CASE(2, 0)
#undef TG_BWD_CASE
    return hipErrorInvalidValue;
}

}  // namespace tg
