// TaylorGrid forward (value and spatial gradient) and the query adjoint dq, per brick.
//
// One workgroup per brick of B^dim cells.  It stages the (B+1)^dim vertex coefficient
// blocks that the brick's cells touch into LDS as FP32 (converting BF16/FP16 storage on
// the way), with coalesced row loads, then evaluates every query bucketed to the brick
// (its primary records) reading corners from LDS:
//   f = sum_b w_b T_b(d_b),  grad f = sum_b (grad w_b T_b + w_b grad T_b)      (Sec. 3.1, Eq. 2-4)
// Results are written in the caller's query order: f and grad f as separate arrays, or
// packed as one 16-byte row (f, grad f) per query, which takes one store (the queries are
// evaluated in bucket order, so these stores land at scattered rows).  The dq mode evaluates
// the field's Hessian as well and writes dq = g_f grad f + Hess f . g_grad, reading the
// upstream gradients from separate arrays or from one packed row per query.
#include "tg_internal.hpp"

namespace tg {

enum { MODE_FWD = 0, MODE_DQ = 1, MODE_LOSS = 2 };

// The SDF objective evaluated in the forward's epilogue (Sec. 3.2 Eq. 6 and the eikonal term
// of Eq. 8): per query r = f - d, g_f = sign(r) / n, and with an eikonal term
// g_grad = 2 w (|grad f| - 1) grad f / (|grad f| n) (zero where grad f = 0); per workgroup
// the FP64 sums of |r| and (|grad f| - 1)^2.
// With urec != NULL the upstream gradients go to urec, indexed by record position (the
// training step keeps them in bucket order).
struct LossArgs {
    const float* d;     // target SDF, query order
    float* gf;          // upstream gradient of f, query order
    float* gg;          // upstream gradient of grad f (NULL: no eikonal term)
    float4* urec;       // (g_f, g_grad) in record order
    double* partials;   // [2 x gridDim.x]
    float w_eik;
    float surf_k;       // Eq. 7's k (0: every sample weighted 1)
    float inv_n;
    int eik;            // eikonal term on (record mode; query mode tests gg)
    int64_t nq;         // queries: the channel stride of a three-channel field's output
    int packed;         // MODE_FWD: f_out is [n][4] (f, grad f); MODE_DQ: gf is [n][4] (g_f, g_grad)
};

// (v, x, y, z) of one query as a 16-byte row; in 2D the last word is 0.
template <int DIM>
__device__ __forceinline__ float4 pack_row(float v, const float* x)
{
    return make_float4(v, x[0], x[1], DIM == 3 ? x[DIM - 1] : 0.0f);
}

template <int DIM> __device__ __forceinline__ void brick_coords(const Geom& g, int32_t brick, int32_t* bc)
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

// Staged vertex blocks in LDS, unpadded, in the brick's row order.  FP32 storage and 16-bit
// storage with an even coefficient count are copied verbatim (LDS_PACKED: two 16-bit values
// per word, widened when read); 16-bit storage with an odd count is widened while staged.
template <int ST, int C> struct StageFmt {
    static constexpr bool PACKED = ST != ST_F32 && C % 2 == 0;
    static constexpr bool DMA = ST == ST_F32 || PACKED;    // copy global -> LDS directly
    static constexpr int WPV = PACKED ? C / 2 : C;         // LDS words per vertex
};

template <int ST, int C>
__device__ __forceinline__ void lds_vertex(const uint32_t* lds, int lv, float* c)
{
    using F = StageFmt<ST, C>;
    const uint32_t* p = lds + lv * F::WPV;
    if constexpr (F::PACKED) {
#pragma unroll
        for (int k = 0; k < C / 2; ++k) {
            const uint32_t w = p[k];
            if constexpr (ST == ST_BF16) {
                c[2 * k] = bf16_bits_to_float(w & 0xffffu);
                c[2 * k + 1] = bf16_bits_to_float(w >> 16);
            } else {
                c[2 * k] = f16_bits_to_float(w & 0xffffu);
                c[2 * k + 1] = f16_bits_to_float(w >> 16);
            }
        }
    } else if constexpr (C % 2 == 0) {
#pragma unroll
        for (int k = 0; k < C / 2; ++k) {
            const float2 v = reinterpret_cast<const float2*>(p)[k];  // 8-byte aligned: C even
            c[2 * k] = v.x;
            c[2 * k + 1] = v.y;
        }
    } else {
#pragma unroll
        for (int k = 0; k < C; ++k) c[k] = __uint_as_float(p[k]);
    }
}

typedef __attribute__((address_space(3))) void* lds_addr_t;

// Hessian entry index of (a, c) in the packed order xx, xy, xz, yy, yz, zz / xx, xy, yy.
template <int DIM> __host__ __device__ constexpr int hidx(int a, int c)
{
    return DIM == 3 ? (a > c ? hidx<DIM>(c, a) : (a == 0 ? c : (a == 1 ? 2 + c : 5)))
                    : (a > c ? hidx<DIM>(c, a) : (a == 0 ? c : 2));
}

template <int DIM, int K, int ST, int MODE>
__global__ __launch_bounds__(kThreads) void k_forward(Geom g, const int4* __restrict__ items,
                                                     const int32_t* __restrict__ meta, const void* __restrict__ coeffs,
                                                     const float4* __restrict__ rec,
                                                     float* __restrict__ f_out, float* __restrict__ grad_out,
                                                     const float* __restrict__ gf, const float* __restrict__ gg,
                                                     float* __restrict__ dq_out, LossArgs LA)
{
    constexpr int B = BrickEdge<DIM>::value;
    constexpr int C = NumCoeffs<DIM, K>::value;
    using SF = StageFmt<ST, C>;
    constexpr int NV1 = B + 1;
    constexpr int NROWS = DIM == 3 ? NV1 * NV1 : NV1;
    constexpr int ROWW = NV1 * SF::WPV;  // LDS words per row of NV1 vertices along x
    constexpr int NWIN = (NROWS * ROWW + 63) / 64;
    constexpr int NH = DIM == 3 ? 6 : 3;
    __shared__ __align__(16) uint32_t lds[NWIN * 64];

    // Work item = (brick, chunk of up to kFwdChunk primary records), in XCD-aware list order:
    // short runs of neighbouring items per XCD, so the crowded bricks of a surface, which are
    // neighbours in the list, still spread over all XCDs (giving each XCD one contiguous
    // range of items instead was measured slower: the XCDs holding the surface finished last).
    const int32_t total = meta[META_FITEMS];
    const int32_t item = xcd_grouped<kXcdGroup>((int32_t)blockIdx.x, total);
    const int4 wi = item < total ? items[item] : make_int4(0, 0, 0, 0);
    const int32_t brick = wi.x, beg = wi.y, end = wi.z;
    if (beg >= end) {
        if constexpr (MODE == MODE_LOSS) {
            if (threadIdx.x == 0) {
                LA.partials[2 * blockIdx.x] = 0.0;
                LA.partials[2 * blockIdx.x + 1] = 0.0;
            }
        }
        return;
    }
    // A thread's records are kThreads apart; each is loaded before the previous one is
    // evaluated, the first before the brick's coefficients are staged.
    int32_t j = beg + threadIdx.x;
    float4 rnext = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
    if (j < end) rnext = rec[j];

    int32_t bc[3];
    brick_coords<DIM>(g, brick, bc);
    int32_t v0[3], nv[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        v0[a] = bc[a] * B;
        nv[a] = min(B, g.res[a] - 1 - v0[a]) + 1;  // >= 2 for a brick that has queries
    }

    // Stage the brick's vertices.  The (B+1)^dim vertex blocks are NROWS rows of ROWW
    // contiguous words in memory, kept in the same order in LDS; the waves copy them straight
    // from global memory into LDS (global_load_lds), all in flight at once and without
    // passing through registers.  Words of rows or vertices outside the grid are not loaded
    // (no query reads them).
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if constexpr (SF::DMA && ROWW >= 32) {
        // Rows of at least half a wave: a wave copies whole rows, 64 words per load, so the
        // row's position (wave-uniform) is computed once in scalar registers and a lane only
        // adds its word offset.  (Per-lane row and column arithmetic in 64-bit cost ~45 vector
        // instructions per load, most of this kernel's instruction issue.)
        // The rows inside the grid are walked z by z, each wave taking every NW-th y row, with
        // the source pointer advanced by additions (a few scalar instructions per row).
        constexpr int NCH = (ROWW + 63) / 64;
        constexpr int NW = kThreads / 64;
        const int nw0 = nv[0] * SF::WPV;  // words of the row inside the grid
        const int wv = __builtin_amdgcn_readfirstlane(wave);
        const int nz = DIM == 3 ? nv[2] : 1;
        const int64_t ystep = g.stride[1] * SF::WPV;  // words from one y row to the next
        int64_t v00 = (int64_t)v0[0] + (int64_t)v0[1] * g.stride[1];
        if constexpr (DIM == 3) v00 += (int64_t)v0[2] * g.stride[2];
        const uint32_t* zsrc = static_cast<const uint32_t*>(coeffs) + v00 * SF::WPV;
        for (int rz = 0; rz < nz; ++rz) {
            const uint32_t* rsrc = zsrc + wv * ystep;
            for (int ry = wv; ry < nv[1]; ry += NW) {
                const int row = rz * NV1 + ry;
#pragma unroll
                for (int c = 0; c < NCH; ++c) {
                    const int off = c * 64 + lane;
                    if (off < nw0)
                        __builtin_amdgcn_global_load_lds(static_cast<const void*>(rsrc + off),
                                                         (lds_addr_t)(lds + row * ROWW + c * 64), 4, 0, 0);
                }
                rsrc += NW * ystep;
            }
            if constexpr (DIM == 3) zsrc += g.stride[2] * SF::WPV;
        }
    } else if constexpr (SF::DMA) {
        // short rows: 64-word windows of the flattened rows
        const uint32_t* src = static_cast<const uint32_t*>(coeffs);
        for (int w = wave; w < NWIN; w += kThreads / 64) {
            const int base = w * 64;
            const int e = base + lane;
            const int row = e / ROWW, off = e - row * ROWW;
            const int ry = DIM == 3 ? row % NV1 : row;
            const int rz = DIM == 3 ? row / NV1 : 0;
            bool ok = row < NROWS && ry < nv[1] && off < nv[0] * SF::WPV;
            if constexpr (DIM == 3) ok = ok && rz < nv[2];
            if (ok) {
                int64_t vrow = (int64_t)v0[0] + (int64_t)(v0[1] + ry) * g.stride[1];
                if constexpr (DIM == 3) vrow += (int64_t)(v0[2] + rz) * g.stride[2];
                __builtin_amdgcn_global_load_lds(static_cast<const void*>(src + vrow * SF::WPV + off),
                                                 (lds_addr_t)(lds + base), 4, 0, 0);
            }
        }
    } else {
        // 16-bit storage with an odd coefficient count: widen through registers
        for (int e = threadIdx.x; e < NROWS * ROWW; e += kThreads) {
            const int row = e / ROWW, off = e - row * ROWW;
            const int ry = DIM == 3 ? row % NV1 : row;
            const int rz = DIM == 3 ? row / NV1 : 0;
            bool ok = ry < nv[1] && off < nv[0] * C;
            if constexpr (DIM == 3) ok = ok && rz < nv[2];
            if (!ok) continue;
            int64_t vrow = (int64_t)v0[0] + (int64_t)(v0[1] + ry) * g.stride[1];
            if constexpr (DIM == 3) vrow += (int64_t)(v0[2] + rz) * g.stride[2];
            lds[e] = __float_as_uint(load_scalar<ST>(coeffs, vrow * C + off));
        }
    }
    __syncthreads();

    double sum_r = 0.0, sum_e = 0.0;  // loss sums (MODE_LOSS)
    for (; j < end; j += kThreads) {
        const float4 r = rnext;
        if (j + kThreads < end) rnext = rec[j + kThreads];
        const float q[3] = {r.x, r.y, r.z};
        const int32_t idx = __float_as_int(r.w);
        // the loss's target, loaded before the corner loop so that its latency hides behind it
        float dt = 0.0f;
        if constexpr (MODE == MODE_LOSS) {
            dt = LA.d[idx];
            __builtin_amdgcn_sched_barrier(0);  // keep the load here; it is waited for at its use
        }
        AxisLoc L[DIM];
        locate<DIM>(g, q, L);
        int lc[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) lc[a] = min(max(L[a].cell - v0[a], 0), nv[a] - 2);
        const AxisFactors<DIM> F = axis_factors<DIM>(g, L);

        if constexpr (K == kOrderRGB1) {
            // three order-1 channels: value only, written channel-major (f_out[ch][query])
            if constexpr (MODE == MODE_FWD) {
                float fc[kRGB] = {0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int b = 0; b < (1 << DIM); ++b) {
                    int lv = lc[0] + (b & 1) + NV1 * (lc[1] + ((b >> 1) & 1));
                    if constexpr (DIM == 3) lv += NV1 * NV1 * (lc[2] + ((b >> 2) & 1));
                    float c[C];
                    lds_vertex<ST, C>(lds, lv, c);
                    float d[DIM];
                    corner_offset<DIM>(F, b, d);
                    float w, dw[DIM];
                    corner_weight<DIM>(F, b, w, dw);
#pragma unroll
                    for (int ch = 0; ch < kRGB; ++ch) {
                        float T = c[ch * (1 + DIM)];
#pragma unroll
                        for (int a = 0; a < DIM; ++a) T = fmaf(c[ch * (1 + DIM) + 1 + a], d[a], T);
                        fc[ch] = fmaf(w, T, fc[ch]);
                    }
                }
#pragma unroll
                for (int ch = 0; ch < kRGB; ++ch) f_out[ch * LA.nq + idx] = fc[ch];
            }
            continue;
        }

        float f = 0.0f;
        float gr[DIM];
        float hf[NH];
#pragma unroll
        for (int a = 0; a < DIM; ++a) gr[a] = 0.0f;
#pragma unroll
        for (int k = 0; k < NH; ++k) hf[k] = 0.0f;

#pragma unroll
        for (int b = 0; b < (1 << DIM); ++b) {
            int lv = lc[0] + (b & 1) + NV1 * (lc[1] + ((b >> 1) & 1));
            if constexpr (DIM == 3) lv += NV1 * NV1 * (lc[2] + ((b >> 2) & 1));
            float c[C];
            lds_vertex<ST, C>(lds, lv, c);
            float d[DIM];
            corner_offset<DIM>(F, b, d);
            float T, dT[DIM];
            taylor_eval<DIM, K>(c, d, T, dT);
            float w, dw[DIM];
            corner_weight<DIM>(F, b, w, dw);
            f = fmaf(w, T, f);
#pragma unroll
            for (int a = 0; a < DIM; ++a) gr[a] = fmaf(dw[a], T, fmaf(w, dT[a], gr[a]));
            if constexpr (MODE == MODE_DQ) {
                float H[NH];
                taylor_hess<DIM, K>(c, H);
                float d2w[DIM == 3 ? 3 : 1];
                corner_weight_d2<DIM>(F, b, d2w);
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
#pragma unroll
                    for (int cc = a; cc < DIM; ++cc) {
                        const int k = hidx<DIM>(a, cc);
                        float v = fmaf(w, H[k], fmaf(dw[a], dT[cc], dw[cc] * dT[a]));
                        if (a != cc) {
                            const int m = DIM == 3 ? (a == 0 ? cc - 1 : 2) : 0;  // xy, xz, yz
                            v = fmaf(d2w[m], T, v);
                        }
                        hf[k] += v;
                    }
                }
            }
        }
#pragma unroll
        for (int a = 0; a < DIM; ++a)
            if (L[a].clamped) gr[a] = 0.0f;

        if (MODE == MODE_FWD && LA.packed) {
            reinterpret_cast<float4*>(f_out)[idx] = pack_row<DIM>(f, gr);
        } else if constexpr (MODE == MODE_FWD || MODE == MODE_LOSS) {
            if (f_out) f_out[idx] = f;
            if (grad_out) {
#pragma unroll
                for (int a = 0; a < DIM; ++a) grad_out[(int64_t)idx * DIM + a] = gr[a];
            }
        }
        if constexpr (MODE == MODE_LOSS) {
            const bool rec_mode = LA.urec != nullptr;
            const float res = f - dt;
            const float w = surface_weight(LA.surf_k, f, dt);  // held fixed in the gradient
            sum_r += (double)w * (double)fabsf(res);
            const float wn = w * LA.inv_n;
            const float sgf = res > 0.0f ? wn : (res < 0.0f ? -wn : 0.0f);
            float sgg[3] = {0.0f, 0.0f, 0.0f};
            if (rec_mode ? LA.eik != 0 : LA.gg != nullptr) {
                float n2 = 0.0f;
#pragma unroll
                for (int a = 0; a < DIM; ++a) n2 = fmaf(gr[a], gr[a], n2);
                const float nrm = sqrtf(n2);
                const float e = nrm - 1.0f;
                sum_e += (double)e * (double)e;
                const float k = nrm > 0.0f ? 2.0f * LA.w_eik * e / nrm * LA.inv_n : 0.0f;
#pragma unroll
                for (int a = 0; a < DIM; ++a) sgg[a] = k * gr[a];
            }
            if (rec_mode) {
                LA.urec[j] = make_float4(sgf, sgg[0], sgg[1], sgg[2]);
            } else {
                LA.gf[idx] = sgf;
                if (LA.gg) {
#pragma unroll
                    for (int a = 0; a < DIM; ++a) LA.gg[(int64_t)idx * DIM + a] = sgg[a];
                }
            }
        }
        if constexpr (MODE == MODE_DQ) {
            float sf, sg[DIM];
            if (LA.packed) {
                const float4 u = reinterpret_cast<const float4*>(gf)[idx];
                const float uu[3] = {u.y, u.z, u.w};
                sf = u.x;
#pragma unroll
                for (int a = 0; a < DIM; ++a) sg[a] = L[a].clamped ? 0.0f : uu[a];
            } else {
                sf = gf ? gf[idx] : 0.0f;
#pragma unroll
                for (int a = 0; a < DIM; ++a) sg[a] = (gg && !L[a].clamped) ? gg[(int64_t)idx * DIM + a] : 0.0f;
            }
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                float v = sf * gr[a];
#pragma unroll
                for (int cc = 0; cc < DIM; ++cc) v = fmaf(sg[cc], hf[hidx<DIM>(a, cc)], v);
                dq_out[(int64_t)idx * DIM + a] = L[a].clamped ? 0.0f : v;
            }
        }
    }
    if constexpr (MODE == MODE_LOSS) {
        const double tr = block_sum_f64<kThreads>(sum_r);
        const double te = block_sum_f64<kThreads>(sum_e);
        if (threadIdx.x == 0) {
            LA.partials[2 * blockIdx.x] = tr;
            LA.partials[2 * blockIdx.x + 1] = te;
        }
    }
}

template <int MODE>
static hipError_t dispatch(const tg_grid* g, const char* ws, const WsLayout& L, float* f, float* grad_f,
                           const float* gf, const float* gg, float* dq, hipStream_t s, LossArgs LA = LossArgs{})
{
    const float4* rec = reinterpret_cast<const float4*>(ws + L.rec_off);
    const int4* items = reinterpret_cast<const int4*>(ws + L.fitems_off);
    const int32_t* meta = reinterpret_cast<const int32_t*>(ws + L.meta_off);
    const dim3 grid((unsigned)L.fwd_blocks), block(kThreads);
    const void* cf = g->bufs.coeffs;
    const int dim = g->desc.dim, K = g->kord, st = g->desc.storage;
#define TG_FWD_CASE(D, KK, ST)                                                                          \
    if (dim == D && K == KK && st == ST) {                                                              \
        hipLaunchKernelGGL((k_forward<D, KK, ST, MODE>), grid, block, 0, s, g->geom, items, meta, cf, rec, f,       \
                           grad_f, gf, gg, dq, LA);                                                     \
        return hipGetLastError();                                                                       \
    }
#define TG_FWD_ST(D, KK) TG_FWD_CASE(D, KK, ST_F32) TG_FWD_CASE(D, KK, ST_BF16) TG_FWD_CASE(D, KK, ST_F16)
    TG_FWD_ST(3, 2) TG_FWD_ST(3, 1) TG_FWD_ST(3, 0) TG_FWD_ST(2, 2) TG_FWD_ST(2, 1) TG_FWD_ST(2, 0)
    TG_FWD_ST(3, kOrderFull) TG_FWD_ST(2, kOrderFull)
    if constexpr (MODE == MODE_FWD) {
        TG_FWD_ST(3, kOrderRGB1) TG_FWD_ST(2, kOrderRGB1)
    }
#undef TG_FWD_ST
#undef TG_FWD_CASE
    return hipErrorInvalidValue;
}

hipError_t launch_forward(const tg_grid* g, int64_t n, const char* ws, const WsLayout& L, float* f,
                          float* grad_f, hipStream_t s, bool packed)
{
    LossArgs LA{};
    LA.nq = n;
    LA.packed = packed ? 1 : 0;
    return dispatch<MODE_FWD>(g, ws, L, f, packed ? nullptr : grad_f, nullptr, nullptr, nullptr, s, LA);
}

hipError_t launch_forward_loss(const tg_grid* g, int64_t n, const char* ws, const WsLayout& L, const float* d,
                               float eik_weight, float surf_k, float* g_f, float* g_grad, double* loss, float* f,
                               float* grad_f, hipStream_t s, bool record_order, bool finish)
{
    LossArgs LA;
    LA.d = d;
    LA.gf = g_f;
    LA.gg = g_grad;
    LA.urec = record_order ? reinterpret_cast<float4*>(const_cast<char*>(ws) + L.urec_off) : nullptr;
    LA.eik = eik_weight != 0.0f ? 1 : 0;
    LA.partials = reinterpret_cast<double*>(const_cast<char*>(ws) + L.fpart_off);
    LA.w_eik = eik_weight;
    LA.surf_k = surf_k;
    LA.inv_n = n > 0 ? (float)(1.0 / (double)n) : 0.0f;
    if (n > 0) {
        const hipError_t e = dispatch<MODE_LOSS>(g, ws, L, f, grad_f, nullptr, nullptr, nullptr, s, LA);
        if (e != hipSuccess) return e;
    }
    if (!finish) return hipSuccess;
    // no partials at n == 0: the finish kernel then writes a zero loss
    const bool eik = record_order ? LA.eik != 0 : g_grad != nullptr;
    return launch_loss_finish(LA.partials, n > 0 ? L.fwd_blocks : 0, n, eik ? eik_weight : 0.0f, loss, s);
}

hipError_t launch_dq(const tg_grid* g, int64_t n, const char* ws, const WsLayout& L, const float* g_f,
                     const float* g_grad, float* dq, hipStream_t s, bool packed)
{
    LossArgs LA{};
    LA.nq = n;
    LA.packed = packed ? 1 : 0;
    return dispatch<MODE_DQ>(g, ws, L, nullptr, nullptr, g_f, packed ? nullptr : g_grad, dq, s, LA);
}

}  // namespace tg
