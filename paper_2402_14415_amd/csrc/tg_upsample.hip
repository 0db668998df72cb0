// Coarse-to-fine resolution step of the progressive training schedule (Sec. 4.1): a finer
// grid over the same box starts from the field the coarse grid already represents.  Every
// fine vertex stores the value, gradient and Hessian of the coarse field (Eq. 2-4 and their
// exact derivatives) at its position, truncated to the fine order: the series of Eq. 1 of
// the field being refined.
//
// One thread per fine vertex; a block's results go through LDS so that every output array is
// written in contiguous runs.  The fine vertex i on an axis sits at i (r_c - 1) / (r_f - 1)
// in coarse cell units, so its coarse cell and local coordinate come from integer arithmetic:
// a fine vertex on a coarse face takes the cell above it (the top face the last cell), with
// no rounding deciding the side.
#include "tg_internal.hpp"

namespace tg {

template <int DIM, int KC>
__global__ __launch_bounds__(kThreads) void k_upsample(Geom gc, Geom gf, const float* __restrict__ coarse,
                                                       int cf, int ffull, int st_f, float* __restrict__ master,
                                                       void* __restrict__ coeffs, float* __restrict__ mom1,
                                                       float* __restrict__ mom2, int64_t nvert)
{
    constexpr int CC = NumCoeffs<DIM, KC>::value;
    constexpr int NH = DIM == 3 ? 6 : 3;
    constexpr int NOUT = 1 + DIM + DIM * DIM;
    // A block's kThreads consecutive fine vertices are kThreads * cf consecutive words of every
    // output array: the results are staged in LDS and written as contiguous runs.
    __shared__ float sh[kThreads * NOUT];
    for (int64_t v0 = (int64_t)blockIdx.x * kThreads; v0 < nvert; v0 += (int64_t)gridDim.x * kThreads) {
        const int64_t v = v0 + threadIdx.x;
        if (v < nvert) {
            int64_t rem = v;
            AxisLoc L[DIM];
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                const int64_t i = rem % gf.res[a];
                rem /= gf.res[a];
                const int64_t num = i * (int64_t)(gc.res[a] - 1), den = gf.res[a] - 1;
                int64_t cell = num / den;
                float t = (float)(num - cell * den) / (float)den;  // both below 2^16: exact operands, one rounding
                if (cell > gc.res[a] - 2) {
                    cell = gc.res[a] - 2;
                    t = 1.0f;
                }
                L[a].cell = (int32_t)cell;
                L[a].t = t;
                L[a].clamped = false;
            }
            const AxisFactors<DIM> F = axis_factors<DIM>(gc, L);
            float f = 0.0f, gr[DIM], hf[NH];
#pragma unroll
            for (int a = 0; a < DIM; ++a) gr[a] = 0.0f;
#pragma unroll
            for (int k = 0; k < NH; ++k) hf[k] = 0.0f;
#pragma unroll
            for (int b = 0; b < (1 << DIM); ++b) {
                int64_t cv = (int64_t)(L[0].cell + (b & 1)) + (int64_t)(L[1].cell + ((b >> 1) & 1)) * gc.stride[1];
                if constexpr (DIM == 3) cv += (int64_t)(L[2].cell + ((b >> 2) & 1)) * gc.stride[2];
                float c[CC];
#pragma unroll
                for (int k = 0; k < CC; ++k) c[k] = coarse[cv * CC + k];
                float d[DIM];
                corner_offset<DIM>(F, b, d);
                float T, dT[DIM];
                taylor_eval<DIM, KC>(c, d, T, dT);
                float w, dw[DIM];
                corner_weight<DIM>(F, b, w, dw);
                float H[NH];
                taylor_hess<DIM, KC>(c, H);
                float d2w[DIM == 3 ? 3 : 1];
                corner_weight_d2<DIM>(F, b, d2w);
                f = fmaf(w, T, f);
                int k = 0;
#pragma unroll
                for (int a = 0; a < DIM; ++a) {
                    gr[a] = fmaf(dw[a], T, fmaf(w, dT[a], gr[a]));
#pragma unroll
                    for (int cc = a; cc < DIM; ++cc, ++k) {
                        // d2(w T)/dx_a dx_cc; the pure second derivatives of w vanish
                        float h = fmaf(w, H[k], fmaf(dw[a], dT[cc], dw[cc] * dT[a]));
                        if (a != cc) h = fmaf(d2w[DIM == 3 ? (a == 0 ? cc - 1 : 2) : 0], T, h);
                        hf[k] += h;
                    }
                }
            }
            // stored order: value, gradient, Hessian xx, xy(, xz), yy(, yz, zz), first cf of
            // them; or, for the full layout, value, gradient, Hessian row-major
            float out[1 + DIM + DIM * DIM];
            out[0] = f;
#pragma unroll
            for (int a = 0; a < DIM; ++a) out[1 + a] = gr[a];
            if (ffull) {
#pragma unroll
                for (int a = 0; a < DIM; ++a)
#pragma unroll
                    for (int b = 0; b < DIM; ++b) {
                        const int lo = a < b ? a : b, hi = a < b ? b : a;
                        // index of (lo, hi) in the packed order
                        const int k = DIM == 3 ? (lo == 0 ? hi : (lo == 1 ? 2 + hi : 5)) : (lo == 0 ? hi : 2);
                        out[1 + DIM + a * DIM + b] = hf[k];
                    }
            } else {
#pragma unroll
                for (int k = 0; k < NH; ++k) out[1 + DIM + k] = hf[k];
            }
#pragma unroll
            for (int k = 0; k < NOUT; ++k)
                if (k < cf) sh[threadIdx.x * cf + k] = out[k];
        }
        __syncthreads();
        const int64_t nv = min((int64_t)kThreads, nvert - v0);
        for (int e = threadIdx.x; e < nv * cf; e += kThreads) {
            const int64_t gi = v0 * cf + e;
            const float val = sh[e];
            master[gi] = val;
            if (st_f == ST_BF16) store_copy<ST_BF16>(coeffs, gi, val);
            else if (st_f == ST_F16) store_copy<ST_F16>(coeffs, gi, val);
            if (mom1) mom1[gi] = 0.0f;
            if (mom2) mom2[gi] = 0.0f;
        }
        __syncthreads();  // sh is rewritten by the next chunk
    }
}

hipError_t launch_upsample(const tg_grid* coarse, tg_grid* fine, hipStream_t s)
{
    const int dim = coarse->desc.dim, kc = coarse->kord;
    const int ffull = fine->kord == kOrderFull ? 1 : 0;
    const int64_t nvert = fine->nvert;
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nvert + kThreads - 1) / kThreads, 65536));
    const tg_grid_buffers& b = fine->bufs;
    void* cfs = fine->desc.storage == ST_F32 ? nullptr : b.coeffs;
#define TG_UP_CASE(D, K)                                                                                    \
    if (dim == D && kc == K) {                                                                              \
        hipLaunchKernelGGL((k_upsample<D, K>), dim3(nb), dim3(kThreads), 0, s, coarse->geom, fine->geom,     \
                           coarse->bufs.master, fine->C, ffull, fine->desc.storage, b.master, cfs, b.adam_m,      \
                           b.adam_v,                                                                        \
                           nvert);                                                                          \
        return hipGetLastError();                                                                           \
    }
    TG_UP_CASE(3, 2) TG_UP_CASE(3, 1) TG_UP_CASE(3, 0) TG_UP_CASE(2, 2) TG_UP_CASE(2, 1) TG_UP_CASE(2, 0)
    TG_UP_CASE(3, kOrderFull) TG_UP_CASE(2, kOrderFull)
#undef TG_UP_CASE
    return hipErrorInvalidValue;
}

}  // namespace tg
