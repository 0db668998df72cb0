// Radiance-field compositing: the Max optical model along each ray (Sec. 3.3, Eq. 10) with a
// ReLU density, the photometric loss (Sec. 3.3, Eq. 11) and its adjoint, in one launch.
//
// One wavefront per ray: lane l holds samples [l SPL, (l + 1) SPL) in registers, so the
// transmittance (an exclusive prefix sum of sigma delta over the ray) is a lane-local running
// sum started at a wave-wide exclusive scan of the lanes' totals, and the light still to come
// behind a sample (a suffix sum of the weighted colours) is the mirror image.  The inputs are
// the density and colour grids' values at the samples, in the grids' own output layout, and
// the outputs are the upstream gradients those grids' adjoints take.
#include "tg_internal.hpp"

namespace tg {

constexpr int kCompositeThreads = 256;  // 4 rays per workgroup

// SPL consecutive floats at p (16-byte aligned when SPL is a multiple of 4, 8-byte when 2).
template <int SPL>
__device__ __forceinline__ void load_run(const float* __restrict__ p, float* v)
{
    if constexpr (SPL % 4 == 0) {
#pragma unroll
        for (int k = 0; k < SPL; k += 4) {
            const float4 t = *reinterpret_cast<const float4*>(p + k);
            v[k] = t.x;
            v[k + 1] = t.y;
            v[k + 2] = t.z;
            v[k + 3] = t.w;
        }
    } else if constexpr (SPL == 2) {
        const float2 t = *reinterpret_cast<const float2*>(p);
        v[0] = t.x;
        v[1] = t.y;
    } else {
        v[0] = p[0];
    }
}

template <int SPL>
__device__ __forceinline__ void store_run(float* __restrict__ p, const float* v)
{
    if constexpr (SPL % 4 == 0) {
#pragma unroll
        for (int k = 0; k < SPL; k += 4)
            *reinterpret_cast<float4*>(p + k) = make_float4(v[k], v[k + 1], v[k + 2], v[k + 3]);
    } else if constexpr (SPL == 2) {
        *reinterpret_cast<float2*>(p) = make_float2(v[0], v[1]);
    } else {
        p[0] = v[0];
    }
}

// VEC: every lane's SPL samples lie wholly inside the ray or wholly past its end (ns is a
// multiple of SPL) and the arrays are aligned for SPL-wide accesses, so a lane moves its
// samples of each array in 8- or 16-byte accesses.
template <int SPL, bool VEC>
__global__ __launch_bounds__(kCompositeThreads) void k_composite(int64_t n_rays, int32_t ns,
                                                               const float* __restrict__ f,
                                                               const float* __restrict__ col,
                                                               const float* __restrict__ delta,
                                                               const float* __restrict__ target,
                                                               float* __restrict__ rgb_out,
                                                               float* __restrict__ g_f,
                                                               float* __restrict__ g_c,
                                                               double* __restrict__ partials)
{
    constexpr int RPB = kCompositeThreads / 64;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t n = n_rays * (int64_t)ns;  // samples, the channel stride of col and g_c
    const float inv_r = n_rays > 0 ? (float)(1.0 / (double)n_rays) : 0.0f;
    double lsum = 0.0;  // this wave's sum of |C - target|^2 / R
    for (int64_t r = (int64_t)blockIdx.x * RPB + wave; r < n_rays; r += (int64_t)gridDim.x * RPB) {
        const int64_t base = r * ns;
        float fk[SPL], dk[SPL], ak[SPL], ck[SPL][3];
        float lane_a = 0.0f;
        const bool lane_in = lane * SPL < ns;  // (VEC) all of this lane's samples are in the ray
        if constexpr (VEC) {
            float cv[3][SPL];
            if (lane_in) {
                const int64_t o = base + lane * SPL;
                load_run<SPL>(f + o, fk);
                load_run<SPL>(delta + o, dk);
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) load_run<SPL>(col + ch * n + o, cv[ch]);
            } else {
#pragma unroll
                for (int k = 0; k < SPL; ++k) {
                    fk[k] = dk[k] = 0.0f;
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) cv[ch][k] = 0.0f;
                }
            }
#pragma unroll
            for (int k = 0; k < SPL; ++k) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) ck[k][ch] = cv[ch][k];
                ak[k] = fmaxf(fk[k], 0.0f) * dk[k];  // sigma delta, sigma = relu(f)
                lane_a += ak[k];
            }
        } else {
#pragma unroll
            for (int k = 0; k < SPL; ++k) {
                const int i = lane * SPL + k;
                const bool ok = i < ns;
                fk[k] = ok ? f[base + i] : 0.0f;
                dk[k] = ok ? delta[base + i] : 0.0f;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) ck[k][ch] = ok ? col[ch * n + base + i] : 0.0f;
                ak[k] = fmaxf(fk[k], 0.0f) * dk[k];  // sigma delta, sigma = relu(f)
                lane_a += ak[k];
            }
        }
        // exclusive prefix of the lanes' sums of sigma delta
        float incl = lane_a;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const float o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        float run = incl - lane_a;
        float Tk[SPL], wk[SPL], Tn[SPL];  // T_i, T_i alpha_i, T_{i+1} = T_i exp(-a_i)
        float lane_c[3] = {0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k = 0; k < SPL; ++k) {
            Tk[k] = expf(-run);
            run += ak[k];
            Tn[k] = expf(-run);
            wk[k] = Tk[k] * -expm1f(-ak[k]);  // alpha = 1 - exp(-a), accurate for small a
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) lane_c[ch] = fmaf(wk[k], ck[k][ch], lane_c[ch]);
        }
        float C[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float s = lane_c[ch];
#pragma unroll
            for (int d = 32; d >= 1; d >>= 1) s += __shfl_xor(s, d, 64);
            C[ch] = s;
        }
        if (rgb_out && lane == 0) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) rgb_out[r * 3 + ch] = C[ch];
        }
        if (!partials) continue;  // colours only
        float g_rgb[3];
        double l2 = 0.0;
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            const float e = C[ch] - target[r * 3 + ch];
            l2 += (double)e * (double)e;
            g_rgb[ch] = 2.0f * e * inv_r;
        }
        if (lane == 0) lsum += l2 * (double)inv_r;
        // exclusive suffix (over the later lanes) of the weighted colours
        float after[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            float inc = lane_c[ch];
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const float o = __shfl_down(inc, d, 64);
                if (lane + d < 64) inc += o;
            }
            after[ch] = inc - lane_c[ch];
        }
        float gfk[SPL], gck[3][SPL];
#pragma unroll
        for (int k = SPL - 1; k >= 0; --k) {
            // dL/dsigma = delta sum_ch g_ch (T_{i+1} c_i - sum_{j>i} T_j alpha_j c_j)
            float gs = 0.0f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) gs = fmaf(g_rgb[ch], fmaf(Tn[k], ck[k][ch], -after[ch]), gs);
            gs *= dk[k];
            gfk[k] = fk[k] > 0.0f ? gs : 0.0f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) gck[ch][k] = g_rgb[ch] * wk[k];
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) after[ch] = fmaf(wk[k], ck[k][ch], after[ch]);
        }
        if constexpr (VEC) {
            if (lane_in) {
                const int64_t o = base + lane * SPL;
                store_run<SPL>(g_f + o, gfk);
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) store_run<SPL>(g_c + ch * n + o, gck[ch]);
            }
        } else {
#pragma unroll
            for (int k = 0; k < SPL; ++k) {
                const int i = lane * SPL + k;
                if (i < ns) {
                    g_f[base + i] = gfk[k];
#pragma unroll
                    for (int ch = 0; ch < 3; ++ch) g_c[ch * n + base + i] = gck[ch][k];
                }
            }
        }
    }
    if (partials) {
        const double tot = block_sum_f64<kCompositeThreads>(lsum);
        if (threadIdx.x == 0) partials[blockIdx.x] = tot;
    }
}

hipError_t launch_composite(int64_t n_rays, int32_t ns, const float* f, const float* col, const float* delta,
                            const float* target, float* rgb, double* loss, float* g_f, float* g_c, double* partials,
                            hipStream_t s)
{
    constexpr int RPB = kCompositeThreads / 64;
    const int64_t want = (n_rays + RPB - 1) / RPB;
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, kMaxReduceBlocks));
    double* part = loss ? partials : nullptr;
    const int spl = (ns + 63) / 64;
    // the wide-access variant: ns a multiple of the samples per lane, every array aligned
    // (a NULL gradient output, as when only rendering, adds nothing to the alignment test)
    auto aligned = [&](int S) {
        const uintptr_t bytes = (uintptr_t)(S % 4 == 0 ? 16 : S * 4);
        const uintptr_t a = reinterpret_cast<uintptr_t>(f) | reinterpret_cast<uintptr_t>(col) |
                            reinterpret_cast<uintptr_t>(delta) | reinterpret_cast<uintptr_t>(g_f) |
                            reinterpret_cast<uintptr_t>(g_c);
        return S > 1 && ns % S == 0 && a % bytes == 0;
    };
#define TG_COMPOSITE(S)                                                                                     \
    if (spl <= S) {                                                                                         \
        if (aligned(S))                                                                                     \
            hipLaunchKernelGGL((k_composite<S, true>), dim3(nb), dim3(kCompositeThreads), 0, s, n_rays, ns, f, \
                               col, delta, target, rgb, g_f, g_c, part);                                   \
        else                                                                                                \
            hipLaunchKernelGGL((k_composite<S, false>), dim3(nb), dim3(kCompositeThreads), 0, s, n_rays, ns, f, \
                               col, delta, target, rgb, g_f, g_c, part);                                   \
    } else
    TG_COMPOSITE(1) TG_COMPOSITE(2) TG_COMPOSITE(4) TG_COMPOSITE(8) TG_COMPOSITE(16) { return hipErrorInvalidValue; }
#undef TG_COMPOSITE
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss) return e;
    return launch_sum_finish(partials, nb, loss, s);
}

}  // namespace tg
