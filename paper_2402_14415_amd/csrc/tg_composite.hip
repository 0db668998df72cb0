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

template <int SPL>
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
#pragma unroll
        for (int k = SPL - 1; k >= 0; --k) {
            const int i = lane * SPL + k;
            // dL/dsigma = delta sum_ch g_ch (T_{i+1} c_i - sum_{j>i} T_j alpha_j c_j)
            float gs = 0.0f;
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) gs = fmaf(g_rgb[ch], fmaf(Tn[k], ck[k][ch], -after[ch]), gs);
            gs *= dk[k];
            if (i < ns) {
                g_f[base + i] = fk[k] > 0.0f ? gs : 0.0f;
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) g_c[ch * n + base + i] = g_rgb[ch] * wk[k];
            }
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) after[ch] = fmaf(wk[k], ck[k][ch], after[ch]);
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
#define TG_COMPOSITE(S)                                                                                     \
    if (spl <= S) {                                                                                         \
        hipLaunchKernelGGL(k_composite<S>, dim3(nb), dim3(kCompositeThreads), 0, s, n_rays, ns, f, col, delta, \
                           target, rgb, g_f, g_c, part);                                                   \
    } else
    TG_COMPOSITE(1) TG_COMPOSITE(2) TG_COMPOSITE(4) TG_COMPOSITE(8) TG_COMPOSITE(16) { return hipErrorInvalidValue; }
#undef TG_COMPOSITE
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || !loss) return e;
    return launch_sum_finish(partials, nb, loss, s);
}

}  // namespace tg
