// SDF objective (upstream gradients + FP64 loss) and the fused Adam step.
//
// Both are streaming kernels: grid-stride over their elements, FP64 per-block partial sums
// written to the reduction scratch, then a one-block kernel that adds the partials in a
// fixed order (deterministic FP64 result on the device).
#include <mutex>

#include "tg_internal.hpp"

namespace tg {

__device__ __forceinline__ double block_sum(double v)
{
    return block_sum_f64<kThreads>(v);
}

static inline unsigned reduce_blocks(int64_t n, int per_thread)
{
    int64_t b = (n + (int64_t)kThreads * per_thread - 1) / ((int64_t)kThreads * per_thread);
    if (b < 1) b = 1;
    if (b > kMaxReduceBlocks) b = kMaxReduceBlocks;
    return (unsigned)b;
}

// ------------------------------------------------------------------ SDF loss (Eq. 6, Eq. 8)
template <int DIM, bool EIK>
__global__ __launch_bounds__(kThreads) void k_sdf_loss(int64_t n, const float* __restrict__ f,
                                                      const float* __restrict__ grad, const float* __restrict__ d,
                                                      float w_eik, float surf_k, float inv_n, float* __restrict__ gf,
                                                      float* __restrict__ gg, double* __restrict__ partials)
{
    double acc_r = 0.0, acc_e = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const float fi = f[i], di = d[i];
        const float r = fi - di;
        const float w = surface_weight(surf_k, fi, di);  // Eq. 7, held fixed in the gradient
        acc_r += (double)w * (double)fabsf(r);
        const float wn = w * inv_n;
        gf[i] = r > 0.0f ? wn : (r < 0.0f ? -wn : 0.0f);
        if constexpr (EIK) {
            float g[DIM];
            float n2 = 0.0f;
#pragma unroll
            for (int a = 0; a < DIM; ++a) {
                g[a] = grad[i * DIM + a];
                n2 = fmaf(g[a], g[a], n2);
            }
            const float nrm = sqrtf(n2);
            const float e = nrm - 1.0f;
            acc_e += (double)e * (double)e;
            const float k = nrm > 0.0f ? 2.0f * w_eik * e / nrm * inv_n : 0.0f;
#pragma unroll
            for (int a = 0; a < DIM; ++a) gg[i * DIM + a] = k * g[a];
        }
    }
    const double sr = block_sum(acc_r);
    const double se = block_sum(acc_e);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x + 0] = sr;
        partials[2 * blockIdx.x + 1] = se;
    }
}

// One block of 1024 threads adds the per-block partials (loads issued 8 at a time).
constexpr int kFinishReduceThreads = 1024;

// This thread's share of sum_b p[S b + k] (k < S) over the blocks b < nblocks, added to acc.
template <int S>
__device__ __forceinline__ void thread_partial_sums(const double* __restrict__ p, int nblocks, double* acc)
{
    for (int b0 = 0; b0 < nblocks; b0 += 8 * kFinishReduceThreads) {
        double v[8][S];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int b = b0 + u * kFinishReduceThreads + threadIdx.x;
#pragma unroll
            for (int k = 0; k < S; ++k) v[u][k] = b < nblocks ? p[(int64_t)S * b + k] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
#pragma unroll
            for (int k = 0; k < S; ++k) acc[k] += v[u][k];
        }
    }
}

// loss[1] = mean w |r|, loss[2] = mean (|grad f| - 1)^2, loss[0] = loss[1] + w_eik loss[2]
// (+ w_tv *tv when tv is given: a TV value finished earlier on the stream) from the
// (sum w |r|, sum (|grad f| - 1)^2) pairs of nl blocks; with gpart, also *gnorm = the sum of
// ng sum(dC^2) partials (the training step finishes both reductions in one launch).
__global__ __launch_bounds__(kFinishReduceThreads) void k_loss_finish(const double* __restrict__ partials, int nblocks,
                                                                      double inv_n, double w_eik, double* __restrict__ loss,
                                                                      const double* __restrict__ gpart, int ng,
                                                                      double* __restrict__ gnorm, double w_tv,
                                                                      const double* __restrict__ tv)
{
    // both sets of partials are loaded in the same rounds (thread_partial_sums' order per set)
    double acc[2] = {0.0, 0.0}, sg = 0.0;
    if (!gpart) ng = 0;
    for (int b0 = 0; b0 < max(nblocks, ng); b0 += 8 * kFinishReduceThreads) {
        double v[8][2], w[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int b = b0 + u * kFinishReduceThreads + threadIdx.x;
            v[u][0] = b < nblocks ? partials[2 * (int64_t)b] : 0.0;
            v[u][1] = b < nblocks ? partials[2 * (int64_t)b + 1] : 0.0;
            w[u] = b < ng ? gpart[b] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            acc[0] += v[u][0];
            acc[1] += v[u][1];
            sg += w[u];
        }
    }
    const double sr = block_sum_f64<kFinishReduceThreads>(acc[0]);
    const double se = block_sum_f64<kFinishReduceThreads>(acc[1]);
    if (threadIdx.x == 0) {
        loss[1] = sr * inv_n;
        loss[2] = se * inv_n;
        loss[0] = loss[1] + w_eik * loss[2] + (tv ? w_tv * *tv : 0.0);
    }
    if (gpart) {
        sg = block_sum_f64<kFinishReduceThreads>(sg);
        if (threadIdx.x == 0 && gnorm) *gnorm = sg;
    }
}

hipError_t launch_sdf_loss(int dim, int64_t n, const float* f, const float* grad_f, const float* d, float eik_weight,
                           float surf_k, float* g_f, float* g_grad, double* loss, double* partials, hipStream_t s)
{
    const unsigned nb = reduce_blocks(n, 4);
    const float inv_n = n > 0 ? (float)(1.0 / (double)n) : 0.0f;
    const dim3 grid(nb), block(kThreads);
    if (grad_f) {
        if (dim == 3)
            hipLaunchKernelGGL((k_sdf_loss<3, true>), grid, block, 0, s, n, f, grad_f, d, eik_weight, surf_k, inv_n, g_f, g_grad, partials);
        else
            hipLaunchKernelGGL((k_sdf_loss<2, true>), grid, block, 0, s, n, f, grad_f, d, eik_weight, surf_k, inv_n, g_f, g_grad, partials);
    } else {
        hipLaunchKernelGGL((k_sdf_loss<3, false>), grid, block, 0, s, n, f, grad_f, d, eik_weight, surf_k, inv_n, g_f, g_grad, partials);
    }
    const double w = grad_f ? (double)eik_weight : 0.0;
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(kFinishReduceThreads), 0, s, partials, (int)nb,
                       n > 0 ? 1.0 / (double)n : 0.0, w, loss, nullptr, 0, nullptr, 0.0, nullptr);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Adam
// Vectorised by 4 over the first n4*4 elements; the scalar tail is handled by block 0.
template <int ST>
__global__ __launch_bounds__(kThreads) void k_adam(int64_t n, AdamArgs A, float* __restrict__ master,
                                                  float* __restrict__ mom1, float* __restrict__ mom2,
                                                  float* __restrict__ grad, void* __restrict__ coeffs,
                                                  int zero_grad, double* __restrict__ partials)
{
    double ss = 0.0;
    const int64_t n4 = n / 4;
    float4* th4 = reinterpret_cast<float4*>(master);
    float4* m4 = reinterpret_cast<float4*>(mom1);
    float4* v4 = reinterpret_cast<float4*>(mom2);
    float4* g4 = reinterpret_cast<float4*>(grad);
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kThreads) {
        float4 t = th4[i], m = m4[i], v = v4[i];
        const float4 g = g4[i];
        ss += (double)g.x * g.x + (double)g.y * g.y + (double)g.z * g.z + (double)g.w * g.w;
        adam_elem(A, g.x, t.x, m.x, v.x);
        adam_elem(A, g.y, t.y, m.y, v.y);
        adam_elem(A, g.z, t.z, m.z, v.z);
        adam_elem(A, g.w, t.w, m.w, v.w);
        th4[i] = t;
        m4[i] = m;
        v4[i] = v;
        if (zero_grad) g4[i] = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        if constexpr (ST != ST_F32) {
            if constexpr (ST == ST_BF16) {
                const uint2 packed = make_uint2((uint32_t)float_to_bf16_rne(t.x) | ((uint32_t)float_to_bf16_rne(t.y) << 16),
                                                (uint32_t)float_to_bf16_rne(t.z) | ((uint32_t)float_to_bf16_rne(t.w) << 16));
                reinterpret_cast<uint2*>(coeffs)[i] = packed;
            } else {
                const uint2 packed = make_uint2((uint32_t)float_to_f16_rne_sat(t.x) | ((uint32_t)float_to_f16_rne_sat(t.y) << 16),
                                                (uint32_t)float_to_f16_rne_sat(t.z) | ((uint32_t)float_to_f16_rne_sat(t.w) << 16));
                reinterpret_cast<uint2*>(coeffs)[i] = packed;
            }
        }
    }
    if (blockIdx.x == 0) {
        for (int64_t i = n4 * 4 + threadIdx.x; i < n; i += kThreads) {
            float t = master[i], m = mom1[i], v = mom2[i];
            const float g = grad[i];
            ss += (double)g * g;
            adam_elem(A, g, t, m, v);
            master[i] = t;
            mom1[i] = m;
            mom2[i] = v;
            if (zero_grad) grad[i] = 0.0f;
            store_copy<ST>(coeffs, i, t);
        }
    }
    const double tot = block_sum(ss);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kFinishReduceThreads) void k_sum_finish(const double* __restrict__ partials, int nblocks,
                                                                     double scale, double* __restrict__ out)
{
    double acc = 0.0;
    thread_partial_sums<1>(partials, nblocks, &acc);
    acc = block_sum_f64<kFinishReduceThreads>(acc);
    if (threadIdx.x == 0) *out = acc * scale;
}

AdamArgs make_adam_args(const tg_adam_params& p)
{
    const double bc1 = 1.0 - pow((double)p.beta1, (double)p.step);
    const double bc2 = 1.0 - pow((double)p.beta2, (double)p.step);
    AdamArgs A;
    A.lr_over_bc1 = (float)((double)p.lr / bc1);
    A.inv_sqrt_bc2 = (float)(1.0 / sqrt(bc2));
    A.beta1 = p.beta1;
    A.beta2 = p.beta2;
    A.one_minus_beta1 = (float)(1.0 - (double)p.beta1);
    A.one_minus_beta2 = (float)(1.0 - (double)p.beta2);
    A.eps = p.eps;
    A.wd = p.weight_decay;
    return A;
}

hipError_t launch_loss_finish(const double* partials, int64_t nblocks, int64_t n, float eik_weight, double* loss,
                              hipStream_t s, const double* gpart, int64_t ng, double* gnorm, float tv_weight,
                              const double* tv)
{
    hipLaunchKernelGGL(k_loss_finish, dim3(1), dim3(kFinishReduceThreads), 0, s, partials, (int)nblocks,
                       n > 0 ? 1.0 / (double)n : 0.0, (double)eik_weight, loss, gpart, (int)ng, gnorm,
                       (double)tv_weight, tv);
    return hipGetLastError();
}

hipError_t launch_sum_finish(const double* partials, int64_t nblocks, double* out, hipStream_t s)
{
    return launch_sum_finish_scaled(partials, nblocks, 1.0, out, s);
}

hipError_t launch_sum_finish_scaled(const double* partials, int64_t nblocks, double scale, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(kFinishReduceThreads), 0, s, partials, (int)nblocks, scale, out);
    return hipGetLastError();
}

hipError_t launch_adam(const tg_grid* g, const tg_adam_params& p, double* grad_norm_sq, double* partials,
                       bool zero_grad, hipStream_t s)
{
    const int64_t n = g->nvert * g->C;
    const AdamArgs A = make_adam_args(p);
    const unsigned nb = reduce_blocks(n / 4 + 1, 8);
    const dim3 grid(nb), block(kThreads);
    const int zg = zero_grad ? 1 : 0;
    switch (g->desc.storage) {
    case ST_F32:
        hipLaunchKernelGGL(k_adam<ST_F32>, grid, block, 0, s, n, A, g->bufs.master, g->bufs.adam_m, g->bufs.adam_v,
                           g->bufs.grad, g->bufs.coeffs, zg, partials);
        break;
    case ST_BF16:
        hipLaunchKernelGGL(k_adam<ST_BF16>, grid, block, 0, s, n, A, g->bufs.master, g->bufs.adam_m, g->bufs.adam_v,
                           g->bufs.grad, g->bufs.coeffs, zg, partials);
        break;
    default:
        hipLaunchKernelGGL(k_adam<ST_F16>, grid, block, 0, s, n, A, g->bufs.master, g->bufs.adam_m, g->bufs.adam_v,
                           g->bufs.grad, g->bufs.coeffs, zg, partials);
        break;
    }
    if (grad_norm_sq)
        hipLaunchKernelGGL(k_sum_finish, dim3(1), dim3(kFinishReduceThreads), 0, s, partials, (int)nb, 1.0, grad_norm_sq);
    return hipGetLastError();
}

// The storage copy of the master coefficients: round to nearest even, FP16 saturating at
// +-65504 (the conversion the Adam update applies after every step).
template <int ST>
__global__ __launch_bounds__(kThreads) void k_sync_storage(int64_t n, const float* __restrict__ master,
                                                           void* __restrict__ coeffs)
{
    const int64_t n4 = n / 4;
    const float4* th4 = reinterpret_cast<const float4*>(master);
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n4; i += (int64_t)gridDim.x * kThreads) {
        const float4 t = th4[i];
        uint2 packed;
        if constexpr (ST == ST_BF16)
            packed = make_uint2((uint32_t)float_to_bf16_rne(t.x) | ((uint32_t)float_to_bf16_rne(t.y) << 16),
                                (uint32_t)float_to_bf16_rne(t.z) | ((uint32_t)float_to_bf16_rne(t.w) << 16));
        else
            packed = make_uint2((uint32_t)float_to_f16_rne_sat(t.x) | ((uint32_t)float_to_f16_rne_sat(t.y) << 16),
                                (uint32_t)float_to_f16_rne_sat(t.z) | ((uint32_t)float_to_f16_rne_sat(t.w) << 16));
        reinterpret_cast<uint2*>(coeffs)[i] = packed;
    }
    if (blockIdx.x == 0)
        for (int64_t i = n4 * 4 + threadIdx.x; i < n; i += kThreads) store_copy<ST>(coeffs, i, master[i]);
}

hipError_t launch_sync_storage(const tg_grid* g, hipStream_t s)
{
    const int64_t n = g->nvert * g->C;
    if (g->desc.storage == ST_F32 || n == 0) return hipSuccess;
    const dim3 grid(reduce_blocks(n / 4 + 1, 8)), block(kThreads);
    if (g->desc.storage == ST_BF16)
        hipLaunchKernelGGL(k_sync_storage<ST_BF16>, grid, block, 0, s, n, g->bufs.master, g->bufs.coeffs);
    else
        hipLaunchKernelGGL(k_sync_storage<ST_F16>, grid, block, 0, s, n, g->bufs.master, g->bufs.coeffs);
    return hipGetLastError();
}

// ------------------------------------------------------------------ allocation-free loss
// tg_sdf_loss_noalloc keeps its per-block FP64 sums in this file-scope device array instead
// of a caller's workspace: the launch uses at most kMaxReduceBlocks blocks, two sums each.
// Every GPU the library runs on holds its own copy until the process ends; in host code
// `scratch` names a host-side stand-in, so kernels get the device address that
// hipGetSymbolAddress returns for the device, looked up once per device.
constexpr int kNoallocPartials = 2 * kMaxReduceBlocks;
static __device__ __align__(256) double scratch[kNoallocPartials];

constexpr int kMaxScratchDevices = 64;
static std::mutex g_scratch_mutex;
static double* g_scratch_ptr[kMaxScratchDevices] = {};

size_t noalloc_scratch_bytes()
{
    return sizeof(scratch);
}

// The device address of `device`'s copy of the scratch array (that device is made current
// for the lookup, and the previous current device restored).
static hipError_t scratch_address(int device, double** out)
{
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[device]) {
        int cur = -1;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if (cur != device && (e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (cur != device) {
            const hipError_t e2 = hipSetDevice(cur);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        g_scratch_ptr[device] = static_cast<double*>(p);
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}

hipError_t launch_sdf_loss_noalloc(int dim, int64_t n, const float* f, const float* grad_f, const float* d,
                                   float eik_weight, float surf_k, float* g_f, float* g_grad, double* loss,
                                   hipStream_t s)
{
    static_assert(2 * kMaxReduceBlocks <= kNoallocPartials, "the scratch holds every block's two sums");
    hipDevice_t device = -1;
    hipError_t e = hipStreamGetDevice(s, &device);
    if (e != hipSuccess) return e;
    double* partials = nullptr;
    e = scratch_address((int)device, &partials);
    if (e != hipSuccess) return e;
    // each block writes its own two sums before the finishing block reads them: nothing in
    // the scratch needs to start at zero
    return launch_sdf_loss(dim, n, f, grad_f, d, eik_weight, surf_k, g_f, g_grad, loss, partials, s);
}

}  // namespace tg
