// Device-side building blocks of the TaylorGrid query path for gfx950.
//
// The field of a TaylorGrid (arXiv 2402.14415, Sec. 3.1) at a point x is
//   f(x) = sum over the 2^dim corners b of x's cell of  w_b(x) * T_b(x - v_b)      (Eq. 2-4)
// where T_b is vertex v_b's stored Taylor polynomial (Eq. 1) and w_b the multilinear weight.
// This header holds the pieces every kernel shares: the geometry passed to kernels, the
// cell location, coefficient loads in the three storage types, and the per-corner Taylor
// polynomial with its gradient.
#pragma once

#include <hip/hip_runtime.h>
#include <hip/hip_bf16.h>
#include <hip/hip_fp16.h>
#include <stdint.h>

namespace tg {

// Cells per brick edge.  A brick is the unit of query bucketing, of LDS staging in the
// forward, and of gradient ownership in the backward.
template <int DIM> struct BrickEdge;
template <> struct BrickEdge<3> { static constexpr int value = 8; };
template <> struct BrickEdge<2> { static constexpr int value = 16; };

// Kernel order code of order 2 with the full (dim x dim, row-major) Hessian stored.
constexpr int kOrderFull = 3;
// Kernel order code of a three-channel order-1 field (a colour): per vertex the three
// channels' series one after the other, channel-major.
constexpr int kOrderRGB1 = 4;
constexpr int kRGB = 3;

// Coefficients per vertex: binom(DIM + K, K); 1 + DIM + DIM^2 for the full-Hessian layout;
// 3 (1 + DIM) for the three-channel order-1 layout.
template <int DIM, int K> struct NumCoeffs {
    static constexpr int value = K == kOrderFull ? 1 + DIM + DIM * DIM
                                 : K == kOrderRGB1 ? kRGB * (1 + DIM)
                                 : DIM == 3 ? (K == 0 ? 1 : K == 1 ? 4 : 10) : (K == 0 ? 1 : K == 1 ? 3 : 6);
};

enum StorageKind { ST_F32 = 0, ST_BF16 = 1, ST_F16 = 2 };

// Geometry passed by value to every kernel.
struct Geom {
    int32_t res[3];     // vertices per axis
    int32_t nvb[3];     // vertex bricks per axis = ceil(res / B)
    float lo[3], hi[3];
    float h[3];         // vertex spacing
    float inv_h[3];
    float inv_h_lo[3];  // 1/h - inv_h (rounded to FP32): with inv_h, 1/h to about 48 bits
    int64_t stride[3];  // vertex strides (x fastest)
};

// Cell location of one query on one axis (Eq. 2), in FP32 arithmetic.  The clamped
// coordinate's offset x - lo is formed exactly as an unevaluated sum of two floats (the
// two-sum of Knuth), and multiplied by 1/h = inv_h + inv_h_lo with the rounding error of the
// leading product recovered exactly by an FMA (Dekker's product), so s = (x - lo)/h is held
// to about 2^-46 of itself.  The cell is the floor of that two-float value (its low part
// decides when the high part is an integer), so it agrees with a floor taken in FP64
// except for points within about 2^-46 s of a face, where both adjacent cells are correct
// (the field is continuous across the face).  t = s - cell keeps the low part.  FMA
// contraction is off in this function: a fused multiply-add in place of a product or sum
// would break the error-free transformations.  Every kernel calls this same function, so
// the sort, the forward and the adjoint always agree on a query's cell.
struct AxisLoc {
    int32_t cell;  // in [0, res - 2]
    float t;       // local coordinate in [0, 1]
    bool clamped;  // the query lay outside [lo, hi] on this axis
};

__device__ __forceinline__ AxisLoc locate_axis(float q, float lo, float hi, float inv_h, float inv_h_lo,
                                               int32_t res)
{
#pragma clang fp contract(off)
    AxisLoc L;
    L.clamped = (q < lo) || (q > hi);
    const float x = fminf(fmaxf(q, lo), hi);  // a NaN query lands on lo
    // x - lo = dh + dl exactly
    const float dh = x - lo;
    const float xb = dh - x;  // the part of dh that came from -lo
    const float dl = (x - (dh - xb)) + (-lo - xb);
    // (dh + dl) (inv_h + inv_h_lo) = sh + sl
    const float p = dh * inv_h;
    float e = __builtin_fmaf(dh, inv_h, -p);  // exact rounding error of p
    e = __builtin_fmaf(dh, inv_h_lo, __builtin_fmaf(dl, inv_h, e));
    const float sh = p + e;
    const float sl = e - (sh - p);
    float fl = floorf(sh);
    if (sh == fl && sl < 0.0f) fl = fl - 1.0f;
    int32_t c = (int32_t)fl;
    c = c < 0 ? 0 : c;
    c = c > res - 2 ? res - 2 : c;
    L.cell = c;
    L.t = (sh - (float)c) + sl;  // sh - c is exact for sh in [c, c + 2)
    return L;
}

template <int DIM>
__device__ __forceinline__ void locate(const Geom& g, const float* q, AxisLoc* L)
{
#pragma unroll
    for (int a = 0; a < DIM; ++a) L[a] = locate_axis(q[a], g.lo[a], g.hi[a], g.inv_h[a], g.inv_h_lo[a], g.res[a]);
}

// ------------------------------------------------------------------ storage conversions
__device__ __forceinline__ float bf16_bits_to_float(uint32_t bits16)
{
    return __uint_as_float(bits16 << 16);
}

__device__ __forceinline__ uint16_t float_to_bf16_rne(float f)
{
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40u);  // quiet NaN
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float f16_bits_to_float(uint32_t bits16)
{
    return __half2float(__ushort_as_half((unsigned short)bits16));
}

__device__ __forceinline__ uint16_t float_to_f16_rne_sat(float f)
{
    // saturate finite values to the largest FP16 magnitude instead of overflowing to inf
    if (f == f) f = fminf(fmaxf(f, -65504.0f), 65504.0f);
    return (uint16_t)__half_as_ushort(__float2half_rn(f));
}

template <int ST> __device__ __forceinline__ float load_scalar(const void* base, int64_t i)
{
    if constexpr (ST == ST_F32) {
        return static_cast<const float*>(base)[i];
    } else if constexpr (ST == ST_BF16) {
        return bf16_bits_to_float(static_cast<const uint16_t*>(base)[i]);
    } else {
        return f16_bits_to_float(static_cast<const uint16_t*>(base)[i]);
    }
}

// Two consecutive coefficients starting at an even index i (8-byte aligned in FP32).
template <int ST> __device__ __forceinline__ float2 load_pair(const void* base, int64_t i)
{
    if constexpr (ST == ST_F32) {
        return *reinterpret_cast<const float2*>(static_cast<const float*>(base) + i);
    } else {
        const uint32_t v = *reinterpret_cast<const uint32_t*>(static_cast<const uint16_t*>(base) + i);
        if constexpr (ST == ST_BF16) return make_float2(bf16_bits_to_float(v & 0xffffu), bf16_bits_to_float(v >> 16));
        else return make_float2(f16_bits_to_float(v & 0xffffu), f16_bits_to_float(v >> 16));
    }
}

// Load the C coefficients of one vertex from global memory (direct gather).
template <int ST, int C>
__device__ __forceinline__ void load_vertex(const void* base, int64_t vertex, float* out)
{
    const int64_t e0 = vertex * C;
    if constexpr (ST == ST_F32) {
        const float* p = static_cast<const float*>(base) + e0;
        if constexpr (C % 2 == 0) {
            // 8-byte aligned because C is even
#pragma unroll
            for (int k = 0; k < C; k += 2) {
                float2 v = *reinterpret_cast<const float2*>(p + k);
                out[k] = v.x;
                out[k + 1] = v.y;
            }
        } else {
#pragma unroll
            for (int k = 0; k < C; ++k) out[k] = p[k];
        }
    } else {
        const uint16_t* p = static_cast<const uint16_t*>(base) + e0;
        if constexpr (C % 2 == 0) {
#pragma unroll
            for (int k = 0; k < C; k += 2) {
                uint32_t v = *reinterpret_cast<const uint32_t*>(p + k);
                if constexpr (ST == ST_BF16) {
                    out[k] = bf16_bits_to_float(v & 0xffffu);
                    out[k + 1] = bf16_bits_to_float(v >> 16);
                } else {
                    out[k] = f16_bits_to_float(v & 0xffffu);
                    out[k + 1] = f16_bits_to_float(v >> 16);
                }
            }
        } else {
#pragma unroll
            for (int k = 0; k < C; ++k) out[k] = load_scalar<ST>(base, e0 + k);
        }
    }
}

// ------------------------------------------------------------------ Taylor polynomial
// Value and gradient (in x) of sum_alpha c_alpha d^alpha / alpha!  at world offset d = x - v
// (Eq. 1 truncated at order K, with the 1/2! of the quadratic terms; coefficients in
// graded-lex order).
template <int DIM, int K>
__device__ __forceinline__ void taylor_eval(const float* c, const float* d, float& T, float* dT)
{
    if constexpr (K == 0) {
        T = c[0];
#pragma unroll
        for (int a = 0; a < DIM; ++a) dT[a] = 0.0f;
    } else if constexpr (K == 1) {
        T = c[0];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            T = fmaf(c[1 + a], d[a], T);
            dT[a] = c[1 + a];
        }
    } else if constexpr (K == kOrderFull) {
        // c: f, g (DIM), H row-major (DIM x DIM); T = f + d.g + d.H d / 2 and
        // grad T = g + (H + H^T) d / 2
        float Hd[DIM], HTd[DIM];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            Hd[a] = 0.0f;
            HTd[a] = 0.0f;
#pragma unroll
            for (int b = 0; b < DIM; ++b) {
                Hd[a] = fmaf(c[1 + DIM + a * DIM + b], d[b], Hd[a]);
                HTd[a] = fmaf(c[1 + DIM + b * DIM + a], d[b], HTd[a]);
            }
        }
        T = c[0];
#pragma unroll
        for (int a = 0; a < DIM; ++a) {
            T = fmaf(d[a], fmaf(0.5f, Hd[a], c[1 + a]), T);
            dT[a] = c[1 + a] + 0.5f * (Hd[a] + HTd[a]);
        }
    } else if constexpr (DIM == 3) {
        // c: f, gx, gy, gz, hxx, hxy, hxz, hyy, hyz, hzz
        const float Hx = fmaf(c[4], d[0], fmaf(c[5], d[1], c[6] * d[2]));
        const float Hy = fmaf(c[5], d[0], fmaf(c[7], d[1], c[8] * d[2]));
        const float Hz = fmaf(c[6], d[0], fmaf(c[8], d[1], c[9] * d[2]));
        dT[0] = c[1] + Hx;
        dT[1] = c[2] + Hy;
        dT[2] = c[3] + Hz;
        // T = f + d.(g + H d / 2)
        T = fmaf(d[0], fmaf(0.5f, Hx, c[1]), fmaf(d[1], fmaf(0.5f, Hy, c[2]), fmaf(d[2], fmaf(0.5f, Hz, c[3]), c[0])));
    } else {
        // c: f, gx, gy, hxx, hxy, hyy
        const float Hx = fmaf(c[3], d[0], c[4] * d[1]);
        const float Hy = fmaf(c[4], d[0], c[5] * d[1]);
        dT[0] = c[1] + Hx;
        dT[1] = c[2] + Hy;
        T = fmaf(d[0], fmaf(0.5f, Hx, c[1]), fmaf(d[1], fmaf(0.5f, Hy, c[2]), c[0]));
    }
}

// Second derivatives of one corner polynomial: the stored Hessian at order 2, else 0.
// Returned in the order xx, xy, xz, yy, yz, zz (3D) or xx, xy, yy (2D).
template <int DIM, int K>
__device__ __forceinline__ void taylor_hess(const float* c, float* H)
{
    constexpr int NH = DIM == 3 ? 6 : 3;
    if constexpr (K == kOrderFull) {
        // the symmetric part (H + H^T) / 2: only it enters the polynomial
        int k = 0;
#pragma unroll
        for (int a = 0; a < DIM; ++a)
#pragma unroll
            for (int b = a; b < DIM; ++b, ++k) H[k] = 0.5f * (c[1 + DIM + a * DIM + b] + c[1 + DIM + b * DIM + a]);
    } else {
#pragma unroll
        for (int k = 0; k < NH; ++k) H[k] = (K == 2) ? c[1 + DIM + k] : 0.0f;
    }
}

// Per-axis interpolation factors of a located query: W[a][b] is the weight factor of the
// corner with bit b on axis a (1 - t or t), Dw[a][b] its derivative in x, Dd[a][b] the
// world offset x - v on that axis.
template <int DIM> struct AxisFactors {
    float W[DIM][2];
    float Dw[DIM][2];
    float Dd[DIM][2];
};

template <int DIM>
__device__ __forceinline__ AxisFactors<DIM> axis_factors(const Geom& g, const AxisLoc* L)
{
    AxisFactors<DIM> F;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        const float t = L[a].t;
        F.W[a][0] = 1.0f - t;
        F.W[a][1] = t;
        F.Dw[a][0] = -g.inv_h[a];
        F.Dw[a][1] = g.inv_h[a];
        F.Dd[a][0] = t * g.h[a];
        F.Dd[a][1] = (t - 1.0f) * g.h[a];
    }
    return F;
}

// Weight of corner b and its gradient.
template <int DIM>
__device__ __forceinline__ void corner_weight(const AxisFactors<DIM>& F, int b, float& w, float* dw)
{
    if constexpr (DIM == 3) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
        const float wyz = F.W[1][by] * F.W[2][bz];
        w = F.W[0][bx] * wyz;
        dw[0] = F.Dw[0][bx] * wyz;
        dw[1] = F.W[0][bx] * F.Dw[1][by] * F.W[2][bz];
        dw[2] = F.W[0][bx] * F.W[1][by] * F.Dw[2][bz];
    } else {
        const int bx = b & 1, by = (b >> 1) & 1;
        w = F.W[0][bx] * F.W[1][by];
        dw[0] = F.Dw[0][bx] * F.W[1][by];
        dw[1] = F.W[0][bx] * F.Dw[1][by];
    }
}

// Mixed second derivatives of corner b's weight: xy, xz, yz (3D) or xy (2D); the pure
// second derivatives of a multilinear weight vanish.
template <int DIM>
__device__ __forceinline__ void corner_weight_d2(const AxisFactors<DIM>& F, int b, float* d2w)
{
    if constexpr (DIM == 3) {
        const int bx = b & 1, by = (b >> 1) & 1, bz = (b >> 2) & 1;
        d2w[0] = F.Dw[0][bx] * F.Dw[1][by] * F.W[2][bz];
        d2w[1] = F.Dw[0][bx] * F.W[1][by] * F.Dw[2][bz];
        d2w[2] = F.W[0][bx] * F.Dw[1][by] * F.Dw[2][bz];
    } else {
        const int bx = b & 1, by = (b >> 1) & 1;
        d2w[0] = F.Dw[0][bx] * F.Dw[1][by];
    }
}

template <int DIM>
__device__ __forceinline__ void corner_offset(const AxisFactors<DIM>& F, int b, float* d)
{
#pragma unroll
    for (int a = 0; a < DIM; ++a) d[a] = F.Dd[a][(b >> a) & 1];
}

// XCD-aware order of work items.  The hardware deals workgroups round-robin to the 8 XCDs,
// each with its own L2; within every run of 8 G workgroups this hands XCD x the G
// consecutive items x G .. x G + G - 1, so that neighbouring bricks in the list (which share
// the cache lines at their common face) are processed by one L2, while the runs stay short
// enough that crowded stretches of the list still spread over all XCDs.  A bijection of
// [0, n): a trailing partial run and workgroups from n on keep their own index.
template <int G>
__device__ __forceinline__ int32_t xcd_grouped(int32_t bid, int32_t n)
{
    const int32_t run = bid / (8 * G);
    if ((run + 1) * (8 * G) > n) return bid;
    return run * (8 * G) + (bid % 8) * G + (bid / 8) % G;
}
constexpr int kXcdGroup = 4;

// ------------------------------------------------------------------ Adam (shared by the
// stand-alone optimizer kernel and the adjoint kernel that applies it in the same pass)
struct AdamArgs {
    float lr_over_bc1;       // lr / (1 - beta1^t)
    float inv_sqrt_bc2;      // 1 / sqrt(1 - beta2^t)
    float beta1, beta2, one_minus_beta1, one_minus_beta2, eps, wd;
};

// Eq. 7's surface weight of one distance, 1 - |2 sigmoid(k x) - 1|, evaluated as the equal
// 2 / (1 + exp(|k x|)) (2 sigmoid(z) - 1 = tanh(z / 2)): 1 on the surface, 0 once exp overflows.
__device__ __forceinline__ float surface_weight1(float k, float x)
{
    return 2.0f / (1.0f + expf(fabsf(k * x)));
}

// Eq. 7: the larger of the predicted and the true distance's weights; k = 0 weights all by 1.
__device__ __forceinline__ float surface_weight(float k, float f, float d)
{
    return k > 0.0f ? fmaxf(surface_weight1(k, f), surface_weight1(k, d)) : 1.0f;
}

// The square root and the division use the hardware's v_sqrt_f32 and v_rcp_f32 (1 ulp each)
// rather than the correctly rounded sequences, which cost about 25 more instructions per
// element in an epilogue that is bound by instruction issue: the update m / (sqrt(v') + eps)
// moves by about 2^-23 of itself.  A denormal v, where v_sqrt_f32 is least accurate, gives a
// square root far below any usual eps (1e-8 and up); eps = 0 with v = 0 is 0/0 either way.
__device__ __forceinline__ float adam_elem(const AdamArgs& A, float g, float& th, float& m, float& v)
{
    const float gp = fmaf(A.wd, th, g);
    m = fmaf(A.beta1, m, A.one_minus_beta1 * gp);
    v = fmaf(A.beta2, v, A.one_minus_beta2 * gp * gp);
    const float denom = fmaf(__builtin_amdgcn_sqrtf(v), A.inv_sqrt_bc2, A.eps);
    th = th - A.lr_over_bc1 * (m * __builtin_amdgcn_rcpf(denom));
    return th;
}

template <int ST>
__device__ __forceinline__ void store_copy(void* coeffs, int64_t i, float v)
{
    if constexpr (ST == ST_BF16) static_cast<uint16_t*>(coeffs)[i] = float_to_bf16_rne(v);
    else if constexpr (ST == ST_F16) static_cast<uint16_t*>(coeffs)[i] = float_to_f16_rne_sat(v);
}

// Sum of one double over a block of NT threads (a multiple of 64); valid in thread 0.
// Fixed reduction order, so the result does not depend on scheduling.
template <int NT>
__device__ __forceinline__ double block_sum_f64(double v)
{
    __shared__ double part[NT / 64];
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v += __shfl_down(v, d, 64);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) part[wave] = v;
    __syncthreads();
    double r = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) r += part[w];
    return r;
}

// Linear brick index (x fastest) of brick coordinates.
template <int DIM>
__device__ __forceinline__ int32_t brick_linear(const Geom& g, const int32_t* bc)
{
    if constexpr (DIM == 3) return (bc[2] * g.nvb[1] + bc[1]) * g.nvb[0] + bc[0];
    else return bc[1] * g.nvb[0] + bc[0];
}

}  // namespace tg
