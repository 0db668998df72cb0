// Serving kernel: field value and unit normal for a batch of requests against several
// resident grids in one launch.
//
// Requests are small and independent, so no sort is built: every thread evaluates one
// query with direct gathers of its cell's corner coefficient blocks (same cell location,
// corner polynomials and blend as the forward, Sec. 3.1 Eq. 2-4).  The request and grid
// descriptors travel in the kernel arguments, so a launch needs no workspace and no
// host-to-device copy.  Each workgroup serves 256 consecutive points of one request; the
// arithmetic per point never depends on the other requests of the batch.
#include <cstring>

#include "tg_internal.hpp"

namespace tg {

struct QGrid {
    const void* coeffs;
    int32_t res[3];
    float lo[3], hi[3], h[3], inv_h[3];
    float inv_h_lo[3];
    int8_t dim, order, storage, pad_;
};

struct QReq {
    const float* q;
    float* sdf;
    float* normal;
    int64_t n;
    int32_t grid;
    int32_t block_start;
};

struct QTable {
    QGrid grids[TG_QUERY_MAX_GRIDS];
    QReq reqs[TG_QUERY_MAX_REQS];
    int32_t n_reqs;
};
static_assert(sizeof(QTable) < 4000, "query table must fit the kernel argument space");

template <int DIM, int K, int ST>
__device__ __forceinline__ void serve_point(const QGrid& G, const float* qp, float& f, float* gr)
{
    constexpr int C = NumCoeffs<DIM, K>::value;
    Geom g;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        g.res[a] = G.res[a];
        g.lo[a] = G.lo[a];
        g.hi[a] = G.hi[a];
        g.h[a] = G.h[a];
        g.inv_h[a] = G.inv_h[a];
        g.inv_h_lo[a] = G.inv_h_lo[a];
    }
    float q[3];
#pragma unroll
    for (int a = 0; a < DIM; ++a) q[a] = qp[a];
    AxisLoc L[DIM];
    locate<DIM>(g, q, L);
    const AxisFactors<DIM> F = axis_factors<DIM>(g, L);
    const int64_t sy = G.res[0];
    const int64_t sz = (int64_t)G.res[0] * G.res[1];
    int64_t base = L[0].cell + (int64_t)L[1].cell * sy;
    if constexpr (DIM == 3) base += (int64_t)L[2].cell * sz;
    f = 0.0f;
#pragma unroll
    for (int a = 0; a < DIM; ++a) gr[a] = 0.0f;
#pragma unroll
    for (int b = 0; b < (1 << DIM); ++b) {
        int64_t v = base + (b & 1) + ((b >> 1) & 1) * sy;
        if constexpr (DIM == 3) v += ((b >> 2) & 1) * sz;
        float c[C];
        load_vertex<ST, C>(G.coeffs, v, c);
        float d[DIM];
        corner_offset<DIM>(F, b, d);
        float T, dT[DIM];
        taylor_eval<DIM, K>(c, d, T, dT);
        float w, dw[DIM];
        corner_weight<DIM>(F, b, w, dw);
        f = fmaf(w, T, f);
#pragma unroll
        for (int a = 0; a < DIM; ++a) gr[a] = fmaf(dw[a], T, fmaf(w, dT[a], gr[a]));
    }
#pragma unroll
    for (int a = 0; a < DIM; ++a)
        if (L[a].clamped) gr[a] = 0.0f;
}

template <int DIM, int K, int ST>
__device__ __forceinline__ void serve(const QGrid& G, const QReq& R, int64_t i)
{
    float f, gr[DIM];
    serve_point<DIM, K, ST>(G, R.q + i * DIM, f, gr);
    R.sdf[i] = f;
    if (R.normal) {
        float n2 = 0.0f;
#pragma unroll
        for (int a = 0; a < DIM; ++a) n2 = fmaf(gr[a], gr[a], n2);
        const float nrm = sqrtf(n2);
#pragma unroll
        for (int a = 0; a < DIM; ++a) R.normal[i * DIM + a] = nrm > 0.0f ? gr[a] / nrm : 0.0f;
    }
}

__global__ __launch_bounds__(kThreads) void k_query(QTable T)
{
    const int32_t blk = blockIdx.x;
    int r = 0;
    for (int k = 1; k < T.n_reqs; ++k)
        if (T.reqs[k].block_start <= blk) r = k;
    const QReq R = T.reqs[r];
    const int64_t i = (int64_t)(blk - R.block_start) * kThreads + threadIdx.x;
    if (i >= R.n) return;
    const QGrid& G = T.grids[R.grid];
    const int sel = G.dim * 100 + G.order * 10 + G.storage;
    switch (sel) {
#define TG_Q_CASE(D, KK, ST) \
    case D * 100 + KK * 10 + ST: serve<D, KK, ST>(G, R, i); break;
#define TG_Q_ST(D, KK) TG_Q_CASE(D, KK, 0) TG_Q_CASE(D, KK, 1) TG_Q_CASE(D, KK, 2)
        TG_Q_ST(3, 2) TG_Q_ST(3, 1) TG_Q_ST(3, 0) TG_Q_ST(2, 2) TG_Q_ST(2, 1) TG_Q_ST(2, 0)
#undef TG_Q_ST
#undef TG_Q_CASE
    default: break;
    }
}

// Splits the batch into launches of at most TG_QUERY_MAX_REQS requests over at most
// TG_QUERY_MAX_GRIDS distinct grids, preserving request order.
hipError_t launch_query(const tg_grid* const* grids, int32_t n_grids, const tg_request* reqs, int32_t n_reqs,
                        hipStream_t s)
{
    (void)n_grids;
    int32_t i = 0;
    while (i < n_reqs) {
        QTable T;
        std::memset(static_cast<void*>(&T), 0, sizeof(T));
        const tg_grid* slot_grid[TG_QUERY_MAX_GRIDS];
        int ngs = 0;
        int nr = 0;
        int64_t blocks = 0;
        while (i < n_reqs && nr < TG_QUERY_MAX_REQS) {
            const tg_grid* gp = grids[reqs[i].grid];
            int slot = -1;
            for (int k = 0; k < ngs; ++k)
                if (slot_grid[k] == gp) slot = k;
            if (slot < 0) {
                if (ngs == TG_QUERY_MAX_GRIDS) break;
                slot = ngs++;
                slot_grid[slot] = gp;
                QGrid& G = T.grids[slot];
                G.coeffs = gp->bufs.coeffs;
                G.dim = (int8_t)gp->desc.dim;
                G.order = (int8_t)gp->desc.order;
                G.storage = (int8_t)gp->desc.storage;
                for (int a = 0; a < 3; ++a) {
                    G.res[a] = gp->geom.res[a];
                    G.lo[a] = gp->geom.lo[a];
                    G.hi[a] = gp->geom.hi[a];
                    G.h[a] = gp->geom.h[a];
                    G.inv_h[a] = gp->geom.inv_h[a];
                    G.inv_h_lo[a] = gp->geom.inv_h_lo[a];
                }
            }
            const int64_t nb = (reqs[i].n + kThreads - 1) / kThreads;
            if (nr > 0 && blocks + nb > (int64_t)0x7fffffff) break;
            QReq& R = T.reqs[nr++];
            R.q = reqs[i].q;
            R.sdf = reqs[i].sdf;
            R.normal = reqs[i].normal;
            R.n = reqs[i].n;
            R.grid = slot;
            R.block_start = (int32_t)blocks;
            blocks += nb;
            ++i;
        }
        T.n_reqs = nr;
        if (blocks > 0) hipLaunchKernelGGL(k_query, dim3((unsigned)blocks), dim3(kThreads), 0, s, T);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// ------------------------------------------------------------------ field on a lattice
// The grid's field at the points of the lattice s times finer than the grid (for the
// zero-level-set mesh of the field), n = s (res - 1) + 1 points per axis.  Point i on an axis
// lies at i / s in cell units, located exactly: cell c = min(floor(i / s), res - 2), local
// coordinate (i - s c) / s, so a point on a face takes the cell above and the top face the
// last cell.  One thread per cell (s <= kLatCellMax) or per (cell along x, cell along y,
// lattice layer): it gathers the cell's 8 corner blocks once into registers and writes the
// cell's points (s + 1 along an axis for the last cell), or those of its layer, with the
// per-point arithmetic of the forward.
constexpr int32_t kLatCellMax = 4;
template <int K, int ST>
__global__ __launch_bounds__(kThreads) void k_field_lattice(QGrid G, int32_t s, int32_t nx, int32_t ny, int32_t nz,
                                                            float* __restrict__ out)
{
    constexpr int C = NumCoeffs<3, K>::value;
    const int32_t cxn = G.res[0] - 1, cyn = G.res[1] - 1, czn = G.res[2] - 1;
    const bool per_cell = s <= kLatCellMax;
    const int64_t tid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (tid >= (int64_t)cxn * cyn * (per_cell ? czn : nz)) return;
    const int32_t cx = (int32_t)(tid % cxn);
    const int64_t rest = tid / cxn;
    const int32_t cy = (int32_t)(rest % cyn), u = (int32_t)(rest / cyn);
    // the cell along z and the thread's lattice layers [k0, k1)
    const int32_t cz = per_cell ? u : min(u / s, czn - 1);
    const int32_t k0 = per_cell ? u * s : u;
    const int32_t k1 = per_cell ? k0 + s + (cz == czn - 1 ? 1 : 0) : u + 1;
    Geom g;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        g.h[a] = G.h[a];
        g.inv_h[a] = G.inv_h[a];
    }
    const float fs = (float)s;
    AxisLoc L[3];
    L[0].cell = cx;
    L[1].cell = cy;
    L[2].cell = cz;
    L[0].clamped = L[1].clamped = L[2].clamped = false;
    float c[8][C];
    const int64_t sy = G.res[0], sz = (int64_t)G.res[0] * G.res[1];
    const int64_t base = cx + cy * sy + cz * sz;
#pragma unroll
    for (int b = 0; b < 8; ++b)
        load_vertex<ST, C>(G.coeffs, base + (b & 1) + ((b >> 1) & 1) * sy + ((b >> 2) & 1) * sz, c[b]);
    const int32_t mx = s + (cx == cxn - 1 ? 1 : 0), my = s + (cy == cyn - 1 ? 1 : 0);
    for (int32_t k = k0; k < k1; ++k) {
        L[2].t = (float)(k - cz * s) / fs;
        for (int32_t ry = 0; ry < my; ++ry) {
            L[1].t = (float)ry / fs;
            float* row = out + ((int64_t)k * ny + (int64_t)cy * s + ry) * nx + (int64_t)cx * s;
            for (int32_t rx = 0; rx < mx; ++rx) {
                L[0].t = (float)rx / fs;
                const AxisFactors<3> F = axis_factors<3>(g, L);
                float f = 0.0f;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    float d[3];
                    corner_offset<3>(F, b, d);
                    float T, dT[3];
                    taylor_eval<3, K>(c[b], d, T, dT);
                    float w, dw[3];
                    corner_weight<3>(F, b, w, dw);
                    f = fmaf(w, T, f);
                }
                row[rx] = f;
            }
        }
    }
}

hipError_t launch_field_lattice(const tg_grid* g, int32_t s, float* values, hipStream_t st)
{
    QGrid G;
    std::memset(static_cast<void*>(&G), 0, sizeof(G));
    G.coeffs = g->bufs.coeffs;
    G.dim = 3;
    G.order = (int8_t)g->desc.order;
    G.storage = (int8_t)g->desc.storage;
    int32_t n[3];
    for (int a = 0; a < 3; ++a) {
        G.res[a] = g->geom.res[a];
        G.lo[a] = g->geom.lo[a];
        G.hi[a] = g->geom.hi[a];
        G.h[a] = g->geom.h[a];
        G.inv_h[a] = g->geom.inv_h[a];
        G.inv_h_lo[a] = g->geom.inv_h_lo[a];
        n[a] = s * (g->geom.res[a] - 1) + 1;
    }
    const int64_t nthreads = (int64_t)(G.res[0] - 1) * (G.res[1] - 1) * (s <= kLatCellMax ? G.res[2] - 1 : n[2]);
    const dim3 grid((unsigned)((nthreads + kThreads - 1) / kThreads)), block(kThreads);
#define TG_FL_CASE(KK, ST)                                                                                    \
    if (G.order == KK && G.storage == ST) {                                                                 \
        hipLaunchKernelGGL((k_field_lattice<KK, ST>), grid, block, 0, st, G, s, n[0], n[1], n[2], values);      \
        return hipGetLastError();                                                                            \
    }
#define TG_FL_ST(KK) TG_FL_CASE(KK, 0) TG_FL_CASE(KK, 1) TG_FL_CASE(KK, 2)
    TG_FL_ST(2) TG_FL_ST(1) TG_FL_ST(0)
#undef TG_FL_ST
#undef TG_FL_CASE
    return hipErrorInvalidValue;
}

}  // namespace tg
