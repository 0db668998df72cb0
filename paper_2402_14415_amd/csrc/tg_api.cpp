// C ABI of the TaylorGrid library: host-side validation, workspace layout and dispatch.
// Every argument is checked before anything is enqueued; see include/taylorgrid.h.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>

#include <algorithm>
#include <mutex>
#include <unordered_map>

#include "tg_internal.hpp"

namespace {

thread_local std::string g_last_error;

// Sort generation of the workspaces sorts were last written into.  A handle's recorded sort
// is current only while its generation is the workspace's: a later sort into the same
// workspace, by any handle, supersedes it.  The table is the library's only process-wide
// state; it keeps the kMaxWorkspaces most recently sorted workspaces, and a workspace that
// drops out of it reads as holding no sort (calls on it fail with TG_ERR_STATE until it is
// sorted again), so forgetting an entry can never make a stale sort look current.
constexpr size_t kMaxWorkspaces = 1024;
std::mutex g_ws_mutex;
std::unordered_map<const void*, uint64_t> g_ws_gen;
uint64_t g_next_gen = 0;

uint64_t ws_new_generation(const void* ws)
{
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    const uint64_t gen = ++g_next_gen;
    g_ws_gen[ws] = gen;
    if (g_ws_gen.size() > kMaxWorkspaces) {
        auto oldest = g_ws_gen.begin();
        for (auto it = g_ws_gen.begin(); it != g_ws_gen.end(); ++it)
            if (it->second < oldest->second) oldest = it;
        g_ws_gen.erase(oldest);
    }
    return gen;
}

bool ws_generation_is(const void* ws, uint64_t gen)
{
    std::lock_guard<std::mutex> lock(g_ws_mutex);
    const auto it = g_ws_gen.find(ws);
    return it != g_ws_gen.end() && it->second == gen;
}

tg_status fail(tg_status st, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
tg_status fail(tg_status st, const char* fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

tg_status ok()
{
    return TG_OK;
}

tg_status device_status(hipError_t e, const char* what)
{
    if (e == hipSuccess) return ok();
    return fail(TG_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void* p, size_t a)
{
    return (reinterpret_cast<uintptr_t>(p) % a) == 0;
}

size_t align_up(size_t x, size_t a)
{
    return (x + a - 1) / a * a;
}

tg_status check_buffers(const tg_grid_desc& d, const tg_grid_buffers& b)
{
    const void* ptrs[5] = {b.coeffs, b.master, b.grad, b.adam_m, b.adam_v};
    for (int k = 0; k < 5; ++k)
        if (ptrs[k] && !aligned(ptrs[k], 16))
            return fail(TG_ERR_INVALID_ARG, "grid buffer %d is not 16-byte aligned", k);
    if (d.storage == TG_F32 && b.coeffs && b.master && b.coeffs != b.master)
        return fail(TG_ERR_INVALID_ARG, "with FP32 storage, coeffs and master must be the same buffer");
    if (d.storage != TG_F32 && b.coeffs && b.master && b.coeffs == static_cast<const void*>(b.master))
        return fail(TG_ERR_INVALID_ARG, "with 16-bit storage, coeffs and master must be different buffers");
    return ok();
}

}  // namespace

namespace tg {

WsLayout ws_layout(const tg_grid* g, int64_t n)
{
    WsLayout L;
    const int dim = g->desc.dim;
    L.nkeys = 2 * g->nbricks;
    L.sort_blocks = 0;
    L.sort_slice = 0;
    const int64_t want = std::max<int64_t>(1, (n + kSortMinSlice - 1) / kSortMinSlice);
    if (L.nkeys <= kMaxLdsKeys32) {
        L.sort_mode = SORT_LDS32;
        L.sort_blocks = std::min<int64_t>(want, kMaxSortBlocks);
    } else if (L.nkeys <= kMaxLdsKeys16 && (n + kMaxSlice16 - 1) / kMaxSlice16 <= kMaxSortBlocks) {
        L.sort_mode = SORT_LDS16;
        L.sort_blocks = std::min<int64_t>(want, kMaxSortBlocks);
    } else {
        L.sort_mode = SORT_ATOMIC;
    }
    if (L.sort_blocks > 0) L.sort_slice = (n + L.sort_blocks - 1) / L.sort_blocks;
    size_t off = 0;
    L.reduce_off = off;
    off = align_up(off + kReduceBytes, 256);
    L.counts_off = off;
    off = align_up(off + (size_t)L.nkeys * 4, 256);
    L.offs_off = off;
    off = align_up(off + (size_t)(L.nkeys + 1) * 4, 256);
    L.scratch_off = off;
    off = align_up(off + (size_t)L.sort_blocks * (size_t)L.nkeys * 4, 256);
    const int64_t fan = (int64_t)1 << dim;  // records per query, at most
    const int B = dim == 3 ? BrickEdge<3>::value : BrickEdge<2>::value;
    L.acc_floats = (dim == 3 ? (int64_t)B * B * B : (int64_t)B * B) * g->C;
    L.max_fitems = g->nbricks + (n + kFwdChunk - 1) / kFwdChunk;
    L.fwd_blocks = L.max_fitems;
    L.max_bitems = g->nbricks + (n * fan + kBwdItemMax - 1) / kBwdItemMax;
    // A split item's slot is its item index, and split items are among the front items, of
    // which there are fewer than (records / kBwdItem): a front brick has more than kBwdItem
    // records and at most one item per kBwdItem of them.
    L.max_slots = std::min<int64_t>(L.max_bitems, (n * fan + kBwdItem - 1) / kBwdItem);
    // split bricks have more than kBwdItemMax records each
    L.merge_blocks = std::max<int64_t>(1, std::min<int64_t>({g->nbricks, (n * fan) / (kBwdItemMax + 1), 256}));
    L.meta_off = off;
    off = align_up(off + 64, 256);
    L.fitems_off = off;
    off = align_up(off + (size_t)L.max_fitems * 16, 256);
    L.bitems_off = off;
    off = align_up(off + (size_t)L.max_bitems * 16, 256);
    L.splitb_off = off;
    off = align_up(off + (size_t)g->nbricks * 4, 256);
    L.split_off = off;
    off = align_up(off + (size_t)g->nbricks * 8, 256);
    L.fpart_off = off;
    off = align_up(off + (size_t)L.fwd_blocks * 2 * sizeof(double), 256);
    L.bpart_off = off;
    off = align_up(off + (size_t)L.max_bitems * sizeof(double), 256);
    L.rec_off = off;
    off = align_up(off + (size_t)n * ((size_t)1 << dim) * 16, 256);
    L.urec_off = off;
    off = align_up(off + (size_t)n * ((size_t)1 << dim) * 16, 256);
    // Everything above depends only on the brick geometry and n, so grids of one geometry
    // can share a sort (tg_share_sort); the split bricks' partial sums depend on C and come last.
    L.parts_off = off;
    off = align_up(off + (size_t)L.max_slots * (size_t)L.acc_floats * 4, 256);
    L.total = off;
    return L;
}

}  // namespace tg

extern "C" {

int32_t tg_coeffs_per_vertex(int32_t dim, int32_t order)
{
    if ((dim != 2 && dim != 3) || order < 0 || order > 2) return -1;
    int64_t num = 1, den = 1;
    for (int i = 1; i <= order; ++i) {
        num *= dim + i;
        den *= i;
    }
    return (int32_t)(num / den);
}

tg_status tg_create(const tg_grid_desc* desc, const tg_grid_buffers* bufs, tg_grid** out)
{
    if (!desc || !out) return fail(TG_ERR_INVALID_ARG, "tg_create: desc and out must not be NULL");
    const tg_grid_desc d = *desc;
    if (d.dim != 2 && d.dim != 3) return fail(TG_ERR_INVALID_ARG, "tg_create: dim must be 2 or 3 (got %d)", d.dim);
    if (d.order < 0 || d.order > 2) return fail(TG_ERR_INVALID_ARG, "tg_create: order must be 0, 1 or 2 (got %d)", d.order);
    if (d.storage != TG_F32 && d.storage != TG_BF16 && d.storage != TG_F16)
        return fail(TG_ERR_INVALID_ARG, "tg_create: unknown storage type %d", d.storage);
    int64_t nvert = 1;
    for (int a = 0; a < d.dim; ++a) {
        if (d.res[a] < 2 || d.res[a] > 65536)
            return fail(TG_ERR_INVALID_ARG, "tg_create: res[%d] = %d outside [2, 65536]", a, d.res[a]);
        if (!std::isfinite(d.lo[a]) || !std::isfinite(d.hi[a]) || !(d.hi[a] > d.lo[a]))
            return fail(TG_ERR_INVALID_ARG, "tg_create: need finite lo[%d] < hi[%d]", a, a);
        nvert *= d.res[a];
    }
    if (d.hessian != TG_HESSIAN_SYMMETRIC && d.hessian != TG_HESSIAN_FULL)
        return fail(TG_ERR_INVALID_ARG, "tg_create: unknown Hessian layout %d", d.hessian);
    const bool full = d.hessian == TG_HESSIAN_FULL;
    if (full && d.order != 2) return fail(TG_ERR_INVALID_ARG, "tg_create: the full-Hessian layout needs order 2");
    const int32_t nch = d.channels == 0 ? 1 : d.channels;
    if (nch != 1 && nch != 3) return fail(TG_ERR_INVALID_ARG, "tg_create: channels must be 1 or 3 (got %d)", d.channels);
    const bool rgb = nch == 3;
    if (rgb && (d.order != 1 || full))
        return fail(TG_ERR_INVALID_ARG, "tg_create: three channels need order 1 and the symmetric layout");
    const int32_t C = full ? 1 + d.dim + d.dim * d.dim
                           : (rgb ? 3 * (1 + d.dim) : tg_coeffs_per_vertex(d.dim, d.order));
    if (nvert * C > ((int64_t)1 << 40)) return fail(TG_ERR_CAPACITY, "tg_create: grid too large");
    tg_grid_buffers b;
    memset(&b, 0, sizeof(b));
    if (bufs) b = *bufs;
    const tg_status bs = check_buffers(d, b);
    if (bs != TG_OK) return bs;

    tg_grid* g = new (std::nothrow) tg_grid;
    if (!g) return fail(TG_ERR_CAPACITY, "tg_create: out of host memory");
    memset(g, 0, sizeof(*g));
    g->desc = d;
    g->bufs = b;
    g->C = C;
    g->kord = full ? tg::kOrderFull : (rgb ? tg::kOrderRGB1 : d.order);
    g->nvert = nvert;
    constexpr int B3 = tg::BrickEdge<3>::value, B2 = tg::BrickEdge<2>::value;
    const int B = d.dim == 3 ? B3 : B2;
    int64_t nb = 1;
    int64_t stride = 1;
    for (int a = 0; a < 3; ++a) {
        tg::Geom& G = g->geom;
        if (a < d.dim) {
            G.res[a] = d.res[a];
            G.nvb[a] = (d.res[a] + B - 1) / B;
            G.lo[a] = d.lo[a];
            G.hi[a] = d.hi[a];
            const double h = ((double)d.hi[a] - (double)d.lo[a]) / (double)(d.res[a] - 1);
            G.h[a] = (float)h;
            G.inv_h[a] = (float)(1.0 / h);
            G.inv_h_lo[a] = (float)(1.0 / h - (double)G.inv_h[a]);
            G.stride[a] = stride;
            stride *= d.res[a];
            nb *= G.nvb[a];
        } else {
            G.res[a] = 1;
            G.nvb[a] = 1;
            G.lo[a] = 0.0f;
            G.hi[a] = 1.0f;
            G.h[a] = 1.0f;
            G.inv_h[a] = 1.0f;
            G.inv_h_lo[a] = 0.0f;
            G.stride[a] = stride;
        }
    }
    g->nbricks = nb;
    *out = g;
    return ok();
}

tg_status tg_set_buffers(tg_grid* grid, const tg_grid_buffers* bufs)
{
    if (!grid || !bufs) return fail(TG_ERR_INVALID_ARG, "tg_set_buffers: NULL argument");
    const tg_status bs = check_buffers(grid->desc, *bufs);
    if (bs != TG_OK) return bs;
    grid->bufs = *bufs;
    return ok();
}

tg_status tg_destroy(tg_grid* grid)
{
    delete grid;
    return ok();
}

size_t tg_reduce_workspace_bytes(void)
{
    return tg::kReduceBytes;
}

size_t tg_workspace_bytes(const tg_grid* grid, int64_t n)
{
    if (!grid || n < 0 || n > tg::max_sorted_queries(grid->desc.dim)) return 0;
    return tg::ws_layout(grid, n).total;
}

static tg_status check_queries(const char* fn, const tg_grid* grid, const float* q, int64_t n, const void* ws,
                               size_t ws_bytes, tg::WsLayout* L)
{
    if (!grid) return fail(TG_ERR_INVALID_ARG, "%s: grid is NULL", fn);
    if (n < 0) return fail(TG_ERR_INVALID_ARG, "%s: n = %lld is negative", fn, (long long)n);
    if (n > tg::max_sorted_queries(grid->desc.dim))
        return fail(TG_ERR_CAPACITY, "%s: n = %lld exceeds %lld (n 2^dim sort records must stay below 2^31)", fn,
                    (long long)n, (long long)tg::max_sorted_queries(grid->desc.dim));
    if (n > 0 && !q) return fail(TG_ERR_INVALID_ARG, "%s: q is NULL", fn);
    if (!ws) return fail(TG_ERR_INVALID_ARG, "%s: workspace is NULL", fn);
    if (!aligned(ws, 256)) return fail(TG_ERR_INVALID_ARG, "%s: workspace must be 256-byte aligned", fn);
    *L = tg::ws_layout(grid, n);
    if (ws_bytes < L->total)
        return fail(TG_ERR_CAPACITY, "%s: workspace has %zu bytes, needs %zu", fn, ws_bytes, L->total);
    return ok();
}

static tg_status check_sorted(const char* fn, const tg_grid* grid, const float* q, int64_t n, const void* ws)
{
    if (!grid->sort_valid || grid->sort_q != q || grid->sort_n != n || grid->sort_ws != ws ||
        !ws_generation_is(ws, grid->sort_gen))
        return fail(TG_ERR_STATE, "%s: workspace does not hold the sort of these queries (call tg_sort_queries first)", fn);
    return ok();
}

tg_status tg_sort_queries(tg_grid* grid, const float* q, int64_t n, void* ws, size_t ws_bytes, void* stream)
{
    tg::WsLayout L;
    tg_status st = check_queries("tg_sort_queries", grid, q, n, ws, ws_bytes, &L);
    if (st != TG_OK) return st;
    (void)hipGetLastError();
    grid->sort_valid = false;
    // a new generation before anything is enqueued: every earlier sort in ws is superseded
    const uint64_t gen = ws_new_generation(ws);
    const hipError_t e = tg::launch_sort(grid, q, n, static_cast<char*>(ws), L, static_cast<hipStream_t>(stream));
    st = device_status(e, "tg_sort_queries");
    if (st == TG_OK) {
        grid->sort_q = q;
        grid->sort_n = n;
        grid->sort_ws = ws;
        grid->sort_gen = gen;
        grid->sort_valid = true;
    }
    return st;
}

tg_status tg_share_sort(tg_grid* grid, const tg_grid* sorted, const float* q, int64_t n, const void* ws,
                        size_t ws_bytes)
{
    if (!grid || !sorted) return fail(TG_ERR_INVALID_ARG, "tg_share_sort: NULL grid");
    const tg_grid_desc &a = grid->desc, &b = sorted->desc;
    bool same = a.dim == b.dim;
    for (int k = 0; same && k < a.dim; ++k)
        same = a.res[k] == b.res[k] && a.lo[k] == b.lo[k] && a.hi[k] == b.hi[k];
    if (!same) return fail(TG_ERR_INVALID_ARG, "tg_share_sort: the grids differ in dim, res, lo or hi");
    tg::WsLayout L;
    tg_status st = check_queries("tg_share_sort", grid, q, n, ws, ws_bytes, &L);
    if (st != TG_OK) return st;
    st = check_sorted("tg_share_sort", sorted, q, n, ws);
    if (st != TG_OK) return st;
    grid->sort_q = q;
    grid->sort_n = n;
    grid->sort_ws = ws;
    grid->sort_gen = sorted->sort_gen;
    grid->sort_valid = true;
    return ok();
}

tg_status tg_forward(tg_grid* grid, const float* q, int64_t n, void* ws, size_t ws_bytes, float* f, float* grad_f,
                     void* stream)
{
    tg::WsLayout L;
    tg_status st = check_queries("tg_forward", grid, q, n, ws, ws_bytes, &L);
    if (st != TG_OK) return st;
    if (n > 0 && !f) return fail(TG_ERR_INVALID_ARG, "tg_forward: f is NULL");
    if (!grid->bufs.coeffs) return fail(TG_ERR_INVALID_ARG, "tg_forward: grid has no coeffs buffer");
    if (grid->kord == tg::kOrderRGB1 && grad_f)
        return fail(TG_ERR_UNSUPPORTED, "tg_forward: a three-channel grid has no grad_f output");
    st = check_sorted("tg_forward", grid, q, n, ws);
    if (st != TG_OK) return st;
    if (n == 0) return ok();
    (void)hipGetLastError();
    return device_status(tg::launch_forward(grid, n, static_cast<const char*>(ws), L, f, grad_f,
                                            static_cast<hipStream_t>(stream)),
                         "tg_forward");
}

tg_status tg_forward_packed(tg_grid* grid, const float* q, int64_t n, void* ws, size_t ws_bytes, float* fg,
                            void* stream)
{
    tg::WsLayout L;
    tg_status st = check_queries("tg_forward_packed", grid, q, n, ws, ws_bytes, &L);
    if (st != TG_OK) return st;
    if (grid->kord == tg::kOrderRGB1)
        return fail(TG_ERR_UNSUPPORTED, "tg_forward_packed: a three-channel grid has no packed layout");
    if (n > 0 && (!fg || reinterpret_cast<uintptr_t>(fg) % 16 != 0))
        return fail(TG_ERR_INVALID_ARG, "tg_forward_packed: fg must be a 16-byte aligned device pointer");
    if (!grid->bufs.coeffs) return fail(TG_ERR_INVALID_ARG, "tg_forward_packed: grid has no coeffs buffer");
    st = check_sorted("tg_forward_packed", grid, q, n, ws);
    if (st != TG_OK) return st;
    if (n == 0) return ok();
    (void)hipGetLastError();
    return device_status(tg::launch_forward(grid, n, static_cast<const char*>(ws), L, fg, nullptr,
                                            static_cast<hipStream_t>(stream), true),
                         "tg_forward_packed");
}

// TG_BWD_PACKED: g_f is the [n][4] upstream (16-byte aligned, required for n > 0), g_grad NULL,
// single-channel grids only.
static tg_status check_packed_upstream(const char* fn, const tg_grid* grid, int64_t n, const float* g_f,
                                       const float* g_grad)
{
    if (grid->kord == tg::kOrderRGB1)
        return fail(TG_ERR_UNSUPPORTED, "%s: a three-channel grid has no packed layout", fn);
    if (g_grad) return fail(TG_ERR_INVALID_ARG, "%s: TG_BWD_PACKED takes g_grad = NULL", fn);
    if (n > 0 && (!g_f || reinterpret_cast<uintptr_t>(g_f) % 16 != 0))
        return fail(TG_ERR_INVALID_ARG, "%s: TG_BWD_PACKED needs a 16-byte aligned g_f [n][4]", fn);
    return ok();
}

// A three-channel grid's adjoint takes g_f [3][n] and nothing else.
static tg_status check_rgb_upstream(const char* fn, const tg_grid* grid, int64_t n, const float* g_f,
                                    const float* g_grad, const float* dq)
{
    if (grid->kord != tg::kOrderRGB1) return ok();
    if (g_grad || dq) return fail(TG_ERR_UNSUPPORTED, "%s: a three-channel grid takes neither g_grad nor dq", fn);
    if (n > 0 && !g_f) return fail(TG_ERR_INVALID_ARG, "%s: a three-channel grid needs g_f [3][n]", fn);
    return ok();
}

static tg_status refuse_rgb(const char* fn, const tg_grid* grid)
{
    if (grid && grid->kord == tg::kOrderRGB1)
        return fail(TG_ERR_UNSUPPORTED, "%s: not defined for a three-channel grid", fn);
    return ok();
}

tg_status tg_backward(tg_grid* grid, const float* q, int64_t n, void* ws, size_t ws_bytes, const float* g_f,
                      const float* g_grad, float* dq, int32_t flags, void* stream)
{
    tg::WsLayout L;
    tg_status st = check_queries("tg_backward", grid, q, n, ws, ws_bytes, &L);
    if (st != TG_OK) return st;
    if (flags & ~(TG_BWD_ACCUMULATE | TG_BWD_PACKED))
        return fail(TG_ERR_INVALID_ARG, "tg_backward: unknown flags 0x%x", flags);
    if (!grid->bufs.grad) return fail(TG_ERR_INVALID_ARG, "tg_backward: grid has no grad buffer");
    if (dq && !grid->bufs.coeffs) return fail(TG_ERR_INVALID_ARG, "tg_backward: dq needs the coeffs buffer");
    const bool packed = (flags & TG_BWD_PACKED) != 0;
    st = packed ? check_packed_upstream("tg_backward", grid, n, g_f, g_grad)
                : check_rgb_upstream("tg_backward", grid, n, g_f, g_grad, dq);
    if (st != TG_OK) return st;
    st = check_sorted("tg_backward", grid, q, n, ws);
    if (st != TG_OK) return st;
    const bool acc = (flags & TG_BWD_ACCUMULATE) != 0;
    if (n == 0 && acc) return ok();
    (void)hipGetLastError();
    hipStream_t s = static_cast<hipStream_t>(stream);
    const char* w = static_cast<const char*>(ws);
    hipError_t e = tg::launch_backward(grid, n, w, L, g_f, g_grad, acc, s, packed);
    if (e == hipSuccess && dq && n > 0) e = tg::launch_dq(grid, n, w, L, g_f, g_grad, dq, s, packed);
    return device_status(e, "tg_backward");
}

static tg_status check_surface_k(const char* fn, float surface_k)
{
    if (!std::isfinite(surface_k) || surface_k < 0.0f)
        return fail(TG_ERR_INVALID_ARG, "%s: surface_k must be finite and >= 0", fn);
    return ok();
}

tg_status tg_forward_sdf_loss(tg_grid* grid, const float* q, int64_t n, void* ws, size_t ws_bytes, const float* d,
                              float eik_weight, float surface_k, float* g_f, float* g_grad, double* loss, float* f,
                              float* grad_f, void* stream)
{
    tg::WsLayout L;
    tg_status st = check_queries("tg_forward_sdf_loss", grid, q, n, ws, ws_bytes, &L);
    if (st != TG_OK) return st;
    if (n > 0 && (!d || !g_f)) return fail(TG_ERR_INVALID_ARG, "tg_forward_sdf_loss: d and g_f must not be NULL");
    if (!loss) return fail(TG_ERR_INVALID_ARG, "tg_forward_sdf_loss: loss is NULL");
    if (!std::isfinite(eik_weight)) return fail(TG_ERR_INVALID_ARG, "tg_forward_sdf_loss: eik_weight is not finite");
    st = check_surface_k("tg_forward_sdf_loss", surface_k);
    if (st != TG_OK) return st;
    st = refuse_rgb("tg_forward_sdf_loss", grid);
    if (st != TG_OK) return st;
    if (!grid->bufs.coeffs) return fail(TG_ERR_INVALID_ARG, "tg_forward_sdf_loss: grid has no coeffs buffer");
    st = check_sorted("tg_forward_sdf_loss", grid, q, n, ws);
    if (st != TG_OK) return st;
    (void)hipGetLastError();
    return device_status(tg::launch_forward_loss(grid, n, static_cast<const char*>(ws), L, d, eik_weight, surface_k,
                                                 g_f, g_grad, loss, f, grad_f, static_cast<hipStream_t>(stream)),
                         "tg_forward_sdf_loss");
}

static tg_status check_adam(const char* fn, const tg_grid* grid, const tg_adam_params* p)
{
    if (!grid || !p) return fail(TG_ERR_INVALID_ARG, "%s: grid and params must not be NULL", fn);
    const tg_grid_buffers& b = grid->bufs;
    if (!b.master || !b.adam_m || !b.adam_v)
        return fail(TG_ERR_INVALID_ARG, "%s: master, adam_m and adam_v are required", fn);
    if (grid->desc.storage != TG_F32 && !b.coeffs)
        return fail(TG_ERR_INVALID_ARG, "%s: 16-bit storage needs the coeffs buffer", fn);
    if (p->step < 1) return fail(TG_ERR_INVALID_ARG, "%s: step must be >= 1", fn);
    if (!std::isfinite(p->lr) || !(p->beta1 >= 0.0f && p->beta1 < 1.0f) || !(p->beta2 >= 0.0f && p->beta2 < 1.0f) ||
        !(p->eps >= 0.0f) || !std::isfinite(p->weight_decay))
        return fail(TG_ERR_INVALID_ARG, "%s: hyper-parameters out of range", fn);
    return ok();
}

tg_status tg_backward_adam(tg_grid* grid, const float* q, int64_t n, void* ws, size_t ws_bytes, const float* g_f,
                           const float* g_grad, const tg_adam_params* params, double* grad_norm_sq, int32_t flags,
                           void* stream)
{
    tg::WsLayout L;
    tg_status st = check_queries("tg_backward_adam", grid, q, n, ws, ws_bytes, &L);
    if (st != TG_OK) return st;
    st = check_adam("tg_backward_adam", grid, params);
    if (st != TG_OK) return st;
    if (flags & ~(TG_BWD_ADD_GRAD | TG_BWD_PACKED))
        return fail(TG_ERR_INVALID_ARG, "tg_backward_adam: unknown flags 0x%x", flags);
    const bool packed = (flags & TG_BWD_PACKED) != 0;
    st = packed ? check_packed_upstream("tg_backward_adam", grid, n, g_f, g_grad)
                : check_rgb_upstream("tg_backward_adam", grid, n, g_f, g_grad, nullptr);
    if (st != TG_OK) return st;
    const bool add = (flags & TG_BWD_ADD_GRAD) != 0;
    if (add && !grid->bufs.grad) return fail(TG_ERR_INVALID_ARG, "tg_backward_adam: TG_BWD_ADD_GRAD needs bufs.grad");
    st = check_sorted("tg_backward_adam", grid, q, n, ws);
    if (st != TG_OK) return st;
    (void)hipGetLastError();
    return device_status(tg::launch_backward_adam(grid, n, static_cast<const char*>(ws), L, g_f, g_grad, *params,
                                                  grad_norm_sq, static_cast<hipStream_t>(stream), false,
                                                  add ? grid->bufs.grad : nullptr, packed),
                         "tg_backward_adam");
}

// The training step; with sort == false the workspace must hold the sort of (q, n) already.
static tg_status train_step(const char* fn, bool sort, tg_grid* grid, const float* q, const float* d, int64_t n,
                            const tg_sdf_objective* obj, const tg_adam_params* params, double* loss,
                            double* grad_norm_sq, void* ws, size_t ws_bytes, void* const* stage_events, void* stream)
{
    tg::WsLayout L;
    tg_status st = check_queries(fn, grid, q, n, ws, ws_bytes, &L);
    if (st != TG_OK) return st;
    if (n > 0 && !d) return fail(TG_ERR_INVALID_ARG, "%s: d is NULL", fn);
    if (!loss) return fail(TG_ERR_INVALID_ARG, "%s: loss is NULL", fn);
    if (!obj) return fail(TG_ERR_INVALID_ARG, "%s: objective is NULL", fn);
    const float eik_weight = obj->eik_weight, surface_k = obj->surface_k, tv_weight = obj->tv_weight;
    if (!std::isfinite(eik_weight)) return fail(TG_ERR_INVALID_ARG, "%s: eik_weight is not finite", fn);
    st = check_surface_k(fn, surface_k);
    if (st != TG_OK) return st;
    st = refuse_rgb(fn, grid);
    if (st != TG_OK) return st;
    if (!std::isfinite(tv_weight)) return fail(TG_ERR_INVALID_ARG, "%s: tv_weight is not finite", fn);
    const bool tv = tv_weight != 0.0f;
    if (tv && !grid->bufs.grad)
        return fail(TG_ERR_INVALID_ARG, "%s: the TV term needs bufs.grad (it holds the TV gradient)", fn);
    if (!grid->bufs.coeffs) return fail(TG_ERR_INVALID_ARG, "%s: grid has no coeffs buffer", fn);
    st = check_adam(fn, grid, params);
    if (st != TG_OK) return st;
    if (!sort) {
        st = check_sorted(fn, grid, q, n, ws);
        if (st != TG_OK) return st;
    }
    (void)hipGetLastError();
    hipStream_t s = static_cast<hipStream_t>(stream);
    char* w = static_cast<char*>(ws);
    uint64_t gen = grid->sort_gen;
    if (sort) {
        grid->sort_valid = false;
        gen = ws_new_generation(ws);
    }
    auto mark = [&](int k) -> hipError_t {
        return stage_events ? hipEventRecord(static_cast<hipEvent_t>(stage_events[k]), s) : hipSuccess;
    };
    hipError_t e = sort ? tg::launch_sort(grid, q, n, w, L, s) : hipSuccess;
    if (e == hipSuccess) e = mark(0);
    // the TV term reads the coefficients before the update: its gradient goes to bufs.grad,
    // its value to loss[3]
    if (e == hipSuccess && tv)
        e = tg::launch_tv(grid, tv_weight, loss + 3, grid->bufs.grad, false,
                          reinterpret_cast<double*>(w + L.reduce_off), s);
    if (e == hipSuccess)
        e = tg::launch_forward_loss(grid, n, w, L, d, eik_weight, surface_k, nullptr, nullptr, loss, nullptr, nullptr,
                                    s, true, false);
    if (e == hipSuccess) e = mark(1);
    if (e == hipSuccess)
        e = tg::launch_backward_adam(grid, n, w, L, nullptr, nullptr, *params, nullptr, s, true,
                                     tv ? grid->bufs.grad : nullptr);
    // both FP64 reductions (the loss and sum(dC^2)) in one launch
    if (e == hipSuccess)
        e = tg::launch_loss_finish(reinterpret_cast<const double*>(w + L.fpart_off), n > 0 ? L.fwd_blocks : 0, n,
                                   eik_weight, loss, s,
                                   grad_norm_sq ? reinterpret_cast<const double*>(w + L.bpart_off) : nullptr,
                                   L.max_bitems, grad_norm_sq, tv_weight, tv ? loss + 3 : nullptr);
    if (e == hipSuccess) e = mark(2);
    st = device_status(e, fn);
    if (st == TG_OK) {  // the workspace holds this sort: tg_forward / tg_backward may reuse it
        grid->sort_q = q;
        grid->sort_n = n;
        grid->sort_ws = ws;
        grid->sort_gen = gen;
        grid->sort_valid = true;
    }
    return st;
}

tg_status tg_train_step(tg_grid* grid, const float* q, const float* d, int64_t n, const tg_sdf_objective* obj,
                        const tg_adam_params* params, double* loss, double* grad_norm_sq, void* ws, size_t ws_bytes,
                        void* const* stage_events, void* stream)
{
    return train_step("tg_train_step", true, grid, q, d, n, obj, params, loss, grad_norm_sq, ws, ws_bytes, stage_events,
                      stream);
}

tg_status tg_train_step_sorted(tg_grid* grid, const float* q, const float* d, int64_t n, const tg_sdf_objective* obj,
                               const tg_adam_params* params, double* loss, double* grad_norm_sq, void* ws,
                               size_t ws_bytes, void* const* stage_events, void* stream)
{
    return train_step("tg_train_step_sorted", false, grid, q, d, n, obj, params, loss, grad_norm_sq, ws, ws_bytes,
                      stage_events, stream);
}

tg_status tg_sdf_loss(int32_t dim, int64_t n, const float* f, const float* grad_f, const float* d, float eik_weight,
                      float surface_k, float* g_f, float* g_grad, double* loss, void* ws, size_t ws_bytes, void* stream)
{
    if (dim != 2 && dim != 3) return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss: dim must be 2 or 3");
    if (n < 0) return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss: n is negative");
    if (n > 0 && (!f || !d || !g_f)) return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss: f, d and g_f must not be NULL");
    if (n > 0 && grad_f && !g_grad) return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss: g_grad is NULL but grad_f is given");
    if (!loss) return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss: loss is NULL");
    if (!std::isfinite(eik_weight)) return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss: eik_weight is not finite");
    if (check_surface_k("tg_sdf_loss", surface_k) != TG_OK) return TG_ERR_INVALID_ARG;
    if (!ws || !aligned(ws, 256)) return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss: workspace NULL or not 256-byte aligned");
    if (ws_bytes < tg::kReduceBytes) return fail(TG_ERR_CAPACITY, "tg_sdf_loss: workspace smaller than %zu bytes", tg::kReduceBytes);
    (void)hipGetLastError();
    return device_status(tg::launch_sdf_loss(dim, n, f, grad_f, d, eik_weight, surface_k, g_f, g_grad, loss,
                                             static_cast<double*>(ws), static_cast<hipStream_t>(stream)),
                         "tg_sdf_loss");
}

tg_status tg_sdf_loss_noalloc(int32_t dim, int64_t n, const float* f, const float* grad_f, const float* d,
                              float eik_weight, float surface_k, float* g_f, float* g_grad, double* loss, void* stream)
{
    if (dim != 2 && dim != 3) return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss_noalloc: dim must be 2 or 3");
    if (n < 0) return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss_noalloc: n is negative");
    if (n > tg::kMaxQueries)
        return fail(TG_ERR_CAPACITY, "tg_sdf_loss_noalloc: n = %lld exceeds the maximum %lld", (long long)n,
                    (long long)tg::kMaxQueries);
    if (n > 0 && (!f || !d || !g_f))
        return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss_noalloc: f, d and g_f must not be NULL");
    if (n > 0 && grad_f && !g_grad)
        return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss_noalloc: g_grad is NULL but grad_f is given");
    if (!loss) return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss_noalloc: loss is NULL");
    if (!std::isfinite(eik_weight)) return fail(TG_ERR_INVALID_ARG, "tg_sdf_loss_noalloc: eik_weight is not finite");
    if (check_surface_k("tg_sdf_loss_noalloc", surface_k) != TG_OK) return TG_ERR_INVALID_ARG;
    (void)hipGetLastError();
    return device_status(tg::launch_sdf_loss_noalloc(dim, n, f, grad_f, d, eik_weight, surface_k, g_f, g_grad, loss,
                                                     static_cast<hipStream_t>(stream)),
                         "tg_sdf_loss_noalloc");
}

tg_status tg_tv_loss(tg_grid* grid, float weight, double* loss, int32_t flags, void* ws, size_t ws_bytes, void* stream)
{
    if (!grid) return fail(TG_ERR_INVALID_ARG, "tg_tv_loss: grid is NULL");
    if (!loss) return fail(TG_ERR_INVALID_ARG, "tg_tv_loss: loss is NULL");
    if (!std::isfinite(weight)) return fail(TG_ERR_INVALID_ARG, "tg_tv_loss: weight is not finite");
    if (flags & ~TG_BWD_ACCUMULATE) return fail(TG_ERR_INVALID_ARG, "tg_tv_loss: unknown flags 0x%x", flags);
    if (!grid->bufs.master || !grid->bufs.grad)
        return fail(TG_ERR_INVALID_ARG, "tg_tv_loss: master and grad are required");
    if (!ws || !aligned(ws, 256)) return fail(TG_ERR_INVALID_ARG, "tg_tv_loss: workspace NULL or not 256-byte aligned");
    if (ws_bytes < tg::kReduceBytes)
        return fail(TG_ERR_CAPACITY, "tg_tv_loss: workspace smaller than %zu bytes", tg::kReduceBytes);
    (void)hipGetLastError();
    return device_status(tg::launch_tv(grid, weight, loss, grid->bufs.grad, (flags & TG_BWD_ACCUMULATE) != 0,
                                       static_cast<double*>(ws), static_cast<hipStream_t>(stream)),
                         "tg_tv_loss");
}

tg_status tg_upsample(const tg_grid* coarse, tg_grid* fine, void* stream)
{
    if (!coarse || !fine) return fail(TG_ERR_INVALID_ARG, "tg_upsample: NULL grid");
    if (coarse == fine) return fail(TG_ERR_INVALID_ARG, "tg_upsample: coarse and fine are the same handle");
    const tg_grid_desc &c = coarse->desc, &f = fine->desc;
    bool same = c.dim == f.dim;
    for (int k = 0; same && k < c.dim; ++k) same = c.lo[k] == f.lo[k] && c.hi[k] == f.hi[k];
    if (!same) return fail(TG_ERR_INVALID_ARG, "tg_upsample: the grids differ in dim, lo or hi");
    if (refuse_rgb("tg_upsample", coarse) != TG_OK || refuse_rgb("tg_upsample", fine) != TG_OK)
        return TG_ERR_UNSUPPORTED;
    if (!coarse->bufs.master) return fail(TG_ERR_INVALID_ARG, "tg_upsample: the coarse grid has no master buffer");
    if (!fine->bufs.master) return fail(TG_ERR_INVALID_ARG, "tg_upsample: the fine grid has no master buffer");
    if (f.storage != TG_F32 && !fine->bufs.coeffs)
        return fail(TG_ERR_INVALID_ARG, "tg_upsample: 16-bit storage of the fine grid needs its coeffs buffer");
    // the outputs must not overlap the coarse coefficients being read
    const char* c0 = reinterpret_cast<const char*>(coarse->bufs.master);
    const char* c1 = c0 + coarse->nvert * coarse->C * sizeof(float);
    const void* outs[4] = {fine->bufs.master, f.storage != TG_F32 ? fine->bufs.coeffs : nullptr, fine->bufs.adam_m,
                           fine->bufs.adam_v};
    const size_t out_bytes[4] = {fine->nvert * fine->C * sizeof(float),
                                 fine->nvert * fine->C * (f.storage != TG_F32 ? sizeof(uint16_t) : 0),
                                 fine->nvert * fine->C * sizeof(float), fine->nvert * fine->C * sizeof(float)};
    for (int k = 0; k < 4; ++k) {
        const char* o0 = static_cast<const char*>(outs[k]);
        if (o0 && o0 < c1 && c0 < o0 + out_bytes[k])
            return fail(TG_ERR_INVALID_ARG, "tg_upsample: a fine buffer overlaps the coarse master");
    }
    (void)hipGetLastError();
    return device_status(tg::launch_upsample(coarse, fine, static_cast<hipStream_t>(stream)), "tg_upsample");
}

tg_status tg_iou_counts(int64_t n, const float* f, const float* d, int64_t* counts, void* ws, size_t ws_bytes,
                        void* stream)
{
    if (n < 0 || n > tg::kMaxQueries) return fail(TG_ERR_INVALID_ARG, "tg_iou_counts: n out of range");
    if (n > 0 && (!f || !d)) return fail(TG_ERR_INVALID_ARG, "tg_iou_counts: f and d must not be NULL");
    if (!counts) return fail(TG_ERR_INVALID_ARG, "tg_iou_counts: counts is NULL");
    if (!ws || !aligned(ws, 256)) return fail(TG_ERR_INVALID_ARG, "tg_iou_counts: workspace NULL or not 256-byte aligned");
    if (ws_bytes < tg::kReduceBytes)
        return fail(TG_ERR_CAPACITY, "tg_iou_counts: workspace smaller than %zu bytes", tg::kReduceBytes);
    (void)hipGetLastError();
    return device_status(tg::launch_iou(n, f, d, counts, static_cast<int64_t*>(ws), static_cast<hipStream_t>(stream)),
                         "tg_iou_counts");
}

tg_status tg_field_lattice(const tg_grid* grid, int32_t s, float* values, void* stream)
{
    if (!grid) return fail(TG_ERR_INVALID_ARG, "tg_field_lattice: grid is NULL");
    if (grid->desc.dim != 3) return fail(TG_ERR_UNSUPPORTED, "tg_field_lattice: needs a 3D grid");
    if (grid->kord != grid->desc.order)
        return fail(TG_ERR_UNSUPPORTED, "tg_field_lattice: needs a single-channel grid in the symmetric layout");
    if (s < 1 || s > 64) return fail(TG_ERR_INVALID_ARG, "tg_field_lattice: s = %d outside 1..64", s);
    if (!grid->bufs.coeffs) return fail(TG_ERR_INVALID_ARG, "tg_field_lattice: grid has no coeffs buffer");
    if (!values) return fail(TG_ERR_INVALID_ARG, "tg_field_lattice: values is NULL");
    int64_t npts = 1;
    for (int a = 0; a < 3; ++a) npts *= (int64_t)s * (grid->desc.res[a] - 1) + 1;
    if (npts >= ((int64_t)1 << 31))
        return fail(TG_ERR_CAPACITY, "tg_field_lattice: %lld lattice points (at most 2^31 - 1)", (long long)npts);
    (void)hipGetLastError();
    return device_status(tg::launch_field_lattice(grid, s, values, static_cast<hipStream_t>(stream)),
                         "tg_field_lattice");
}

static bool mesh_cells(const int32_t* n, int64_t* ncell)
{
    if (!n) return false;
    int64_t c = 1;
    for (int a = 0; a < 3; ++a) {
        if (n[a] < 2 || n[a] > 65536) return false;
        c *= n[a] - 1;
    }
    *ncell = c;
    return true;
}

size_t tg_mesh_workspace_bytes(const int32_t* n)
{
    int64_t ncell;
    if (!mesh_cells(n, &ncell) || ncell > tg::kMaxMeshCells) return 0;
    return tg::mesh_workspace_bytes(ncell);
}

tg_status tg_mesh(const int32_t* n, const float* lo, const float* hi, const float* values, float* tri,
                  int64_t max_tris, int64_t* n_tris, void* ws, size_t ws_bytes, void* stream)
{
    int64_t ncell;
    if (!mesh_cells(n, &ncell)) return fail(TG_ERR_INVALID_ARG, "tg_mesh: every n[a] must be in 2..65536");
    if (ncell > tg::kMaxMeshCells)
        return fail(TG_ERR_CAPACITY, "tg_mesh: more than %lld cells", (long long)tg::kMaxMeshCells);
    if (!lo || !hi) return fail(TG_ERR_INVALID_ARG, "tg_mesh: lo and hi must not be NULL");
    for (int a = 0; a < 3; ++a)
        if (!std::isfinite(lo[a]) || !std::isfinite(hi[a]) || !(hi[a] > lo[a]))
            return fail(TG_ERR_INVALID_ARG, "tg_mesh: need finite lo[%d] < hi[%d]", a, a);
    if (!values || !n_tris) return fail(TG_ERR_INVALID_ARG, "tg_mesh: values and n_tris must not be NULL");
    if (max_tris < 0) return fail(TG_ERR_INVALID_ARG, "tg_mesh: max_tris is negative");
    if (max_tris > 0 && !tri) return fail(TG_ERR_INVALID_ARG, "tg_mesh: tri is NULL");
    if (!ws || !aligned(ws, 256)) return fail(TG_ERR_INVALID_ARG, "tg_mesh: workspace NULL or not 256-byte aligned");
    if (ws_bytes < tg::mesh_workspace_bytes(ncell))
        return fail(TG_ERR_CAPACITY, "tg_mesh: workspace has %zu bytes, needs %zu", ws_bytes,
                    tg::mesh_workspace_bytes(ncell));
    (void)hipGetLastError();
    return device_status(tg::launch_mesh(n, lo, hi, values, tri, max_tris, n_tris, static_cast<char*>(ws),
                                         static_cast<hipStream_t>(stream)),
                         "tg_mesh");
}

size_t tg_chamfer_workspace_bytes(int64_t na, int64_t nb)
{
    if (na < 1 || nb < 1 || na > tg::kMaxQueries || nb > tg::kMaxQueries) return 0;
    return tg::chamfer_workspace_bytes(na, nb);
}

tg_status tg_chamfer(const float* a, int64_t na, const float* b, int64_t nb, int32_t norm, double* out, void* ws,
                     size_t ws_bytes, void* stream)
{
    if (na < 1 || nb < 1 || na > tg::kMaxQueries || nb > tg::kMaxQueries)
        return fail(TG_ERR_INVALID_ARG, "tg_chamfer: point counts must be in 1..%lld", (long long)tg::kMaxQueries);
    if (norm != 1 && norm != 2) return fail(TG_ERR_INVALID_ARG, "tg_chamfer: norm must be 1 (L1) or 2 (Euclidean)");
    if (!a || !b || !out) return fail(TG_ERR_INVALID_ARG, "tg_chamfer: a, b and out must not be NULL");
    if (!ws || !aligned(ws, 256)) return fail(TG_ERR_INVALID_ARG, "tg_chamfer: workspace NULL or not 256-byte aligned");
    const size_t need = tg::chamfer_workspace_bytes(na, nb);
    if (ws_bytes < need) return fail(TG_ERR_CAPACITY, "tg_chamfer: workspace has %zu bytes, needs %zu", ws_bytes, need);
    (void)hipGetLastError();
    return device_status(tg::launch_chamfer(a, na, b, nb, norm, out, static_cast<char*>(ws),
                                            static_cast<hipStream_t>(stream)),
                         "tg_chamfer");
}

tg_status tg_composite(int64_t n_rays, int32_t n_samples, const float* f, const float* c, const float* delta,
                       const float* target, float* rgb, double* loss, float* g_f, float* g_c, void* ws,
                       size_t ws_bytes, void* stream)
{
    if (n_rays < 0) return fail(TG_ERR_INVALID_ARG, "tg_composite: n_rays is negative");
    if (n_samples < 1 || n_samples > 1024) return fail(TG_ERR_INVALID_ARG, "tg_composite: n_samples must be in 1..1024");
    if (n_rays > tg::kMaxQueries / n_samples)
        return fail(TG_ERR_CAPACITY, "tg_composite: more than %lld samples", (long long)tg::kMaxQueries);
    if (n_rays > 0 && (!f || !c || !delta)) return fail(TG_ERR_INVALID_ARG, "tg_composite: f, c and delta must not be NULL");
    if (target && !loss) return fail(TG_ERR_INVALID_ARG, "tg_composite: a target needs loss");
    if (loss && n_rays > 0 && (!target || !g_f || !g_c))
        return fail(TG_ERR_INVALID_ARG, "tg_composite: with loss, target, g_f and g_c must not be NULL");
    if (!ws || !aligned(ws, 256)) return fail(TG_ERR_INVALID_ARG, "tg_composite: workspace NULL or not 256-byte aligned");
    if (ws_bytes < tg::kReduceBytes) return fail(TG_ERR_CAPACITY, "tg_composite: workspace smaller than %zu bytes", tg::kReduceBytes);
    (void)hipGetLastError();
    return device_status(tg::launch_composite(n_rays, n_samples, f, c, delta, target, rgb, loss, g_f, g_c,
                                              static_cast<double*>(ws), static_cast<hipStream_t>(stream)),
                         "tg_composite");
}

tg_status tg_adam_step(tg_grid* grid, const tg_adam_params* p, double* grad_norm_sq, void* ws, size_t ws_bytes,
                       int32_t flags, void* stream)
{
    tg_status st = check_adam("tg_adam_step", grid, p);
    if (st != TG_OK) return st;
    if (flags & ~TG_ADAM_ZERO_GRAD) return fail(TG_ERR_INVALID_ARG, "tg_adam_step: unknown flags 0x%x", flags);
    if (!grid->bufs.grad) return fail(TG_ERR_INVALID_ARG, "tg_adam_step: master, grad, adam_m and adam_v are required");
    if (!ws || !aligned(ws, 256)) return fail(TG_ERR_INVALID_ARG, "tg_adam_step: workspace NULL or not 256-byte aligned");
    if (ws_bytes < tg::kReduceBytes) return fail(TG_ERR_CAPACITY, "tg_adam_step: workspace smaller than %zu bytes", tg::kReduceBytes);
    (void)hipGetLastError();
    return device_status(tg::launch_adam(grid, *p, grad_norm_sq, static_cast<double*>(ws), (flags & TG_ADAM_ZERO_GRAD) != 0,
                                         static_cast<hipStream_t>(stream)),
                         "tg_adam_step");
}

tg_status tg_sync_storage(tg_grid* grid, void* stream)
{
    if (!grid) return fail(TG_ERR_INVALID_ARG, "tg_sync_storage: grid is NULL");
    if (grid->desc.storage == TG_F32) return ok();
    if (!grid->bufs.master || !grid->bufs.coeffs)
        return fail(TG_ERR_INVALID_ARG, "tg_sync_storage: master and coeffs are required");
    (void)hipGetLastError();
    return device_status(tg::launch_sync_storage(grid, static_cast<hipStream_t>(stream)), "tg_sync_storage");
}

tg_status tg_query(const tg_grid* const* grids, int32_t n_grids, const tg_request* reqs, int32_t n_reqs, void* stream)
{
    if (n_reqs < 0) return fail(TG_ERR_INVALID_ARG, "tg_query: n_reqs is negative");
    if (n_reqs == 0) return ok();
    if (!grids || n_grids < 1 || !reqs) return fail(TG_ERR_INVALID_ARG, "tg_query: grids and reqs must not be NULL");
    for (int32_t k = 0; k < n_grids; ++k) {
        if (!grids[k] || !grids[k]->bufs.coeffs)
            return fail(TG_ERR_INVALID_ARG, "tg_query: grid %d is NULL or has no coeffs", k);
        if (grids[k]->kord == tg::kOrderFull)
            return fail(TG_ERR_UNSUPPORTED, "tg_query: grid %d stores the full Hessian (serve the symmetric layout)", k);
        if (grids[k]->kord == tg::kOrderRGB1)
            return fail(TG_ERR_UNSUPPORTED, "tg_query: grid %d has three channels (serving answers SDF queries)", k);
    }
    for (int32_t i = 0; i < n_reqs; ++i) {
        const tg_request& r = reqs[i];
        if (r.grid < 0 || r.grid >= n_grids) return fail(TG_ERR_INVALID_ARG, "tg_query: request %d names grid %d", i, r.grid);
        if (r.n < 0 || r.n > 0x7fffffffLL) return fail(TG_ERR_INVALID_ARG, "tg_query: request %d has n = %lld", i, (long long)r.n);
        if (r.n > 0 && (!r.q || !r.sdf)) return fail(TG_ERR_INVALID_ARG, "tg_query: request %d has a NULL q or sdf", i);
    }
    (void)hipGetLastError();
    return device_status(tg::launch_query(grids, n_grids, reqs, n_reqs, static_cast<hipStream_t>(stream)), "tg_query");
}

const char* tg_status_string(tg_status status)
{
    switch (status) {
    case TG_OK: return "ok";
    case TG_ERR_INVALID_ARG: return "invalid argument";
    case TG_ERR_UNSUPPORTED: return "unsupported";
    case TG_ERR_DEVICE: return "device error";
    case TG_ERR_CAPACITY: return "capacity exceeded";
    case TG_ERR_STATE: return "workspace state mismatch";
    }
    return "unknown status";
}

const char* tg_last_error(void)
{
    return g_last_error.c_str();
}

}  // extern "C"
