// Query bucketing for the TaylorGrid forward and adjoint.
//
// Queries are bucketed by brick of B^dim cells.  Each query emits a "primary" record for
// the brick that contains its cell (read by the forward), and one "secondary" record for
// each neighbouring vertex brick that owns one of its cell's corners: when the cell lies
// on the high boundary layer of its brick along axis a, the corners with bit a set belong
// to the next vertex brick.  Bucket key = 2 * (vertex brick) + (secondary ? 1 : 0), so the
// forward workgroup of a brick reads one range and the backward workgroup that owns a
// brick of vertices reads one contiguous range (primary + secondary) and scatters only
// into its own vertices.
//
// Counting sort without global atomics (device-scope atomics are slow on this GPU):
//   1. every block takes a contiguous slice of the queries and counts its records per key
//      in an LDS histogram (LDS integer atomics), writing one row of a [blocks x keys]
//      matrix;
//   2. a column scan turns the matrix into per-(block, key) offsets and per-key totals,
//      and one block scans the totals into the key offsets and builds the work lists;
//   3. every block recomputes its records and places each at key offset + its block's
//      column offset + a rank drawn from an LDS counter.
// Grids with more keys than fit an LDS histogram use a slower path with global atomic
// counters.
#include "tg_internal.hpp"

namespace tg {

template <int DIM>
__device__ __forceinline__ void query_keys(const Geom& g, const float* q, int32_t* keys, int& nk)
{
    constexpr int B = BrickEdge<DIM>::value;
    AxisLoc L[DIM];
    locate<DIM>(g, q, L);
    int32_t cb[DIM];
    int bound = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        cb[a] = L[a].cell / B;
        if (L[a].cell - cb[a] * B == B - 1) bound |= 1 << a;
    }
    nk = 0;
#pragma unroll
    for (int e = 0; e < (1 << DIM); ++e) {
        if (e & ~bound) continue;
        int32_t vb[3];
#pragma unroll
        for (int a = 0; a < DIM; ++a) vb[a] = cb[a] + ((e >> a) & 1);
        keys[nk++] = 2 * brick_linear<DIM>(g, vb) + (e != 0 ? 1 : 0);
    }
}

constexpr int kSortUnroll = 8;  // queries per thread whose loads are issued together

template <int DIM>
__device__ __forceinline__ void load_query(const float* __restrict__ q, int64_t i, float* out)
{
#pragma unroll
    for (int a = 0; a < DIM; ++a) out[a] = q[i * DIM + a];
}

// ------------------------------------------------------------------ work lists
// Splits every brick's buckets into work items so that crowded bricks are shared among
// several workgroups.  Forward: up to kFwdChunk primary records per item.  Backward: a
// brick with more than kBwdItem records (primary + secondary) is split into items of
// kBwdItem records, listed first (they are the longest and start first); every other brick
// is one item, listed from the end of the array backwards, including bricks no query
// touches (the item writes their zero gradient).  A split item's index doubles as its
// partial-sum slot; a merge kernel adds the slots of a brick in order.
// Runs in one block of kThreads threads after the bucket offsets are final.
struct WorkPtrs {
    int2* fitems;
    int4* bitems;
    int32_t* split_first;  // first item of each split brick, in order
    int32_t* meta;
    int64_t max_bitems;
};

constexpr int kFinishThreads = 1024;
constexpr int kFinishPer = 8;  // bricks per thread and pass

// Block-wide exclusive scan of NV values per thread; returns this thread's exclusive
// offsets in start[] and the block totals in total[].
template <int NV>
__device__ __forceinline__ void block_scan_multi(const int32_t* val, int32_t* start, int32_t* total)
{
    __shared__ int32_t wt[NV][kFinishThreads / 64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t incl[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        incl[v] = val[v];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t o = __shfl_up(incl[v], d, 64);
            if (lane >= d) incl[v] += o;
        }
        if (lane == 63) wt[v][wave] = incl[v];
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        int32_t before = 0, all = 0;
        for (int w = 0; w < kFinishThreads / 64; ++w) {
            if (w < wave) before += wt[v][w];
            all += wt[v][w];
        }
        start[v] = before + incl[v] - val[v];
        total[v] = all;
    }
    __syncthreads();
}

__device__ void build_work(const int32_t* offs, int64_t nbricks, WorkPtrs W)
{
    int32_t carry[4] = {0, 0, 0, 0};  // forward items, split items, whole items, split bricks
    for (int64_t tile = 0; tile < nbricks; tile += (int64_t)kFinishThreads * kFinishPer) {
        const int64_t b0 = tile + (int64_t)threadIdx.x * kFinishPer;
        int32_t o[kFinishPer + 1][3];
#pragma unroll
        for (int k = 0; k < kFinishPer; ++k) {
            const int64_t b = b0 + k;
            o[k][0] = o[k][1] = o[k][2] = 0;
            if (b < nbricks) {
                o[k][0] = offs[2 * b];
                o[k][1] = offs[2 * b + 1];
                o[k][2] = offs[2 * b + 2];
            }
        }
        int32_t cnt[kFinishPer][3], tot[4] = {0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < kFinishPer; ++k) {
            const bool ok = b0 + k < nbricks;
            cnt[k][0] = ok ? (o[k][1] - o[k][0] + kFwdChunk - 1) / kFwdChunk : 0;
            const int32_t nb = ok ? (o[k][2] - o[k][0] + kBwdItem - 1) / kBwdItem : 0;
            cnt[k][1] = nb > 1 ? nb : 0;
            cnt[k][2] = ok && nb <= 1 ? 1 : 0;
            tot[0] += cnt[k][0];
            tot[1] += cnt[k][1];
            tot[2] += cnt[k][2];
            tot[3] += nb > 1 ? 1 : 0;
        }
        int32_t start[4], all[4];
        block_scan_multi<4>(tot, start, all);
        int32_t pos[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) pos[v] = carry[v] + start[v];
#pragma unroll
        for (int k = 0; k < kFinishPer; ++k) {
            const int32_t b = (int32_t)(b0 + k);
            for (int32_t j = 0; j < cnt[k][0]; ++j) W.fitems[pos[0] + j] = make_int2(b, j);
            for (int32_t j = 0; j < cnt[k][1]; ++j) W.bitems[pos[1] + j] = make_int4(b, j, cnt[k][1], pos[1]);
            if (cnt[k][1]) W.split_first[pos[3]++] = pos[1];
            if (cnt[k][2]) W.bitems[W.max_bitems - 1 - pos[2]] = make_int4(b, 0, 1, -1);
            pos[0] += cnt[k][0];
            pos[1] += cnt[k][1];
            pos[2] += cnt[k][2];
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) carry[v] += all[v];
    }
    if (threadIdx.x == 0) {
        W.meta[META_FITEMS] = carry[0];
        W.meta[META_BSPLIT] = carry[1];
        W.meta[META_BWHOLE] = carry[2];
        W.meta[META_NSPLITB] = carry[3];
    }
}

__global__ __launch_bounds__(kFinishThreads) void k_build_work(const int32_t* __restrict__ offs, int64_t nbricks, WorkPtrs W)
{
    build_work(offs, nbricks, W);
}

// ------------------------------------------------------------------ LDS-histogram path
template <int DIM>
__global__ __launch_bounds__(kSortThreads) void k_sort_count(Geom g, const float* __restrict__ q, int64_t n,
                                                             int64_t slice, int32_t nkeys,
                                                             int32_t* __restrict__ mat)
{
    extern __shared__ uint32_t hist[];
    for (int k = threadIdx.x; k < nkeys; k += kSortThreads) hist[k] = 0u;
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * slice;
    const int64_t end = min(n, beg + slice);
    for (int64_t i0 = beg; i0 < end; i0 += (int64_t)kSortThreads * kSortUnroll) {
        float x[kSortUnroll][3];
#pragma unroll
        for (int u = 0; u < kSortUnroll; ++u) {
            const int64_t i = i0 + threadIdx.x + (int64_t)u * kSortThreads;
            x[u][0] = x[u][1] = x[u][2] = 0.0f;
            if (i < end) load_query<DIM>(q, i, x[u]);
        }
#pragma unroll
        for (int u = 0; u < kSortUnroll; ++u) {
            const int64_t i = i0 + threadIdx.x + (int64_t)u * kSortThreads;
            if (i >= end) continue;
            int32_t keys[1 << DIM];
            int nk;
            query_keys<DIM>(g, x[u], keys, nk);
            for (int k = 0; k < nk; ++k) atomicAdd(&hist[keys[k]], 1u);
        }
    }
    __syncthreads();
    int32_t* row = mat + (int64_t)blockIdx.x * nkeys;
    for (int k = threadIdx.x; k < nkeys; k += kSortThreads) row[k] = (int32_t)hist[k];
}

// Column scan of the [nblk x nkeys] matrix (each thread one key): per-(block, key) offsets
// within the key, and per-key totals.
__global__ __launch_bounds__(kThreads) void k_sort_colscan(int32_t* __restrict__ mat, int32_t nblk, int32_t nkeys,
                                                          int32_t* __restrict__ total)
{
    const int32_t key = blockIdx.x * kThreads + threadIdx.x;
    if (key >= nkeys) return;
    int32_t run = 0;
    int32_t b = 0;
    for (; b + 8 <= nblk; b += 8) {
        int32_t v[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) v[u] = mat[(int64_t)(b + u) * nkeys + key];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            mat[(int64_t)(b + u) * nkeys + key] = run;
            run += v[u];
        }
    }
    for (; b < nblk; ++b) {
        const int32_t v = mat[(int64_t)b * nkeys + key];
        mat[(int64_t)b * nkeys + key] = run;
        run += v;
    }
    total[key] = run;
}

// One block: exclusive scan of the per-key totals into offs[0..nkeys], then the work lists.
__global__ __launch_bounds__(kFinishThreads) void k_sort_finish(const int32_t* __restrict__ total, int32_t nkeys,
                                                               int32_t* __restrict__ offs, WorkPtrs W)
{
    constexpr int KP = 16;  // keys per thread and pass
    int32_t carry = 0;
    for (int32_t base = 0; base < nkeys; base += kFinishThreads * KP) {
        int32_t v[KP];
        int32_t s = 0;
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            const int32_t k = base + threadIdx.x * KP + u;
            v[u] = k < nkeys ? total[k] : 0;
            s += v[u];
        }
        int32_t start[1], all[1];
        block_scan_multi<1>(&s, start, all);
        int32_t run = carry + start[0];
#pragma unroll
        for (int u = 0; u < KP; ++u) {
            const int32_t k = base + threadIdx.x * KP + u;
            if (k < nkeys) offs[k] = run;
            run += v[u];
        }
        carry += all[0];
    }
    if (threadIdx.x == 0) offs[nkeys] = carry;
    __syncthreads();
    build_work(offs, nkeys / 2, W);
}

template <int DIM>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter(Geom g, const float* __restrict__ q, int64_t n,
                                                               int64_t slice, int32_t nkeys,
                                                               const int32_t* __restrict__ mat,
                                                               const int32_t* __restrict__ offs,
                                                               float4* __restrict__ rec)
{
    extern __shared__ uint32_t cursor[];
    const int32_t* row = mat + (int64_t)blockIdx.x * nkeys;
    for (int k = threadIdx.x; k < nkeys; k += kSortThreads) cursor[k] = (uint32_t)(offs[k] + row[k]);
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * slice;
    const int64_t end = min(n, beg + slice);
    for (int64_t i0 = beg; i0 < end; i0 += (int64_t)kSortThreads * kSortUnroll) {
        float x[kSortUnroll][3];
#pragma unroll
        for (int u = 0; u < kSortUnroll; ++u) {
            const int64_t i = i0 + threadIdx.x + (int64_t)u * kSortThreads;
            x[u][0] = x[u][1] = x[u][2] = 0.0f;
            if (i < end) load_query<DIM>(q, i, x[u]);
        }
#pragma unroll
        for (int u = 0; u < kSortUnroll; ++u) {
            const int64_t i = i0 + threadIdx.x + (int64_t)u * kSortThreads;
            if (i >= end) continue;
            int32_t keys[1 << DIM];
            int nk;
            query_keys<DIM>(g, x[u], keys, nk);
            const float4 r = make_float4(x[u][0], x[u][1], x[u][2], __int_as_float((int32_t)i));
            for (int k = 0; k < nk; ++k) rec[atomicAdd(&cursor[keys[k]], 1u)] = r;
        }
    }
}

// ------------------------------------------------------------------ global-atomic path
__global__ void k_zero_i32(int32_t* __restrict__ p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0;
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_bucket_count(Geom g, const float* __restrict__ q, int64_t n,
                                                          int32_t* __restrict__ counts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[3] = {0.0f, 0.0f, 0.0f};
    load_query<DIM>(q, i, x);
    int32_t keys[1 << DIM];
    int nk;
    query_keys<DIM>(g, x, keys, nk);
    for (int k = 0; k < nk; ++k) atomicAdd(&counts[keys[k]], 1);
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_bucket_scatter(Geom g, const float* __restrict__ q, int64_t n,
                                                            int32_t* __restrict__ cursor, float4* __restrict__ rec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[3] = {0.0f, 0.0f, 0.0f};
    load_query<DIM>(q, i, x);
    int32_t keys[1 << DIM];
    int nk;
    query_keys<DIM>(g, x, keys, nk);
    const float4 r = make_float4(x[0], x[1], x[2], __int_as_float((int32_t)i));
    for (int k = 0; k < nk; ++k) rec[atomicAdd(&cursor[keys[k]], 1)] = r;
}

// Inclusive scan of one value across the 256 threads of a block; the block total goes to
// *total.
__device__ __forceinline__ int32_t block_inclusive_scan(int32_t v, int32_t* total)
{
    __shared__ int32_t wave_tot[kThreads / 64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    if (lane == 63) wave_tot[wave] = v;
    __syncthreads();
    int32_t before = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        const int32_t t = wave_tot[w];
        if (w < wave) before += t;
        all += t;
    }
    __syncthreads();
    *total = all;
    return v + before;
}

// Pass 1: total of each tile of kScanTile keys.
__global__ __launch_bounds__(kThreads) void k_scan_tiles(const int32_t* __restrict__ counts,
                                                        int32_t* __restrict__ tile_tot)
{
    const int4* p = reinterpret_cast<const int4*>(counts + (int64_t)blockIdx.x * kScanTile) + threadIdx.x * 4;
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int4 v = p[k];
        s += v.x + v.y + v.z + v.w;
    }
    int32_t total;
    block_inclusive_scan(s, &total);
    if (threadIdx.x == 0) tile_tot[blockIdx.x] = total;
}

// Pass 2: exclusive scan of the tile totals in place (one block, up to 4096 tiles).
__global__ __launch_bounds__(1024) void k_scan_top(int32_t* __restrict__ tile_tot, int32_t ntiles)
{
    __shared__ int32_t wave_tot[16];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int32_t v[4];
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int32_t i = threadIdx.x * 4 + k;
        v[k] = i < ntiles ? tile_tot[i] : 0;
        s += v[k];
    }
    int32_t incl = s;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) wave_tot[wave] = incl;
    __syncthreads();
    int32_t before = 0;
    for (int w = 0; w < wave; ++w) before += wave_tot[w];
    int32_t run = before + incl - s;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int32_t i = threadIdx.x * 4 + k;
        if (i < ntiles) tile_tot[i] = run;
        run += v[k];
    }
}

// Pass 3: exclusive offsets of every key; the counters become the scatter cursors.
__global__ __launch_bounds__(kThreads) void k_scan_apply(int32_t* __restrict__ counts,
                                                        const int32_t* __restrict__ tile_off,
                                                        int32_t* __restrict__ offs)
{
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 16;
    int4* pc = reinterpret_cast<int4*>(counts + base);
    int4* po = reinterpret_cast<int4*>(offs + base);
    int32_t v[16];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int4 t = pc[k];
        v[4 * k + 0] = t.x;
        v[4 * k + 1] = t.y;
        v[4 * k + 2] = t.z;
        v[4 * k + 3] = t.w;
    }
    int32_t s = 0;
#pragma unroll
    for (int k = 0; k < 16; ++k) s += v[k];
    int32_t total;
    const int32_t incl = block_inclusive_scan(s, &total);
    int32_t run = tile_off[blockIdx.x] + incl - s;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const int32_t c = v[k];
        v[k] = run;
        run += c;
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const int4 t = make_int4(v[4 * k], v[4 * k + 1], v[4 * k + 2], v[4 * k + 3]);
        po[k] = t;
        pc[k] = t;
    }
}

static inline unsigned blocks_for(int64_t n, int per)
{
    return (unsigned)((n + per - 1) / per);
}

hipError_t launch_sort(const tg_grid* g, const float* q, int64_t n, char* ws, const WsLayout& L, hipStream_t s)
{
    int32_t* offs = reinterpret_cast<int32_t*>(ws + L.offs_off);
    float4* rec = reinterpret_cast<float4*>(ws + L.rec_off);
    const int dim = g->desc.dim;
    WorkPtrs W;
    W.fitems = reinterpret_cast<int2*>(ws + L.fitems_off);
    W.bitems = reinterpret_cast<int4*>(ws + L.bitems_off);
    W.max_bitems = L.max_bitems;
    W.split_first = reinterpret_cast<int32_t*>(ws + L.splitb_off);
    W.meta = reinterpret_cast<int32_t*>(ws + L.meta_off);
    if (L.lds_path) {
        int32_t* mat = reinterpret_cast<int32_t*>(ws + L.scratch_off);
        int32_t* total = reinterpret_cast<int32_t*>(ws + L.counts_off);
        const int32_t nkeys = (int32_t)L.nkeys;
        const size_t lds = (size_t)nkeys * sizeof(uint32_t);
        const dim3 gb((unsigned)L.sort_blocks), tb(kSortThreads);
        if (dim == 3)
            hipLaunchKernelGGL(k_sort_count<3>, gb, tb, lds, s, g->geom, q, n, L.sort_slice, nkeys, mat);
        else
            hipLaunchKernelGGL(k_sort_count<2>, gb, tb, lds, s, g->geom, q, n, L.sort_slice, nkeys, mat);
        hipLaunchKernelGGL(k_sort_colscan, dim3(blocks_for(nkeys, kThreads)), dim3(kThreads), 0, s, mat,
                           (int32_t)L.sort_blocks, nkeys, total);
        hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(kFinishThreads), 0, s, total, nkeys, offs, W);
        if (n > 0) {
            if (dim == 3)
                hipLaunchKernelGGL(k_sort_scatter<3>, gb, tb, lds, s, g->geom, q, n, L.sort_slice, nkeys, mat, offs, rec);
            else
                hipLaunchKernelGGL(k_sort_scatter<2>, gb, tb, lds, s, g->geom, q, n, L.sort_slice, nkeys, mat, offs, rec);
        }
        return hipGetLastError();
    }
    int32_t* counts = reinterpret_cast<int32_t*>(ws + L.counts_off);
    int32_t* tiles = reinterpret_cast<int32_t*>(ws + L.tiles_off);
    hipLaunchKernelGGL(k_zero_i32, dim3(blocks_for(L.nkeys_pad, kThreads)), dim3(kThreads), 0, s, counts, L.nkeys_pad);
    if (n > 0) {
        if (dim == 3)
            hipLaunchKernelGGL(k_bucket_count<3>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, g->geom, q, n, counts);
        else
            hipLaunchKernelGGL(k_bucket_count<2>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, g->geom, q, n, counts);
    }
    hipLaunchKernelGGL(k_scan_tiles, dim3((unsigned)L.ntiles), dim3(kThreads), 0, s, counts, tiles);
    hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, tiles, (int32_t)L.ntiles);
    hipLaunchKernelGGL(k_scan_apply, dim3((unsigned)L.ntiles), dim3(kThreads), 0, s, counts, tiles, offs);
    hipLaunchKernelGGL(k_build_work, dim3(1), dim3(kFinishThreads), 0, s, offs, g->nbricks, W);
    if (n > 0) {
        if (dim == 3)
            hipLaunchKernelGGL(k_bucket_scatter<3>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, g->geom, q, n, counts, rec);
        else
            hipLaunchKernelGGL(k_bucket_scatter<2>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, g->geom, q, n, counts, rec);
    }
    return hipGetLastError();
}

}  // namespace tg
