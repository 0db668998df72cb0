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
//      matrix.  Up to 40704 keys the counters are 32-bit; up to 81920 keys two 16-bit
//      counters share a word (a block then takes at most 65535 queries, and a query adds
//      at most one record to a key, so a counter cannot overflow);
//   2. a column scan turns the matrix into per-(block, key) offsets and per-key totals;
//   3. the key totals are scanned into key offsets and the work lists are built: with
//      32-bit counters by every block of step 4 itself (so no separate pass), with packed
//      counters by one block;
//   4. every block recomputes its records and places each at key offset + its block's
//      column offset + a rank drawn from an LDS counter.
// Grids with more keys than that use a slower path with global atomic counters.
#include "tg_internal.hpp"

namespace tg {

// Calls emit(key) for each bucket key of the query at x: the primary key of its cell's
// brick, then the secondary key of every neighbouring vertex brick that owns a corner.
template <int DIM, typename F>
__device__ __forceinline__ void for_each_key(const Geom& g, const float* x, F&& emit)
{
    constexpr int B = BrickEdge<DIM>::value;
    AxisLoc L[DIM];
    locate<DIM>(g, x, L);
    int32_t cb[DIM];
    int bound = 0;
#pragma unroll
    for (int a = 0; a < DIM; ++a) {
        cb[a] = L[a].cell / B;
        if (L[a].cell - cb[a] * B == B - 1) bound |= 1 << a;
    }
#pragma unroll
    for (int e = 0; e < (1 << DIM); ++e) {
        if (e & ~bound) continue;
        int32_t vb[3];
#pragma unroll
        for (int a = 0; a < DIM; ++a) vb[a] = cb[a] + ((e >> a) & 1);
        emit(2 * brick_linear<DIM>(g, vb) + (e != 0 ? 1 : 0));
    }
}

constexpr int kSortUnroll = 8;  // queries per thread whose loads are issued together

// Writes one sorted record at pos: the query's coordinates and a tag.  A primary record's
// tag is the query index; a secondary record's tag is kRecSecondary | (position of the same
// query's primary record), so that per-query data kept in record order (the training
// step's upstream gradients) is found from either copy.  for_each_key emits the primary key
// first, so p0 holds the primary position when the secondaries are written.
__device__ __forceinline__ void put_record(float4* rec, int32_t pos, const float* x, int64_t i, int32_t key,
                                           int32_t& p0)
{
    int32_t tag;
    if (key & 1) {
        tag = p0 | kRecSecondary;
    } else {
        p0 = pos;
        tag = (int32_t)i;
    }
    rec[pos] = make_float4(x[0], x[1], x[2], __int_as_float(tag));
}

template <int DIM>
__device__ __forceinline__ void load_query(const float* __restrict__ q, int64_t i, float* out)
{
#pragma unroll
    for (int a = 0; a < DIM; ++a) out[a] = q[i * DIM + a];
}

// ------------------------------------------------------------------ work lists
// Splits every brick's buckets into work items so that crowded bricks are shared among
// several workgroups; an item carries its record range.  Forward: up to kFwdChunk primary
// records per item.  Backward: up to kBwdItemMax records (primary + secondary) per item; the
// items of bricks with more than kBwdItem records are listed first (the longest work starts
// first), every other brick is one item listed from the end of the array backwards,
// including bricks no query touches (the item writes their zero gradient).  A split brick's
// items are consecutive and an item's index doubles as its partial-sum slot: the adjoint's
// merge launch adds the slots of a brick in order (the adjoint with Adam takes a split brick
// whole in its first item, or merges in the item that finishes last).
struct WorkPtrs {
    int4* fitems;  // (brick, first record, end record, 0)
    int4* bitems;  // (brick, first record, end record, items of the brick)
    int32_t* split_first;  // first item of each split brick, in order
    int2* split;           // per split brick: (0, its first item), the adjoint's arrival count
    int32_t* meta;
    int64_t max_bitems;
};

constexpr int kFinishThreads = 512;
constexpr int kFinishBricks = 8;  // bricks per thread and pass

// Block-wide exclusive scan of NV values per thread; returns this thread's exclusive
// offsets in start[] and the block totals in total[].  The waves' totals are scanned by
// the first wave, so that a thread reads two words per value from LDS.
template <int NV, int NT>
__device__ __forceinline__ void block_scan_multi(const int32_t* val, int32_t* start, int32_t* total)
{
    constexpr int NW = NT / 64;
    static_assert(NW <= 64, "one wave scans the wave totals");
    __shared__ int32_t wt[NV][NW + 1];  // wave totals, then their exclusive prefix; [NW]: block total
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
    if (wave == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int32_t t = lane < NW ? wt[v][lane] : 0;
            int32_t it = t;
#pragma unroll
            for (int d = 1; d < NW; d <<= 1) {
                const int32_t o = __shfl_up(it, d, 64);
                if (lane >= d) it += o;
            }
            if (lane < NW) wt[v][lane] = it - t;
            if (lane == NW - 1) wt[v][NW] = it;
        }
    }
    __syncthreads();
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        start[v] = wt[v][wave] + incl[v] - val[v];
        total[v] = wt[v][NW];
    }
    __syncthreads();  // wt is reused by the next call
}

// The five work-list quantities of a brick with tp primary and ts secondary records:
// records, forward items, front backward items, back backward items, split bricks.
__device__ __forceinline__ void brick_counts(int32_t tp, int32_t ts, bool exists, int32_t* v)
{
    const int32_t nr = tp + ts;
    const int32_t nb = (nr + kBwdItemMax - 1) / kBwdItemMax;
    v[0] += nr;
    v[1] += (tp + kFwdChunk - 1) / kFwdChunk;
    v[2] += nr > kBwdItem ? nb : 0;
    v[3] += (exists && nr <= kBwdItem) ? 1 : 0;
    v[4] += nb > 1 ? 1 : 0;
}

// Writes the work items of brick b (when emit), whose running positions (the exclusive
// scan of brick_counts over the bricks before it) are pos[]; advances pos[] past the brick.
__device__ __forceinline__ void brick_items(int64_t b, int32_t tp, int32_t ts, int32_t* pos, const WorkPtrs& W,
                                            bool emit = true)
{
    const int32_t r0 = pos[0], rp = r0 + tp, r1 = rp + ts;  // primary, secondary ends
    pos[0] = r1;
    const int32_t nf = (tp + kFwdChunk - 1) / kFwdChunk;
    if (emit)
        for (int32_t j = 0; j < nf; ++j)
            W.fitems[pos[1] + j] = make_int4((int32_t)b, r0 + j * kFwdChunk, min(rp, r0 + (j + 1) * kFwdChunk), 0);
    pos[1] += nf;
    const int32_t nr = tp + ts;
    const int32_t nb = (nr + kBwdItemMax - 1) / kBwdItemMax;
    const bool front = nr > kBwdItem;
    if (emit) {
        if (front) {
            for (int32_t j = 0; j < nb; ++j)
                W.bitems[pos[2] + j] =
                    make_int4((int32_t)b, r0 + j * kBwdItemMax, min(r1, r0 + (j + 1) * kBwdItemMax), nb);
            if (nb > 1) {
                W.split_first[pos[4]] = pos[2];
                W.split[b] = make_int2(0, pos[2]);
            }
        } else {
            W.bitems[W.max_bitems - 1 - pos[3]] = make_int4((int32_t)b, r0, r1, 1);
        }
    }
    // written without branches, so that the positions stay in registers
    pos[2] += front ? nb : 0;
    pos[3] += front ? 0 : 1;
    pos[4] += nb > 1 ? 1 : 0;
}

__device__ __forceinline__ void write_meta(const int32_t* carry, const WorkPtrs& W)
{
    W.meta[META_FITEMS] = carry[1];
    W.meta[META_BFRONT] = carry[2];
    W.meta[META_BBACK] = carry[3];
    W.meta[META_NSPLITB] = carry[4];
}

// One block: from the per-key totals, the exclusive key offsets offs[0..nkeys] (and a
// copy in cursor[], when given, for the atomic scatter) and the work lists, in passes of
// kFinishThreads * kFinishBricks bricks.
__global__ __launch_bounds__(kFinishThreads) void k_sort_finish(const int32_t* total, int64_t nbricks,
                                                               int32_t* __restrict__ offs, int32_t* cursor, WorkPtrs W)
{
    int32_t carry[5] = {0, 0, 0, 0, 0};
    for (int64_t pass = 0; pass < nbricks; pass += (int64_t)kFinishThreads * kFinishBricks) {
        const int64_t b0 = pass + (int64_t)threadIdx.x * kFinishBricks;
        int32_t tp[kFinishBricks], ts[kFinishBricks];
#pragma unroll
        for (int k = 0; k < kFinishBricks; ++k) {
            const bool ok = b0 + k < nbricks;
            tp[k] = ok ? total[2 * (b0 + k)] : 0;
            ts[k] = ok ? total[2 * (b0 + k) + 1] : 0;
        }
        int32_t v[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < kFinishBricks; ++k) brick_counts(tp[k], ts[k], b0 + k < nbricks, v);
        int32_t pos[5], all[5];
        block_scan_multi<5, kFinishThreads>(v, pos, all);
#pragma unroll
        for (int u = 0; u < 5; ++u) pos[u] += carry[u];
#pragma unroll
        for (int k = 0; k < kFinishBricks; ++k) {
            const int64_t b = b0 + k;
            if (b >= nbricks) break;
            offs[2 * b] = pos[0];
            offs[2 * b + 1] = pos[0] + tp[k];
            if (cursor) {
                cursor[2 * b] = pos[0];
                cursor[2 * b + 1] = pos[0] + tp[k];
            }
            brick_items(b, tp[k], ts[k], pos, W);
        }
#pragma unroll
        for (int u = 0; u < 5; ++u) carry[u] += all[u];
    }
    if (threadIdx.x == 0) {
        offs[2 * nbricks] = carry[0];
        write_meta(carry, W);
    }
}

// ------------------------------------------------------------------ LDS-histogram path
// Counter of `key` in the LDS histogram: a 32-bit word, or half of one (PACK16).
template <bool PACK16>
__device__ __forceinline__ uint32_t lds_count_add(uint32_t* hist, int32_t key)
{
    if constexpr (PACK16) {
        const uint32_t sh = (uint32_t)(key & 1) << 4;
        return (atomicAdd(&hist[key >> 1], 1u << sh) >> sh) & 0xffffu;
    } else {
        return atomicAdd(&hist[key], 1u);
    }
}

template <bool PACK16>
__host__ __device__ constexpr int32_t lds_words(int32_t nkeys)
{
    return PACK16 ? (nkeys + 1) >> 1 : nkeys;
}

template <int DIM, bool PACK16>
__global__ __launch_bounds__(kSortThreads) void k_sort_count(Geom g, const float* __restrict__ q, int64_t n,
                                                             int64_t slice, int32_t nkeys,
                                                             int32_t* __restrict__ mat)
{
    extern __shared__ uint32_t hist[];
    const int32_t nw = lds_words<PACK16>(nkeys);
    for (int k = threadIdx.x; k < nw; k += kSortThreads) hist[k] = 0u;
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
            for_each_key<DIM>(g, x[u], [&](int32_t key) { lds_count_add<PACK16>(hist, key); });
        }
    }
    __syncthreads();
    int32_t* row = mat + (int64_t)blockIdx.x * nkeys;
    for (int k = threadIdx.x; k < nkeys; k += kSortThreads) {
        const uint32_t w = hist[PACK16 ? k >> 1 : k];
        row[k] = PACK16 ? (int32_t)((w >> ((k & 1) << 4)) & 0xffffu) : (int32_t)w;
    }
}

// Column scan of the [nblk x nkeys] matrix: per-(block, key) offsets within the key, and
// per-key totals.  A workgroup takes 64 keys (one per lane) and splits the rows among its
// waves: each wave sums its rows (kept in registers), the waves' sums are scanned through
// LDS, and each wave rewrites its rows as running offsets.
constexpr int kColWaves = 16;
constexpr int kColRows = kMaxSortBlocks / kColWaves;  // rows per wave at most
static_assert(kMaxSortBlocks % kColWaves == 0, "the matrix rows must split evenly over the waves");
__global__ __launch_bounds__(64 * kColWaves) void k_sort_colscan(int32_t* __restrict__ mat, int32_t nblk,
                                                                int32_t nkeys, int32_t* __restrict__ total)
{
    __shared__ int32_t gsum[kColWaves][64];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int32_t key = blockIdx.x * 64 + lane;
    const bool ok = key < nkeys;
    const int32_t per = (nblk + kColWaves - 1) / kColWaves;
    const int32_t r0 = min(nblk, wave * per), r1 = min(nblk, r0 + per);
    int32_t v[kColRows];
    int32_t s = 0;
#pragma unroll
    for (int u = 0; u < kColRows; ++u) {
        v[u] = (ok && r0 + u < r1) ? mat[(int64_t)(r0 + u) * nkeys + key] : 0;
        s += v[u];
    }
    gsum[wave][lane] = s;
    __syncthreads();
    int32_t run = 0, all = 0;
#pragma unroll
    for (int w = 0; w < kColWaves; ++w) {
        const int32_t t = gsum[w][lane];
        run += w < wave ? t : 0;
        all += t;
    }
    if (!ok) return;
    if (wave == 0) total[key] = all;
#pragma unroll
    for (int u = 0; u < kColRows; ++u) {
        if (r0 + u < r1) mat[(int64_t)(r0 + u) * nkeys + key] = run;
        run += v[u];
    }
}

// Places the records of queries [beg, end).  32-bit counters (cursor) start at the block's
// position for each key; packed 16-bit counters hold ranks only, and the key's base (bucket
// offset + block offset) is read from global memory.
template <int DIM, bool PACK16>
__device__ __forceinline__ void place_queries(const Geom& g, const float* __restrict__ q, int64_t beg, int64_t end,
                                              const int32_t* __restrict__ row, const int32_t* __restrict__ offs,
                                              uint32_t* cursor, float4* __restrict__ rec)
{
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
            int32_t p0 = 0;
            for_each_key<DIM>(g, x[u], [&](int32_t key) {
                int32_t pos;
                if constexpr (PACK16) pos = offs[key] + row[key] + (int32_t)lds_count_add<true>(cursor, key);
                else pos = (int32_t)lds_count_add<false>(cursor, key);
                put_record(rec, pos, x[u], i, key, p0);
            });
        }
    }
}

// Packed 16-bit path: places the records after k_sort_finish has written the key offsets.
template <int DIM>
__global__ __launch_bounds__(kSortThreads) void k_sort_scatter16(Geom g, const float* __restrict__ q, int64_t n,
                                                                 int64_t slice, int32_t nkeys,
                                                                 const int32_t* __restrict__ mat,
                                                                 const int32_t* __restrict__ offs,
                                                                 float4* __restrict__ rec)
{
    extern __shared__ uint32_t cursor[];
    for (int k = threadIdx.x; k < lds_words<true>(nkeys); k += kSortThreads) cursor[k] = 0u;
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * slice;
    place_queries<DIM, true>(g, q, beg, min(n, beg + slice), mat + (int64_t)blockIdx.x * nkeys, offs, cursor, rec);
}

// 32-bit path: places the records and builds the work lists on the way.  Every block scans
// the key totals itself (the same integer arithmetic in every block, so all agree), which
// gives the offsets of all keys, and starts its LDS cursor of a key at the key's offset plus
// the block's column offset; block b writes the work items of its share of bricks
// [b s, (b + 1) s), s = ceil(bricks / blocks), and block 0 the list sizes.  This takes the
// place of a separate single-block pass over the totals.
constexpr int kPlaceBricks = 4;  // bricks per thread and pass of the key scan
template <int DIM>
__global__ __launch_bounds__(kSortThreads) void k_sort_place(Geom g, const float* __restrict__ q, int64_t n,
                                                             int64_t slice, int64_t nbricks,
                                                             const int32_t* __restrict__ mat,
                                                             const int32_t* __restrict__ total,
                                                             float4* __restrict__ rec, WorkPtrs W)
{
    extern __shared__ uint32_t cursor[];
    const int64_t nkeys = 2 * nbricks;
    const int32_t* row = mat + (int64_t)blockIdx.x * nkeys;
    const int64_t share = (nbricks + gridDim.x - 1) / gridDim.x;
    const int64_t s0 = (int64_t)blockIdx.x * share, s1 = min(nbricks, s0 + share);
    int32_t carry[5] = {0, 0, 0, 0, 0};
    for (int64_t pass = 0; pass < nbricks; pass += (int64_t)kSortThreads * kPlaceBricks) {
        const int64_t b0 = pass + (int64_t)threadIdx.x * kPlaceBricks;
        int32_t tp[kPlaceBricks], ts[kPlaceBricks], cp[kPlaceBricks], cs[kPlaceBricks];
#pragma unroll
        for (int k = 0; k < kPlaceBricks; ++k) {
            const bool ok = b0 + k < nbricks;
            tp[k] = ok ? total[2 * (b0 + k)] : 0;
            ts[k] = ok ? total[2 * (b0 + k) + 1] : 0;
            cp[k] = ok ? row[2 * (b0 + k)] : 0;
            cs[k] = ok ? row[2 * (b0 + k) + 1] : 0;
        }
        int32_t v[5] = {0, 0, 0, 0, 0};
#pragma unroll
        for (int k = 0; k < kPlaceBricks; ++k) brick_counts(tp[k], ts[k], b0 + k < nbricks, v);
        int32_t pos[5], all[5];
        block_scan_multi<5, kSortThreads>(v, pos, all);
#pragma unroll
        for (int u = 0; u < 5; ++u) pos[u] += carry[u];
#pragma unroll
        for (int k = 0; k < kPlaceBricks; ++k) {
            const int64_t b = b0 + k;
            if (b >= nbricks) break;
            cursor[2 * b] = (uint32_t)(pos[0] + cp[k]);
            cursor[2 * b + 1] = (uint32_t)(pos[0] + tp[k] + cs[k]);
            brick_items(b, tp[k], ts[k], pos, W, b >= s0 && b < s1);
        }
#pragma unroll
        for (int u = 0; u < 5; ++u) carry[u] += all[u];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) write_meta(carry, W);
    __syncthreads();
    const int64_t beg = (int64_t)blockIdx.x * slice;
    place_queries<DIM, false>(g, q, beg, min(n, beg + slice), row, nullptr, cursor, rec);
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
    for_each_key<DIM>(g, x, [&](int32_t key) { atomicAdd(&counts[key], 1); });
}

template <int DIM>
__global__ __launch_bounds__(kThreads) void k_bucket_scatter(Geom g, const float* __restrict__ q, int64_t n,
                                                            int32_t* __restrict__ cursor, float4* __restrict__ rec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    float x[3] = {0.0f, 0.0f, 0.0f};
    load_query<DIM>(q, i, x);
    int32_t p0 = 0;
    for_each_key<DIM>(g, x, [&](int32_t key) { put_record(rec, atomicAdd(&cursor[key], 1), x, i, key, p0); });
}

static inline unsigned blocks_for(int64_t n, int per)
{
    return (unsigned)((n + per - 1) / per);
}

template <int DIM, bool PACK16>
static hipError_t launch_lds_sort(const tg_grid* g, const float* q, int64_t n, const WsLayout& L, int32_t* mat,
                                  int32_t* total, int32_t* offs, float4* rec, const WorkPtrs& W, hipStream_t s)
{
    const int32_t nkeys = (int32_t)L.nkeys;
    const size_t lds = (size_t)lds_words<PACK16>(nkeys) * sizeof(uint32_t);
    const dim3 gb((unsigned)L.sort_blocks), tb(kSortThreads);
    const void* place = PACK16 ? (const void*)k_sort_scatter16<DIM> : (const void*)k_sort_place<DIM>;
    if (lds > 65536) {
        // allow the full LDS of a CU, less the kernel's static LDS, for these kernels (the
        // same value every time, so a race between threads is harmless)
        for (const void* f : {(const void*)k_sort_count<DIM, PACK16>, place}) {
            hipFuncAttributes fa;
            hipError_t e = hipFuncGetAttributes(&fa, f);
            if (e == hipSuccess)
                e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)(kLdsBytes - (int64_t)fa.sharedSizeBytes));
            if (e != hipSuccess) return e;
        }
    }
    hipLaunchKernelGGL((k_sort_count<DIM, PACK16>), gb, tb, lds, s, g->geom, q, n, L.sort_slice, nkeys, mat);
    hipLaunchKernelGGL(k_sort_colscan, dim3(blocks_for(nkeys, 64)), dim3(64 * kColWaves), 0, s, mat,
                       (int32_t)L.sort_blocks, nkeys, total);
    if constexpr (PACK16) {
        hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(kFinishThreads), 0, s, total, g->nbricks, offs, nullptr, W);
        if (n > 0)
            hipLaunchKernelGGL(k_sort_scatter16<DIM>, gb, tb, lds, s, g->geom, q, n, L.sort_slice, nkeys, mat, offs,
                               rec);
    } else {
        // also when there are no queries: it writes the work lists
        hipLaunchKernelGGL(k_sort_place<DIM>, gb, tb, lds, s, g->geom, q, n, L.sort_slice, g->nbricks, mat, total,
                           rec, W);
    }
    return hipGetLastError();
}

hipError_t launch_sort(const tg_grid* g, const float* q, int64_t n, char* ws, const WsLayout& L, hipStream_t s)
{
    int32_t* offs = reinterpret_cast<int32_t*>(ws + L.offs_off);
    int32_t* counts = reinterpret_cast<int32_t*>(ws + L.counts_off);
    float4* rec = reinterpret_cast<float4*>(ws + L.rec_off);
    const int dim = g->desc.dim;
    WorkPtrs W;
    W.fitems = reinterpret_cast<int4*>(ws + L.fitems_off);
    W.bitems = reinterpret_cast<int4*>(ws + L.bitems_off);
    W.max_bitems = L.max_bitems;
    W.split_first = reinterpret_cast<int32_t*>(ws + L.splitb_off);
    W.split = reinterpret_cast<int2*>(ws + L.split_off);
    W.meta = reinterpret_cast<int32_t*>(ws + L.meta_off);
    if (L.sort_mode != SORT_ATOMIC) {
        int32_t* mat = reinterpret_cast<int32_t*>(ws + L.scratch_off);
        const bool p16 = L.sort_mode == SORT_LDS16;
        if (dim == 3)
            return p16 ? launch_lds_sort<3, true>(g, q, n, L, mat, counts, offs, rec, W, s)
                       : launch_lds_sort<3, false>(g, q, n, L, mat, counts, offs, rec, W, s);
        return p16 ? launch_lds_sort<2, true>(g, q, n, L, mat, counts, offs, rec, W, s)
                   : launch_lds_sort<2, false>(g, q, n, L, mat, counts, offs, rec, W, s);
    }
    hipLaunchKernelGGL(k_zero_i32, dim3(blocks_for(L.nkeys, kThreads)), dim3(kThreads), 0, s, counts, L.nkeys);
    if (n > 0) {
        if (dim == 3)
            hipLaunchKernelGGL(k_bucket_count<3>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, g->geom, q, n, counts);
        else
            hipLaunchKernelGGL(k_bucket_count<2>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, g->geom, q, n, counts);
    }
    // the finish kernel turns the counts into cursors in place (each thread reads its keys
    // before writing them)
    hipLaunchKernelGGL(k_sort_finish, dim3(1), dim3(kFinishThreads), 0, s, counts, g->nbricks, offs, counts, W);
    if (n > 0) {
        if (dim == 3)
            hipLaunchKernelGGL(k_bucket_scatter<3>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, g->geom, q, n, counts, rec);
        else
            hipLaunchKernelGGL(k_bucket_scatter<2>, dim3(blocks_for(n, kThreads)), dim3(kThreads), 0, s, g->geom, q, n, counts, rec);
    }
    return hipGetLastError();
}

}  // namespace tg
