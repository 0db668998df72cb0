// Host-side internals shared by the C-ABI layer and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "taylorgrid.h"
#include "tg_device.hpp"

struct tg_grid {
    tg_grid_desc desc;
    tg_grid_buffers bufs;
    tg::Geom geom;
    int32_t C;          // coefficients per vertex
    int32_t kord;       // kernel order code: the order, or kOrderFull for the full Hessian
    int64_t nvert;      // vertices
    int64_t nbricks;    // vertex bricks (launch size of the forward and backward)
    // last sort written by tg_sort_queries (or taken over by tg_share_sort) on this handle;
    // current while sort_gen is the workspace's sort generation
    const float* sort_q;
    int64_t sort_n;
    const void* sort_ws;
    uint64_t sort_gen;
    bool sort_valid;
};

namespace tg {

constexpr int kThreads = 256;
constexpr int kSortThreads = 1024;       // threads per block of the LDS-histogram sort
constexpr int64_t kLdsBytes = 160 * 1024; // LDS one workgroup may allocate on gfx950
constexpr int64_t kMaxLdsKeys32 = (kLdsBytes - 1024) / 4;  // 32-bit LDS counters (1 KB left for a scan)
constexpr int64_t kMaxLdsKeys16 = kLdsBytes / 2;  // packed 16-bit LDS counters
constexpr int64_t kMaxSlice16 = 65535;   // queries per block with 16-bit counters
constexpr int kMaxSortBlocks = 256;      // rows of the [blocks x keys] count matrix
constexpr int64_t kSortMinSlice = 4096;  // queries per sort block, at least
enum SortMode { SORT_LDS32 = 0, SORT_LDS16 = 1, SORT_ATOMIC = 2 };
constexpr int kFwdChunk = 1024;          // primary records per forward work item
constexpr int32_t kRecSecondary = (int32_t)0x80000000;  // record tag bit: secondary bucket copy
constexpr int kBwdItem = 512;            // records staged per pass of a backward work item
constexpr int kBwdItemMax = 2048;        // records per backward work item (4 passes)
// The adjoint with Adam stages every record of a split brick in the brick's first item (no
// partial sums) up to this many records; larger bricks keep their items.
constexpr int kBwdWholeMax = 8192;
constexpr int64_t kMaxMeshCells = (int64_t)1 << 28;  // 12 triangles per cell stay below 2^32
constexpr int kMaxReduceBlocks = 2048;  // FP64 partials: 4 per block
constexpr size_t kReduceBytes = (size_t)kMaxReduceBlocks * 4 * sizeof(double);
constexpr int64_t kMaxQueries = (int64_t)1 << 28;  // points per call of the unsorted measures
// Queries per sorted call: a query makes up to 2^dim sort records (its primary bucket and the
// neighbouring vertex bricks that own corners of its cell), whose positions are int32.
constexpr int64_t max_sorted_queries(int dim)
{
    return (int64_t)0x7fffffff >> dim;
}

// Workspace layout of one grid for n queries.  Offsets are from the workspace base and
// 256-byte aligned.
struct WsLayout {
    size_t reduce_off;   // FP64 reduction partials (tg_sdf_loss, tg_adam_step)
    size_t counts_off;   // int32 [nkeys]: per-key totals, or counts then cursors (atomic path)
    size_t offs_off;     // int32 [nkeys + 1]: exclusive bucket offsets (+ total at [nkeys])
    size_t scratch_off;  // int32 [sort_blocks x nkeys]: per-block key counts, then offsets
    size_t meta_off;     // int32 [16]: work-item totals
    size_t fitems_off;   // int4 [max_fitems]: forward work items (brick, first record, end, 0)
    size_t bitems_off;   // int4 [max_bitems]: backward items (brick, first record, end, items of
                         // the brick): split bricks' items from the front, whole bricks from the back
    size_t splitb_off;   // int32 [nbricks]: first backward item of each split brick
    size_t split_off;    // int2 [nbricks]: per split brick, (items finished, first item); the
                         // sort writes (0, first), the adjoint with Adam counts and resets
    size_t parts_off;    // float [max_slots x brick accumulator]: partial sums of split bricks
    size_t fpart_off;    // double [2 x fwd_blocks]: per-workgroup loss sums of the fused forward
    size_t bpart_off;    // double [max_bitems]: per-workgroup sum(dC^2) of the fused adjoint
    size_t rec_off;      // float4 [n * 2^dim]: sorted query records (x, y, z, tag)
    size_t urec_off;     // float4 [n * 2^dim]: upstream gradients (g_f, g_grad) in record order
    size_t total;
    int64_t nkeys;       // 2 * nbricks (primary / secondary bucket of every vertex brick)
    int sort_mode;       // SortMode
    int64_t sort_blocks; // blocks of the LDS-histogram sort
    int64_t sort_slice;  // queries per sort block
    int64_t max_fitems;  // bound on forward work items
    int64_t fwd_blocks;  // workgroups of a forward launch
    int64_t max_bitems;  // bound on backward work items
    int64_t max_slots;   // bound on partial-sum slots of split backward bricks
    int64_t merge_blocks;  // workgroups of the merge launch (the adjoint without Adam)
    int64_t acc_floats;  // floats in one brick accumulator (B^dim * C)
};

// Meta words in the workspace.
// Backward items: "front" items belong to bricks with more than one pass of records (listed
// from the front of the array, heaviest work first), "back" items to the other bricks
// (listed from the end); a brick with more than kBwdItemMax records is split into several
// items ("split" bricks), whose partial sums the merge launch adds (the adjoint with Adam
// takes the brick whole in its first item up to kBwdWholeMax records, else merges in the
// item that finishes last).
enum { META_FITEMS = 0, META_BFRONT = 1, META_BBACK = 2, META_NSPLITB = 3 };

WsLayout ws_layout(const tg_grid* g, int64_t n);

// Kernel launchers (return the launch status).
hipError_t launch_sort(const tg_grid* g, const float* q, int64_t n, char* ws, const WsLayout& L,
                       hipStream_t s);
// packed: f (forward) or g_f (adjoint, dq) is [n][4], one row (value, gradient) per query, and
// grad_f / g_grad are unused.
hipError_t launch_forward(const tg_grid* g, int64_t n, const char* ws, const WsLayout& L, float* f,
                          float* grad_f, hipStream_t s, bool packed = false);
hipError_t launch_dq(const tg_grid* g, int64_t n, const char* ws, const WsLayout& L, const float* g_f,
                     const float* g_grad, float* dq, hipStream_t s, bool packed = false);
hipError_t launch_backward(const tg_grid* g, int64_t n, const char* ws, const WsLayout& L,
                           const float* g_f, const float* g_grad, bool accumulate, hipStream_t s,
                           bool packed = false);
hipError_t launch_sdf_loss(int dim, int64_t n, const float* f, const float* grad_f, const float* d,
                           float eik_weight, float surf_k, float* g_f, float* g_grad, double* loss,
                           double* partials, hipStream_t s);
hipError_t launch_adam(const tg_grid* g, const tg_adam_params& p, double* grad_norm_sq, double* partials,
                       bool zero_grad, hipStream_t s);
// With finish = false the loss partials stay in the workspace (fpart_off, fwd_blocks pairs)
// for a later launch_loss_finish.
hipError_t launch_forward_loss(const tg_grid* g, int64_t n, const char* ws, const WsLayout& L, const float* d,
                               float eik_weight, float surf_k, float* g_f, float* g_grad, double* loss, float* f,
                               float* grad_f, hipStream_t s, bool record_order = false, bool finish = true);
// extra_grad (may be NULL): a stored gradient added to every coefficient's adjoint before
// the update (the TV term's, written beforehand).
hipError_t launch_backward_adam(const tg_grid* g, int64_t n, const char* ws, const WsLayout& L, const float* g_f,
                                const float* g_grad, const tg_adam_params& p, double* grad_norm_sq, hipStream_t s,
                                bool record_order = false, const float* extra_grad = nullptr, bool packed = false);
// Also sums ng sum(dC^2) partials into *gnorm when gpart is given, and adds tv_weight * *tv
// to the total when tv is given.
hipError_t launch_loss_finish(const double* partials, int64_t nblocks, int64_t n, float eik_weight, double* loss,
                              hipStream_t s, const double* gpart = nullptr, int64_t ng = 0, double* gnorm = nullptr,
                              float tv_weight = 0.0f, const double* tv = nullptr);
// TV of the master coefficients: *tv_out = TV (FP64), grad (=, or += when accumulating)
// weight * dTV/dC.  partials: kMaxReduceBlocks doubles.
hipError_t launch_tv(const tg_grid* g, float weight, double* tv_out, float* grad, bool accumulate,
                     double* partials, hipStream_t s);
// The fine grid's master (and storage copy) from the coarse field's value, gradient and
// Hessian at the fine vertices; the fine moments (when present) are zeroed.
hipError_t launch_upsample(const tg_grid* coarse, tg_grid* fine, hipStream_t s);
// Quality measures: IoU counts (partials: 2 int64 per block, kMaxReduceBlocks blocks at most),
// the marching-tetrahedra mesh (ws: mesh_workspace_bytes) and the Chamfer distance (ws:
// chamfer_workspace_bytes).
hipError_t launch_iou(int64_t n, const float* f, const float* d, int64_t* counts, int64_t* partials, hipStream_t s);
size_t mesh_workspace_bytes(int64_t ncell);
hipError_t launch_mesh(const int* n, const float* lo, const float* hi, const float* values, float* tri,
                       int64_t max_tris, int64_t* n_tris, char* ws, hipStream_t s);
size_t chamfer_workspace_bytes(int64_t na, int64_t nb);
hipError_t launch_chamfer(const float* a, int64_t na, const float* b, int64_t nb, int norm, double* out, char* ws,
                          hipStream_t s);
hipError_t launch_sum_finish(const double* partials, int64_t nblocks, double* out, hipStream_t s);
hipError_t launch_sum_finish_scaled(const double* partials, int64_t nblocks, double scale, double* out, hipStream_t s);
hipError_t launch_composite(int64_t n_rays, int32_t ns, const float* f, const float* col, const float* delta,
                            const float* target, float* rgb, double* loss, float* g_f, float* g_c, double* partials,
                            hipStream_t s);
AdamArgs make_adam_args(const tg_adam_params& p);
// coeffs = the storage rounding of master (16-bit storage; nothing to do for FP32).
hipError_t launch_sync_storage(const tg_grid* g, hipStream_t s);
// launch_sdf_loss with its FP64 partial sums in the library's static device scratch (the
// stream's device's copy) instead of a workspace; allocates nothing.
hipError_t launch_sdf_loss_noalloc(int dim, int64_t n, const float* f, const float* grad_f, const float* d,
                                   float eik_weight, float surf_k, float* g_f, float* g_grad, double* loss,
                                   hipStream_t s);
size_t noalloc_scratch_bytes();
// The field of a 3D single-channel symmetric-layout grid at the lattice s times finer than
// the grid, values [nz][ny][nx] with n = s (res - 1) + 1 (fewer than 2^31 points).
hipError_t launch_field_lattice(const tg_grid* g, int32_t s, float* values, hipStream_t st);
hipError_t launch_query(const tg_grid* const* grids, int32_t n_grids, const tg_request* reqs, int32_t n_reqs,
                        hipStream_t s);

}  // namespace tg
