// SDF quality measures (the paper evaluates reconstructions by IoU and Chamfer distance,
// Sec. 4.1): IoU counts of the inside sets on sample points, the field of a grid sampled on a
// lattice, a zero-level-set mesh of a sampled field by marching cubes, and the Chamfer
// distance between two point sets.
//
// Mesh (marching cubes; Sec. 4.1 extracts its meshes with marching cubes and prints no
// variant).  A lattice cell has corners c = bx + 2 by + 4 bz; a corner is inside when its
// value is < 0.  The 12 edges are numbered axis by axis (x, y, z), each axis's four in
// increasing order of their lower corner; a crossing edge (ends on different sides) carries
// the vertex p_a + v_a / (v_a - v_b) (p_b - p_a), a its lower end.  The triangles of each of
// the 256 inside/outside patterns come from a table built at compile time by one rule: walk
// every face of the cube counterclockwise as seen from outside, join each crossing where the
// walk enters the inside set to the next crossing where it leaves it (so a face with inside
// corners on a diagonal separates them); the joins form closed loops; each loop, started at
// its smallest edge and taken in increasing order of that edge, is cut into the fan
// (e0, e_i, e_i+1).  The walk's direction puts every triangle's normal (p1 - p0) x (p2 - p0)
// from the inside to the outside, and neighbouring cells put the same joins on a shared face,
// so the mesh is closed wherever the inside set is.  Triangles are written cell by cell (x
// fastest), then in table order: a first pass counts each cell's triangles and lists the
// cells that cross the level set with their offsets within the block, a scan of the block
// totals places the lists, which are compacted into one, and a last pass writes their
// triangles.
#include "tg_internal.hpp"

namespace tg {

constexpr int kMeshThreads = 256;
constexpr int kMeshCellsPerThread = 8;
constexpr int kMeshCellsPerBlock = kMeshThreads * kMeshCellsPerThread;

// ------------------------------------------------------------------ marching cubes table
constexpr int kCubeEdge[12][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7},   // along x
                                  {0, 2}, {1, 3}, {4, 6}, {5, 7},   // along y
                                  {0, 4}, {1, 5}, {2, 6}, {3, 7}};  // along z
constexpr int kMcMaxTris = 5;

struct McCase {
    uint8_t ntri;
    uint8_t edge[3 * kMcMaxTris];
};
struct McTable {
    McCase c[256];
};

constexpr int cube_edge_of(int a, int b)
{
    const int lo = a < b ? a : b, hi = a < b ? b : a;
    for (int k = 0; k < 12; ++k)
        if (kCubeEdge[k][0] == lo && kCubeEdge[k][1] == hi) return k;
    return -1;
}

// The triangles of every inside/outside pattern, by the face-walk rule described above.
constexpr McTable make_mc_table()
{
    McTable T{};
    for (int pat = 0; pat < 256; ++pat) {
        int next[12] = {-1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1, -1};
        for (int axis = 0; axis < 3; ++axis) {
            const int u = (axis + 1) % 3, v = (axis + 2) % 3;
            for (int side = 0; side < 2; ++side) {
                // the face's corners, counterclockwise about the outward normal
                const int sq[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
                int walk[4] = {0, 0, 0, 0};
                for (int k = 0; k < 4; ++k) {
                    const int kk = side == 1 ? k : (4 - k) % 4;  // the inner face runs the other way
                    walk[k] = (side << axis) | (sq[kk][0] << u) | (sq[kk][1] << v);
                }
                int enter_at[2] = {0, 0}, enter_edge[2] = {0, 0}, leave_at[2] = {0, 0}, leave_edge[2] = {0, 0};
                int ne = 0, nl = 0;
                for (int k = 0; k < 4; ++k) {
                    const int a = walk[k], b = walk[(k + 1) % 4];
                    const int ia = (pat >> a) & 1, ib = (pat >> b) & 1;
                    if (ia == ib) continue;
                    if (ia) {
                        leave_at[nl] = k;
                        leave_edge[nl++] = cube_edge_of(a, b);
                    } else {
                        enter_at[ne] = k;
                        enter_edge[ne++] = cube_edge_of(a, b);
                    }
                }
                for (int j = 0; j < ne; ++j) {
                    int best = 0, best_gap = 5;
                    for (int l = 0; l < nl; ++l) {
                        const int gap = (leave_at[l] - enter_at[j] + 4) % 4;
                        if (gap < best_gap) {
                            best_gap = gap;
                            best = l;
                        }
                    }
                    next[enter_edge[j]] = leave_edge[best];
                }
            }
        }
        bool seen[12] = {false, false, false, false, false, false, false, false, false, false, false, false};
        int nt = 0;
        for (int e0 = 0; e0 < 12; ++e0) {
            if (next[e0] < 0 || seen[e0]) continue;
            int loop[12] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
            int len = 0;
            for (int e = e0; !seen[e]; e = next[e]) {
                seen[e] = true;
                loop[len++] = e;
            }
            for (int i = 1; i + 1 < len; ++i) {
                T.c[pat].edge[3 * nt + 0] = (uint8_t)loop[0];
                T.c[pat].edge[3 * nt + 1] = (uint8_t)loop[i];
                T.c[pat].edge[3 * nt + 2] = (uint8_t)loop[i + 1];
                ++nt;
            }
        }
        T.c[pat].ntri = (uint8_t)nt;
    }
    return T;
}

constexpr McTable kMcHostTable = make_mc_table();
__constant__ McTable kMc = kMcHostTable;

constexpr int mc_max_tris()
{
    int m = 0;
    for (int p = 0; p < 256; ++p) m = kMcHostTable.c[p].ntri > m ? kMcHostTable.c[p].ntri : m;
    return m;
}
static_assert(mc_max_tris() <= kMcMaxTris, "a cube yields at most five triangles");
static_assert(kMcHostTable.c[1].ntri == 1 && kMcHostTable.c[0].ntri == 0 && kMcHostTable.c[255].ntri == 0,
              "one inside corner: one triangle; uniform cubes: none");

struct Lattice {
    int nx, ny, nz;
    float lo[3], h[3];
};

// Cell coordinates of cell c (x fastest); cells number below 2^28, so 32-bit division is exact.
__device__ __forceinline__ void cell_of(const Lattice& L, int64_t c, int& i, int& j, int& k)
{
    const uint32_t cc = (uint32_t)c, cx = (uint32_t)(L.nx - 1), cy = (uint32_t)(L.ny - 1);
    const uint32_t row = cc / cx;
    i = (int)(cc - row * cx);
    k = (int)(row / cy);
    j = (int)(row - (uint32_t)k * cy);
}

__device__ __forceinline__ void cell_values(const Lattice& L, const float* __restrict__ v, int i, int j, int k,
                                            float* cv)
{
#pragma unroll
    for (int c = 0; c < 8; ++c)
        cv[c] = v[((int64_t)(k + ((c >> 2) & 1)) * L.ny + (j + ((c >> 1) & 1))) * L.nx + (i + (c & 1))];
}

// Inside/outside pattern of a cell's corners (bit c set when corner c is inside).
__device__ __forceinline__ int cell_pattern(const float* cv)
{
    int p = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) p |= (cv[c] < 0.0f ? 1 : 0) << c;
    return p;
}

// Per block: kMeshCellsPerBlock consecutive cells, thread t taking cells q kMeshThreads + t
// (q < kMeshCellsPerThread), so that the 64 lanes of a wave read neighbouring lattice values.
// The block's cells that cross the level set (count > 0) are listed in cell order from
// blist[block * kMeshCellsPerBlock] with the exclusive prefix of the block's triangle counts
// at each of them in boff (nothing is written for the many cells that do not cross), their
// number in scnt and the block's triangle total in bsum.
__global__ __launch_bounds__(kMeshThreads) void k_mesh_count(Lattice L, const float* __restrict__ v, int64_t ncell,
                                                            uint32_t* __restrict__ boff, uint32_t* __restrict__ bsum,
                                                            uint32_t* __restrict__ blist, uint32_t* __restrict__ scnt)
{
    constexpr int kWaves = kMeshThreads / 64;
    static_assert(kMeshThreads == 256, "one thread per sign pattern stages the triangle counts");
    // per (q, wave): the wave's sums, in cell order
    __shared__ uint32_t wtot[kMeshCellsPerThread * kWaves];
    // triangles of every sign pattern (an LDS read instead of a per-lane gather from the table)
    __shared__ uint8_t ntri[256];
    ntri[threadIdx.x] = kMc.c[threadIdx.x].ntri;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int64_t cb = (int64_t)blockIdx.x * kMeshCellsPerBlock + threadIdx.x;
    // per cell: its triangle count in the high half-word and 1 if it crosses in the low one
    // (the block's sums stay below 2^16: at most 5 triangles per cell)
    uint32_t x[kMeshCellsPerThread], incl[kMeshCellsPerThread];
#pragma unroll
    for (int q = 0; q < kMeshCellsPerThread; ++q) {
        const int64_t c = cb + (int64_t)q * kMeshThreads;
        uint32_t n = 0;
        if (c < ncell) {
            int i, j, k;
            cell_of(L, c, i, j, k);
            float cv[8];
            cell_values(L, v, i, j, k, cv);
            n = ntri[cell_pattern(cv)];
        }
        x[q] = (n << 16) | (n > 0 ? 1u : 0u);
    }
#pragma unroll
    for (int q = 0; q < kMeshCellsPerThread; ++q) {
        uint32_t sc = x[q];
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t o = __shfl_up(sc, d, 64);
            if (lane >= d) sc += o;
        }
        incl[q] = sc;
        if (lane == 63) wtot[q * kWaves + wave] = sc;
    }
    __syncthreads();
    uint32_t* mine = blist + (int64_t)blockIdx.x * kMeshCellsPerBlock;
    uint32_t* mine_off = boff + (int64_t)blockIdx.x * kMeshCellsPerBlock;
    uint32_t all = 0;  // sums of the entries of earlier q
#pragma unroll
    for (int q = 0; q < kMeshCellsPerThread; ++q) {
        uint32_t before = all;
#pragma unroll
        for (int w = 0; w < kWaves; ++w) {
            const uint32_t t = wtot[q * kWaves + w];
            if (w < wave) before += t;
            all += t;
        }
        if (x[q] & 0xffffu) {
            const uint32_t ex = before + incl[q] - x[q];
            mine[ex & 0xffffu] = (uint32_t)(cb + (int64_t)q * kMeshThreads);
            mine_off[ex & 0xffffu] = ex >> 16;
        }
    }
    if (threadIdx.x == 0) {
        bsum[blockIdx.x] = all >> 16;
        scnt[blockIdx.x] = all & 0xffffu;
    }
}

// Gathers every block's list of crossing cells into one list at the block's scanned offset,
// with each cell's first triangle (the block's scanned triangle offset bsum added).
__global__ __launch_bounds__(kMeshThreads) void k_mesh_list(const uint32_t* __restrict__ blist,
                                                           const uint32_t* __restrict__ boff,
                                                           const uint32_t* __restrict__ scnt,
                                                           const uint32_t* __restrict__ soff,
                                                           const uint32_t* __restrict__ bsum,
                                                           uint32_t* __restrict__ list, uint32_t* __restrict__ lofs,
                                                           int64_t nb)
{
    for (int64_t b = blockIdx.x; b < nb; b += gridDim.x) {
        const uint32_t m = scnt[b], base = soff[b], tb = bsum[b];
        for (uint32_t r = threadIdx.x; r < m; r += kMeshThreads) {
            list[base + r] = blist[b * kMeshCellsPerBlock + r];
            lofs[base + r] = tb + boff[b * kMeshCellsPerBlock + r];
        }
    }
}

// One block: exclusive scans of the blocks' triangle totals (tri, in place) and crossing-cell
// counts (scnt into soff); *ntri and *nlist = their sums.  Each thread takes 4 consecutive
// entries of a pass.
__global__ __launch_bounds__(1024) void k_mesh_scan_blocks(uint32_t* __restrict__ tri, const uint32_t* __restrict__ scnt,
                                                          uint32_t* __restrict__ soff, int64_t nb,
                                                          int64_t* __restrict__ ntri, int64_t* __restrict__ nlist)
{
    constexpr int kPer = 4, kPass = 1024 * kPer;
    __shared__ uint32_t wsum[2][16];
    __shared__ uint32_t carry[2];
    if (threadIdx.x == 0) carry[0] = carry[1] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t b0 = 0; b0 < nb; b0 += kPass) {
        const int64_t b = b0 + (int64_t)threadIdx.x * kPer;
        uint32_t x[2][kPer], t[2] = {0u, 0u}, incl[2];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            x[0][k] = b + k < nb ? tri[b + k] : 0u;
            x[1][k] = b + k < nb ? scnt[b + k] : 0u;
            t[0] += x[0][k];
            t[1] += x[1][k];
        }
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            incl[u] = t[u];
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t o = __shfl_up(incl[u], d, 64);
                if (lane >= d) incl[u] += o;
            }
            if (lane == 63) wsum[u][wave] = incl[u];
        }
        __syncthreads();
        uint32_t run[2] = {carry[0], carry[1]};
        for (int w = 0; w < wave; ++w) {
            run[0] += wsum[0][w];
            run[1] += wsum[1][w];
        }
        const uint32_t end0 = run[0] + incl[0], end1 = run[1] + incl[1];
        run[0] += incl[0] - t[0];
        run[1] += incl[1] - t[1];
#pragma unroll
        for (int k = 0; k < kPer; ++k) {
            if (b + k < nb) {
                tri[b + k] = run[0];
                soff[b + k] = run[1];
            }
            run[0] += x[0][k];
            run[1] += x[1][k];
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            carry[0] = end0;
            carry[1] = end1;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        *ntri = (int64_t)carry[0];
        *nlist = (int64_t)carry[1];
    }
}

__device__ __forceinline__ void corner_pos(const Lattice& L, int i, int j, int k, int c, float* p)
{
    p[0] = L.lo[0] + (float)(i + (c & 1)) * L.h[0];
    p[1] = L.lo[1] + (float)(j + ((c >> 1) & 1)) * L.h[1];
    p[2] = L.lo[2] + (float)(k + ((c >> 2) & 1)) * L.h[2];
}

// One thread per cell that crosses the level set (the compacted list, *nlist of them).
__global__ __launch_bounds__(kMeshThreads) void k_mesh_emit(Lattice L, const float* __restrict__ v,
                                                           const uint32_t* __restrict__ list,
                                                           const int64_t* __restrict__ nlist,
                                                           const uint32_t* __restrict__ lofs, float* __restrict__ tri,
                                                           int64_t max_tris)
{
    const int64_t nl = *nlist;
    for (int64_t li = (int64_t)blockIdx.x * kMeshThreads + threadIdx.x; li < nl;
         li += (int64_t)gridDim.x * kMeshThreads) {
        const int64_t c = list[li];
        int i, j, k;
        cell_of(L, c, i, j, k);
        float cv[8];
        cell_values(L, v, i, j, k, cv);
        const McCase& mc = kMc.c[cell_pattern(cv)];
        const int64_t out0 = lofs[li];
        for (int t = 0; t < mc.ntri; ++t) {
            const int64_t out = out0 + t;
            if (out >= max_tris) break;  // past the caller's capacity: counted, not written
            for (int m = 0; m < 3; ++m) {
                const int e = mc.edge[3 * t + m];
                const int a = kCubeEdge[e][0], b = kCubeEdge[e][1];
                float pa[3], pb[3];
                corner_pos(L, i, j, k, a, pa);
                corner_pos(L, i, j, k, b, pb);
                const float va = cv[a], vb = cv[b];
                const float tt = va / (va - vb);
                for (int x = 0; x < 3; ++x) tri[(out * 3 + m) * 3 + x] = fmaf(tt, pb[x] - pa[x], pa[x]);
            }
        }
    }
}

// Workspace sections: per-block crossing-cell lists and their triangle offsets [nb * cells
// per block each], the compacted list and its triangle offsets [ncell each], per-block
// triangle totals / offsets, crossing-cell counts and offsets [nb each], the number of
// crossing cells and of triangles (int64).
struct MeshWs {
    size_t boff, blist, list, lofs, bsum, scnt, soff, nlist, total;
};

static MeshWs mesh_ws(int64_t ncell)
{
    const int64_t nb = std::max<int64_t>(1, (ncell + kMeshCellsPerBlock - 1) / kMeshCellsPerBlock);
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    MeshWs W;
    size_t off = 0;
    W.boff = off;
    off = up(off + (size_t)nb * kMeshCellsPerBlock * 4);
    W.blist = off;
    off = up(off + (size_t)nb * kMeshCellsPerBlock * 4);
    W.list = off;
    off = up(off + (size_t)ncell * 4);
    W.lofs = off;
    off = up(off + (size_t)ncell * 4);
    W.bsum = off;
    off = up(off + (size_t)nb * 4);
    W.scnt = off;
    off = up(off + (size_t)nb * 4);
    W.soff = off;
    off = up(off + (size_t)nb * 4);
    W.nlist = off;
    off = up(off + 8);
    W.total = off;
    return W;
}

size_t mesh_workspace_bytes(int64_t ncell)
{
    return mesh_ws(ncell).total;
}

hipError_t launch_mesh(const int* n, const float* lo, const float* hi, const float* values, float* tri,
                       int64_t max_tris, int64_t* n_tris, char* ws, hipStream_t s)
{
    Lattice L;
    L.nx = n[0];
    L.ny = n[1];
    L.nz = n[2];
    for (int a = 0; a < 3; ++a) {
        L.lo[a] = lo[a];
        L.h[a] = (float)(((double)hi[a] - (double)lo[a]) / (double)(n[a] - 1));
    }
    const int64_t ncell = (int64_t)(n[0] - 1) * (n[1] - 1) * (n[2] - 1);
    const int64_t nb = (ncell + kMeshCellsPerBlock - 1) / kMeshCellsPerBlock;
    const MeshWs W = mesh_ws(ncell);
    uint32_t* boff = reinterpret_cast<uint32_t*>(ws + W.boff);
    uint32_t* blist = reinterpret_cast<uint32_t*>(ws + W.blist);
    uint32_t* list = reinterpret_cast<uint32_t*>(ws + W.list);
    uint32_t* lofs = reinterpret_cast<uint32_t*>(ws + W.lofs);
    uint32_t* bsum = reinterpret_cast<uint32_t*>(ws + W.bsum);
    uint32_t* scnt = reinterpret_cast<uint32_t*>(ws + W.scnt);
    uint32_t* soff = reinterpret_cast<uint32_t*>(ws + W.soff);
    int64_t* nlist = reinterpret_cast<int64_t*>(ws + W.nlist);
    if (nb > 0)
        hipLaunchKernelGGL(k_mesh_count, dim3((unsigned)nb), dim3(kMeshThreads), 0, s, L, values, ncell, boff, bsum,
                           blist, scnt);
    hipLaunchKernelGGL(k_mesh_scan_blocks, dim3(1), dim3(1024), 0, s, bsum, scnt, soff, nb, n_tris, nlist);
    if (nb > 0) {
        const unsigned nlb = (unsigned)std::min<int64_t>(nb, 4096);
        hipLaunchKernelGGL(k_mesh_list, dim3(nlb), dim3(kMeshThreads), 0, s, blist, boff, scnt, soff, bsum, list,
                           lofs, nb);
        // at most every cell crosses; the kernel reads the actual count on the device
        const unsigned ne = (unsigned)std::min<int64_t>((ncell + kMeshThreads - 1) / kMeshThreads, 4096);
        hipLaunchKernelGGL(k_mesh_emit, dim3(ne), dim3(kMeshThreads), 0, s, L, values, list, nlist, lofs, tri,
                           max_tris);
    }
    return hipGetLastError();
}

// ------------------------------------------------------------------ IoU
__global__ __launch_bounds__(kThreads) void k_iou(int64_t n, const float* __restrict__ f, const float* __restrict__ d,
                                                 int64_t* __restrict__ partials)
{
    int64_t inter = 0, uni = 0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
        const bool a = f[i] < 0.0f, b = d[i] < 0.0f;
        inter += (a && b) ? 1 : 0;
        uni += (a || b) ? 1 : 0;
    }
    // exact integer sums (as doubles: every count is below 2^53)
    const double si = block_sum_f64<kThreads>((double)inter);
    const double su = block_sum_f64<kThreads>((double)uni);
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = (int64_t)si;
        partials[2 * blockIdx.x + 1] = (int64_t)su;
    }
}

constexpr int kFinishThreads = 256;

__global__ __launch_bounds__(kFinishThreads) void k_iou_finish(const int64_t* __restrict__ partials, int nb,
                                                              int64_t* __restrict__ counts)
{
    // exact: every count and sum is an integer below 2^53
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < nb; k += kFinishThreads) {
        a += (double)partials[2 * k];
        b += (double)partials[2 * k + 1];
    }
    a = block_sum_f64<kFinishThreads>(a);
    b = block_sum_f64<kFinishThreads>(b);
    if (threadIdx.x == 0) {
        counts[0] = (int64_t)a;
        counts[1] = (int64_t)b;
    }
}

hipError_t launch_iou(int64_t n, const float* f, const float* d, int64_t* counts, int64_t* partials, hipStream_t s)
{
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + kThreads * 4 - 1) / (kThreads * 4),
                                                                        kMaxReduceBlocks));
    hipLaunchKernelGGL(k_iou, dim3(nb), dim3(kThreads), 0, s, n, f, d, partials);
    hipLaunchKernelGGL(k_iou_finish, dim3(1), dim3(kFinishThreads), 0, s, partials, (int)nb, counts);
    return hipGetLastError();
}

// ------------------------------------------------------------------ Chamfer
// Exact nearest points on a bucket grid of the destination set.  The grid covers the bounding
// box of the destination's finite points with cubic cells (at most one cell per point,
// at most kNnDimMax along an axis); a point's cell is floor((x - org) / cs) per axis, clamped
// to the grid (non-finite coordinates included), so it is monotone in x.  The points are
// counting-sorted by cell (x fastest).  A source point visits the rings of cells around its
// own cell (ring r: the cells whose largest index difference is r), nearest first.  Every
// point of a cell in ring r + 1 differs from the source by at least r cells along one axis,
// so by at least r cs in the L1 and Euclidean norms (less a rounding allowance): the search
// stops once its best distance is below that bound, or when the rings leave the grid.  A point
// whose bound is not met within kNnNearRings rings (far from the other set, where the rings
// would grow large and serialise its thread) is listed instead, and a brute-force pass over
// the destination points (split over many workgroups) finishes the listed points.  The
// minimum is the one a comparison with every point finds (the same FP32 distances).
struct NnGrid {
    float org[3];
    float cs, inv_cs;
    float slack;  // rounding allowance of the ring bound
    int32_t dims[3];
    int32_t pad_;
};
constexpr int kNnDimMax = 1024;
constexpr int64_t kNnMaxCells = (int64_t)1 << 24;
constexpr int kNnBoxBlocks = 1024;
constexpr int kNnScanThreads = 1024;
constexpr int kNnScanPer = 4;  // cells per thread of the start scan
constexpr int kNnScanCells = kNnScanThreads * kNnScanPer;
constexpr int kNnNearRings = 2;   // rings a point searches before it is left to the brute-force pass
constexpr int kNnFarChunks = 16;  // workgroups along the list of far points (kThreads points each)
constexpr int kNnFarSplits = 256;  // workgroups along the destination points

static int64_t nn_max_cells(int64_t nd)
{
    return std::min<int64_t>(kNnMaxCells, std::max<int64_t>(1, nd));
}

__device__ __forceinline__ int32_t nn_axis_cell(float x, float org, float inv_cs, int32_t dim)
{
    float f = floorf((x - org) * inv_cs);
    if (!(f >= 0.0f)) f = 0.0f;  // NaN too
    if (f > (float)(dim - 1)) f = (float)(dim - 1);
    return (int32_t)f;
}

// Per block: min and max of the finite coordinates on every axis (part[6 block ..]).
__global__ __launch_bounds__(kThreads) void k_nn_box(const float* __restrict__ p, int64_t n, float* __restrict__ part)
{
    __shared__ float red[6][kThreads / 64];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float x = p[3 * i + a];
            if (isfinite(x)) {
                v[a] = fminf(v[a], x);
                v[3 + a] = fmaxf(v[3 + a], x);
            }
        }
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const float o = __shfl_xor(v[k], d, 64);
            v[k] = k < 3 ? fminf(v[k], o) : fmaxf(v[k], o);
        }
        if (lane == 0) red[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        float r = red[k][0];
        for (int w = 1; w < kThreads / 64; ++w) r = k < 3 ? fminf(r, red[k][w]) : fmaxf(r, red[k][w]);
        part[6 * blockIdx.x + k] = r;
    }
}

// One block: the box from the block partials; then thread 0 picks the cell size, the
// smallest of 2 emax 2^(-k/8) whose grid has at most max_cells cells (emax the largest
// extent).
__global__ __launch_bounds__(kThreads) void k_nn_setup(const float* __restrict__ part, int nblk, int64_t max_cells,
                                                      NnGrid* __restrict__ G, int32_t* __restrict__ nfar)
{
    __shared__ float red[6][kThreads / 64];
    float v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int b = threadIdx.x; b < nblk; b += kThreads)
#pragma unroll
        for (int k = 0; k < 6; ++k) v[k] = k < 3 ? fminf(v[k], part[6 * b + k]) : fmaxf(v[k], part[6 * b + k]);
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < 6; ++k) {
#pragma unroll
        for (int d = 32; d >= 1; d >>= 1) {
            const float o = __shfl_xor(v[k], d, 64);
            v[k] = k < 3 ? fminf(v[k], o) : fmaxf(v[k], o);
        }
        if (lane == 0) red[k][wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    *nfar = 0;
    float lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
        lo[a] = red[a][0];
        hi[a] = red[3 + a][0];
        for (int w = 1; w < kThreads / 64; ++w) {
            lo[a] = fminf(lo[a], red[a][w]);
            hi[a] = fmaxf(hi[a], red[3 + a][w]);
        }
    }
    double ext[3], emax = 0.0, amax = 0.0;
    for (int a = 0; a < 3; ++a) {
        if (!(lo[a] <= hi[a])) lo[a] = hi[a] = 0.0f;  // no finite coordinate
        ext[a] = (double)hi[a] - (double)lo[a];
        emax = fmax(emax, ext[a]);
        amax = fmax(amax, fmax(fabs((double)lo[a]), fabs((double)hi[a])));
    }
    double cs = emax > 0.0 ? 2.0 * emax : 1.0;
    int64_t dims[3] = {1, 1, 1};
    if (emax > 0.0) {
        for (int k = 1; k <= 8 * 40; ++k) {
            const double c = 2.0 * emax * exp2(-(double)k / 8.0);
            int64_t d[3], prod = 1;
            for (int a = 0; a < 3; ++a) {
                d[a] = std::min<int64_t>(kNnDimMax, (int64_t)floor(ext[a] / c) + 1);
                prod *= d[a];
            }
            if (prod > max_cells) break;
            cs = c;
            for (int a = 0; a < 3; ++a) dims[a] = d[a];
        }
    }
    NnGrid g;
    for (int a = 0; a < 3; ++a) {
        g.org[a] = lo[a];
        g.dims[a] = (int32_t)dims[a];
    }
    g.cs = (float)cs;
    g.inv_cs = (float)(1.0 / cs);
    // cell faces and FP32 differences are off by a few units in the last place of the
    // coordinates' magnitude; a generous allowance keeps the bound below every such error
    g.slack = (float)(1e-5 * (amax + cs));
    g.pad_ = 0;
    *G = g;
}

__global__ __launch_bounds__(kThreads) void k_nn_zero(int32_t* __restrict__ p, int64_t n)
{
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) p[i] = 0;
}

__device__ __forceinline__ int32_t nn_cell(const NnGrid& g, float x, float y, float z)
{
    const int32_t cx = nn_axis_cell(x, g.org[0], g.inv_cs, g.dims[0]);
    const int32_t cy = nn_axis_cell(y, g.org[1], g.inv_cs, g.dims[1]);
    const int32_t cz = nn_axis_cell(z, g.org[2], g.inv_cs, g.dims[2]);
    return cx + g.dims[0] * (cy + g.dims[1] * cz);
}

// Runs of neighbouring lanes of a wave with the same cell (c < 0: the lane has no point).  The
// run's first lane (head) stands for it in one atomic, which keeps the many repeated points of
// a triangle mesh (listed cell by cell) from queueing on one counter.
struct WaveRun {
    int head;  // lane of the run's first lane (-1 for a lane without a point)
    int off;   // position in the run
    int len;   // lanes in the run
};
__device__ __forceinline__ WaveRun wave_run(int32_t c)
{
    const int lane = threadIdx.x & 63;
    const int32_t cp = __shfl_up(c, 1, 64);
    const bool valid = c >= 0;
    const uint64_t heads = __ballot(valid && (lane == 0 || cp != c));
    const uint64_t stops = heads | __ballot(!valid);
    const uint64_t upto = heads & ((2ull << lane) - 1);  // heads at or below this lane
    WaveRun r;
    r.head = upto ? 63 - __builtin_clzll(upto) : -1;
    r.off = lane - r.head;
    const uint64_t after = r.head >= 0 ? stops & ~((2ull << r.head) - 1) : 0ull;
    r.len = (after ? __builtin_ctzll(after) : 64) - r.head;
    return r;
}

// Grid-stride loops over whole waves (the run detection needs every lane of the wave).
__global__ __launch_bounds__(kThreads) void k_nn_count(const float* __restrict__ p, int64_t n,
                                                      const NnGrid* __restrict__ G, int32_t* __restrict__ cnt)
{
    const NnGrid g = *G;
    const int lane = threadIdx.x & 63;
    for (int64_t i0 = (int64_t)blockIdx.x * kThreads + (threadIdx.x & ~63); i0 < n;
         i0 += (int64_t)gridDim.x * kThreads) {
        const int64_t i = i0 + lane;
        const int32_t c = i < n ? nn_cell(g, p[3 * i], p[3 * i + 1], p[3 * i + 2]) : -1;
        const WaveRun r = wave_run(c);
        if (c >= 0 && r.off == 0) atomicAdd(&cnt[c], r.len);
    }
}

// Exclusive scan of the kNnScanPer cells of each thread across the block; *total = the
// block's sum.
__device__ __forceinline__ void nn_block_scan(const int32_t* v, int32_t* ex, int32_t* wsum, int32_t* total)
{
    int32_t t = 0;
#pragma unroll
    for (int k = 0; k < kNnScanPer; ++k) t += v[k];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    int32_t incl = t;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t o = __shfl_up(incl, d, 64);
        if (lane >= d) incl += o;
    }
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    int32_t before = 0, all = 0;
    for (int w = 0; w < kNnScanThreads / 64; ++w) {
        if (w < wave) before += wsum[w];
        all += wsum[w];
    }
    int32_t run = before + incl - t;
#pragma unroll
    for (int k = 0; k < kNnScanPer; ++k) {
        ex[k] = run;
        run += v[k];
    }
    *total = all;
}

__global__ __launch_bounds__(kNnScanThreads) void k_nn_scan_blocks(const int32_t* __restrict__ cnt, int64_t ncell,
                                                                  int32_t* __restrict__ bsum)
{
    __shared__ int32_t wsum[kNnScanThreads / 64];
    const int64_t c0 = (int64_t)blockIdx.x * kNnScanCells + (int64_t)threadIdx.x * kNnScanPer;
    int32_t v[kNnScanPer], ex[kNnScanPer], total;
#pragma unroll
    for (int k = 0; k < kNnScanPer; ++k) v[k] = c0 + k < ncell ? cnt[c0 + k] : 0;
    nn_block_scan(v, ex, wsum, &total);
    if (threadIdx.x == 0) bsum[blockIdx.x] = total;
}

// One block: exclusive scan of the block sums in place.
__global__ __launch_bounds__(kNnScanThreads) void k_nn_scan_top(int32_t* __restrict__ bsum, int64_t nb)
{
    __shared__ int32_t wsum[kNnScanThreads / 64];
    __shared__ int32_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t b0 = 0; b0 < nb; b0 += kNnScanThreads) {
        const int64_t b = b0 + threadIdx.x;
        const int32_t x = b < nb ? bsum[b] : 0;
        int32_t incl = x;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int32_t o = __shfl_up(incl, d, 64);
            if (lane >= d) incl += o;
        }
        if (lane == 63) wsum[wave] = incl;
        __syncthreads();
        int32_t before = carry;
        for (int w = 0; w < wave; ++w) before += wsum[w];
        if (b < nb) bsum[b] = before + incl - x;
        __syncthreads();
        if (threadIdx.x == kNnScanThreads - 1) carry = before + incl;
        __syncthreads();
    }
}

// start[c] = first sorted position of cell c (start[ncell] = the total), cursor[c] = start[c].
__global__ __launch_bounds__(kNnScanThreads) void k_nn_scan_apply(const int32_t* __restrict__ cnt, int64_t ncell,
                                                                 const int32_t* __restrict__ boff,
                                                                 int32_t* __restrict__ start,
                                                                 int32_t* __restrict__ cursor)
{
    __shared__ int32_t wsum[kNnScanThreads / 64];
    const int64_t c0 = (int64_t)blockIdx.x * kNnScanCells + (int64_t)threadIdx.x * kNnScanPer;
    int32_t v[kNnScanPer], ex[kNnScanPer], total;
#pragma unroll
    for (int k = 0; k < kNnScanPer; ++k) v[k] = c0 + k < ncell ? cnt[c0 + k] : 0;
    nn_block_scan(v, ex, wsum, &total);
    const int32_t base = boff[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kNnScanPer; ++k) {
        const int64_t c = c0 + k;
        if (c < ncell) {
            start[c] = base + ex[k];
            cursor[c] = base + ex[k];
            if (c == ncell - 1) start[ncell] = base + ex[k] + v[k];
        }
    }
}

__global__ __launch_bounds__(kThreads) void k_nn_scatter(const float* __restrict__ p, int64_t n,
                                                        const NnGrid* __restrict__ G, int32_t* __restrict__ cursor,
                                                        float4* __restrict__ pts)
{
    const NnGrid g = *G;
    const int lane = threadIdx.x & 63;
    for (int64_t i0 = (int64_t)blockIdx.x * kThreads + (threadIdx.x & ~63); i0 < n;
         i0 += (int64_t)gridDim.x * kThreads) {
        const int64_t i = i0 + lane;
        float x = 0.0f, y = 0.0f, z = 0.0f;
        int32_t c = -1;
        if (i < n) {
            x = p[3 * i];
            y = p[3 * i + 1];
            z = p[3 * i + 2];
            c = nn_cell(g, x, y, z);
        }
        const WaveRun r = wave_run(c);
        int32_t base = 0;
        if (c >= 0 && r.off == 0) base = atomicAdd(&cursor[c], r.len);
        base = __shfl(base, r.head >= 0 ? r.head : lane, 64);
        if (c >= 0) pts[base + r.off] = make_float4(x, y, z, 0.0f);
    }
}

// NORM 1: the L1 distance; NORM 2: the squared Euclidean distance (its square root is taken
// once per source).
template <int NORM>
__device__ __forceinline__ float nn_scan_range(const float4* __restrict__ pts, int32_t b, int32_t e, float x, float y,
                                               float z, float best)
{
#pragma unroll 4
    for (int32_t j = b; j < e; ++j) {
        const float4 q = pts[j];
        const float dx = q.x - x, dy = q.y - y, dz = q.z - z;
        if constexpr (NORM == 1) best = fminf(best, fabsf(dx) + fabsf(dy) + fabsf(dz));
        else best = fminf(best, fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
    }
    return best;
}

// partials[block] = sum over the block's sources of the distance to the nearest destination,
// for the sources whose search completes within kNnNearRings rings; the others are appended
// to far_idx (their best distance so far, as float bits, to far_min).
template <int NORM>
__global__ __launch_bounds__(kThreads) void k_nn_search(const float* __restrict__ src, int64_t ns,
                                                       const NnGrid* __restrict__ G, const int32_t* __restrict__ start,
                                                       const float4* __restrict__ pts, double* __restrict__ partials,
                                                       int32_t* __restrict__ nfar, int32_t* __restrict__ far_idx,
                                                       uint32_t* __restrict__ far_min)
{
    const NnGrid g = *G;
    const int32_t rmax = max(g.dims[0], max(g.dims[1], g.dims[2]));
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < ns; i += (int64_t)gridDim.x * kThreads) {
        const float x = src[3 * i], y = src[3 * i + 1], z = src[3 * i + 2];
        const int32_t cx = nn_axis_cell(x, g.org[0], g.inv_cs, g.dims[0]);
        const int32_t cy = nn_axis_cell(y, g.org[1], g.inv_cs, g.dims[1]);
        const int32_t cz = nn_axis_cell(z, g.org[2], g.inv_cs, g.dims[2]);
        float best = INFINITY;
        // every cell of ring r is at least (r - 1) cs away
        auto bound_met = [&](int32_t r) {
            const float lb = (float)(r - 1) * g.cs - g.slack;
            return r >= 1 && lb > 0.0f && best <= (NORM == 1 ? lb : lb * lb);
        };
        // rings 0 and 1 together: the 3 x 3 rows of the cube around the cell, each a contiguous
        // run of up to 3 cells whose 4 cell starts are loaded up front
        {
            const int32_t xl = max(cx - 1, 0), xr = min(cx + 1, g.dims[0] - 1);
            int32_t sa[9], sm0[9], sm1[9], se[9];
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                const int32_t yy = cy - 1 + q % 3, zz = cz - 1 + q / 3;
                const bool in = yy >= 0 && yy < g.dims[1] && zz >= 0 && zz < g.dims[2];
                // the row of the clamped indices, so that no address leaves the grid
                const int32_t row = g.dims[0] * (min(max(yy, 0), g.dims[1] - 1) +
                                                 g.dims[1] * min(max(zz, 0), g.dims[2] - 1));
                sa[q] = in ? start[row + xl] : 0;
                sm0[q] = in ? start[row + cx] : 0;
                sm1[q] = in ? start[row + cx + 1] : 0;
                se[q] = in ? start[row + xr + 1] : 0;
            }
            // lower bounds of the distance to the neighbouring cells along each axis: the
            // point's distance to the shared cell face, less the rounding allowance
            const float lx = x - fmaf((float)cx, g.cs, g.org[0]);
            const float ly = y - fmaf((float)cy, g.cs, g.org[1]), lz = z - fmaf((float)cz, g.cs, g.org[2]);
            const float gx[3] = {fmaxf(lx - g.slack, 0.0f), 0.0f, fmaxf(g.cs - lx - g.slack, 0.0f)};
            const float gy[3] = {fmaxf(ly - g.slack, 0.0f), 0.0f, fmaxf(g.cs - ly - g.slack, 0.0f)};
            const float gz[3] = {fmaxf(lz - g.slack, 0.0f), 0.0f, fmaxf(g.cs - lz - g.slack, 0.0f)};
            auto lower = [&](float bx, float by, float bz) {
                return NORM == 1 ? bx + by + bz : fmaf(bx, bx, fmaf(by, by, bz * bz));
            };
            // the cell itself first, then its row's other cells, then the other rows, each
            // trimmed to the cells whose bound is below the best distance found
            best = nn_scan_range<NORM>(pts, sm0[4], sm1[4], x, y, z, best);
            if (lower(gx[0], 0.0f, 0.0f) < best) best = nn_scan_range<NORM>(pts, sa[4], sm0[4], x, y, z, best);
            if (lower(gx[2], 0.0f, 0.0f) < best) best = nn_scan_range<NORM>(pts, sm1[4], se[4], x, y, z, best);
#pragma unroll
            for (int q = 0; q < 9; ++q) {
                if (q == 4) continue;
                const float by = gy[q % 3], bz = gz[q / 3];
                if (lower(0.0f, by, bz) < best) {
                    const int32_t b = lower(gx[0], by, bz) < best ? sa[q] : sm0[q];
                    const int32_t e = lower(gx[2], by, bz) < best ? se[q] : sm1[q];
                    best = nn_scan_range<NORM>(pts, b, e, x, y, z, best);
                }
            }
        }
        int32_t r = 2;
        for (; r <= min(rmax, kNnNearRings); ++r) {
            if (bound_met(r)) break;
            const int32_t z0 = max(cz - r, 0), z1 = min(cz + r, g.dims[2] - 1);
            const int32_t y0 = max(cy - r, 0), y1 = min(cy + r, g.dims[1] - 1);
            const int32_t x0 = max(cx - r, 0), x1 = min(cx + r, g.dims[0] - 1);
            for (int32_t zz = z0; zz <= z1; ++zz) {
                for (int32_t yy = y0; yy <= y1; ++yy) {
                    const int32_t row = g.dims[0] * (yy + g.dims[1] * zz);
                    if (zz == cz - r || zz == cz + r || yy == cy - r || yy == cy + r) {
                        // a row on the ring's faces: every cell of the row in range, contiguous
                        best = nn_scan_range<NORM>(pts, start[row + x0], start[row + x1 + 1], x, y, z, best);
                    } else {
                        if (cx - r >= 0)
                            best = nn_scan_range<NORM>(pts, start[row + cx - r], start[row + cx - r + 1], x, y, z, best);
                        if (cx + r < g.dims[0])
                            best = nn_scan_range<NORM>(pts, start[row + cx + r], start[row + cx + r + 1], x, y, z, best);
                    }
                }
            }
        }
        // complete when every ring was visited or the next ring's bound is met
        if (r > rmax || bound_met(r)) {
            acc += NORM == 1 ? (double)best : (double)sqrtf(best);
        } else {
            const int32_t k = atomicAdd(nfar, 1);
            far_idx[k] = (int32_t)i;
            far_min[k] = __float_as_uint(best);
        }
    }
    const double tot = block_sum_f64<kThreads>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// The listed far sources against every destination point: kNnFarChunks x kNnFarSplits
// workgroups, every lane of a wave reading the same destination point; each workgroup's
// minimum over its split enters far_min with an integer atomic min (the bits of non-negative
// floats order as the floats).
template <int NORM>
__global__ __launch_bounds__(kThreads) void k_nn_far(const float* __restrict__ src, const int32_t* __restrict__ nfar_p,
                                                    const int32_t* __restrict__ far_idx, const float4* __restrict__ pts,
                                                    int64_t nd, uint32_t* __restrict__ far_min)
{
    const int32_t nfar = *nfar_p;
    const int32_t chunk = blockIdx.x % kNnFarChunks, split = blockIdx.x / kNnFarChunks;
    const int64_t per = (nd + kNnFarSplits - 1) / kNnFarSplits;
    const int64_t d0 = (int64_t)split * per, d1 = min(nd, d0 + per);
    for (int32_t k0 = chunk * kThreads; k0 < nfar; k0 += kNnFarChunks * kThreads) {
        const int32_t k = k0 + threadIdx.x;
        float x = 0.0f, y = 0.0f, z = 0.0f;
        if (k < nfar) {
            const int64_t i = far_idx[k];
            x = src[3 * i];
            y = src[3 * i + 1];
            z = src[3 * i + 2];
        }
        float best = INFINITY;
        // the destination index is the same in every lane: wave-uniform loads, no LDS
#pragma unroll 8
        for (int64_t j = d0; j < d1; ++j) {
            const float4 p = pts[j];
            const float dx = p.x - x, dy = p.y - y, dz = p.z - z;
            if constexpr (NORM == 1) best = fminf(best, fabsf(dx) + fabsf(dy) + fabsf(dz));
            else best = fminf(best, fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
        }
        if (k < nfar) atomicMin(&far_min[k], __float_as_uint(best));
    }
}

// *part = sum over the far sources of their distance to the nearest destination.
template <int NORM>
__global__ __launch_bounds__(kThreads) void k_nn_far_sum(const int32_t* __restrict__ nfar_p,
                                                        const uint32_t* __restrict__ far_min, double* __restrict__ part)
{
    const int32_t nfar = *nfar_p;
    double acc = 0.0;
    for (int32_t k = threadIdx.x; k < nfar; k += kThreads) {
        const float m = __uint_as_float(far_min[k]);
        acc += NORM == 1 ? (double)m : (double)sqrtf(m);
    }
    const double tot = block_sum_f64<kThreads>(acc);
    if (threadIdx.x == 0) *part = tot;
}

// Workspace of one direction's grid (offsets from the section's base, 256-byte aligned).
struct NnWs {
    size_t grid, box, cnt, bsum, start, cursor, pts, nfar, far_idx, far_min, total;
};

// nd destination points (bucketed), ns source points (the far list).
static NnWs nn_ws(int64_t nd, int64_t ns)
{
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const int64_t mc = nn_max_cells(nd);
    NnWs W;
    size_t off = 0;
    W.grid = off;
    off = up(off + sizeof(NnGrid));
    W.box = off;
    off = up(off + (size_t)kNnBoxBlocks * 6 * 4);
    W.cnt = off;
    off = up(off + (size_t)mc * 4);
    W.bsum = off;
    off = up(off + (size_t)((mc + kNnScanCells - 1) / kNnScanCells) * 4);
    W.start = off;
    off = up(off + (size_t)(mc + 1) * 4);
    W.cursor = off;
    off = up(off + (size_t)mc * 4);
    W.pts = off;
    off = up(off + (size_t)nd * 16);
    W.nfar = off;
    off = up(off + 4);
    W.far_idx = off;
    off = up(off + (size_t)ns * 4);
    W.far_min = off;
    off = up(off + (size_t)ns * 4);
    W.total = off;
    return W;
}

size_t chamfer_workspace_bytes(int64_t na, int64_t nb)
{
    return kReduceBytes + nn_ws(nb, na).total + nn_ws(na, nb).total;
}

// Builds the bucket grid of dst in the section at base and sums the nearest distances of
// src's points into partials (nblk + 1 of them: one per search block, then the far sources').
static void nn_direction(const float* src, int64_t ns, const float* dst, int64_t nd, int norm, char* base,
                         double* partials, unsigned nblk, hipStream_t s)
{
    const NnWs W = nn_ws(nd, ns);
    int32_t* nfar = reinterpret_cast<int32_t*>(base + W.nfar);
    int32_t* far_idx = reinterpret_cast<int32_t*>(base + W.far_idx);
    uint32_t* far_min = reinterpret_cast<uint32_t*>(base + W.far_min);
    NnGrid* G = reinterpret_cast<NnGrid*>(base + W.grid);
    float* box = reinterpret_cast<float*>(base + W.box);
    int32_t* cnt = reinterpret_cast<int32_t*>(base + W.cnt);
    int32_t* bsum = reinterpret_cast<int32_t*>(base + W.bsum);
    int32_t* start = reinterpret_cast<int32_t*>(base + W.start);
    int32_t* cursor = reinterpret_cast<int32_t*>(base + W.cursor);
    float4* pts = reinterpret_cast<float4*>(base + W.pts);
    const int64_t mc = nn_max_cells(nd);
    const int64_t nsb = (mc + kNnScanCells - 1) / kNnScanCells;
    const unsigned gbox = (unsigned)std::min<int64_t>((nd + kThreads - 1) / kThreads, kNnBoxBlocks);
    const unsigned gpts = (unsigned)std::min<int64_t>((nd + kThreads - 1) / kThreads, 8192);
    const unsigned gz = (unsigned)std::min<int64_t>((mc + kThreads - 1) / kThreads, 8192);
    hipLaunchKernelGGL(k_nn_box, dim3(gbox), dim3(kThreads), 0, s, dst, nd, box);
    hipLaunchKernelGGL(k_nn_setup, dim3(1), dim3(kThreads), 0, s, box, (int)gbox, mc, G, nfar);
    hipLaunchKernelGGL(k_nn_zero, dim3(gz), dim3(kThreads), 0, s, cnt, mc);
    hipLaunchKernelGGL(k_nn_count, dim3(gpts), dim3(kThreads), 0, s, dst, nd, G, cnt);
    hipLaunchKernelGGL(k_nn_scan_blocks, dim3((unsigned)nsb), dim3(kNnScanThreads), 0, s, cnt, mc, bsum);
    hipLaunchKernelGGL(k_nn_scan_top, dim3(1), dim3(kNnScanThreads), 0, s, bsum, nsb);
    hipLaunchKernelGGL(k_nn_scan_apply, dim3((unsigned)nsb), dim3(kNnScanThreads), 0, s, cnt, mc, bsum, start,
                       cursor);
    hipLaunchKernelGGL(k_nn_scatter, dim3(gpts), dim3(kThreads), 0, s, dst, nd, G, cursor, pts);
    auto search = norm == 1 ? k_nn_search<1> : k_nn_search<2>;
    auto far = norm == 1 ? k_nn_far<1> : k_nn_far<2>;
    auto far_sum = norm == 1 ? k_nn_far_sum<1> : k_nn_far_sum<2>;
    hipLaunchKernelGGL(search, dim3(nblk), dim3(kThreads), 0, s, src, ns, G, start, pts, partials, nfar, far_idx,
                       far_min);
    hipLaunchKernelGGL(far, dim3(kNnFarChunks * kNnFarSplits), dim3(kThreads), 0, s, src, nfar, far_idx, pts, nd,
                       far_min);
    hipLaunchKernelGGL(far_sum, dim3(1), dim3(kThreads), 0, s, nfar, far_min, partials + nblk);
}

__global__ __launch_bounds__(kFinishThreads) void k_chamfer_finish(const double* __restrict__ pa, int na_b,
                                                                  int64_t na, const double* __restrict__ pb,
                                                                  int nb_b, int64_t nb, double* __restrict__ out)
{
    double a = 0.0, b = 0.0;
    for (int k = threadIdx.x; k < na_b; k += kFinishThreads) a += pa[k];
    for (int k = threadIdx.x; k < nb_b; k += kFinishThreads) b += pb[k];
    a = block_sum_f64<kFinishThreads>(a);
    b = block_sum_f64<kFinishThreads>(b);
    if (threadIdx.x == 0) {
        out[1] = a / (double)na;
        out[2] = b / (double)nb;
        out[0] = out[1] + out[2];
    }
}

hipError_t launch_chamfer(const float* a, int64_t na, const float* b, int64_t nb, int norm, double* out, char* ws,
                          hipStream_t s)
{
    double* partials = reinterpret_cast<double*>(ws);
    const int half = kMaxReduceBlocks * 2;  // the reduction area holds 4 kMaxReduceBlocks doubles
    // search blocks of each direction, one partial left for its far sources
    const unsigned ga = (unsigned)std::min<int64_t>((na + kThreads - 1) / kThreads, half - 1);
    const unsigned gb = (unsigned)std::min<int64_t>((nb + kThreads - 1) / kThreads, half - 1);
    char* sec_b = ws + kReduceBytes;  // the grid of b (searched by a's points)
    char* sec_a = sec_b + nn_ws(nb, na).total;
    nn_direction(a, na, b, nb, norm, sec_b, partials, ga, s);
    nn_direction(b, nb, a, na, norm, sec_a, partials + half, gb, s);
    hipLaunchKernelGGL(k_chamfer_finish, dim3(1), dim3(kFinishThreads), 0, s, partials, (int)ga + 1, na,
                       partials + half, (int)gb + 1, nb, out);
    return hipGetLastError();
}

}  // namespace tg
