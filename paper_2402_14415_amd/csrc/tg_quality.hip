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

__device__ __forceinline__ int cell_count(const float* cv)
{
    return kMc.c[cell_pattern(cv)].ntri;
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
    // per (q, wave): the wave's sums, in cell order
    __shared__ uint32_t wtot[kMeshCellsPerThread * kWaves];
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
            n = (uint32_t)cell_count(cv);
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
// counts (scnt into soff); *ntri and *nlist = their sums.
__global__ __launch_bounds__(1024) void k_mesh_scan_blocks(uint32_t* __restrict__ tri, const uint32_t* __restrict__ scnt,
                                                          uint32_t* __restrict__ soff, int64_t nb,
                                                          int64_t* __restrict__ ntri, int64_t* __restrict__ nlist)
{
    __shared__ uint32_t wsum[2][16];
    __shared__ uint32_t carry[2];
    if (threadIdx.x == 0) carry[0] = carry[1] = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int64_t b0 = 0; b0 < nb; b0 += 1024) {
        const int64_t b = b0 + threadIdx.x;
        uint32_t x[2] = {b < nb ? tri[b] : 0u, b < nb ? scnt[b] : 0u}, incl[2];
#pragma unroll
        for (int u = 0; u < 2; ++u) {
            incl[u] = x[u];
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t o = __shfl_up(incl[u], d, 64);
                if (lane >= d) incl[u] += o;
            }
            if (lane == 63) wsum[u][wave] = incl[u];
        }
        __syncthreads();
        uint32_t before[2] = {carry[0], carry[1]};
        for (int w = 0; w < wave; ++w) {
            before[0] += wsum[0][w];
            before[1] += wsum[1][w];
        }
        if (b < nb) {
            tri[b] = before[0] + incl[0] - x[0];
            soff[b] = before[1] + incl[1] - x[1];
        }
        __syncthreads();
        if (threadIdx.x == 1023) {
            carry[0] = before[0] + incl[0];
            carry[1] = before[1] + incl[1];
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
constexpr int kNnThreads = 256;
constexpr int kNnPerThread = 4;   // source points per thread (each staged point is read once for all)
constexpr int kNnTile = 2048;     // destination points per LDS tile (a multiple of 4)

// The destination set of one direction is split over S groups of workgroups (enough
// workgroups to fill the GPU when the source set is small): mins[split * ns + i] = the
// smallest squared distance from source i to split `split` of the destinations.  Brute
// force: destination tiles are staged in LDS as x, y, z arrays (padded to a multiple of 4
// with points at infinity), read 4 points at a time, and every thread compares each with
// its kNnPerThread source points held in registers.
constexpr int kNnTargetBlocks = 2048;

// NORM 1: the L1 distance |dx| + |dy| + |dz|; NORM 2: the squared Euclidean distance (the
// square root is taken once per source, in k_nn_reduce).
template <int NORM>
__global__ __launch_bounds__(kNnThreads) void k_nn_min(const float* __restrict__ src, int64_t ns,
                                                      const float* __restrict__ dst, int64_t nd, int64_t chunks,
                                                      int64_t tiles_per_split, float* __restrict__ mins)
{
    __shared__ __align__(16) float tx[kNnTile], ty[kNnTile], tz[kNnTile];
    constexpr int CHUNK = kNnThreads * kNnPerThread;
    const int64_t chunk = blockIdx.x % chunks, split = blockIdx.x / chunks;
    const int64_t s0 = chunk * CHUNK;
    const int64_t dbeg = split * tiles_per_split * kNnTile, dend = min(nd, dbeg + tiles_per_split * kNnTile);
    float px[kNnPerThread], py[kNnPerThread], pz[kNnPerThread], best[kNnPerThread];
#pragma unroll
    for (int r = 0; r < kNnPerThread; ++r) {
        const int64_t si = s0 + threadIdx.x + (int64_t)r * kNnThreads;
        const bool ok = si < ns;
        px[r] = ok ? src[3 * si] : 0.0f;
        py[r] = ok ? src[3 * si + 1] : 0.0f;
        pz[r] = ok ? src[3 * si + 2] : 0.0f;
        best[r] = INFINITY;
    }
    for (int64_t d0 = dbeg; d0 < dend; d0 += kNnTile) {
        const int cnt = (int)min((int64_t)kNnTile, dend - d0);
        const int cnt4 = (cnt + 3) & ~3;
        __syncthreads();
        for (int q = threadIdx.x; q < cnt4; q += kNnThreads) {
            const bool ok = q < cnt;
            tx[q] = ok ? dst[3 * (d0 + q)] : INFINITY;
            ty[q] = ok ? dst[3 * (d0 + q) + 1] : INFINITY;
            tz[q] = ok ? dst[3 * (d0 + q) + 2] : INFINITY;
        }
        __syncthreads();
        for (int q = 0; q < cnt4; q += 4) {
            const float4 X = *reinterpret_cast<const float4*>(tx + q);
            const float4 Y = *reinterpret_cast<const float4*>(ty + q);
            const float4 Z = *reinterpret_cast<const float4*>(tz + q);
            const float xs[4] = {X.x, X.y, X.z, X.w}, ys[4] = {Y.x, Y.y, Y.z, Y.w}, zs[4] = {Z.x, Z.y, Z.z, Z.w};
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int r = 0; r < kNnPerThread; ++r) {
                    const float dx = xs[u] - px[r], dy = ys[u] - py[r], dz = zs[u] - pz[r];
                    if constexpr (NORM == 1) best[r] = fminf(best[r], fabsf(dx) + fabsf(dy) + fabsf(dz));
                    else best[r] = fminf(best[r], fmaf(dx, dx, fmaf(dy, dy, dz * dz)));
                }
        }
    }
#pragma unroll
    for (int r = 0; r < kNnPerThread; ++r) {
        const int64_t si = s0 + threadIdx.x + (int64_t)r * kNnThreads;
        if (si < ns) mins[split * ns + si] = best[r];
    }
}

// partials[block] = sum over this block's sources of the distance to the nearest destination
// (the smallest of the splits' distances; for NORM 2, its square root).
template <int NORM>
__global__ __launch_bounds__(kThreads) void k_nn_reduce(const float* __restrict__ mins, int64_t ns, int64_t nsplit,
                                                       double* __restrict__ partials)
{
    double acc = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < ns; i += (int64_t)gridDim.x * kThreads) {
        float m = mins[i];
        for (int64_t sp = 1; sp < nsplit; ++sp) m = fminf(m, mins[sp * ns + i]);
        acc += NORM == 1 ? (double)m : (double)sqrtf(m);
    }
    const double tot = block_sum_f64<kThreads>(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = tot;
}

// Splits of the destination set for sources ns: enough workgroups to fill the GPU, at least
// one tile of destinations per split.
static int64_t nn_splits(int64_t ns, int64_t nd)
{
    constexpr int CHUNK = kNnThreads * kNnPerThread;
    const int64_t chunks = (ns + CHUNK - 1) / CHUNK, tiles = (nd + kNnTile - 1) / kNnTile;
    return std::max<int64_t>(1, std::min<int64_t>({(kNnTargetBlocks + chunks - 1) / chunks, tiles, 64}));
}

size_t chamfer_workspace_bytes(int64_t na, int64_t nb)
{
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    return kReduceBytes + up((size_t)na * nn_splits(na, nb) * 4) + up((size_t)nb * nn_splits(nb, na) * 4);
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
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    const int64_t sa = nn_splits(na, nb), sb = nn_splits(nb, na);
    float* mins_a = reinterpret_cast<float*>(ws + kReduceBytes);
    float* mins_b = reinterpret_cast<float*>(ws + kReduceBytes + up((size_t)na * sa * 4));
    constexpr int CHUNK = kNnThreads * kNnPerThread;
    const int64_t ca = (na + CHUNK - 1) / CHUNK, cb = (nb + CHUNK - 1) / CHUNK;
    const int64_t ta = ((nb + kNnTile - 1) / kNnTile + sa - 1) / sa;  // destination tiles per split
    const int64_t tb = ((na + kNnTile - 1) / kNnTile + sb - 1) / sb;
    auto nn_min = norm == 1 ? k_nn_min<1> : k_nn_min<2>;
    auto nn_reduce = norm == 1 ? k_nn_reduce<1> : k_nn_reduce<2>;
    hipLaunchKernelGGL(nn_min, dim3((unsigned)(ca * sa)), dim3(kNnThreads), 0, s, a, na, b, nb, ca, ta, mins_a);
    hipLaunchKernelGGL(nn_min, dim3((unsigned)(cb * sb)), dim3(kNnThreads), 0, s, b, nb, a, na, cb, tb, mins_b);
    const int half = kMaxReduceBlocks / 2;
    const unsigned ga = (unsigned)std::min<int64_t>((na + kThreads - 1) / kThreads, half);
    const unsigned gb = (unsigned)std::min<int64_t>((nb + kThreads - 1) / kThreads, half);
    hipLaunchKernelGGL(nn_reduce, dim3(ga), dim3(kThreads), 0, s, mins_a, na, sa, partials);
    hipLaunchKernelGGL(nn_reduce, dim3(gb), dim3(kThreads), 0, s, mins_b, nb, sb, partials + half);
    hipLaunchKernelGGL(k_chamfer_finish, dim3(1), dim3(kFinishThreads), 0, s, partials, (int)ga, na, partials + half,
                       (int)gb, nb, out);
    return hipGetLastError();
}

}  // namespace tg
