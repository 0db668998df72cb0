/*
 * taylorgrid.h -- C ABI of the MI355X (gfx950) TaylorGrid query path.
 *
 * TaylorGrid (arXiv 2402.14415, Sec. 3.1) represents a field f: R^n -> R (n = 2 or 3) by a
 * dense grid whose vertices each store the low-order Taylor series of f at that vertex
 * (value, gradient and, at order 2, the symmetric Hessian).  A query point is located in
 * its cell (Eq. 2); each corner's Taylor polynomial (Eq. 1) is evaluated at the point's
 * offset from that corner (Eq. 3); the corner values are blended with multilinear weights
 * (Eq. 4).  The grid is optimised directly, with no network (Sec. 3.1, Sec. 4.1), which
 * needs the adjoint of that map; the SDF task adds an L1 reconstruction term (Eq. 6) and
 * an eikonal term (Eq. 8) that needs the field's spatial gradient.  Beyond that path: the
 * rest of the SDF objective (Eq. 7's surface weight, the TV term), the coarse-to-fine step of
 * progressive training, the radiance-field form (Sec. 3.3: compositing, photometric loss,
 * a three-channel colour grid) and quality measures (IoU, a zero-level-set mesh, Chamfer).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  Grid geometry: res[a] vertices on axis a span the closed box [lo[a], hi[a]]; vertex i
 *    sits at lo + i*h, h = (hi - lo)/(res - 1).  Queries outside the box are clamped to it;
 *    the spatial gradient is zero along a clamped axis.  The cell of a point is
 *    floor((x - lo)/h) capped at res - 2 (a point on the high face uses the last cell).
 *  Coefficient layout: [res_z][res_y][res_x][C] (x fastest; 2D: [res_y][res_x][C]), C =
 *    tg_coeffs_per_vertex(dim, order) values per vertex holding the partial derivatives of
 *    f at the vertex in graded-lexicographic order (3D order 2: f, fx, fy, fz, fxx, fxy,
 *    fxz, fyy, fyz, fzz; 2D order 2: f, fx, fy, fxx, fxy, fyy), in world units.  Two
 *    further layouts (tg_grid_desc): the full Hessian (f, the gradient, all dim^2 second
 *    derivatives row-major) and three channels at order 1 (each channel's f and gradient in
 *    turn).
 *  Queries: q is [n][dim] FP32, row-major.  Outputs are in the caller's query order.
 *  Memory: every pointer argument is DEVICE memory unless marked (host).  The library
 *    never allocates, copies or frees device memory; buffers belong to the caller and must
 *    outlive the calls that use them.  Workspaces are caller-allocated device buffers of at
 *    least the size the matching *_workspace_bytes function returns; their content is
 *    private to the library between the calls documented to share it.
 *  Streams: `stream` is a hipStream_t passed as void* (NULL = the null stream).  Every
 *    call only enqueues work and returns; results are ready when the stream reaches them.
 *  Errors: arguments are validated on the host before anything is enqueued; on failure
 *    the call returns a non-zero tg_status and enqueues nothing (outputs untouched).  A
 *    launch failure is reported as TG_ERR_DEVICE.  tg_last_error() returns a thread-local
 *    description of the last failure.  No call aborts or throws.
 *  Sizes: n = 0 is a no-op returning TG_OK.  Calls that sort queries take n <= (2^31 - 1) /
 *    2^dim (a query makes up to 2^dim int32-indexed sort records); the others n <= 2^28.
 *  Sorting: tg_forward, tg_backward, tg_forward_sdf_loss and tg_backward_adam read the
 *    bucketing of (q, n) that tg_sort_queries (or tg_train_step) wrote into ws, and fail with
 *    TG_ERR_STATE without it; one sort serves any number of these calls.
 *  Concurrency: calls on different grid handles may run concurrently.  Calls on one
 *    handle must be serialised by the caller (the handle records the last sort).
 */
#ifndef TAYLORGRID_H
#define TAYLORGRID_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TG_OK = 0,
    TG_ERR_INVALID_ARG = 1, /* a NULL, out-of-range or inconsistent argument */
    TG_ERR_UNSUPPORTED = 2, /* valid request this library does not implement */
    TG_ERR_DEVICE = 3,      /* HIP reported an error on launch */
    TG_ERR_CAPACITY = 4,    /* workspace too small or size beyond the supported maximum */
    TG_ERR_STATE = 5        /* workspace does not hold the sort this call needs */
} tg_status;

typedef enum { TG_F32 = 0, TG_BF16 = 1, TG_F16 = 2 } tg_dtype;

/* Grid geometry and storage type (host struct, copied by tg_create). */
typedef struct {
    int32_t dim;     /* 2 or 3 */
    int32_t res[3];  /* vertices per axis, each in [2, 65536]; res[2] unused when dim == 2 */
    int32_t order;   /* Taylor order K: 0, 1 or 2 */
    float lo[3];     /* box corner; lo[2] unused when dim == 2 */
    float hi[3];     /* hi[a] > lo[a], both finite */
    int32_t storage; /* tg_dtype of `coeffs` */
    int32_t hessian; /* order 2 only: TG_HESSIAN_SYMMETRIC (default, 0) stores the dim(dim+1)/2
                        distinct entries; TG_HESSIAN_FULL stores all dim^2 entries (row-major),
                        1 + dim + dim^2 coefficients per vertex (13 in 3D) */
    int32_t channels; /* 1 (default 0 means 1), or 3 with order 1: a three-channel field such as
                         the radiance form's colour (Sec. 3.3), each vertex storing the three
                         channels' series one after the other (3 (1 + dim) coefficients, 12 in
                         3D); tg_forward writes f [3][n] (grad_f must be NULL) and tg_backward /
                         tg_backward_adam take g_f [3][n] (g_grad and dq must be NULL).  The SDF
                         calls, tg_query and tg_upsample refuse it (TG_ERR_UNSUPPORTED). */
} tg_grid_desc;

#define TG_HESSIAN_SYMMETRIC 0
#define TG_HESSIAN_FULL 1

/* Device buffers of one grid, all with the coefficient layout above (host struct).
 * A pointer may be NULL when no call that needs it is made. */
typedef struct {
    void* coeffs;  /* storage dtype; read by tg_forward, tg_query; rewritten by tg_adam_step
                      when storage != TG_F32 (round-to-nearest-even copy of master) */
    float* master; /* FP32 master coefficients updated by tg_adam_step; when storage ==
                      TG_F32 it must equal `coeffs` */
    float* grad;   /* FP32 gradient: written (or accumulated) by tg_backward, read by
                      tg_adam_step */
    float* adam_m; /* FP32 first moment */
    float* adam_v; /* FP32 second moment */
} tg_grid_buffers;

typedef struct tg_grid tg_grid; /* opaque host-side handle: geometry + buffer pointers */

/* Weights of the SDF objective of Sec. 3.2, Eq. 8 (host struct): L = L_recon (Eq. 6, weighted
 * by Eq. 7 with k = surface_k; 0 = unweighted) + eik_weight L_eik + tv_weight L_TV. */
typedef struct {
    float eik_weight; /* lambda_1 (finite) */
    float surface_k;  /* k of Eq. 7 (finite, >= 0) */
    float tv_weight;  /* lambda_2 (finite; 0 = no TV term) */
} tg_sdf_objective;

/* Adam hyper-parameters (host struct).  step counts from 1. */
typedef struct {
    float lr, beta1, beta2, eps, weight_decay;
    int64_t step;
} tg_adam_params;

/* One serving request (host struct): n query points against grid index `grid`. */
typedef struct {
    int32_t grid;    /* index into the grids array of tg_query */
    int32_t pad_;
    int64_t n;       /* number of points, >= 0 */
    const float* q;  /* [n][dim] */
    float* sdf;      /* [n] field value */
    float* normal;   /* [n][dim] unit gradient (zero where the gradient vanishes); NULL = skip */
} tg_request;

/* Flags. */
#define TG_BWD_ACCUMULATE 1  /* tg_backward: grad += contribution (default: grad = contribution,
                                which saves the training loop a separate zeroing pass over grad) */
#define TG_ADAM_ZERO_GRAD 1  /* tg_adam_step: zero grad after reading it */
#define TG_BWD_ADD_GRAD 1    /* tg_backward_adam: add bufs.grad (e.g. tg_tv_loss's gradient) to the
                                adjoint before the update */
#define TG_BWD_PACKED 2      /* tg_backward, tg_backward_adam: g_f is [n][4], each query's
                                (g_f, g_grad) in one 16-byte row (in 2D the last word is ignored),
                                the layout tg_forward_packed writes; g_grad must be NULL */

/* binom(dim + order, order), or -1 when dim is not 2/3 or order is not 0..2. */
int32_t tg_coeffs_per_vertex(int32_t dim, int32_t order);

/* Create a handle (host only; nothing is enqueued).  The descriptor is copied; buffers may
 * be NULL and set later with tg_set_buffers.  *out receives the handle on success. */
tg_status tg_create(const tg_grid_desc* desc, const tg_grid_buffers* bufs, tg_grid** out);

/* Replace the buffer pointers of a handle (host only). */
tg_status tg_set_buffers(tg_grid* grid, const tg_grid_buffers* bufs);

/* Free a handle (host only).  NULL is accepted. */
tg_status tg_destroy(tg_grid* grid);

/* Device workspace bytes that tg_sort_queries, tg_forward and tg_backward need for n
 * queries on this grid (the sort, sized for the worst case), plus the reduction scratch
 * that tg_sdf_loss and tg_adam_step use.  0 on an invalid handle or n. */
size_t tg_workspace_bytes(const tg_grid* grid, int64_t n);

/* Bytes of reduction scratch that tg_sdf_loss and tg_adam_step need (a constant). */
size_t tg_reduce_workspace_bytes(void);

/* Bucket the queries by brick of cells (an implementation step that makes the grid
 * gathers of tg_forward and the adjoint scatter of tg_backward local; it has no
 * counterpart in the paper).  Writes the sort into `ws`, and records (q, n, ws) in the
 * handle: tg_forward and tg_backward on the same (q, n, ws) reuse it, until another sort
 * is written into ws (by any handle).  The queries must not change between this call and
 * the calls that reuse the sort. */
tg_status tg_sort_queries(tg_grid* grid, const float* q, int64_t n, void* ws, size_t ws_bytes,
                          void* stream);

/* Let `grid` reuse the sort of (q, n) that `sorted` holds in ws (host only; nothing is
 * enqueued).  The bucketing depends only on the cell geometry, so grids with the same dim,
 * res, lo and hi (compared exactly) bucket the same queries identically, whatever their
 * order, channels or storage; a field with several grids on one vertex lattice (the density
 * and colour grids of the radiance form, Sec. 3.3) sorts its samples once.  ws_bytes must cover
 * tg_workspace_bytes(grid, n), which grows with the coefficient count: size a shared
 * workspace for the grid with the most coefficients per vertex.  Errors: TG_ERR_INVALID_ARG
 * for a NULL handle or different geometry, TG_ERR_CAPACITY for a short workspace,
 * TG_ERR_STATE when ws does not hold sorted's current sort of (q, n).  A workspace is known
 * by its address: any later tg_sort_queries or tg_train_step into ws supersedes the sort
 * for every handle that shares it (their calls then fail with TG_ERR_STATE).  Calls that
 * share a workspace must be ordered on one stream: each uses its reduction and partial-sum
 * sections. */
tg_status tg_share_sort(tg_grid* grid, const tg_grid* sorted, const float* q, int64_t n, const void* ws,
                        size_t ws_bytes);

/* Field value and spatial gradient at each query (Sec. 3.1, Eq. 2-4):
 *   f[i] = sum over the 2^dim corners b of the cell of w_b(x) T_b(x - v_b),
 *   grad_f[i][a] = df/dx_a (0 on a clamped axis).
 * Requires the sort of (q, n) in ws (TG_ERR_STATE otherwise).  grad_f may be NULL. */
tg_status tg_forward(tg_grid* grid, const float* q, int64_t n, void* ws, size_t ws_bytes,
                     float* f, float* grad_f, void* stream);

/* tg_forward (Sec. 3.1, Eq. 2-4) with each query's value and gradient packed in one 16-byte
 * row: fg[i] = (f[i], grad_f[i][0], grad_f[i][1], grad_f[i][2]), fg [n][4] (in 2D the last
 * word is written 0), the same values as tg_forward's.  The queries are evaluated in bucket
 * order, so their outputs land at scattered rows: one aligned 16-byte store per query costs
 * about half of tg_forward's two.  tg_backward with TG_BWD_PACKED takes the upstream
 * gradients in the same layout.  fg: device, 16-byte aligned, written only.  Single-channel
 * grids only (TG_ERR_UNSUPPORTED for a three-channel grid); TG_ERR_INVALID_ARG for a NULL or
 * misaligned fg with n > 0; requires the sort of (q, n) in ws (TG_ERR_STATE otherwise). */
tg_status tg_forward_packed(tg_grid* grid, const float* q, int64_t n, void* ws, size_t ws_bytes,
                            float* fg, void* stream);

/* SDF objective (Sec. 3.2, Eq. 6 with the adaptive weight of Eq. 7, plus the eikonal term
 * of Eq. 8):
 *   L = mean_i w_i |f_i - d_i| + eik_weight * mean_i (|grad_f_i| - 1)^2,
 *   w_i = max(w'(f_i), w'(d_i)),  w'(x) = 1 - |2 sigmoid(surface_k x) - 1|,
 * written as loss[0] = L, loss[1] = weighted L1 mean, loss[2] = eikonal mean, in FP64
 * (device).  surface_k >= 0 (finite); 0 gives w = 1, the unweighted L1.  The weight is a
 * per-sample importance: it is held fixed in the gradient.  Writes the upstream gradients
 * g_f[i] = dL/df_i and, if grad_f != NULL, g_grad[i][a] = dL/d(grad_f_i)_a.  grad_f == NULL
 * drops the eikonal term (g_grad unused).  ws must hold tg_reduce_workspace_bytes(). */
tg_status tg_sdf_loss(int32_t dim, int64_t n, const float* f, const float* grad_f, const float* d,
                      float eik_weight, float surface_k, float* g_f, float* g_grad, double* loss,
                      void* ws, size_t ws_bytes, void* stream);

/* tg_sdf_loss for callers that cannot allocate device memory (code under HIP graph capture,
 * serving loops and harnesses that forbid allocation): no workspace argument.  Its FP64
 * per-block sums go to a static device array of the library (32 KiB, one per GPU, held until
 * the process ends, looked up on the stream's device at its first use there); nothing is
 * allocated, and nothing in it needs to start at zero.  Results are identical to
 * tg_sdf_loss's.  n <= 2^28 (TG_ERR_CAPACITY beyond).  Every call on one GPU shares that
 * GPU's array: calls that overlap on one GPU (on different streams, or from several host
 * threads without ordering) race and give wrong losses; order them on one stream. */
tg_status tg_sdf_loss_noalloc(int32_t dim, int64_t n, const float* f, const float* grad_f, const float* d,
                              float eik_weight, float surface_k, float* g_f, float* g_grad, double* loss,
                              void* stream);

/* Total variation of the coefficient grid (the L_TV term of Sec. 3.2, Eq. 8; the paper
 * cites the regulariser of Plenoxels and prints no formula).  For every vertex v and stored
 * coefficient channel c, with Delta_a(v, c) = master(v + e_a, c) - master(v, c) along each
 * axis a (0 on the grid's last layer along a):
 *   loss[0] = TV = (1/|V|) sum_v sum_c sqrt(sum_a Delta_a(v, c)^2)   (FP64, device),
 *   grad (=, or += with TG_BWD_ACCUMULATE) weight * dTV/dC   (0 for terms whose differences
 *   are all 0).
 * Reads bufs.master, writes bufs.grad (both required).  One pass: every workgroup stages a
 * tile of vertices with a one-vertex halo in LDS.  ws must hold tg_reduce_workspace_bytes(). */
tg_status tg_tv_loss(tg_grid* grid, float weight, double* loss, int32_t flags, void* ws,
                     size_t ws_bytes, void* stream);

/* Coarse-to-fine step of the progressive training schedule (Sec. 4.1 trains progressively,
 * from coarse to fine resolution): the fine grid, over the same box (dim, lo and hi compared
 * exactly), takes the field the coarse grid represents.  Every fine vertex v stores the
 * coarse field's value, gradient and Hessian at v (Eq. 2-4 and their exact derivatives) in
 * the stored order (value; gradient; Hessian xx, xy, xz, yy, yz, zz / xx, xy, yy), truncated
 * to the fine order: fine master (FP32) and, for 16-bit storage, its round-to-nearest-even
 * copy in coeffs.  Fine adam_m and adam_v, when present, are zeroed (a new optimisation
 * stage; the Adam step count is the caller's).  A fine vertex i on axis a lies at
 * i (res_c - 1) / (res_f - 1) in coarse cell units, located in exact integer arithmetic; on
 * a coarse face it takes the cell above (the top face: the last cell), where the gradient
 * and Hessian are that cell's one-sided values.  Reads the coarse master; the fine buffers
 * must not overlap it.  Any orders and resolutions (finer or not). */
tg_status tg_upsample(const tg_grid* coarse, tg_grid* fine, void* stream);

/* Quality measures (the paper reports IoU and Chamfer distance of its reconstructions,
 * Sec. 4.1; these evaluate a fitted grid against a known shape).
 *
 * IoU counts of the inside sets A = {i : f[i] < 0} and B = {i : d[i] < 0} over n sample
 * points (f: the grid's values, e.g. from tg_forward; d: the reference SDF):
 *   counts[0] = |A and B|, counts[1] = |A or B|   (device int64 [2]; IoU = counts[0] /
 *   counts[1], 1 when both are empty).  Exact integer counts.  ws must hold
 *   tg_reduce_workspace_bytes(). */
tg_status tg_iou_counts(int64_t n, const float* f, const float* d, int64_t* counts, void* ws,
                        size_t ws_bytes, void* stream);

/* The field of a grid on the lattice s times finer than the grid, for the zero-level-set mesh
 * of the learned field (Sec. 4.1 meshes its fields with marching cubes): values [nz][ny][nx]
 * (device FP32, x fastest), n[a] = s (res[a] - 1) + 1, point (i, j, k) at lo + (i, j, k) h / s
 * (h the cell size); every s-th point is a grid vertex.  Each value is the field of Sec. 3.1,
 * Eq. 2-4 (in FP32), at its point located exactly: on axis a point i lies in cell
 * c = min(floor(i / s), res[a] - 2) at local coordinate (i - s c) / s, so a point on a cell
 * face takes the cell above (the top face: the last cell).  3D grids of one channel in the
 * symmetric layout (TG_ERR_UNSUPPORTED otherwise), 1 <= s <= 64, fewer than 2^31 points
 * (TG_ERR_CAPACITY).  No workspace. */
tg_status tg_field_lattice(const tg_grid* grid, int32_t s, float* values, void* stream);

/* Device workspace bytes of tg_mesh for a lattice of n[0] x n[1] x n[2] points (host array);
 * 0 when n is invalid or the lattice has more than 2^28 cells. */
size_t tg_mesh_workspace_bytes(const int32_t* n);

/* Zero-level-set mesh of a field sampled on a lattice, by marching cubes (Sec. 4.1 extracts
 * its meshes with marching cubes).  values [n[2]][n[1]][n[0]] (device, x fastest) at the
 * points lo + i (hi - lo) / (n - 1) (n, lo, hi host arrays of 3; every n[a] in 2..65536, at
 * most 2^28 cells).  A cell's corners are c = bx + 2 by + 4 bz; a corner with value < 0 is
 * inside.  Edges are numbered axis by axis, each axis's four by increasing lower corner:
 * (0,1) (2,3) (4,5) (6,7), (0,2) (1,3) (4,6) (5,7), (0,4) (1,5) (2,6) (3,7); an edge whose
 * ends differ carries the vertex p_a + v_a / (v_a - v_b) (p_b - p_a), a its lower end.  The
 * triangles of a cell: walk each face counterclockwise as seen from outside the cube and join
 * every crossing where the walk enters the inside set to the next crossing where it leaves it
 * (a face with inside corners on a diagonal separates them); the joins form loops; each loop
 * (e0, e1, ..., started at its smallest edge, loops in increasing order of that edge) gives
 * the fan (e0, e_i, e_i+1).  Every triangle's normal (p1 - p0) x (p2 - p0) points from the
 * inside to the outside, and the mesh is closed wherever the inside set is.  Triangles are
 * written to tri [max_tris][3][3] (device, xyz per vertex) cell by cell (x fastest), then in
 * that order; *n_tris (device int64) receives the total, of which only the first max_tris are
 * written (call again with a larger buffer if it is larger).  ws must hold
 * tg_mesh_workspace_bytes(n). */
tg_status tg_mesh(const int32_t* n, const float* lo, const float* hi, const float* values,
                  float* tri, int64_t max_tris, int64_t* n_tris, void* ws, size_t ws_bytes,
                  void* stream);

/* Bytes of device workspace tg_chamfer needs for na and nb points (a bucket grid and a
 * bucketed copy of each set, and the reduction partials); 0 if a count is out of range. */
size_t tg_chamfer_workspace_bytes(int64_t na, int64_t nb);

/* Chamfer distance between point sets a [na][3] and b [nb][3] (device; na, nb >= 1), the CD
 * of Sec. 4.1 (the paper's "Chamfer-L1", computed there with PyTorch3D's code): out (device
 * double [3]) = {mean_a min_b |a - b| + mean_b min_a |a - b|, the first mean, the second
 * mean}, with |.| the L1 norm |dx| + |dy| + |dz| (norm = 1) or the Euclidean norm (norm = 2).
 * Exact nearest points: each set is bucketed on a grid of cubic cells over its bounding box,
 * and a point of the other set searches the rings of cells around its own until no unvisited
 * cell can hold a nearer point, which finds the minimum over every pair; distances in FP32,
 * means in FP64 (a direction's mean is the same whichever argument the set is).  ws must hold
 * tg_chamfer_workspace_bytes(na, nb); TG_ERR_CAPACITY if smaller. */
tg_status tg_chamfer(const float* a, int64_t na, const float* b, int64_t nb, int32_t norm, double* out,
                     void* ws, size_t ws_bytes, void* stream);

/* Radiance-field compositing (Sec. 3.3): the Max optical model of Eq. 10 along n_rays rays
 * of n_samples samples each, with a ReLU density, and the photometric loss of Eq. 11 with
 * its adjoint, in one launch.  Sample i of ray r is element r*n_samples + i of:
 *   f [N]      the density grid's value (N = n_rays * n_samples; tg_forward output),
 *   c [3][N]   the three colour channels (channel-major: the tg_forward output of a
 *              three-channel colour grid),
 *   delta [N]  the distance to the next sample along the ray (>= 0),
 * and per ray
 *   sigma_i = max(f_i, 0), T_i = exp(-sum_{j<i} sigma_j delta_j),
 *   C(r) = sum_i T_i (1 - exp(-sigma_i delta_i)) c_i.
 * rgb (may be NULL) [n_rays][3] receives C(r).  With loss != NULL (then target [n_rays][3],
 * g_f and g_c are required unless n_rays == 0):
 *   loss (device FP64) = (1/n_rays) sum_r |C(r) - target_r|^2 (0 for no rays),
 *   g_f [N] = dL/df_i (0 where f_i <= 0) and g_c [3][N] = dL/dc_i, the upstream gradients
 *   of the density grid's and the three-channel colour grid's adjoints (their g_f).
 * 1 <= n_samples <= 1024.  All arrays are device memory and must not overlap the outputs.
 * ws must hold tg_reduce_workspace_bytes(). */
tg_status tg_composite(int64_t n_rays, int32_t n_samples, const float* f, const float* c,
                       const float* delta, const float* target, float* rgb, double* loss,
                       float* g_f, float* g_c, void* ws, size_t ws_bytes, void* stream);

/* Adjoint of tg_forward (the exact transpose of the map C -> (f, grad f), which is linear
 * in the coefficients; the paper prints no formula).  For upstream gradients g_f [n] and
 * g_grad [n][dim] (either may be NULL = zero) it writes, for every vertex of the grid,
 *   grad[v][alpha] (=, or += with TG_BWD_ACCUMULATE) sum over queries of
 *     g_f w_b m_alpha(d_b) + sum_a g_grad_a (dw_b/dx_a m_alpha(d_b) + w_b dm_alpha/dd_a(d_b)),
 * with m_alpha(d) = d^alpha / alpha! the Taylor monomials of Eq. 1.  Vertices no query
 * touches are written 0 (or left unchanged when accumulating).  If dq != NULL it also
 * writes dq[i][a] = g_f df/dx_a + sum_c g_grad_c d2f/dx_a dx_c (0 on a clamped axis).
 * Requires the sort of (q, n) in ws; needs bufs.grad (and bufs.coeffs when dq != NULL).
 * With TG_BWD_PACKED in flags, g_f is [n][4] ((g_f, g_grad) of a query in one 16-byte row,
 * 16-byte aligned, required for n > 0) and g_grad must be NULL; a single-channel grid only.
 * The result does not depend on the order of the queries up to FP32 rounding of the sums. */
tg_status tg_backward(tg_grid* grid, const float* q, int64_t n, void* ws, size_t ws_bytes,
                      const float* g_f, const float* g_grad, float* dq, int32_t flags,
                      void* stream);

/* tg_forward and tg_sdf_loss in one pass, for training: the loss of Sec. 3.2 (Eq. 6 with
 * Eq. 7's weight, plus the eikonal term of Eq. 8) is evaluated where f and grad f are computed,
 * so they need not make a round trip through memory.  Writes g_f [n] and, when g_grad !=
 * NULL, g_grad [n][dim] exactly as tg_sdf_loss would from tg_forward's outputs, and loss[3]
 * (device FP64, as tg_sdf_loss; the sums are added in another order).  g_grad == NULL drops
 * the eikonal term.  f and grad_f (either may be NULL) receive tg_forward's outputs.
 * d [n] is the target SDF in query order.  Requires the sort of (q, n) in ws. */
tg_status tg_forward_sdf_loss(tg_grid* grid, const float* q, int64_t n, void* ws, size_t ws_bytes,
                              const float* d, float eik_weight, float surface_k, float* g_f,
                              float* g_grad, double* loss, float* f, float* grad_f, void* stream);

/* tg_backward followed by tg_adam_step in one pass, for training: every vertex brick's
 * coefficient adjoint (overwrite semantics) is handed straight to the Adam update of that
 * brick's master, moments and storage copy, so the gradient is never written (bufs.grad is
 * neither read nor written).  The update is tg_adam_step's, element for element.  If
 * grad_norm_sq != NULL (device double) it receives sum(dC^2) in FP64.  Requires the sort of
 * (q, n) in ws, bufs.master, bufs.adam_m, bufs.adam_v (and bufs.coeffs for 16-bit storage).
 * Must not overlap any other call that touches the same grid's buffers. */
tg_status tg_backward_adam(tg_grid* grid, const float* q, int64_t n, void* ws, size_t ws_bytes,
                           const float* g_f, const float* g_grad, const tg_adam_params* params,
                           double* grad_norm_sq, int32_t flags, void* stream);
/* flags: 0, or TG_BWD_ADD_GRAD, which adds bufs.grad (required then; read, not written) to
 * every coefficient's adjoint before its update, and counts it in grad_norm_sq: a gradient
 * computed beforehand, such as the TV term's from tg_tv_loss; TG_BWD_PACKED as for
 * tg_backward. */

/* One SDF-fitting step (Sec. 3.2: the grid is optimised directly against the objective of
 * Eq. 8) in one call: tg_sort_queries, then tg_forward_sdf_loss, then
 * tg_backward_adam, except that the upstream gradients are kept in the workspace in bucket
 * order, so they never make a round trip through memory in query order.  q [n][dim] and d [n]
 * as in those calls; loss (device FP64) as tg_sdf_loss, with the TV value added as below;
 * grad_norm_sq (device double, may be NULL) receives
 * sum(dC^2).  Afterwards ws holds the sort of (q, n), so tg_forward / tg_backward may reuse
 * it.  The same buffer requirements as tg_backward_adam; must not overlap any other call on
 * the same grid.  ws must hold tg_workspace_bytes(grid, n). */
tg_status tg_train_step(tg_grid* grid, const float* q, const float* d, int64_t n,
                        const tg_sdf_objective* obj, const tg_adam_params* params, double* loss,
                        double* grad_norm_sq, void* ws, size_t ws_bytes, void* const* stage_events,
                        void* stream);
/* obj: the objective's weights (host struct, required).  With obj->tv_weight != 0 the step
 * first runs tg_tv_loss on the current coefficients into bufs.grad (required then; its
 * contents are overwritten) and value loss[3], and the adjoint adds it before the update
 * (TG_BWD_ADD_GRAD); loss then holds 4 doubles and
 *   loss[0] = loss[1] + eik_weight loss[2] + tv_weight loss[3].
 * With tv_weight == 0, loss holds 3 doubles and bufs.grad is not touched. */
/* stage_events: NULL, or a host array of 3 hipEvent_t that are recorded on the stream after
 * the sort, after the forward with the loss terms (and the TV term) and after the adjoint
 * with Adam and the
 * final FP64 reductions of the loss and the gradient norm (for timing). */

/* tg_train_step without its sort: the workspace must already hold the sort of (q, n) for this
 * handle (tg_sort_queries, or tg_share_sort), else TG_ERR_STATE.  Arguments, buffers and
 * results are tg_train_step's; stage_events[0] is recorded when the step starts.  The
 * bucketing of a batch depends only on its queries (Sec. 3.1's cell location), not on the
 * coefficients a step updates, so a loop may sort a batch ahead of its step: into a second
 * workspace through a second handle on the same buffers, on another stream ordered by events. */
tg_status tg_train_step_sorted(tg_grid* grid, const float* q, const float* d, int64_t n,
                               const tg_sdf_objective* obj, const tg_adam_params* params, double* loss,
                               double* grad_norm_sq, void* ws, size_t ws_bytes, void* const* stage_events,
                               void* stream);

/* One Adam step over every coefficient.  The grid is optimised directly by gradient descent
 * with no network (Sec. 3.1); Sec. 4.1 trains it with a fixed learning rate and names no
 * optimizer.  This is Adam with bias correction, eps added to the corrected root, and weight
 * decay added to the gradient:
 *   g' = grad + wd*master; m = b1 m + (1-b1) g'; v = b2 v + (1-b2) g'^2;
 *   master -= lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps)
 * then, when storage != TG_F32, coeffs = round_to_nearest_even(master) (FP16 saturates to
 * +-65504).  If grad_norm_sq != NULL (device double) it receives sum(grad^2) in FP64.
 * TG_ADAM_ZERO_GRAD zeroes grad afterwards.  ws must hold tg_reduce_workspace_bytes(). */
tg_status tg_adam_step(tg_grid* grid, const tg_adam_params* params, double* grad_norm_sq,
                       void* ws, size_t ws_bytes, int32_t flags, void* stream);

/* Serving: field value (Sec. 3.1, Eq. 2-4) and unit normal, the normalised spatial gradient
 * of that field (the SDF's normal, Sec. 3.2), for a batch of requests against several
 * resident grids, in one launch per group of up to TG_QUERY_MAX_REQS requests referencing up
 * to TG_QUERY_MAX_GRIDS distinct grids (larger batches are split into several launches).
 * grids (host array of handles) and reqs (host array) are read during the call only; no
 * workspace or sort is needed.  The arithmetic per query is the same as tg_forward's, so a
 * request's result does not depend on which other requests share the launch. */
#define TG_QUERY_MAX_REQS 32
#define TG_QUERY_MAX_GRIDS 16
tg_status tg_query(const tg_grid* const* grids, int32_t n_grids, const tg_request* reqs,
                   int32_t n_reqs, void* stream);

/* Write the storage copy `coeffs` from `master` (16-bit storage): round to nearest even,
 * FP16 saturating at +-65504 -- the conversion tg_adam_step applies after every update, for a
 * master set outside the library (initial values, a checkpoint).  FP32 storage: nothing to
 * do (coeffs is master).  Needs bufs.master and bufs.coeffs for 16-bit storage. */
tg_status tg_sync_storage(tg_grid* grid, void* stream);

/* Static description of a status code; never NULL. */
const char* tg_status_string(tg_status status);

/* Thread-local description of the last failing call on this thread ("" if none). */
const char* tg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TAYLORGRID_H */
