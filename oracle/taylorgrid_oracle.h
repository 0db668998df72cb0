/*
 * FP64 CPU oracle of the TaylorGrid query path (arXiv 2402.14415, Sec. 3.1, Eq. 1-4).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU path; only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.  It shares no
 * code, header, table or constant with the GPU library.
 *
 * Conventions (the readings of the paper that this oracle fixes):
 *  - A grid has res[a] vertices on axis a spanning the closed box [lo[a], hi[a]]; vertex
 *    i sits at lo + i*h with h = (hi - lo) / (res - 1).  Vertex (i0, i1, i2) has linear
 *    index i0 + res0*(i1 + res1*i2) (x fastest); its coefficient block is contiguous.
 *  - Coefficients per vertex: the partial derivatives d^alpha f(v) for every multi-index
 *    alpha with |alpha| <= order, in graded-lexicographic order (3D, order 2:
 *    1, x, y, z, xx, xy, xz, yy, yz, zz; 2D: 1, x, y, xx, xy, yy).
 *  - Offsets x - v are in world units; the Taylor polynomial is sum_alpha
 *    C_alpha * (x - v)^alpha / alpha!  (Eq. 1, which carries the 1/2! factor).
 *  - Queries outside the box are clamped to it; the spatial gradient is zero on a
 *    clamped axis (x does not move with q there).
 *  - The cell is floor((x - lo)/h), capped at res - 2 so a point on the high face uses
 *    the last cell with local coordinate 1.
 *
 * Every function is serial per query and written for clarity, not speed.
 */
#ifndef TAYLORGRID_ORACLE_H
#define TAYLORGRID_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    int32_t dim;      /* 2 or 3 */
    int32_t res[3];   /* vertices per axis, >= 2 (res[2] ignored when dim == 2) */
    int32_t order;    /* Taylor order K, 0..4 */
    double lo[3];
    double hi[3];
} og_geom;

/* Number of coefficients per vertex: binom(dim + order, order). */
int32_t og_num_coeffs(int32_t dim, int32_t order);

/* Writes the exponent table (num_coeffs rows of 3 ints) in graded-lex order. */
int32_t og_exponents(int32_t dim, int32_t order, int32_t* exps);

/* Forward: f[n] and, if grad != NULL, grad[n*dim] (value and spatial gradient).
 * If hess != NULL it also receives the spatial Hessian hess[n*dim*dim]. */
void og_forward(const og_geom* g, const double* coeffs, const double* q, int64_t n,
                double* f, double* grad, double* hess);

/* Adjoint: dcoeffs += d<gf,f> + <gg,grad f> / dcoeffs and, if dq != NULL,
 * dq = d(...)/dq.  gf may be NULL (treated as 0); gg may be NULL (treated as 0). */
void og_backward(const og_geom* g, const double* coeffs, const double* q, int64_t n,
                 const double* gf, const double* gg, double* dcoeffs, double* dq);

/* SDF objective: L = mean|f - d| + w_eik * mean(|grad f| - 1)^2.
 * out[0] = L, out[1] = mean|f-d|, out[2] = mean(|grad f|-1)^2.  Also writes the upstream
 * gradients gf = dL/df and gg = dL/d(grad f) (gg may be NULL when grad is NULL). */
void og_sdf_loss(int32_t dim, int64_t n, const double* f, const double* grad, const double* d,
                 double w_eik, double* gf, double* gg, double* out);

/* One Adam step (bias-corrected, eps added to the corrected root, L2 weight decay added
 * to the gradient) on n parameters, in place on theta, m and v.  Returns sum(g^2). */
double og_adam(int64_t n, double* theta, double* m, double* v, const double* grad,
               double lr, double beta1, double beta2, double eps, double weight_decay,
               int64_t step);

#ifdef __cplusplus
}
#endif
#endif
