/*
 * FP64 CPU oracle of the TaylorGrid query path (arXiv 2402.14415, Sec. 3.1, Eq. 1-4).
 *
 * TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the benchmark's
 * CPU-baseline leg to check the GPU path.  Nothing in the GPU library calls it.
 *
 * The query path computes, for each point (Sec. 3.1):
 *   Eq. 2  the Taylor voxel (cell) that contains the point;
 *   Eq. 3  for every corner v_i of that cell, the stored low-order Taylor polynomial
 *          T'(x - v_i; S(v_i)) of Eq. 1 evaluated at the point;
 *   Eq. 4  the trilinear (bilinear in 2D) interpolation of those corner values.
 * The spatial gradient and the adjoint are not printed in the paper; they are the exact
 * derivatives of that composite, written out below term by term.
 */
#include "taylorgrid_oracle.h"

#include <math.h>
#include <stdlib.h>

#define OG_MAX_COEFFS 35 /* binom(3 + 4, 4) */

static double factorial(int k)
{
    double r = 1.0;
    for (int i = 2; i <= k; ++i) r *= (double)i;
    return r;
}

int32_t og_num_coeffs(int32_t dim, int32_t order)
{
    int64_t num = 1, den = 1;
    for (int i = 1; i <= order; ++i) {
        num *= dim + i;
        den *= i;
    }
    return (int32_t)(num / den);
}

/* Multi-indices alpha with |alpha| <= order; degree by degree, and inside one degree in
 * descending lexicographic order of (alpha_x, alpha_y, alpha_z). */
int32_t og_exponents(int32_t dim, int32_t order, int32_t* exps)
{
    int n = 0;
    for (int k = 0; k <= order; ++k) {
        for (int a = k; a >= 0; --a) {
            if (dim == 2) {
                exps[3 * n + 0] = a;
                exps[3 * n + 1] = k - a;
                exps[3 * n + 2] = 0;
                ++n;
            } else {
                for (int b = k - a; b >= 0; --b) {
                    exps[3 * n + 0] = a;
                    exps[3 * n + 1] = b;
                    exps[3 * n + 2] = k - a - b;
                    ++n;
                }
            }
        }
    }
    return n;
}

/* Taylor monomial d^alpha / alpha! (Eq. 1).  A negative exponent stands for the
 * derivative of a monomial that does not depend on that axis, which is zero. */
static double monomial(const int32_t* alpha, const double* d, int dim)
{
    double r = 1.0;
    for (int a = 0; a < dim; ++a) {
        if (alpha[a] < 0) return 0.0;
        for (int p = 0; p < alpha[a]; ++p) r *= d[a];
        r /= factorial(alpha[a]);
    }
    return r;
}

/* d/dd_a of d^alpha/alpha! is d^(alpha - e_a)/(alpha - e_a)!; same rule twice for the
 * second derivative. */
static double monomial_d1(const int32_t* alpha, const double* d, int dim, int a)
{
    int32_t beta[3] = {alpha[0], alpha[1], alpha[2]};
    beta[a] -= 1;
    return monomial(beta, d, dim);
}

static double monomial_d2(const int32_t* alpha, const double* d, int dim, int a, int c)
{
    int32_t beta[3] = {alpha[0], alpha[1], alpha[2]};
    beta[a] -= 1;
    beta[c] -= 1;
    return monomial(beta, d, dim);
}

/* Eq. 2: the cell that contains the (clamped) point, and the point's local coordinate. */
typedef struct {
    int64_t cell[3];
    double t[3];
    double h[3];
    double x[3];
    int clamped[3];
} og_loc;

static void locate(const og_geom* g, const double* q, og_loc* L)
{
    for (int a = 0; a < g->dim; ++a) {
        double h = (g->hi[a] - g->lo[a]) / (double)(g->res[a] - 1);
        double x = q[a];
        L->clamped[a] = 0;
        if (x < g->lo[a]) { x = g->lo[a]; L->clamped[a] = 1; }
        if (x > g->hi[a]) { x = g->hi[a]; L->clamped[a] = 1; }
        double s = (x - g->lo[a]) / h;
        int64_t i = (int64_t)floor(s);
        if (i > g->res[a] - 2) i = g->res[a] - 2;
        if (i < 0) i = 0;
        L->cell[a] = i;
        L->t[a] = s - (double)i;
        L->h[a] = h;
        L->x[a] = x;
    }
}

/* One corner b of the located cell: its vertex index, the world-space offset d = x - v_b,
 * the interpolation weight w_b (Eq. 4) and the weight's first and second derivatives
 * with respect to x. */
typedef struct {
    int64_t vertex;
    double d[3];
    double w;
    double dw[3];
    double d2w[3][3];
} og_corner;

static void corner(const og_geom* g, const og_loc* L, int b, og_corner* K)
{
    const int dim = g->dim;
    double factor[3], dfactor[3];
    int64_t stride = 1;
    K->vertex = 0;
    for (int a = 0; a < dim; ++a) {
        int ba = (b >> a) & 1;
        int64_t vi = L->cell[a] + ba;
        K->vertex += vi * stride;
        stride *= g->res[a];
        double v = g->lo[a] + (double)vi * L->h[a];
        K->d[a] = L->x[a] - v;
        factor[a] = ba ? L->t[a] : 1.0 - L->t[a];
        dfactor[a] = (ba ? 1.0 : -1.0) / L->h[a];
    }
    K->w = 1.0;
    for (int a = 0; a < dim; ++a) K->w *= factor[a];
    for (int a = 0; a < dim; ++a) {
        K->dw[a] = dfactor[a];
        for (int c = 0; c < dim; ++c)
            if (c != a) K->dw[a] *= factor[c];
    }
    for (int a = 0; a < dim; ++a)
        for (int c = 0; c < dim; ++c) {
            if (a == c) {
                K->d2w[a][c] = 0.0; /* multilinear: no square terms */
                continue;
            }
            double r = dfactor[a] * dfactor[c];
            for (int e = 0; e < dim; ++e)
                if (e != a && e != c) r *= factor[e];
            K->d2w[a][c] = r;
        }
}

/* Value, gradient and Hessian of the TaylorGrid field at one query. */
static void eval_query(const og_geom* g, const double* coeffs, const int32_t* exps, int nc,
                       const double* q, double* f_out, double* grad_out, double* hess_out)
{
    const int dim = g->dim;
    og_loc L;
    locate(g, q, &L);
    double f = 0.0, grad[3] = {0, 0, 0}, hess[3][3] = {{0}};
    for (int b = 0; b < (1 << dim); ++b) {
        og_corner K;
        corner(g, &L, b, &K);
        const double* C = coeffs + K.vertex * nc;
        /* Eq. 1/3: T'(x - v_b; S(v_b)) and its derivatives in x. */
        double T = 0.0, dT[3] = {0, 0, 0}, d2T[3][3] = {{0}};
        for (int k = 0; k < nc; ++k) {
            const int32_t* alpha = exps + 3 * k;
            T += C[k] * monomial(alpha, K.d, dim);
            for (int a = 0; a < dim; ++a) {
                dT[a] += C[k] * monomial_d1(alpha, K.d, dim, a);
                for (int c = 0; c < dim; ++c) d2T[a][c] += C[k] * monomial_d2(alpha, K.d, dim, a, c);
            }
        }
        /* Eq. 4: interpolate the corner values (product rule for the derivatives). */
        f += K.w * T;
        for (int a = 0; a < dim; ++a) {
            grad[a] += K.dw[a] * T + K.w * dT[a];
            for (int c = 0; c < dim; ++c)
                hess[a][c] += K.d2w[a][c] * T + K.dw[a] * dT[c] + K.dw[c] * dT[a] + K.w * d2T[a][c];
        }
    }
    /* On a clamped axis the field does not move with the query. */
    for (int a = 0; a < dim; ++a)
        if (L.clamped[a]) {
            grad[a] = 0.0;
            for (int c = 0; c < dim; ++c) hess[a][c] = hess[c][a] = 0.0;
        }
    *f_out = f;
    if (grad_out)
        for (int a = 0; a < dim; ++a) grad_out[a] = grad[a];
    if (hess_out)
        for (int a = 0; a < dim; ++a)
            for (int c = 0; c < dim; ++c) hess_out[a * dim + c] = hess[a][c];
}

void og_forward(const og_geom* g, const double* coeffs, const double* q, int64_t n,
                double* f, double* grad, double* hess)
{
    int32_t exps[3 * OG_MAX_COEFFS];
    const int nc = og_exponents(g->dim, g->order, exps);
    const int dim = g->dim;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i)
        eval_query(g, coeffs, exps, nc, q + i * dim, f + i, grad ? grad + i * dim : NULL,
                   hess ? hess + i * dim * dim : NULL);
}

/* The field value and gradient are linear in the coefficients, so the adjoint of
 * (f, grad f) with respect to C is the transpose of that linear map:
 *   dC[v_b][alpha] += gf * w_b m_alpha(d_b)
 *                   + sum_a gg_a (dw_b/dx_a m_alpha(d_b) + w_b dm_alpha/dd_a(d_b)).
 * The adjoint with respect to the query is dq_a = gf df/dx_a + sum_c gg_c d2f/dx_a dx_c. */
void og_backward(const og_geom* g, const double* coeffs, const double* q, int64_t n,
                 const double* gf, const double* gg, double* dcoeffs, double* dq)
{
    int32_t exps[3 * OG_MAX_COEFFS];
    const int nc = og_exponents(g->dim, g->order, exps);
    const int dim = g->dim;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double* qi = q + i * dim;
        og_loc L;
        locate(g, qi, &L);
        double s_f = gf ? gf[i] : 0.0;
        double s_g[3] = {0, 0, 0};
        for (int a = 0; a < dim; ++a)
            s_g[a] = (gg && !L.clamped[a]) ? gg[i * dim + a] : 0.0;
        for (int b = 0; b < (1 << dim); ++b) {
            og_corner K;
            corner(g, &L, b, &K);
            double* dC = dcoeffs + K.vertex * nc;
            for (int k = 0; k < nc; ++k) {
                const int32_t* alpha = exps + 3 * k;
                double m = monomial(alpha, K.d, dim);
                double contrib = s_f * K.w * m;
                for (int a = 0; a < dim; ++a)
                    contrib += s_g[a] * (K.dw[a] * m + K.w * monomial_d1(alpha, K.d, dim, a));
#pragma omp atomic update
                dC[k] += contrib;
            }
        }
        if (dq) {
            double f, grad[3], hess[9];
            eval_query(g, coeffs, exps, nc, qi, &f, grad, hess);
            for (int a = 0; a < dim; ++a) {
                double r = 0.0;
                if (!L.clamped[a]) {
                    r = s_f * grad[a];
                    for (int c = 0; c < dim; ++c) r += s_g[c] * hess[a * dim + c];
                }
                dq[i * dim + a] = r;
            }
        }
    }
}

/* Sec. 3.2, Eq. 6 (unweighted; an L1 residual of the scalar SDF) plus the eikonal term of
 * Eq. 8 in its usual form mean (|grad f| - 1)^2. */
void og_sdf_loss(int32_t dim, int64_t n, const double* f, const double* grad, const double* d,
                 double w_eik, double* gf, double* gg, double* out)
{
    double recon = 0.0, eik = 0.0;
    const double inv_n = n > 0 ? 1.0 / (double)n : 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double r = f[i] - d[i];
        recon += fabs(r);
        gf[i] = (r > 0.0 ? 1.0 : (r < 0.0 ? -1.0 : 0.0)) * inv_n;
        if (grad) {
            double nrm2 = 0.0;
            for (int a = 0; a < dim; ++a) nrm2 += grad[i * dim + a] * grad[i * dim + a];
            double nrm = sqrt(nrm2);
            double e = nrm - 1.0;
            eik += e * e;
            for (int a = 0; a < dim; ++a)
                gg[i * dim + a] = nrm > 0.0 ? w_eik * 2.0 * e * grad[i * dim + a] / nrm * inv_n : 0.0;
        }
    }
    out[1] = recon * inv_n;
    out[2] = eik * inv_n;
    out[0] = out[1] + w_eik * out[2];
}

double og_adam(int64_t n, double* theta, double* m, double* v, const double* grad,
               double lr, double beta1, double beta2, double eps, double weight_decay,
               int64_t step)
{
    const double bc1 = 1.0 - pow(beta1, (double)step);
    const double bc2 = 1.0 - pow(beta2, (double)step);
    double sumsq = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double g = grad[i] + weight_decay * theta[i];
        m[i] = beta1 * m[i] + (1.0 - beta1) * g;
        v[i] = beta2 * v[i] + (1.0 - beta2) * g * g;
        double mhat = m[i] / bc1;
        double vhat = v[i] / bc2;
        theta[i] -= lr * mhat / (sqrt(vhat) + eps);
        sumsq += grad[i] * grad[i];
    }
    return sumsq;
}
