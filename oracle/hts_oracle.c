/*
 * hts_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of what one iteration of hyperbolic
 * t-SNE computes, following "Accelerating hyperbolic t-SNE" (arXiv
 * 2401.13708).  Used only by the tests, the smoke check and the CPU-baseline
 * leg of the benchmark; the product path never loads it.  It shares no code
 * with the HIP library.
 *
 * Readings taken where the paper is silent or inconsistent are marked
 * "reading:" next to the code they affect.
 *
 * Build: gcc -O2 -ffp-contract=off -fopenmp -fPIC -shared (no fast-math).
 */
#include "hts_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

static int g_threads = 0;

void ora_set_threads(int32_t nthreads) { g_threads = nthreads; }

int32_t ora_get_threads(void) {
#ifdef _OPENMP
    return g_threads > 0 ? g_threads : omp_get_max_threads();
#else
    return 1;
#endif
}

#ifdef _OPENMP
#define NTH() (ora_get_threads())
#endif

/* ======================================================================
 * Geometry of the Poincare disk (Sec. 2-C, Sec. 4-B)
 * ====================================================================== */

/* acosh(1 + t) for t >= 0, written as log1p(t + sqrt(t (t + 2))): the same
 * function, but it keeps full relative accuracy when t is tiny (points near
 * the origin), where 1 + t would round to 1. */
static double acosh1p(double t) { return log1p(t + sqrt(t * (t + 2.0))); }

/* t = 2 |a - b|^2 / ((1 - |a|^2)(1 - |b|^2)), the argument of eq. (8) minus 1 */
static double dist_arg(double ax, double ay, double bx, double by) {
    double dx = ax - bx, dy = ay - by;
    double al = 1.0 - (ax * ax + ay * ay);
    double be = 1.0 - (bx * bx + by * by);
    return 2.0 * (dx * dx + dy * dy) / (al * be);
}

/* Poincare distance, eq. (8) (Sec. 2-C) */
double ora_dist(double ax, double ay, double bx, double by) {
    return acosh1p(dist_arg(ax, ay, bx, by));
}

/* Variation of the distance with respect to the first point, eq. (13)
 * (Sec. 4-B):
 *   4 ((|b|^2 - 2<a,b> + 1) a / alpha - b) / (alpha beta sqrt(gamma^2 - 1)).
 * Written with |b|^2 - 2<a,b> + 1 = |a-b|^2 + alpha and gamma^2 - 1 =
 * t (t + 2), which are identities, so the numerator becomes
 * (a - b) + (|a-b|^2 / alpha) a.  Coincident points give 0. */
void ora_dist_grad(double ax, double ay, double bx, double by, double *g) {
    double dx = ax - bx, dy = ay - by;
    double dd = dx * dx + dy * dy;
    double al = 1.0 - (ax * ax + ay * ay);
    double be = 1.0 - (bx * bx + by * by);
    double t = 2.0 * dd / (al * be);
    double sh = sqrt(t * (t + 2.0));
    if (sh == 0.0) { g[0] = g[1] = 0.0; return; }
    double c = 4.0 / (al * be * sh);
    g[0] = c * (dx + (dd / al) * ax);
    g[1] = c * (dy + (dd / al) * ay);
}

/* Mobius addition, eq. (17) (Sec. 4-B) */
void ora_mobius_add(double ax, double ay, double bx, double by, double *out) {
    double ab = ax * bx + ay * by;
    double a2 = ax * ax + ay * ay;
    double b2 = bx * bx + by * by;
    double num_a = 1.0 + 2.0 * ab + b2;
    double num_b = 1.0 - a2;
    double den = 1.0 + 2.0 * ab + a2 * b2;
    out[0] = (num_a * ax + num_b * bx) / den;
    out[1] = (num_a * ay + num_b * by) / den;
}

/* Exponential map at y, eq. (16):  y (+) tanh(lambda_y |v| / 2) v / |v|,
 * with lambda_y = 2 / (1 - |y|^2) from eq. (7).  exp_y(0) = y. */
void ora_exp_map(double yx, double yy, double vx, double vy, double *out) {
    double nv = sqrt(vx * vx + vy * vy);
    if (nv == 0.0) { out[0] = yx; out[1] = yy; return; }
    double lam = 2.0 / (1.0 - (yx * yx + yy * yy));
    double s = tanh(lam * nv / 2.0) / nv;
    ora_mobius_add(yx, yy, s * vx, s * vy, out);
}

/* Einstein midpoint, eq. (11) (Sec. 4-A): the points are mapped to the Klein
 * model, v = 2 y / (1 + |y|^2), averaged with weights gamma(v) =
 * 1 / sqrt(1 - |v|^2), and the average is mapped back to the Poincare disk,
 * y = v / (1 + sqrt(1 - |v|^2)).  For this v, gamma(v) v = lambda_y y and
 * gamma(v) = (1 + |y|^2) / (1 - |y|^2) exactly; the sums use these forms
 * because 1 - |v|^2 cancels to a few digits near the rim. */
void ora_einstein_midpoint(const double *Y, int64_t n, double *out) {
    double sx = 0.0, sy = 0.0, sg = 0.0;
    for (int64_t j = 0; j < n; ++j) {
        double x = Y[2 * j], y = Y[2 * j + 1];
        double r2 = x * x + y * y;
        double a = 1.0 - r2;
        sx += 2.0 * x / a;
        sy += 2.0 * y / a;
        sg += (1.0 + r2) / a;
    }
    double kx = sx / sg, ky = sy / sg;
    double den = 1.0 + sqrt(1.0 - (kx * kx + ky * ky));
    out[0] = kx / den;
    out[1] = ky / den;
}

/* ======================================================================
 * Input affinities P (Sec. 2-A, eq. (1); truncation as in Sec. 2-A/4-B)
 * ====================================================================== */

typedef struct { double d2; int32_t j; } cand_t;

static int cand_cmp(const void *pa, const void *pb) {
    const cand_t *a = (const cand_t *)pa, *b = (const cand_t *)pb;
    if (a->d2 < b->d2) return -1;
    if (a->d2 > b->d2) return 1;
    return (a->j > b->j) - (a->j < b->j);
}

/* Exact k nearest neighbours of selected rows.  reading: exact brute force;
 * squared distances summed in a fixed order (dimension ascending, each term
 * added with one fused multiply-add); ties broken by the smaller index; the
 * point itself excluded. */
int ora_knn_rows(const double *X, int64_t n, int32_t d, int32_t k,
                 const int64_t *rows, int64_t nrows,
                 int32_t *idx_out, double *d2_out) {
    if (n < 2 || d < 1 || k < 1 || k >= n) return -1;
    int err = 0;
#pragma omp parallel num_threads(NTH())
    {
        cand_t *c = (cand_t *)malloc(sizeof(cand_t) * (size_t)(n - 1));
        if (!c) {
#pragma omp atomic write
            err = -2;
        }
#pragma omp for schedule(dynamic, 4)
        for (int64_t r = 0; r < nrows; ++r) {
            if (!c) continue;
            int64_t i = rows ? rows[r] : r;
            const double *xi = X + i * d;
            int64_t m = 0;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                const double *xj = X + j * d;
                double s = 0.0;
                for (int32_t t = 0; t < d; ++t) {
                    double dl = xi[t] - xj[t];
                    s = fma(dl, dl, s);
                }
                c[m].d2 = s;
                c[m].j = (int32_t)j;
                ++m;
            }
            qsort(c, (size_t)m, sizeof(cand_t), cand_cmp);
            for (int32_t t = 0; t < k; ++t) {
                idx_out[r * k + t] = c[t].j;
                if (d2_out) d2_out[r * k + t] = c[t].d2;
            }
        }
        free(c);
    }
    return err;
}

/* Conditional probabilities p_{j|i} over the k neighbours of each row, with
 * the bandwidth chosen so that the perplexity equals the target (Sec. 2-A).
 * reading: the Gaussian of eq. (1) is exp(-|xi-xj|^2 / (2 sigma_i^2)) with
 * sigma_i a standard deviation; it is parametrised by beta = 1/(2 sigma^2).
 * The entropy uses the natural log with target ln(perplexity).  beta starts at
 * 1 and is found by bisection (doubling/halving until bracketed) for a fixed
 * 100 steps, so the result is converged to double precision. */
static void row_entropy_p(const double *d2, int32_t k, double beta, double *p,
                          double *H) {
    double dmin = d2[0];
    for (int32_t t = 1; t < k; ++t) if (d2[t] < dmin) dmin = d2[t];
    double s = 0.0, sd = 0.0;
    for (int32_t t = 0; t < k; ++t) {
        double D = d2[t] - dmin;
        double e = exp(-beta * D);
        p[t] = e;
        s += e;
        sd += D * e;
    }
    for (int32_t t = 0; t < k; ++t) p[t] /= s;
    /* H = -sum p ln p = ln s + beta sum p D */
    *H = log(s) + beta * sd / s;
}

int ora_cond_p(const double *d2, int64_t n, int32_t k, double perplexity,
               double *p_out, double *beta_out) {
    if (n < 1 || k < 1 || !(perplexity > 0.0) || perplexity >= k) return -1;
    double target = log(perplexity);
#pragma omp parallel for num_threads(NTH()) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        const double *di = d2 + i * k;
        double *pi = p_out + i * k;
        double beta = 1.0, lo = -INFINITY, hi = INFINITY, H;
        for (int it = 0; it < 100; ++it) {
            row_entropy_p(di, k, beta, pi, &H);
            if (H > target) {           /* too flat: sharpen */
                lo = beta;
                beta = isinf(hi) ? beta * 2.0 : 0.5 * (beta + hi);
            } else {
                hi = beta;
                beta = isinf(lo) ? beta * 0.5 : 0.5 * (beta + lo);
            }
        }
        row_entropy_p(di, k, beta, pi, &H);
        if (beta_out) beta_out[i] = beta;
    }
    return 0;
}

typedef struct { int64_t key; double v; } trip_t;

static int trip_cmp(const void *pa, const void *pb) {
    const trip_t *a = (const trip_t *)pa, *b = (const trip_t *)pb;
    return (a->key > b->key) - (a->key < b->key);
}

/* Symmetrisation p_ij = (p_{j|i} + p_{i|j}) / 2 of eq. (1).  reading: divided
 * by n as well, so that sum P = 1 as the cost of eq. (3) requires. */
int ora_symmetrize(const int32_t *knn, const double *pc, int64_t n, int32_t k,
                   int64_t *row_ptr, int32_t *col, double *val, int64_t cap_nnz,
                   int64_t *nnz_out) {
    int64_t m = 2 * n * (int64_t)k;
    trip_t *tr = (trip_t *)malloc(sizeof(trip_t) * (size_t)m);
    if (!tr) return -2;
    int64_t q = 0;
    for (int64_t i = 0; i < n; ++i)
        for (int32_t t = 0; t < k; ++t) {
            int64_t j = knn[i * k + t];
            double p = pc[i * k + t];
            tr[q].key = i * n + j; tr[q].v = p; ++q;
            tr[q].key = j * n + i; tr[q].v = p; ++q;
        }
    qsort(tr, (size_t)m, sizeof(trip_t), trip_cmp);
    int64_t nnz = 0;
    for (int64_t a = 0; a < m; ++a)
        if (a == 0 || tr[a].key != tr[a - 1].key) ++nnz;
    *nnz_out = nnz;
    if (nnz > cap_nnz) { free(tr); return -4; }
    for (int64_t i = 0; i <= n; ++i) row_ptr[i] = 0;
    int64_t e = -1;
    for (int64_t a = 0; a < m; ++a) {
        if (a == 0 || tr[a].key != tr[a - 1].key) {
            ++e;
            col[e] = (int32_t)(tr[a].key % n);
            val[e] = tr[a].v;
            row_ptr[tr[a].key / n + 1]++;
        } else {
            val[e] += tr[a].v;
        }
    }
    for (int64_t i = 0; i < n; ++i) row_ptr[i + 1] += row_ptr[i];
    for (int64_t a = 0; a < nnz; ++a) val[a] /= (2.0 * (double)n);
    free(tr);
    return 0;
}

int ora_build_affinities(const double *X, int64_t n, int32_t d, double perplexity,
                         int32_t k, int32_t *knn_out, int64_t *row_ptr,
                         int32_t *col, double *val, int64_t cap_nnz,
                         int64_t *nnz_out) {
    if (n < 2 || d < 1 || k < 1 || k >= n || !(perplexity > 0.0) ||
        perplexity >= k)
        return -1;
    double *d2 = (double *)malloc(sizeof(double) * (size_t)(n * k));
    double *pc = (double *)malloc(sizeof(double) * (size_t)(n * k));
    int32_t *kn = knn_out ? knn_out : (int32_t *)malloc(sizeof(int32_t) * (size_t)(n * k));
    int rc = -2;
    if (d2 && pc && kn) {
        rc = ora_knn_rows(X, n, d, k, NULL, n, kn, d2);
        if (rc == 0) rc = ora_cond_p(d2, n, k, perplexity, pc, NULL);
        if (rc == 0) rc = ora_symmetrize(kn, pc, n, k, row_ptr, col, val, cap_nnz, nnz_out);
    }
    free(d2);
    free(pc);
    if (!knn_out) free(kn);
    return rc;
}

/* ======================================================================
 * Cost and exact gradient (eqs. (3), (12)-(15), Sec. 4-B)
 * ====================================================================== */

/* w = (1 + d^2)^-1, the unnormalised hyperbolic Student-t kernel of eq. (12) */
static double kernel_w(double d) { return 1.0 / (1.0 + d * d); }

/* Z^H = sum over ordered pairs k != l of (1 + d_kl^2)^-1, eq. (12)/(15).
 * reading: the subscripts "ij" in the printed Z are the summation indices. */
static double z_all_pairs(const double *Y, int64_t n) {
    double *zi = (double *)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for num_threads(NTH()) schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j)
            if (j != i) s += kernel_w(ora_dist(Y[2 * i], Y[2 * i + 1], Y[2 * j], Y[2 * j + 1]));
        zi[i] = s;
    }
    double z = 0.0;
    for (int64_t i = 0; i < n; ++i) z += zi[i];
    free(zi);
    return z;
}

int ora_z_exact(const double *Y, int64_t n, double *z_out) {
    if (n < 2) return -1;
    *z_out = z_all_pairs(Y, n);
    return 0;
}

/* KL(P || Q^H) of eq. (3) with q from eq. (12); with exaggeration a the
 * objective is sum a p ln(a p) - sum a p ln w + ln Z, whose gradient is the
 * exaggerated gradient below (for a = 1 it is the KL divergence itself). */
int ora_kl_cost(const double *Y, int64_t n, const int64_t *row_ptr,
                const int32_t *col, const double *val, double exaggeration,
                double *cost_out) {
    if (n < 2) return -1;
    double z = z_all_pairs(Y, n);
    double c = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int64_t j = col[e];
            double p = exaggeration * val[e];
            if (p <= 0.0) continue;
            double w = kernel_w(ora_dist(Y[2 * i], Y[2 * i + 1], Y[2 * j], Y[2 * j + 1]));
            c += p * (log(p) - log(w));
        }
    *cost_out = c + log(z);
    return 0;
}

/* CO-SNE (Sec. 4-C): the cost lambda1 KL(P||Q) + (lambda2 / n) sum_i
 * (|x_i|^2 - |y_i|^2)^2, with xnorm2[i] = |x_i|^2 of the input point.
 * reading: the printed variation of the second part has the sign of
 * +(4 lambda2 / n)(|x_i|^2 - |y_i|^2) y_i; the derivative of the stated cost is
 * -(4 lambda2 / n)(|x_i|^2 - |y_i|^2) y_i, which is what is used (the finite
 * differences of the cost decide it). */
int ora_cosne_cost(const double *Y, int64_t n, const int64_t *row_ptr, const int32_t *col,
                   const double *val, const double *xnorm2, double lambda1, double lambda2,
                   double *cost_out) {
    if (n < 2 || !xnorm2) return -1;
    double kl = 0.0;
    int rc = ora_kl_cost(Y, n, row_ptr, col, val, 1.0, &kl);
    if (rc != 0) return rc;
    double h = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double y2 = Y[2 * i] * Y[2 * i] + Y[2 * i + 1] * Y[2 * i + 1];
        double e = xnorm2[i] - y2;
        h += e * e;
    }
    *cost_out = lambda1 * kl + lambda2 / (double)n * h;
    return 0;
}

/* gradient of ora_cosne_cost from the KL gradient g_kl (exact or
 * Barnes-Hut): g = lambda1 g_kl - (4 lambda2 / n)(|x_i|^2 - |y_i|^2) y_i */
int ora_cosne_gradient(const double *Y, int64_t n, const double *xnorm2, double lambda1,
                       double lambda2, const double *g_kl, double *g_out) {
    if (n < 1 || !xnorm2 || !g_kl || !g_out) return -1;
    for (int64_t i = 0; i < n; ++i) {
        double y2 = Y[2 * i] * Y[2 * i] + Y[2 * i + 1] * Y[2 * i + 1];
        double c = 4.0 * lambda2 / (double)n * (xnorm2[i] - y2);
        g_out[2 * i] = lambda1 * g_kl[2 * i] - c * Y[2 * i];
        g_out[2 * i + 1] = lambda1 * g_kl[2 * i + 1] - c * Y[2 * i + 1];
    }
    return 0;
}


/* One pair's term w^m d (d d_ij / d y_i), the common factor of both sums of
 * eq. (15).  reading: eq. (14) prints (1 + d^2)^-1 dd/dy; the derivative of
 * ln (1 + d^2)^-1 is -2 d (1 + d^2)^-1 dd/dy, so the factor d_ij is kept. */
static void pair_term(double ix, double iy, double jx, double jy, double *wd,
                      double *f) {
    double d = ora_dist(ix, iy, jx, jy);
    double g[2];
    ora_dist_grad(ix, iy, jx, jy, g);
    *wd = kernel_w(d);
    f[0] = d * g[0];
    f[1] = d * g[1];
}

/* attractive sum of eq. (15) for row i: sum_j p_ij w_ij d_ij dd_ij/dy_i */
static void attract_row(const double *Y, const int64_t *row_ptr,
                        const int32_t *col, const double *val, int64_t i,
                        double *fa) {
    fa[0] = fa[1] = 0.0;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        int64_t j = col[e];
        if (j == i) continue;
        double w, f[2];
        pair_term(Y[2 * i], Y[2 * i + 1], Y[2 * j], Y[2 * j + 1], &w, f);
        fa[0] += val[e] * w * f[0];
        fa[1] += val[e] * w * f[1];
    }
}

/* Exact gradient, eqs. (14)-(15) with the factor d restored:
 *   g_i = 4 sum_{j != i} (a p_ij - w_ij / Z) w_ij d_ij dd_ij/dy_i.
 * Returned as the Euclidean variation (no metric rescaling). */
int ora_gradient_exact(const double *Y, int64_t n, const int64_t *row_ptr,
                       const int32_t *col, const double *val,
                       double exaggeration, double *grad, double *z_out) {
    if (n < 2) return -1;
    double *zi = (double *)malloc(sizeof(double) * (size_t)n);
    double *fr = (double *)malloc(sizeof(double) * (size_t)(2 * n));
    if (!zi || !fr) { free(zi); free(fr); return -2; }
#pragma omp parallel for num_threads(NTH()) schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double rx = 0.0, ry = 0.0, s = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double w, f[2];
            pair_term(Y[2 * i], Y[2 * i + 1], Y[2 * j], Y[2 * j + 1], &w, f);
            rx += w * w * f[0];
            ry += w * w * f[1];
            s += w;
        }
        fr[2 * i] = rx;
        fr[2 * i + 1] = ry;
        zi[i] = s;
    }
    double z = 0.0;
    for (int64_t i = 0; i < n; ++i) z += zi[i];
#pragma omp parallel for num_threads(NTH()) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double fa[2];
        attract_row(Y, row_ptr, col, val, i, fa);
        grad[2 * i] = 4.0 * (exaggeration * fa[0] - fr[2 * i] / z);
        grad[2 * i + 1] = 4.0 * (exaggeration * fa[1] - fr[2 * i + 1] / z);
    }
    if (z_out) *z_out = z;
    free(zi);
    free(fr);
    return 0;
}

int ora_gradient_exact_rows(const double *Y, int64_t n, const int64_t *row_ptr,
                            const int32_t *col, const double *val,
                            double exaggeration, const int64_t *rows,
                            int64_t nrows, double z, double *grad_rows) {
    if (n < 2 || !(z > 0.0)) return -1;
#pragma omp parallel for num_threads(NTH()) schedule(dynamic, 1)
    for (int64_t r = 0; r < nrows; ++r) {
        int64_t i = rows[r];
        double rx = 0.0, ry = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double w, f[2];
            pair_term(Y[2 * i], Y[2 * i + 1], Y[2 * j], Y[2 * j + 1], &w, f);
            rx += w * w * f[0];
            ry += w * w * f[1];
        }
        double fa[2];
        attract_row(Y, row_ptr, col, val, i, fa);
        grad_rows[2 * r] = 4.0 * (exaggeration * fa[0] - rx / z);
        grad_rows[2 * r + 1] = 4.0 * (exaggeration * fa[1] - ry / z);
    }
    return 0;
}

/* ======================================================================
 * Polar quadtree with the equal-embedding-length radial split (Sec. 4-A)
 * ====================================================================== */

typedef struct {
    double r_lo, r_hi, p_lo, p_hi; /* polar quadrilateral [r_lo,r_hi] x [p_lo,p_hi) */
    double a_lo[2], a_hi[2];       /* directions of its two angular bounds (the split rays) */
    int32_t depth;
    int32_t child[4];              /* -1: empty sub-cell (no node) */
    int32_t count;                 /* points in the subtree */
    int32_t is_leaf;
    int32_t npts, cap;             /* leaf payload */
    int64_t *pts;
} onode;

struct ora_tree {
    int64_t n;
    int32_t max_depth;
    int32_t split_rule; /* 0: equal radial lengths, eq. (10); 1: equal areas, eq. (9) */
    double *px, *py;   /* point coordinates (full precision) */
    double *r;         /* radius of the FP32-rounded coordinates */
    double *xs, *ys;   /* the FP32-rounded coordinates */
    onode *nodes;
    int64_t nn, capn;
    /* pre-order export, filled after the build */
    int64_t *pre;      /* node ids in pre-order */
    int32_t *pre_first, *pre_next;
    int64_t *perm;     /* points in leaf order */
    double *mid;       /* Einstein midpoints, pre-order */
    double *rcell;     /* cell diameters, pre-order */
    double *ecent;     /* Euclidean centres of mass, pre-order (h-SNE term) */
    double *ediam;     /* Euclidean cell diameters, pre-order (h-SNE term) */
};

/* reading: the radius and the angular position are taken from the
 * coordinates rounded to single precision, so that the tree depends only on
 * the stored single-precision embedding; r = sqrt(x^2 + y^2) in double (the
 * products are exact, the sum and the root rounded once each). */
static void polar_of(double x, double y, double *r, double *xs, double *ys) {
    *xs = (double)(float)x;
    *ys = (double)(float)y;
    *r = sqrt(*xs * *xs + *ys * *ys);
}

/* The angular split of Sec. 2-D halves a cell's angular range at
 * mid_phi = (max_phi + min_phi) / 2.  reading: the half is decided without
 * computing the angle of the point (an angle from atan2 differs in its last
 * bit between math libraries): the split ray of a cell is a direction
 * vector built from those of its bounds -- the negative x-axis for the root
 * (the ray at pi), the bound min_phi turned by a right angle at depth 1
 * (widths pi), and below that the normalised sum of the two bound
 * directions, each operation rounded on its own in double -- and a point
 * (x, y) lies in the upper half iff c y - s x >= 0 with (c, s) that
 * direction rounded to single precision.  With single-precision coordinates
 * both products are exact in double and the one rounding of the difference
 * keeps its sign, so the decision is exact; points on the ray go to the upper
 * half, as phi >= mid_phi sends them.  The root: phi >= pi iff y < 0, or
 * y = 0 and x < 0 (the origin takes the lower half there and the upper half
 * below, where it lies on every ray). */
static void ang_mid(int32_t depth, const double *lo, const double *hi, double *mid) {
    if (depth == 0) {
        mid[0] = -1.0;
        mid[1] = 0.0;
        return;
    }
    if (depth == 1) {
        mid[0] = -lo[1];
        mid[1] = lo[0];
        return;
    }
    double sx = lo[0] + hi[0], sy = lo[1] + hi[1];
    double h = sqrt(sx * sx + sy * sy);
    mid[0] = sx / h;
    mid[1] = sy / h;
}

static int ang_bit(int32_t depth, const double *mid, double xs, double ys) {
    if (depth == 0) return ys < 0.0 || (ys == 0.0 && xs < 0.0);
    double c = (double)(float)mid[0], s = (double)(float)mid[1];
    return c * ys - s * xs >= 0.0;
}

static int32_t new_node(ora_tree *t, double rlo, double rhi, double plo,
                        double phi, const double *alo, const double *ahi, int32_t depth) {
    if (t->nn == t->capn) {
        int64_t nc = t->capn ? 2 * t->capn : 64;
        onode *nb = (onode *)realloc(t->nodes, sizeof(onode) * (size_t)nc);
        if (!nb) return -1;
        t->nodes = nb;
        t->capn = nc;
    }
    onode *o = &t->nodes[t->nn];
    memset(o, 0, sizeof(*o));
    o->r_lo = rlo; o->r_hi = rhi; o->p_lo = plo; o->p_hi = phi;
    o->a_lo[0] = alo[0]; o->a_lo[1] = alo[1];
    o->a_hi[0] = ahi[0]; o->a_hi[1] = ahi[1];
    o->depth = depth;
    o->child[0] = o->child[1] = o->child[2] = o->child[3] = -1;
    o->is_leaf = 1;
    return (int32_t)t->nn++;
}

/* Radial split point of a cell with embedding radii [lo, hi].
 * rule 0, eq. (10): the mean of the two radii (equal lengths in the disk).
 * rule 1, eq. (9): the hyperbolic radius rho = 2 artanh(r) whose cosh is the
 * mean of cosh(rho_lo) and cosh(rho_hi), so that both halves of the annulus
 * have the same hyperbolic area (2 pi (cosh rho - 1) inside radius rho).
 * Written in the embedding radius with cosh(rho) = 1 + 2u, u = r^2/(1-r^2):
 * the mean of the cosh values is 1 + (u_lo + u_hi), and r^2 = u/(1+u) gives
 * mid^2 = s / (2 + s) with s = u_lo + u_hi (the same number as the cosh and
 * acosh form, without their cancellation near r = 0). */
double ora_radial_mid(double lo, double hi, int32_t rule) {
    if (rule == 0) return (lo + hi) * 0.5;
    double ulo = lo * lo / (1.0 - lo * lo);
    double uhi = hi * hi / (1.0 - hi * hi);
    double sum = ulo + uhi;
    return sqrt(sum / (2.0 + sum));
}

/* Split of a cell into four (Sec. 4-A): the angular range is halved at its
 * split ray (ang_mid, ang_bit), and the radial range at ora_radial_mid.
 * Children are numbered 2 * [r >= mid_r] + [upper angular half]. */
static int digit_of(const ora_tree *t, const onode *o, int64_t p) {
    double mr = ora_radial_mid(o->r_lo, o->r_hi, t->split_rule);
    double am[2];
    ang_mid(o->depth, o->a_lo, o->a_hi, am);
    return 2 * (t->r[p] >= mr) + ang_bit(o->depth, am, t->xs[p], t->ys[p]);
}

static int32_t child_of(ora_tree *t, int32_t nid, int64_t p) {
    onode *o = &t->nodes[nid];
    int dg = digit_of(t, o, p);
    if (o->child[dg] >= 0) return o->child[dg];
    double mr = ora_radial_mid(o->r_lo, o->r_hi, t->split_rule);
    double mp = (o->p_lo + o->p_hi) * 0.5;
    double am[2], alo[2], ahi[2];
    ang_mid(o->depth, o->a_lo, o->a_hi, am);
    double rlo = (dg & 2) ? mr : o->r_lo, rhi = (dg & 2) ? o->r_hi : mr;
    double plo = (dg & 1) ? mp : o->p_lo, phi = (dg & 1) ? o->p_hi : mp;
    for (int c = 0; c < 2; ++c) {
        alo[c] = (dg & 1) ? am[c] : o->a_lo[c];
        ahi[c] = (dg & 1) ? o->a_hi[c] : am[c];
    }
    int32_t depth = o->depth + 1;
    int32_t c = new_node(t, rlo, rhi, plo, phi, alo, ahi, depth);
    if (c < 0) return -1;
    t->nodes[nid].child[dg] = c; /* re-fetch: new_node may have moved the array */
    return c;
}

static int leaf_push(onode *o, int64_t p) {
    if (o->npts == o->cap) {
        int32_t nc = o->cap ? 2 * o->cap : 1;
        int64_t *nb = (int64_t *)realloc(o->pts, sizeof(int64_t) * (size_t)nc);
        if (!nb) return -1;
        o->pts = nb;
        o->cap = nc;
    }
    o->pts[o->npts++] = p;
    return 0;
}

/* Insertion of one point (Sec. 2-D: O(log n) insertion; Sec. 4-A: a leaf
 * stores a single point).  reading: a leaf that receives a second point is
 * split and both points move down; at the maximum depth a leaf keeps every
 * point that reaches it (identical positions cannot be separated). */
static int insert_point(ora_tree *t, int32_t nid, int64_t p, int count_here) {
    for (;;) {
        if (count_here) t->nodes[nid].count++;
        count_here = 1;
        onode *o = &t->nodes[nid];
        if (o->is_leaf) {
            if (o->npts == 0 || o->depth == t->max_depth) return leaf_push(o, p);
            int64_t q = o->pts[0];
            o->npts = 0;
            o->is_leaf = 0;
            int32_t cq = child_of(t, nid, q);
            if (cq < 0) return -1;
            if (insert_point(t, cq, q, 1) < 0) return -1;
        }
        int32_t c = child_of(t, nid, p);
        if (c < 0) return -1;
        nid = c;
    }
}

static ora_tree *tree_alloc(const double *Y, int64_t n, int32_t max_depth, int32_t rule) {
    ora_tree *t = (ora_tree *)calloc(1, sizeof(ora_tree));
    if (!t) return NULL;
    t->n = n;
    t->max_depth = max_depth;
    t->split_rule = rule;
    t->px = (double *)malloc(sizeof(double) * (size_t)n);
    t->py = (double *)malloc(sizeof(double) * (size_t)n);
    t->r = (double *)malloc(sizeof(double) * (size_t)n);
    t->xs = (double *)malloc(sizeof(double) * (size_t)n);
    t->ys = (double *)malloc(sizeof(double) * (size_t)n);
    if (!t->px || !t->py || !t->r || !t->xs || !t->ys) { ora_tree_free(t); return NULL; }
    for (int64_t i = 0; i < n; ++i) {
        t->px[i] = Y[2 * i];
        t->py[i] = Y[2 * i + 1];
        polar_of(t->px[i], t->py[i], &t->r[i], &t->xs[i], &t->ys[i]);
    }
    return t;
}

/* reading: the root is the annulus [min_i r_i, max_i r_i] x [0, 2 pi) over
 * the current points (Sec. 4-A), rebuilt for every embedding. */
static int32_t make_root(ora_tree *t) {
    double rmin = INFINITY, rmax = -INFINITY;
    for (int64_t i = 0; i < t->n; ++i) {
        if (t->r[i] < rmin) rmin = t->r[i];
        if (t->r[i] > rmax) rmax = t->r[i];
    }
    const double east[2] = {1.0, 0.0};  /* both bounds of the root: angle 0 = 2 pi */
    return new_node(t, rmin, rmax, 0.0, 2.0 * M_PI, east, east, 0);
}

/* Hyperbolic diameter of a polar quadrilateral (Sec. 4-A).  The largest
 * distance inside the cell is between two of its corners: the diagonal, the
 * outer arc's end points or a radial edge (the paper checks the diagonal, one
 * radial and one polar edge).  reading: when the angular width is pi or more
 * (root and first level) the far corner is taken pi away from the first one,
 * which gives the antipodal pair 4 artanh(r_hi) on the outer circle. */
static double cell_diameter(const onode *o) {
    double dphi = o->p_hi - o->p_lo;
    if (dphi >= M_PI) dphi = M_PI;
    double rr[2] = {o->r_lo, o->r_hi};
    double pp[2] = {o->p_lo, o->p_lo + dphi};
    double cx[4], cy[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            cx[2 * a + b] = rr[a] * cos(pp[b]);
            cy[2 * a + b] = rr[a] * sin(pp[b]);
        }
    double best = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b) {
            double dd = ora_dist(cx[a], cy[a], cx[b], cy[b]);
            if (dd > best) best = dd;
        }
    return best;
}

/* Euclidean diameter of a cell: the largest Euclidean distance between two
 * of its corners, with the same reading for angular widths of pi or more as
 * the hyperbolic diameter above (the far corner pi away from the first). */
static double cell_diameter_euclid(const onode *o) {
    double dphi = o->p_hi - o->p_lo;
    if (dphi >= M_PI) dphi = M_PI;
    double rr[2] = {o->r_lo, o->r_hi};
    double pp[2] = {o->p_lo, o->p_lo + dphi};
    double cx[4], cy[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            cx[2 * a + b] = rr[a] * cos(pp[b]);
            cy[2 * a + b] = rr[a] * sin(pp[b]);
        }
    double best = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b) {
            double dx = cx[a] - cx[b], dy = cy[a] - cy[b];
            double dd = sqrt(dx * dx + dy * dy);
            if (dd > best) best = dd;
        }
    return best;
}

static int64_t g_pre_pos;
static int64_t g_perm_pos;

static void preorder(ora_tree *t, int32_t nid) {
    int64_t me = g_pre_pos++;
    t->pre[me] = nid;
    t->pre_first[me] = (int32_t)g_perm_pos;
    onode *o = &t->nodes[nid];
    if (o->is_leaf) {
        for (int32_t a = 0; a < o->npts; ++a) t->perm[g_perm_pos++] = o->pts[a];
    } else {
        for (int c = 0; c < 4; ++c)
            if (o->child[c] >= 0) preorder(t, o->child[c]);
    }
    t->pre_next[me] = (int32_t)g_pre_pos;
}

/* pre-order layout, Einstein midpoints (eq. (11)) from each cell's own
 * points, and cell diameters */
static int finish_tree(ora_tree *t) {
    int64_t m = t->nn;
    t->pre = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    t->pre_first = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    t->pre_next = (int32_t *)malloc(sizeof(int32_t) * (size_t)m);
    t->perm = (int64_t *)malloc(sizeof(int64_t) * (size_t)t->n);
    t->mid = (double *)malloc(sizeof(double) * (size_t)(2 * m));
    t->rcell = (double *)malloc(sizeof(double) * (size_t)m);
    t->ecent = (double *)malloc(sizeof(double) * (size_t)(2 * m));
    t->ediam = (double *)malloc(sizeof(double) * (size_t)m);
    if (!t->pre || !t->pre_first || !t->pre_next || !t->perm || !t->mid || !t->rcell ||
        !t->ecent || !t->ediam)
        return -2;
    g_pre_pos = 0;
    g_perm_pos = 0;
    preorder(t, 0);
    double *buf = (double *)malloc(sizeof(double) * (size_t)(2 * t->n));
    if (!buf) return -2;
    for (int64_t k = 0; k < m; ++k) {
        const onode *o = &t->nodes[t->pre[k]];
        int64_t f = t->pre_first[k];
        for (int32_t a = 0; a < o->count; ++a) {
            int64_t p = t->perm[f + a];
            buf[2 * a] = t->px[p];
            buf[2 * a + 1] = t->py[p];
        }
        ora_einstein_midpoint(buf, o->count, &t->mid[2 * k]);
        t->rcell[k] = cell_diameter(o);
        /* centre of mass of the cell's points in the disk coordinates */
        double sx = 0.0, sy = 0.0;
        for (int32_t a = 0; a < o->count; ++a) {
            sx += buf[2 * a];
            sy += buf[2 * a + 1];
        }
        t->ecent[2 * k] = sx / (double)o->count;
        t->ecent[2 * k + 1] = sy / (double)o->count;
        t->ediam[k] = cell_diameter_euclid(o);
    }
    free(buf);
    return 0;
}

int ora_tree_build(const double *Y, int64_t n, int32_t max_depth,
                   ora_tree **out) {
    return ora_tree_build_rule(Y, n, max_depth, 0, out);
}

int ora_tree_build_rule(const double *Y, int64_t n, int32_t max_depth,
                        int32_t split_rule, ora_tree **out) {
    if (n < 2 || max_depth < 1 || max_depth > 30) return -1;
    if (split_rule != 0 && split_rule != 1) return -1;
    ora_tree *t = tree_alloc(Y, n, max_depth, split_rule);
    if (!t) return -2;
    if (make_root(t) < 0) { ora_tree_free(t); return -2; }
    for (int64_t p = 0; p < n; ++p)
        if (insert_point(t, 0, p, 1) < 0) { ora_tree_free(t); return -2; }
    if (finish_tree(t) < 0) { ora_tree_free(t); return -2; }
    *out = t;
    return 0;
}

/* second, independent construction: recursive partition of the point set */
static int partition(ora_tree *t, int32_t nid, int64_t *idx, int64_t cnt,
                     int64_t *tmp) {
    onode *o = &t->nodes[nid];
    o->count = (int32_t)cnt;
    if (cnt == 1 || o->depth == t->max_depth) {
        for (int64_t a = 0; a < cnt; ++a)
            if (leaf_push(&t->nodes[nid], idx[a]) < 0) return -1;
        return 0;
    }
    o->is_leaf = 0;
    int64_t start[5] = {0, 0, 0, 0, 0};
    for (int64_t a = 0; a < cnt; ++a)
        start[digit_of(t, &t->nodes[nid], idx[a]) + 1]++;
    for (int c = 0; c < 4; ++c) start[c + 1] += start[c];
    int64_t fill[4] = {start[0], start[1], start[2], start[3]};
    for (int64_t a = 0; a < cnt; ++a) {
        int dg = digit_of(t, &t->nodes[nid], idx[a]);
        tmp[fill[dg]++] = idx[a];
    }
    memcpy(idx, tmp, sizeof(int64_t) * (size_t)cnt);
    for (int c = 0; c < 4; ++c) {
        int64_t m = start[c + 1] - start[c];
        if (m == 0) continue;
        int32_t ch = child_of(t, nid, idx[start[c]]);
        if (ch < 0) return -1;
        if (partition(t, ch, idx + start[c], m, tmp) < 0) return -1;
    }
    return 0;
}

int ora_tree_build_partition(const double *Y, int64_t n, int32_t max_depth,
                             ora_tree **out) {
    return ora_tree_build_partition_rule(Y, n, max_depth, 0, out);
}

int ora_tree_build_partition_rule(const double *Y, int64_t n, int32_t max_depth,
                                  int32_t split_rule, ora_tree **out) {
    if (n < 2 || max_depth < 1 || max_depth > 30) return -1;
    if (split_rule != 0 && split_rule != 1) return -1;
    ora_tree *t = tree_alloc(Y, n, max_depth, split_rule);
    if (!t) return -2;
    int64_t *idx = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *tmp = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int rc = (idx && tmp && make_root(t) >= 0) ? 0 : -2;
    if (rc == 0) {
        for (int64_t p = 0; p < n; ++p) idx[p] = p;
        rc = partition(t, 0, idx, n, tmp) < 0 ? -2 : 0;
    }
    free(idx);
    free(tmp);
    if (rc == 0) rc = finish_tree(t);
    if (rc != 0) { ora_tree_free(t); return rc; }
    *out = t;
    return 0;
}

void ora_tree_free(ora_tree *t) {
    if (!t) return;
    for (int64_t k = 0; k < t->nn; ++k) free(t->nodes[k].pts);
    free(t->nodes);
    free(t->px); free(t->py); free(t->r); free(t->xs); free(t->ys);
    free(t->pre); free(t->pre_first); free(t->pre_next);
    free(t->perm); free(t->mid); free(t->rcell);
    free(t->ecent); free(t->ediam);
    free(t);
}

int64_t ora_tree_num_nodes(const ora_tree *t) { return t->nn; }

int ora_tree_export(const ora_tree *t, int32_t *count, int32_t *depth,
                    int32_t *first, int32_t *next, double *mid, double *r_cell,
                    double *bounds, int64_t *perm) {
    for (int64_t k = 0; k < t->nn; ++k) {
        const onode *o = &t->nodes[t->pre[k]];
        if (count) count[k] = o->count;
        if (depth) depth[k] = o->depth;
        if (first) first[k] = t->pre_first[k];
        if (next) next[k] = t->pre_next[k];
        if (mid) { mid[2 * k] = t->mid[2 * k]; mid[2 * k + 1] = t->mid[2 * k + 1]; }
        if (r_cell) r_cell[k] = t->rcell[k];
        if (bounds) {
            bounds[4 * k] = o->r_lo; bounds[4 * k + 1] = o->r_hi;
            bounds[4 * k + 2] = o->p_lo; bounds[4 * k + 3] = o->p_hi;
        }
    }
    if (perm) memcpy(perm, t->perm, sizeof(int64_t) * (size_t)t->n);
    return 0;
}

/* ======================================================================
 * Barnes-Hut repulsion over the polar quadtree (eq. (19), Sec. 4-B)
 * ====================================================================== */

typedef struct {
    const ora_tree *t;
    const int64_t *pos_of_node; /* node id -> pre-order position */
    double theta;
    int64_t i;
    double yx, yy;
    double fx, fy, z;
    int64_t tests, accepts, pairs;
    int64_t covered; /* points stood for: N_cell per accepted cell, 1 per leaf pair */
} bh_state;

/* Depth-first traversal (Sec. 4-B): at an internal node the condition
 * r_cell / d^H(y_i, y_cell) < theta decides whether the whole cell is replaced
 * by N_cell copies of its Einstein midpoint (eq. (19)); otherwise the
 * children are visited.  Leaves are evaluated point by point.
 * reading: the traversal also accumulates the normaliser Z from the same
 * terms (N_cell w for an accepted cell, w for a leaf point); the test is
 * strict, so theta = 0 never approximates; the query itself is skipped. */
static void bh_visit(bh_state *s, int32_t nid) {
    const onode *o = &s->t->nodes[nid];
    if (o->is_leaf) {
        for (int32_t a = 0; a < o->npts; ++a) {
            int64_t j = o->pts[a];
            if (j == s->i) continue;
            double w, f[2];
            pair_term(s->yx, s->yy, s->t->px[j], s->t->py[j], &w, f);
            s->fx += w * w * f[0];
            s->fy += w * w * f[1];
            s->z += w;
            s->pairs++;
            s->covered++;
        }
        return;
    }
    int64_t k = s->pos_of_node[nid];
    const double *m = &s->t->mid[2 * k];
    double rc = s->t->rcell[k];
    double d = ora_dist(s->yx, s->yy, m[0], m[1]);
    s->tests++;
    if (rc / d < s->theta) {
        double w, f[2];
        pair_term(s->yx, s->yy, m[0], m[1], &w, f);
        double nc = (double)o->count;
        s->fx += nc * w * w * f[0];
        s->fy += nc * w * w * f[1];
        s->z += nc * w;
        s->accepts++;
        s->covered += o->count;
        return;
    }
    for (int c = 0; c < 4; ++c)
        if (o->child[c] >= 0) bh_visit(s, o->child[c]);
}

/* Barnes-Hut gradient rows for a subset of the queries, with Z given (the
 * sum over all queries, which the subset cannot form): the same traversal
 * per query as ora_gradient_bh.  counters as there, summed over the subset. */
int ora_gradient_bh_rows(const double *Y, int64_t n, const int64_t *row_ptr,
                         const int32_t *col, const double *val, double exaggeration,
                         const ora_tree *t, double theta, const int64_t *rows,
                         int64_t nrows, double z, double *grad_rows, int64_t *counters) {
    if (n < 2 || !t || t->n != n || !(theta >= 0.0) || isinf(theta) || !(z > 0.0)) return -1;
    int64_t m = t->nn;
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    int64_t *cnt = (int64_t *)calloc((size_t)(4 * (nrows > 0 ? nrows : 1)), sizeof(int64_t));
    if (!pos || !cnt) { free(pos); free(cnt); return -2; }
    for (int64_t k = 0; k < m; ++k) pos[t->pre[k]] = k;
    for (int64_t r = 0; r < nrows; ++r)
        if (rows[r] < 0 || rows[r] >= n) { free(pos); free(cnt); return -1; }
#pragma omp parallel for num_threads(NTH()) schedule(dynamic, 16)
    for (int64_t r = 0; r < nrows; ++r) {
        const int64_t i = rows[r];
        bh_state s;
        memset(&s, 0, sizeof(s));
        s.t = t;
        s.pos_of_node = pos;
        s.theta = theta;
        s.i = i;
        s.yx = Y[2 * i];
        s.yy = Y[2 * i + 1];
        bh_visit(&s, 0);
        double fa[2];
        attract_row(Y, row_ptr, col, val, i, fa);
        grad_rows[2 * r] = 4.0 * (exaggeration * fa[0] - s.fx / z);
        grad_rows[2 * r + 1] = 4.0 * (exaggeration * fa[1] - s.fy / z);
        cnt[4 * r] = s.tests;
        cnt[4 * r + 1] = s.accepts;
        cnt[4 * r + 2] = s.pairs;
        cnt[4 * r + 3] = s.covered;
    }
    if (counters) {
        counters[0] = counters[1] = counters[2] = counters[3] = 0;
        for (int64_t r = 0; r < nrows; ++r)
            for (int a = 0; a < 4; ++a) counters[a] += cnt[4 * r + a];
    }
    free(pos);
    free(cnt);
    return 0;
}

int ora_gradient_bh(const double *Y, int64_t n, const int64_t *row_ptr,
                    const int32_t *col, const double *val, double exaggeration,
                    const ora_tree *t, double theta, double *grad,
                    double *z_out, int64_t *counters) {
    if (n < 2 || !t || t->n != n || !(theta >= 0.0) || isinf(theta)) return -1;
    int64_t m = t->nn;
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    double *fr = (double *)malloc(sizeof(double) * (size_t)(2 * n));
    double *zi = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t *cnt = (int64_t *)calloc((size_t)(4 * n), sizeof(int64_t));
    if (!pos || !fr || !zi || !cnt) { free(pos); free(fr); free(zi); free(cnt); return -2; }
    for (int64_t k = 0; k < m; ++k) pos[t->pre[k]] = k;
#pragma omp parallel for num_threads(NTH()) schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        bh_state s;
        memset(&s, 0, sizeof(s));
        s.t = t;
        s.pos_of_node = pos;
        s.theta = theta;
        s.i = i;
        s.yx = Y[2 * i];
        s.yy = Y[2 * i + 1];
        bh_visit(&s, 0);
        fr[2 * i] = s.fx;
        fr[2 * i + 1] = s.fy;
        zi[i] = s.z;
        cnt[4 * i] = s.tests;
        cnt[4 * i + 1] = s.accepts;
        cnt[4 * i + 2] = s.pairs;
        cnt[4 * i + 3] = s.covered;
    }
    double z = 0.0;
    for (int64_t i = 0; i < n; ++i) z += zi[i];
#pragma omp parallel for num_threads(NTH()) schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        double fa[2];
        attract_row(Y, row_ptr, col, val, i, fa);
        grad[2 * i] = 4.0 * (exaggeration * fa[0] - fr[2 * i] / z);
        grad[2 * i + 1] = 4.0 * (exaggeration * fa[1] - fr[2 * i + 1] / z);
    }
    if (z_out) *z_out = z;
    if (counters) {
        counters[0] = counters[1] = counters[2] = counters[3] = 0;
        for (int64_t i = 0; i < n; ++i) {
            counters[0] += cnt[4 * i];
            counters[1] += cnt[4 * i + 1];
            counters[2] += cnt[4 * i + 2];
            counters[3] += cnt[4 * i + 3];
        }
    }
    free(pos); free(fr); free(zi); free(cnt);
    return 0;
}

/* ======================================================================
 * h-SNE (Sec. 4-C): a Euclidean Student-t term on the disk coordinates
 * ======================================================================
 * reading: the printed h-SNE variation is the sum of a Euclidean t-SNE
 * gradient of the disk coordinates (the form of eq. (4)) and lambda times the
 * hyperbolic one of eq. (14); the printed minus sign in front of the second
 * part and its missing factor d are taken as misprints (with them it would
 * ascend the hyperbolic KL divergence).  The cost whose gradient this sum is
 * reads KL(P || Q^E) + lambda KL(P || Q^H), with
 * q^E_ij = (1 + |y_i - y_j|^2)^-1 / sum_{k != l} (1 + |y_k - y_l|^2)^-1.
 * The Euclidean part is accelerated over the same polar quadtree: an internal
 * cell is replaced by N_cell copies of its centre of mass when
 * ediam / |y_i - c| < theta (ediam: the Euclidean cell diameter). */

static double euclid_w(double ix, double iy, double jx, double jy, double *dx, double *dy) {
    *dx = ix - jx;
    *dy = iy - jy;
    return 1.0 / (1.0 + (*dx) * (*dx) + (*dy) * (*dy));
}

/* Euclidean attractive sum for row i: sum_j p_ij w_ij (y_i - y_j) */
static void euclid_attract_row(const double *Y, const int64_t *row_ptr, const int32_t *col,
                               const double *val, int64_t i, double *fa) {
    fa[0] = fa[1] = 0.0;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
        int64_t j = col[e];
        if (j == i) continue;
        double dx, dy;
        double w = euclid_w(Y[2 * i], Y[2 * i + 1], Y[2 * j], Y[2 * j + 1], &dx, &dy);
        fa[0] += val[e] * w * dx;
        fa[1] += val[e] * w * dy;
    }
}

/* KL(P || Q^E); with exaggeration a, sum a p ln(a p) - sum a p ln w + ln Z as
 * for the hyperbolic cost */
int ora_euclid_cost(const double *Y, int64_t n, const int64_t *row_ptr, const int32_t *col,
                    const double *val, double exaggeration, double *cost_out) {
    if (n < 2) return -1;
    double z = 0.0, dx, dy;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = 0; j < n; ++j)
            if (j != i) z += euclid_w(Y[2 * i], Y[2 * i + 1], Y[2 * j], Y[2 * j + 1], &dx, &dy);
    double c = 0.0;
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
            int64_t j = col[e];
            double p = exaggeration * val[e];
            if (p <= 0.0) continue;
            double w = euclid_w(Y[2 * i], Y[2 * i + 1], Y[2 * j], Y[2 * j + 1], &dx, &dy);
            c += p * (log(p) - log(w));
        }
    *cost_out = c + log(z);
    return 0;
}

/* exact Euclidean gradient: g_i = 4 sum_{j != i} (a p_ij - w_ij / Z) w_ij (y_i - y_j) */
int ora_gradient_euclid_exact(const double *Y, int64_t n, const int64_t *row_ptr,
                              const int32_t *col, const double *val, double exaggeration,
                              double *grad, double *z_out) {
    if (n < 2) return -1;
    double *zi = (double *)malloc(sizeof(double) * (size_t)n);
    double *fr = (double *)malloc(sizeof(double) * (size_t)(2 * n));
    if (!zi || !fr) { free(zi); free(fr); return -2; }
#pragma omp parallel for num_threads(NTH()) schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        double rx = 0.0, ry = 0.0, sz = 0.0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx, dy;
            double w = euclid_w(Y[2 * i], Y[2 * i + 1], Y[2 * j], Y[2 * j + 1], &dx, &dy);
            rx += w * w * dx;
            ry += w * w * dy;
            sz += w;
        }
        fr[2 * i] = rx;
        fr[2 * i + 1] = ry;
        zi[i] = sz;
    }
    double z = 0.0;
    for (int64_t i = 0; i < n; ++i) z += zi[i];
    for (int64_t i = 0; i < n; ++i) {
        double fa[2];
        euclid_attract_row(Y, row_ptr, col, val, i, fa);
        grad[2 * i] = 4.0 * (exaggeration * fa[0] - fr[2 * i] / z);
        grad[2 * i + 1] = 4.0 * (exaggeration * fa[1] - fr[2 * i + 1] / z);
    }
    if (z_out) *z_out = z;
    free(zi);
    free(fr);
    return 0;
}

/* the same depth-first traversal as bh_visit, with Euclidean distances,
 * centres of mass and diameters */
static void bh_visit_euclid(bh_state *s, int32_t nid) {
    const onode *o = &s->t->nodes[nid];
    if (o->is_leaf) {
        for (int32_t a = 0; a < o->npts; ++a) {
            int64_t j = o->pts[a];
            if (j == s->i) continue;
            double dx, dy;
            double w = euclid_w(s->yx, s->yy, s->t->px[j], s->t->py[j], &dx, &dy);
            s->fx += w * w * dx;
            s->fy += w * w * dy;
            s->z += w;
            s->pairs++;
            s->covered++;
        }
        return;
    }
    int64_t k = s->pos_of_node[nid];
    const double *c = &s->t->ecent[2 * k];
    double dx, dy;
    double w = euclid_w(s->yx, s->yy, c[0], c[1], &dx, &dy);
    double d = sqrt(dx * dx + dy * dy);
    s->tests++;
    if (s->t->ediam[k] / d < s->theta) {
        double nc = (double)o->count;
        s->fx += nc * w * w * dx;
        s->fy += nc * w * w * dy;
        s->z += nc * w;
        s->accepts++;
        s->covered += o->count;
        return;
    }
    for (int ch = 0; ch < 4; ++ch)
        if (o->child[ch] >= 0) bh_visit_euclid(s, o->child[ch]);
}

int ora_gradient_euclid_bh(const double *Y, int64_t n, const int64_t *row_ptr,
                           const int32_t *col, const double *val, double exaggeration,
                           const ora_tree *t, double theta, double *grad, double *z_out,
                           int64_t *counters) {
    if (n < 2 || !t || t->n != n || !(theta >= 0.0) || isinf(theta)) return -1;
    int64_t m = t->nn;
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)m);
    double *fr = (double *)malloc(sizeof(double) * (size_t)(2 * n));
    double *zi = (double *)malloc(sizeof(double) * (size_t)n);
    int64_t *cnt = (int64_t *)calloc((size_t)(4 * n), sizeof(int64_t));
    if (!pos || !fr || !zi || !cnt) { free(pos); free(fr); free(zi); free(cnt); return -2; }
    for (int64_t k = 0; k < m; ++k) pos[t->pre[k]] = k;
#pragma omp parallel for num_threads(NTH()) schedule(dynamic, 64)
    for (int64_t i = 0; i < n; ++i) {
        bh_state s;
        memset(&s, 0, sizeof(s));
        s.t = t;
        s.pos_of_node = pos;
        s.theta = theta;
        s.i = i;
        s.yx = Y[2 * i];
        s.yy = Y[2 * i + 1];
        bh_visit_euclid(&s, 0);
        fr[2 * i] = s.fx;
        fr[2 * i + 1] = s.fy;
        zi[i] = s.z;
        cnt[4 * i] = s.tests;
        cnt[4 * i + 1] = s.accepts;
        cnt[4 * i + 2] = s.pairs;
        cnt[4 * i + 3] = s.covered;
    }
    double z = 0.0;
    for (int64_t i = 0; i < n; ++i) z += zi[i];
    for (int64_t i = 0; i < n; ++i) {
        double fa[2];
        euclid_attract_row(Y, row_ptr, col, val, i, fa);
        grad[2 * i] = 4.0 * (exaggeration * fa[0] - fr[2 * i] / z);
        grad[2 * i + 1] = 4.0 * (exaggeration * fa[1] - fr[2 * i + 1] / z);
    }
    if (z_out) *z_out = z;
    if (counters) {
        counters[0] = counters[1] = counters[2] = counters[3] = 0;
        for (int64_t i = 0; i < n; ++i) {
            counters[0] += cnt[4 * i];
            counters[1] += cnt[4 * i + 1];
            counters[2] += cnt[4 * i + 2];
            counters[3] += cnt[4 * i + 3];
        }
    }
    free(pos); free(fr); free(zi); free(cnt);
    return 0;
}

int ora_tree_export_euclid(const ora_tree *t, double *cent, double *diam) {
    for (int64_t k = 0; k < t->nn; ++k) {
        if (cent) { cent[2 * k] = t->ecent[2 * k]; cent[2 * k + 1] = t->ecent[2 * k + 1]; }
        if (diam) diam[k] = t->ediam[k];
    }
    return 0;
}

/* ======================================================================
 * Riemannian gradient step (eqs. (7), (16)-(18); optimiser of Sec. 5)
 * ====================================================================== */

/* One step for every point:
 *   g_hat = s(y) g with s = lambda_y^-2 = (1 - |y|^2)^2 / 4 (the inverse of
 *           the metric of eq. (7)); reading: metric_power = 1 uses lambda^-1
 *           as the sentence before eq. (14) literally says;
 *   gains  (delta-bar-delta, Sec. 5): +0.2 where sign(g_hat) != sign(u),
 *           x0.8 otherwise, never below min_gain;
 *   u      <- momentum u - eta gains g_hat;
 *   y      <- exp_y(u), eq. (16); reading: the momentum vector is reused at
 *           the new point without transport;
 *   proj   eq. (18); reading: "y/|y| - eps" is read as (1 - eps) y / |y|,
 *           applied when |y| >= 1, tested as |y|^2 >= 1 - 2^-50: a point
 *           on the circle up to the rounding of its double-precision norm
 *           counts as on it (else 1 - |y|^2 could round to 0 next). */
#define ON_CIRCLE (1.0 - 0x1p-50)
int ora_step(double *Y, double *update, double *gains, const double *grad,
             int64_t n, double eta, double momentum, double min_gain,
             double boundary_eps, int32_t metric_power) {
    if (n < 1 || !(eta > 0.0) || (metric_power != 1 && metric_power != 2)) return -1;
    for (int64_t i = 0; i < n; ++i) {
        double x = Y[2 * i], y = Y[2 * i + 1];
        double a = 1.0 - (x * x + y * y);
        double s = metric_power == 2 ? a * a / 4.0 : a / 2.0;
        for (int c = 0; c < 2; ++c) {
            double gh = s * grad[2 * i + c];
            double u = update[2 * i + c];
            double g = gains[2 * i + c];
            g = ((gh > 0.0) != (u > 0.0)) ? g + 0.2 : g * 0.8;
            if (g < min_gain) g = min_gain;
            gains[2 * i + c] = g;
            update[2 * i + c] = momentum * u - eta * g * gh;
        }
        double out[2];
        ora_exp_map(x, y, update[2 * i], update[2 * i + 1], out);
        double r2 = out[0] * out[0] + out[1] * out[1];
        if (r2 >= ON_CIRCLE) {
            double nr = sqrt(r2);
            out[0] = (1.0 - boundary_eps) * out[0] / nr;
            out[1] = (1.0 - boundary_eps) * out[1] / nr;
        }
        Y[2 * i] = out[0];
        Y[2 * i + 1] = out[1];
    }
    return 0;
}
