/*
 * hts_oracle.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow FP64 CPU reference of one iteration of hyperbolic t-SNE in the
 * Poincare disk, written from "Accelerating hyperbolic t-SNE" (arXiv
 * 2401.13708).  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load it.  It shares no code, header, table or helper with
 * the HIP library; both are written independently from the paper.
 *
 * All arrays are host arrays.  Points Y are n x 2 row-major doubles inside the
 * unit disk; CSR affinities are (row_ptr int64[n+1], col int32[nnz], val
 * double[nnz]) with columns ascending in each row and sum(val) = 1.
 *
 * Return codes: 0 ok, -1 invalid argument, -2 out of memory, -4 capacity.
 *
 * Pins -- what fixes each function other than itself (tests/test_oracle_*.py;
 * a dropped term, a wrong sign or index, or a transposed operand in the
 * function fails at least one of them):
 *   ora_dist            closed form d(0, y) = 2 artanh|y|; symmetry and the
 *                       triangle inequality; invariance under Mobius
 *                       translation; the boundary example of Sec. 5
 *                       (2 ln 19999); relative accuracy at tiny separations
 *   ora_dist_grad       central finite differences of ora_dist; the printed
 *                       form of eq. (13); the Euclidean limit near the origin
 *   ora_mobius_add,     exp_y(0) = y, exp_0(v) = tanh|v| v/|v|,
 *   ora_exp_map         d(y, exp_y v) = lambda_y |v|; Mobius identities
 *   ora_einstein_midpoint  one point gives itself, {y, -y} gives 0, rotation
 *                       equivariance, gyro-covariance, inside the Klein hull
 *   ora_knn_rows        brute force (N <= 64); ties by index; any row subset
 *                       equals the same rows of the full computation
 *   ora_cond_p          the entropy reaches ln(perplexity) to 1e-10
 *   ora_symmetrize,     P symmetric, non-negative, sums to 1, pattern
 *   ora_build_affinities  kNN union its transpose
 *   ora_kl_cost         the two-point closed form a ln a - (a - 1)(ln 2 + ln w);
 *                       a dense sum of p ln(p / q) (N <= 64)
 *   ora_gradient_exact  central finite differences of ora_kl_cost (the printed
 *                       eq. (14) without the factor d fails them); Z by brute
 *                       force; rotation covariance; the near-origin limit of
 *                       Euclidean t-SNE (Sec. 2-B)
 *   ora_gradient_exact_rows  all rows equal ora_gradient_exact
 *   ora_z_exact         the brute-force sum over ordered pairs
 *   ora_cosne_cost,     finite differences of the cost (the printed sign of
 *   ora_cosne_gradient  the variation fails them)
 *   ora_tree_build(_rule)  the recursive partition (ora_tree_build_partition)
 *                       on random, duplicate-heavy and near-ray inputs; brute
 *                       force (N <= 64); structural invariants; every point in
 *                       one leaf; the split's sign test against exact
 *                       rational arithmetic; points on a ray go to the upper
 *                       half
 *   ora_radial_mid      eq. (10) mid = (lo + hi)/2; eq. (9) against its printed
 *                       acosh / cosh form and against equal hyperbolic areas
 *   ora_tree_export     midpoints equal ora_einstein_midpoint of the cells;
 *                       cell diameters by dense sampling of the cell boundary;
 *                       the root's closed form; the shrink factor -> 1/2
 *   ora_gradient_bh     theta = 0 equals the exact gradient and Z (also with
 *                       duplicates); every query covers every other point
 *                       once (sum of N_c + leaf pairs = n (n - 1)); the error
 *                       lies in Table 3's band at theta = 0.5 and grows with
 *                       theta
 *   ora_gradient_bh_rows  all rows equal ora_gradient_bh, with its counters
 *   ora_euclid_cost,    finite differences; the two-point closed form; the
 *   ora_gradient_euclid_*  h-SNE sum against finite differences of its cost
 *                       (the printed minus sign fails them); theta = 0 equals
 *                       exact; cell centres of mass and diameters by brute
 *                       force
 *   ora_step            an independent restatement of the update rule;
 *                       zero gradient and update keep the points; the gain
 *                       floor; projection back into the disk; metric power 1
 */
#ifndef HTS_ORACLE_H
#define HTS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- geometry (Sec. 2-C, Sec. 4-B) ---- */
double ora_dist(double ax, double ay, double bx, double by);           /* eq. (8) */
void ora_dist_grad(double ax, double ay, double bx, double by, double *g); /* eq. (13): d d(a,b)/d a */
void ora_mobius_add(double ax, double ay, double bx, double by, double *out); /* eq. (17) */
void ora_exp_map(double yx, double yy, double vx, double vy, double *out);    /* eq. (16) */
void ora_einstein_midpoint(const double *Y, int64_t n, double *out);          /* eq. (11) */

/* ---- input affinities (Sec. 2-A, eq. (1); truncated Gaussians) ---- */
int ora_knn_rows(const double *X, int64_t n, int32_t d, int32_t k,
                 const int64_t *rows, int64_t nrows,
                 int32_t *idx_out, double *d2_out);
int ora_cond_p(const double *d2, int64_t n, int32_t k, double perplexity,
               double *p_out, double *beta_out);
int ora_symmetrize(const int32_t *knn, const double *pc, int64_t n, int32_t k,
                   int64_t *row_ptr, int32_t *col, double *val, int64_t cap_nnz,
                   int64_t *nnz_out);
int ora_build_affinities(const double *X, int64_t n, int32_t d, double perplexity,
                         int32_t k, int32_t *knn_out, int64_t *row_ptr,
                         int32_t *col, double *val, int64_t cap_nnz,
                         int64_t *nnz_out);

/* ---- cost and exact gradient (eqs. (3), (12)-(15)) ---- */
int ora_kl_cost(const double *Y, int64_t n, const int64_t *row_ptr,
                const int32_t *col, const double *val, double exaggeration,
                double *cost_out);
/* CO-SNE (Sec. 4-C): cost lambda1 KL + (lambda2/n) sum (|x_i|^2 - |y_i|^2)^2 and
 * its gradient from a KL gradient g_kl */
int ora_cosne_cost(const double *Y, int64_t n, const int64_t *row_ptr, const int32_t *col,
                   const double *val, const double *xnorm2, double lambda1, double lambda2,
                   double *cost_out);
int ora_cosne_gradient(const double *Y, int64_t n, const double *xnorm2, double lambda1,
                       double lambda2, const double *g_kl, double *g_out);
int ora_gradient_exact(const double *Y, int64_t n, const int64_t *row_ptr,
                       const int32_t *col, const double *val,
                       double exaggeration, double *grad, double *z_out);
/* exact gradient rows for a subset of queries; z is given (sum over all pairs) */
int ora_gradient_exact_rows(const double *Y, int64_t n, const int64_t *row_ptr,
                            const int32_t *col, const double *val,
                            double exaggeration, const int64_t *rows,
                            int64_t nrows, double z, double *grad_rows);
int ora_z_exact(const double *Y, int64_t n, double *z_out);

/* ---- polar quadtree (Sec. 2-D, Sec. 4-A) ---- */
typedef struct ora_tree ora_tree;
int ora_tree_build(const double *Y, int64_t n, int32_t max_depth,
                   ora_tree **out);                       /* by insertion */
int ora_tree_build_partition(const double *Y, int64_t n, int32_t max_depth,
                             ora_tree **out);             /* by recursive split */
/* the same with a radial split rule: 0 equal lengths (eq. (10)), 1 equal
 * hyperbolic areas (eq. (9)) */
int ora_tree_build_rule(const double *Y, int64_t n, int32_t max_depth,
                        int32_t split_rule, ora_tree **out);
int ora_tree_build_partition_rule(const double *Y, int64_t n, int32_t max_depth,
                                  int32_t split_rule, ora_tree **out);
double ora_radial_mid(double lo, double hi, int32_t split_rule);
void ora_tree_free(ora_tree *t);
int64_t ora_tree_num_nodes(const ora_tree *t);
/* pre-order export; any pointer may be NULL.  mid is n_nodes x 2, bounds is
 * n_nodes x 4 (r_lo, r_hi, phi_lo, phi_hi), perm is the leaf-order point list */
int ora_tree_export(const ora_tree *t, int32_t *count, int32_t *depth,
                    int32_t *first, int32_t *next, double *mid, double *r_cell,
                    double *bounds, int64_t *perm);

/* ---- Barnes-Hut gradient (eq. (19) and the traversal of Sec. 4-B) ---- */
int ora_gradient_bh(const double *Y, int64_t n, const int64_t *row_ptr,
                    const int32_t *col, const double *val, double exaggeration,
                    const ora_tree *t, double theta, double *grad,
                    double *z_out, int64_t *counters);
/* counters: NULL or int64[4] receiving, summed over the queries, the node
 * tests, the accepted cells, the exact leaf pairs and the points the query
 * accounted for (N_cell per accepted cell plus 1 per leaf pair); every query
 * meets each other point exactly once, so the last one equals n (n - 1). */

/* the same gradient for the query rows rows[0..nrows) only, with Z given */
int ora_gradient_bh_rows(const double *Y, int64_t n, const int64_t *row_ptr,
                         const int32_t *col, const double *val, double exaggeration,
                         const ora_tree *t, double theta, const int64_t *rows,
                         int64_t nrows, double z, double *grad_rows, int64_t *counters);

/* ---- h-SNE (Sec. 4-C): the Euclidean Student-t term of the disk coordinates ----
 * cost KL(P || Q^E) with q^E_ij proportional to (1 + |y_i - y_j|^2)^-1; its
 * exact gradient; and the same accelerated over the polar quadtree with
 * Euclidean centres of mass and the criterion ediam / |y_i - c| < theta.
 * The h-SNE gradient is the Euclidean one plus lambda times the hyperbolic. */
int ora_euclid_cost(const double *Y, int64_t n, const int64_t *row_ptr, const int32_t *col,
                    const double *val, double exaggeration, double *cost_out);
int ora_gradient_euclid_exact(const double *Y, int64_t n, const int64_t *row_ptr,
                              const int32_t *col, const double *val, double exaggeration,
                              double *grad, double *z_out);
int ora_gradient_euclid_bh(const double *Y, int64_t n, const int64_t *row_ptr,
                           const int32_t *col, const double *val, double exaggeration,
                           const ora_tree *t, double theta, double *grad, double *z_out,
                           int64_t *counters);
/* per node (pre-order): centre of mass (n_nodes x 2) and Euclidean diameter */
int ora_tree_export_euclid(const ora_tree *t, double *cent, double *diam);

/* ---- Riemannian step (eqs. (7), (16)-(18), Sec. 5 optimiser) ---- */
int ora_step(double *Y, double *update, double *gains, const double *grad,
             int64_t n, double eta, double momentum, double min_gain,
             double boundary_eps, int32_t metric_power);

/* threads used by the parallel loops (0 = OpenMP default) */
void ora_set_threads(int32_t nthreads);
int32_t ora_get_threads(void);

#ifdef __cplusplus
}
#endif
#endif
