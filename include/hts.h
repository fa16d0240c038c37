/*
 * hts.h -- C ABI of the MI355X (gfx950) hyperbolic t-SNE gradient library.
 *
 * Computes one iteration of hyperbolic t-SNE in the Poincare disk as defined
 * in "Accelerating hyperbolic t-SNE" (arXiv 2401.13708): the sparse
 * attractive sum over the affinities P, the repulsive sum with its
 * normaliser Z (exactly, or by Barnes-Hut over a polar quadtree), and the
 * Riemannian gradient step.
 *
 * Conventions shared by every entry point
 *  - Every array argument is a DEVICE pointer owned by the caller, contiguous
 *    and naturally aligned, unless marked "host".  The library never frees or
 *    keeps a caller pointer beyond the call.
 *  - Points are n x 2 row-major (x, y) pairs strictly inside the unit disk.
 *    dtype HTS_F32: float arrays; HTS_F64: double arrays.  Y, P values,
 *    gradients, update and gains of one call share the dtype.
 *  - Affinities P are CSR: row_ptr int64[n+1], col_idx int32[nnz] (columns
 *    ascending in each row, no diagonal), p_val[nnz] with sum 1.
 *  - stream is a hipStream_t (NULL: the null stream).  Calls are asynchronous
 *    on it except those marked "sync", which return after the stream has
 *    drained.  Calls on one context must not overlap on different streams.
 *  - Arguments are validated before anything is launched; a failed check
 *    returns HTS_EINVAL and launches nothing.  hts_last_error() gives the
 *    message of the last failure on the calling thread.
 *  - Numerical faults found on the device (NaN or infinite gradients,
 *    points outside the disk) set a device error word that the next sync
 *    call or hts_check() reports as HTS_ENUMERIC.
 */
#ifndef HTS_H
#define HTS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum hts_status {
    HTS_OK = 0,
    HTS_EINVAL = -1,     /* invalid argument (nothing launched) */
    HTS_ENOMEM = -2,     /* device allocation failed */
    HTS_EDEVICE = -3,    /* HIP runtime error */
    HTS_ECAPACITY = -4,  /* an output capacity is too small; the size needed is returned */
    HTS_ENUMERIC = -5    /* the device error word is set */
} hts_status;

typedef enum hts_dtype { HTS_F32 = 0, HTS_F64 = 1 } hts_dtype;

/* device error word bits */
#define HTS_ERR_NONFINITE_GRAD 1u
#define HTS_ERR_OUTSIDE_DISK 2u
#define HTS_ERR_NONFINITE_Y 4u
#define HTS_ERR_BAD_INDEX 8u      /* a CSR column outside [0, n) was skipped */
#define HTS_ERR_TREE_OVERFLOW 16u /* node storage exhausted (internal error) */

typedef struct hts_ctx_s *hts_ctx;
typedef struct hts_tree_s *hts_tree;
typedef void *hts_stream;

/* Message of the last failed call on this thread ("" if none). */
const char *hts_last_error(void);

/* Library version string. */
const char *hts_version(void);

/* Context on one device: owns the device error word and grow-on-demand
 * workspaces.  device: HIP device ordinal.  *out receives the handle. */
hts_status hts_create(int32_t device, hts_ctx *out);
hts_status hts_destroy(hts_ctx ctx);

/* sync: waits for the stream, returns HTS_ENUMERIC if the device error word
 * is set (and clears it), otherwise HTS_OK.  *bits_out (host, may be NULL)
 * receives the word. */
hts_status hts_check(hts_ctx ctx, hts_stream stream, uint32_t *bits_out);

/* ------------------------------------------------------------------------
 * Input affinities P -- Sec. 2-A, eq. (1), truncated to the k nearest
 * neighbours (Sec. 2-A, Sec. 4-B) and symmetrised.  sync.
 *  X          n x d row-major input points, dtype x_dtype.
 *  perplexity target perplexity of every conditional row, 0 < perplexity < k.
 *  k          neighbours per point, 1 <= k < n, k <= 128.
 *  knn_idx    n x k int32 output (nearest first; ties by smaller index) or NULL.
 *  row_ptr, col_idx, p_val   CSR output of P = (P_c + P_c^T) / (2 n), p_val
 *             in p_dtype; cap_nnz entries available (2 n k always suffice).
 *  nnz_out    host: number of entries written, or needed on HTS_ECAPACITY.
 * The k-NN search is exact: squared distances are summed in double precision
 * over the dimensions in ascending order with fused multiply-adds.  The
 * bandwidth of row i solves perplexity(P_i) = perplexity by 100 bisection
 * steps in double precision.
 * ---------------------------------------------------------------------- */
hts_status hts_build_affinities(hts_ctx ctx, hts_stream stream, const void *X,
                                int64_t n, int32_t d, int32_t x_dtype,
                                double perplexity, int32_t k, int32_t *knn_idx,
                                int64_t *row_ptr, int32_t *col_idx, void *p_val,
                                int32_t p_dtype, int64_t cap_nnz,
                                int64_t *nnz_out);

/* ------------------------------------------------------------------------
 * Polar quadtree -- Sec. 2-D and Sec. 4-A.  The root is the annulus
 * [min r, max r] x [0, 2 pi) of the current points; every cell splits at the
 * angular middle and at the radial middle in embedding radius (eq. (10)); a
 * leaf holds one point, or all points that reach max_depth; internal nodes
 * carry the Einstein midpoint of their points (eq. (11)) and their hyperbolic
 * diameter.  Nodes are kept in depth-first pre-order, children in the order
 * 2 * [outer half] + [upper angular half].
 * ---------------------------------------------------------------------- */

/* Tree storage for up to n_max points; max_depth in [1, 24] (20 is the
 * default of the tree readings).  Allocates device memory once.  A tree may
 * be destroyed after its context (hts_tree_destroy is then the only valid
 * call on it). */
hts_status hts_tree_create(hts_ctx ctx, int64_t n_max, int32_t max_depth,
                           hts_tree *out);
hts_status hts_tree_destroy(hts_tree tree);

/* sync.  Job layout: the tree will hold n_jobs independent embeddings side
 * by side (one tree per job, built, traversed and stepped in the same
 * launches).  Job j owns the n_per_job[j] >= 2 consecutive points after
 * those of jobs 0..j-1 of the concatenated Y; the sum must not exceed n_max.
 * The job index is kept above the 2 max_depth cell bits of a 64-bit sort
 * key, so ceil(log2(n_jobs)) + 2 max_depth must not exceed 64 (HTS_EINVAL).
 * n_per_job is a host array.  A new tree holds one job of whatever n the
 * next build is given; after this call every build must be given exactly
 * the layout's total.  Jobs in one layout see only their own points: their
 * results are those of the same jobs built and traversed alone. */
hts_status hts_tree_set_jobs(hts_tree tree, int32_t n_jobs,
                             const int64_t *n_per_job);

/* Radial split rule of later builds (Sec. 2-D, Sec. 4-A): 0 (default) splits
 * a cell's radial range at the mean embedding radius, eq. (10); 1 splits it
 * into two parts of equal hyperbolic area, eq. (9) (mid^2 = s / (2 + s) with
 * s = lo^2/(1-lo^2) + hi^2/(1-hi^2), the same point written in the embedding
 * radius).  The angular split is the same for both. */
hts_status hts_tree_set_split(hts_tree tree, int32_t split_rule);

/* Builds the tree of Y (n points, 2 <= n <= n_max) on the stream (one tree
 * per job of the layout).  The tree keeps its own copy of everything it
 * needs; Y may change afterwards. */
hts_status hts_build_polar_tree(hts_ctx ctx, hts_stream stream, const void *Y,
                                int64_t n, int32_t y_dtype, hts_tree tree);

/* sync.  Copies the last built tree out in pre-order.  *n_nodes_out (host)
 * receives the node count M; every non-NULL device array must hold cap
 * entries (M <= cap, else HTS_ECAPACITY): count[M] points per node,
 * depth[M], first[M] (position of the node's first point in perm), next[M]
 * (pre-order index after the node's subtree), mid[2M] (midpoint, double),
 * r_cell[M] (hyperbolic diameter, double), perm[n] (int32 point indices in
 * leaf order). */
hts_status hts_tree_export(hts_ctx ctx, hts_stream stream, hts_tree tree,
                           int64_t *n_nodes_out, int64_t cap, int32_t *count,
                           int32_t *depth, int32_t *first, int32_t *next,
                           double *mid, double *r_cell, int32_t *perm);

/* ------------------------------------------------------------------------
 * Gradients -- eqs. (12)-(15) of Sec. 4-B, with the factor d_ij that the
 * derivative of ln(1 + d^2)^-1 carries:
 *   g_i = 4 ( a sum_j p_ij w_ij d_ij dd_ij/dy_i - (1/Z) sum_{j!=i} w_ij^2 d_ij dd_ij/dy_i ),
 *   w_ij = (1 + d_ij^2)^-1,  Z = sum over ordered pairs k != l of w_kl,
 * with a = exaggeration > 0.  grad (n x 2) receives this Euclidean variation
 * (no metric rescaling); *z_dev (device double) receives Z.
 * Single precision: forces in float with float accumulation; the distance
 * argument 2|yi-yj|^2 / ((1-|yi|^2)(1-|yj|^2)) and the criterion in double;
 * Z from float partial sums (one per subtree walk) added up in double.
 * ---------------------------------------------------------------------- */

/* Exact O(n^2) repulsion.  kl_dev: NULL, or a device double that receives
 * the cost of eq. (3) with q_ij = w_ij / Z (eq. (12)), summed over the
 * non-zeros of P:  sum_ij a p_ij (ln(a p_ij) - ln w_ij) + ln Z,  which is
 * KL(P || Q) for a = 1 (sum P = 1) and in general the objective whose
 * gradient grad holds.  Its terms are formed and summed in double (from the
 * stored coordinates) in a fixed order. */
hts_status hts_gradient_exact(hts_ctx ctx, hts_stream stream, const void *Y,
                              int64_t n, int32_t dtype, const int64_t *row_ptr,
                              const int32_t *col_idx, const void *p_val,
                              double exaggeration, void *grad, double *z_dev,
                              double *kl_dev);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, serving loops that forbid allocation): hts_gradient_exact with
 * the same arguments, results and kernels, but every byte of workspace it
 * needs comes from one fixed device region per GPU (18 MiB, held by each GPU
 * the library runs on until the process ends) instead of the context's
 * grow-on-demand buffers, so the call allocates and frees nothing and sets
 * no timing events.  n <= HTS_NOALLOC_MAX_N, else HTS_ECAPACITY.  All calls
 * on one GPU share the region and it keeps the last call's contents:
 * calls that overlap on one GPU (other streams, other contexts, other
 * threads) race and must not be issued. */
#define HTS_NOALLOC_MAX_N 65536
hts_status hts_gradient_exact_noalloc(hts_ctx ctx, hts_stream stream,
                                      const void *Y, int64_t n, int32_t dtype,
                                      const int64_t *row_ptr,
                                      const int32_t *col_idx, const void *p_val,
                                      double exaggeration, void *grad,
                                      double *z_dev, double *kl_dev);

/* Barnes-Hut repulsion (eq. (19)): a cell whose diameter r_cell and midpoint
 * m satisfy r_cell / d(y_i, m) < theta stands for its N_cell points;
 * theta = 0 evaluates every pair.  tree must have been built from the same Y.
 * stats_dev: NULL or device uint64[12] to which the call ADDS, in [0..5],
 * the number of node tests, accepted cells and exact leaf pairs (per query),
 * the node visits and the visits with at least one interaction (per wave),
 * and the points the queries accounted for (N_cell per accepted cell plus 1
 * per leaf pair; each query meets every other point once, so one call adds
 * n (n - 1)); [6..11] receive the same six counts restricted to the second
 * traversal kernel (the walks of the small subtrees), so the first kernel's
 * share is the difference. */
hts_status hts_gradient_bh(hts_ctx ctx, hts_stream stream, const void *Y,
                           int64_t n, int32_t dtype, const int64_t *row_ptr,
                           const int32_t *col_idx, const void *p_val,
                           double exaggeration, hts_tree tree, double theta,
                           void *grad, double *z_dev, uint64_t *stats_dev);

/* The same for every job of the tree's layout at once (hts_tree_set_jobs).
 * Y, grad: the concatenated n x 2 arrays.  P: one CSR over the concatenated
 * rows whose column indices are global (a job's columns lie in its own
 * range).  exaggeration_dev: device double[n_jobs], the exaggeration of each
 * job; z_dev: device double[n_jobs], receives each job's Z.  stats_dev as
 * above, summed over the jobs.  Each job's gradient and Z equal those of the
 * job alone through hts_gradient_bh, bit for bit. */
hts_status hts_gradient_bh_jobs(hts_ctx ctx, hts_stream stream, const void *Y,
                                int64_t n, int32_t dtype, const int64_t *row_ptr,
                                const int32_t *col_idx, const void *p_val,
                                const double *exaggeration_dev, hts_tree tree,
                                double theta, void *grad, double *z_dev,
                                uint64_t *stats_dev);

/* h-SNE variant (Sec. 4-C).  The printed h-SNE variation is read as the sum
 * of a Euclidean t-SNE gradient of the disk coordinates and lambda times the
 * hyperbolic gradient above (the printed minus sign of the second part and
 * its missing factor d taken as misprints): the gradient of
 *   KL(P||Q^E) + lambda KL(P||Q^H),  q^E_ij = v_ij / Z^E,  v_ij = (1 + |y_i - y_j|^2)^-1,
 *   g_i = 4 ( a sum_j p_ij v_ij (y_i - y_j) - (1/Z^E) sum_{j!=i} v_ij^2 (y_i - y_j) )
 *         + lambda g^H_i  (g^H as from hts_gradient_bh).
 * Both parts are accelerated over the same polar quadtree: the Euclidean
 * part replaces a cell by N_cell copies of its centre of mass c when
 * ediam / |y_i - c| < theta, ediam being the largest Euclidean distance
 * between two corners of the cell (angular widths of pi or more read as pi).
 * tree: built from the same Y, one job.  lambda: finite, >= 0.
 * z_dev: device double[2], receives Z^E then Z^H.  stats_dev: NULL or device
 * uint64[24]: [0..11] the counters of hts_gradient_bh for the Euclidean
 * traversal, [12..23] for the hyperbolic one (added to).  The first call
 * allocates the tree's Euclidean node records (cap entries). */
hts_status hts_gradient_hsne(hts_ctx ctx, hts_stream stream, const void *Y,
                             int64_t n, int32_t dtype, const int64_t *row_ptr,
                             const int32_t *col_idx, const void *p_val,
                             double exaggeration, double lambda, hts_tree tree,
                             double theta, void *grad, double *z_dev,
                             uint64_t *stats_dev);

/* CO-SNE variant (Sec. 4-C): turns the KL gradient in grad (from either
 * gradient call, same Y) into the gradient of
 *   lambda1 KL(P||Q) + (lambda2 / n) sum_i (|x_i|^2 - |y_i|^2)^2,
 * in place: grad_i <- lambda1 grad_i - (4 lambda2 / n)(|x_i|^2 - |y_i|^2) y_i,
 * the derivative of that cost (the paper prints the second term with the
 * opposite sign).  xnorm2: device double[n], the squared norms of the input
 * points as the caller defines them; lambda2 >= 0. */
hts_status hts_cosne_terms(hts_ctx ctx, hts_stream stream, const void *Y,
                           int64_t n, int32_t dtype, const double *xnorm2,
                           double lambda1, double lambda2, void *grad);

/* ------------------------------------------------------------------------
 * Riemannian step -- eqs. (7), (16)-(18) and the optimiser of Sec. 5.  In
 * place on Y, update and gains (n x 2 each):
 *   g_hat = s(y) grad, s = (1-|y|^2)^2 / 4 (metric_power 2: inverse metric)
 *           or (1-|y|^2) / 2 (metric_power 1);
 *   gains += 0.2 where sign(g_hat) != sign(update), else *= 0.8, >= min_gain;
 *   update = momentum * update - eta * gains * g_hat;
 *   y = exp_y(update) (Mobius addition), then y = (1 - boundary_eps) y / |y|
 *       if |y| >= 1 (eq. (18)).
 * The exponential map and the projection run in double precision.
 * ---------------------------------------------------------------------- */
hts_status hts_step(hts_ctx ctx, hts_stream stream, void *Y, void *update,
                    void *gains, const void *grad, int64_t n, int32_t dtype,
                    double eta, double momentum, double min_gain,
                    double boundary_eps, int32_t metric_power);

/* One whole iteration of the Barnes-Hut path -- Sec. 4-B and Sec. 5: the
 * polar tree of Y (as hts_build_polar_tree), the gradient (as
 * hts_gradient_bh, into grad and z_dev[0]) and the step (as hts_step), in one
 * asynchronous call on the stream, with results bit for bit those of the
 * three calls.  One job only; tree as for hts_build_polar_tree
 * (n <= n_max); the other arguments as for the three calls. */
hts_status hts_iteration_bh(hts_ctx ctx, hts_stream stream, void *Y, void *update, void *gains,
                            int64_t n, int32_t dtype, const int64_t *row_ptr,
                            const int32_t *col_idx, const void *p_val, double exaggeration,
                            hts_tree tree, double theta, void *grad, double *z_dev, double eta,
                            double momentum, double min_gain, double boundary_eps,
                            int32_t metric_power);

/* The step for every job of a tree's layout: n must be the layout's total;
 * eta_dev and momentum_dev are device double[n_jobs] (each job's learning
 * rate and momentum). */
hts_status hts_step_jobs(hts_ctx ctx, hts_stream stream, hts_tree tree, void *Y,
                         void *update, void *gains, const void *grad, int64_t n,
                         int32_t dtype, const double *eta_dev,
                         const double *momentum_dev, double min_gain,
                         double boundary_eps, int32_t metric_power);

/* Optimiser schedule of Sec. 5 per job, on the device: for each of n_jobs
 * jobs with iteration counter it_dev[j] (device int32), writes
 * exaggeration_dev[j] = exaggeration and momentum_dev[j] = momentum_early
 * while it_dev[j] < ee_iters, else 1 and momentum_late; then increments
 * it_dev[j].  Jobs of one layout may be at different iterations. */
hts_status hts_jobs_schedule(hts_ctx ctx, hts_stream stream, int32_t n_jobs,
                             int32_t *it_dev, int32_t ee_iters, double exaggeration,
                             double momentum_early, double momentum_late,
                             double *exaggeration_dev, double *momentum_dev);

/* Traversal work split (a tuning parameter, not part of the method): the
 * Barnes-Hut walk hands every rejected cell of at most item_points points to
 * a separate short walk.  Results differ between settings only by the order
 * of floating-point sums.  Default 288; applies to later calls on ctx. */
hts_status hts_set_item_points(hts_ctx ctx, int32_t item_points);

/* Size of the list that carries those short walks between the two kernels of
 * the traversal: each 64-query wave of the first kernel hands over at most
 * items_per_wave (>= 0) of them (40 bytes and a 64-lane partial force each)
 * and makes the others itself.  The split depends only on the wave, so every
 * setting gives the same result up to the order of floating-point sums, and
 * each setting gives it run after run; smaller lists use less device memory
 * and run slower once waves exceed their share.  Default 256 (every walk a
 * wave records; larger values act as 256); applies to later calls on ctx. */
hts_status hts_set_item_list(hts_ctx ctx, int32_t items_per_wave);

/* Launch shape of the traversal's second kernel (the short walks of the item
 * list): at most `workgroups` workgroups of `waves_per_workgroup` 64-lane
 * waves (1, 2 or 4), striding over the list.  workgroups = 0 (the default)
 * sizes the grid to 32 waves per wave of the first kernel, about one wave per
 * walk, so that each freed wave slot takes the next walk; with the default of
 * one wave per workgroup no slot waits for a workgroup's other waves.  Every
 * walk writes its own partials, so the result does not depend on the shape at
 * all (bit for bit).  Applies to later calls on ctx. */
hts_status hts_set_traversal_launch(hts_ctx ctx, int32_t workgroups, int32_t waves_per_workgroup);

/* Where the Barnes-Hut gradient computes its attractive term (the first sum
 * of eq. (15)): 1 in the traversal's first launch, beside the walks of the
 * large cells (its waves then compete with those chains for issue, and are
 * hidden when the chains are long), 2 in the last workgroups of the second
 * launch (they start after the work items and fill the chip while the longest
 * walks finish), 0 automatic (1 when the largest job of the tree's layout has
 * at least 131072 points, else 2).  The result does not depend on the choice
 * (bit for bit).  HTS_EINVAL for another value or a NULL ctx.  Applies to
 * later calls on ctx. */
hts_status hts_set_attract_launch(hts_ctx ctx, int32_t where);

/* Workspace generation of ctx (host, *gen_out).  The context keeps device
 * workspaces that grow on demand, and a job layout (hts_tree_set_jobs)
 * replaces its tree's tables; either reallocation changes this counter.
 * Launches recorded into a HIP graph reference the device memory of the
 * moment of capture: replaying such a graph is valid only while the counter
 * keeps the value it had when the graph was captured (re-capture otherwise). */
hts_status hts_workspace_generation(hts_ctx ctx, uint64_t *gen_out);

/* ------------------------------------------------------------------------
 * Kernel timing with HIP events on the caller's stream (for benchmarks).
 * While enabled, each launch of a timed kernel class is bracketed by events.
 * hts_timing_read (sync) adds the elapsed milliseconds and launch counts of
 * the classes into ms_out[HTS_KCLASS_COUNT] / launches_out[...] (host) and
 * resets them.
 * ---------------------------------------------------------------------- */
enum {
    HTS_K_TREE = 0,      /* whole tree build */
    HTS_K_ATTRACT = 1,   /* attractive CSR kernel */
    HTS_K_TRAVERSE = 2,  /* Barnes-Hut traversal, walk of the large cells */
    HTS_K_EXACT = 3,     /* exact repulsion kernel */
    HTS_K_FINALIZE = 4,  /* Z reduction and combine */
    HTS_K_STEP = 5,      /* Riemannian step */
    HTS_K_KNN = 6,       /* exact k-NN */
    HTS_K_ITEMS = 7,     /* Barnes-Hut traversal, walks of the small subtrees */
    HTS_KCLASS_COUNT = 8
};
hts_status hts_timing_enable(hts_ctx ctx, int32_t on);
hts_status hts_timing_read(hts_ctx ctx, double *ms_out, int64_t *launches_out);

#ifdef __cplusplus
}
#endif
#endif /* HTS_H */
