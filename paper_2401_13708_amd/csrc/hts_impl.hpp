// hts_impl.hpp -- internals of the HIP library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>

#include "hts.h"

namespace hts {

constexpr int kWave = 64;
constexpr int kBlock = 256;

// ---------------------------------------------------------------- records
// Per-point record read by the gradient kernels: coordinates in the working
// precision plus ia = 1 / (1 - |y|^2) computed in double from the stored
// coordinates, so the distance argument never cancels near the rim.
template <typename T> struct PointRec;
template <> struct alignas(16) PointRec<float> { float x, y; double ia; };
template <> struct alignas(16) PointRec<double> { double x, y, ia, pad; };

// Node record of the polar quadtree in pre-order, read with scalar loads by
// the traversal.  next_depth packs the pre-order index after the subtree
// (low 26 bits) and the depth (high 6 bits); a node is a leaf iff next is
// its own index + 1.  Internal nodes: (mx, my) is the Einstein midpoint,
// ib = 1 / (1 - |m|^2), c = cosh(r_cell / theta) - 1 (set per theta).
// Leaves: (mx, my, ib) is the leaf's first point and c holds the position of
// that point in the sorted order (as an int64 bit pattern).
template <typename T> struct NodeRec;
template <> struct alignas(16) NodeRec<float> {
    float mx, my;
    int32_t count;
    uint32_t next_depth;
    double ib;
    double c;
};
template <> struct alignas(16) NodeRec<double> {
    double mx, my;
    int32_t count;
    uint32_t next_depth;
    double ib;
    double c;
    double pad;
};
// traversal counters per stats block of the Barnes-Hut calls: node tests,
// accepted cells, exact leaf pairs, wave node visits, visits with at least one
// interaction, points accounted for (N_cell per accepted cell, 1 per pair)
constexpr int kBhStats = 6;
constexpr int kNextBits = 26;
constexpr uint32_t kNextMask = (1u << kNextBits) - 1u;
constexpr int64_t kMaxNodes = (int64_t)1 << kNextBits;

// Job layout as the kernels see it.  Query block qb of job j covers the
// global points off[j] + 64 (qb - job_qb[j]) ... (at most 64, within the job).
struct Jobs {
    const int64_t *off;
    const int32_t *job_qb;
    const int32_t *qb_job;
    const int32_t *pjob;
    int32_t J;
    __device__ __forceinline__ void block(int64_t qb, int64_t &start, int &cnt, int &job) const {
        job = qb_job[qb];
        start = off[job] + (int64_t)64 * (qb - job_qb[job]);
        const int64_t e = off[job + 1] - start;
        cnt = e < 64 ? (int)e : 64;
    }
};

// double-double triple used for the prefix sums of the midpoint summands
struct DD3 { double hi[3]; double lo[3]; };
// double-double pair for the prefix sums of the coordinates (Euclidean centres)
struct DD2 { double hi[2]; double lo[2]; };

// ---------------------------------------------------------------- handles
struct Timing {
    bool on = false;
    std::vector<hipEvent_t> pool;
    struct Rec { int cls; hipEvent_t a, b; };
    std::vector<Rec> recs;
    size_t used = 0;
};

struct Buffer {
    void *p = nullptr;
    size_t bytes = 0;
    uint64_t *gen = nullptr;  // the owning context's generation, bumped on reallocation
};

}  // namespace hts

struct hts_ctx_s {
    int device = 0;
    int32_t item_points = 288;  // Barnes-Hut work-item size S (hts_set_item_points)
    int32_t list_items = 256;   // item-list entries per phase-A wave (hts_set_item_list)
    int32_t items_grid = 0;     // phase-B workgroups at most, 0: automatic (hts_set_traversal_launch)
    int32_t items_waves = 1;    // waves per phase-B workgroup
    int32_t attract_at = 0;     // attractive rows: 0 automatic, 1 phase A, 2 phase B (hts_set_attract_launch)
    uint32_t *d_err = nullptr;
    // changes whenever device memory that launches on this context referenced
    // is reallocated (a workspace grown, a job layout's tables replaced)
    uint64_t gen = 0;
    hts::Buffer pts, fattr, frep, zpart, part, spare;
    hts::Buffer aff[8];
    hts::Timing timing;
};

struct hts_tree_s {
    hts_ctx ctx = nullptr;
    int device = 0;           // the context's device (the tree may outlive the context)
    int64_t n_max = 0;
    int32_t max_depth = 20;
    int64_t cap_nodes = 0;
    int64_t n = 0;            // points of the last build
    int32_t dtype = -1;       // dtype of the last build
    int64_t nb = 0;           // blocks over n_max
    // job layout: J embeddings side by side, job j owning global points
    // [off[j], off[j+1]); J = 1 with off = {0, n} unless set explicitly
    int32_t J = 1;
    bool jobs_set = false;        // layout given by hts_tree_set_jobs
    int64_t tab_n = -1;           // n the single-job tables were written for
    std::vector<int64_t> h_off;   // host copy of off
    int64_t max_job = 0;          // points of the largest job of the layout
    int64_t *job_off = nullptr;   // [J+1]
    int32_t *job_qb = nullptr;    // [J+1] first query block of each job
    int32_t *qb_job = nullptr;    // [nqb_max] job of each query block
    int32_t *pjob = nullptr;      // [n_max] job of each point
    int64_t nqb = 0;              // query blocks of the layout
    double *root = nullptr;       // [2J] (r_min, r_max) per job
    double *r = nullptr;           // [n_max] radius of every point
    double *mm = nullptr;     // per block: (min, max) of its first and of its last job
    uint64_t *keys_in = nullptr, *keys = nullptr;
    uint32_t *idx_in = nullptr, *perm = nullptr;
    void *sort_tmp = nullptr;
    size_t sort_tmp_bytes = 0;
    int32_t *ncnt_part = nullptr;  // per-block node counts
    hts::DD3 *q_part = nullptr;    // per-block midpoint-sum aggregates
    int32_t *node_start = nullptr; // [n+1]
    hts::DD3 *psum = nullptr;      // [n+1] exclusive prefix sums
    int32_t *d_m = nullptr;        // node count on the device
    void *spts = nullptr;          // sorted PointRec<T>
    void *nodes = nullptr;         // NodeRec<T>[cap_nodes]
    double *r_cell = nullptr;      // [cap_nodes]
    int32_t *node_first = nullptr; // [cap_nodes]
    double *sinhalf = nullptr;     // [32] sin(pi / 2^l), 1 for l <= 1
    int32_t job_bits = 0;          // key bits above the 2 max_depth cell bits
    int32_t split_rule = 0;        // 0: equal radial lengths (eq. (10)); 1: equal areas (eq. (9))
    // Euclidean summaries for the h-SNE term, allocated on first use
    void *enodes = nullptr;        // NodeRec<T>[cap_nodes]
    hts::DD2 *epsum = nullptr;     // [n_max + 1] prefix sums of the sorted coordinates
    hts::DD2 *epart = nullptr;     // [nb] block aggregates
};

namespace hts {

// ---------------------------------------------------------------- host utils
void set_error(const char *fmt, ...);
hts_status fail(hts_status s, const char *fmt, ...);
hts_status hip_fail(hipError_t e, const char *what);
hts_status ensure(Buffer &b, size_t bytes);

#define HTS_HIP(call)                                            \
    do {                                                         \
        hipError_t e__ = (call);                                 \
        if (e__ != hipSuccess) return ::hts::hip_fail(e__, #call); \
    } while (0)

#define HTS_OKR(call)                         \
    do {                                      \
        hts_status s__ = (call);              \
        if (s__ != HTS_OK) return s__;        \
    } while (0)

__host__ __device__ inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

// scoped event pair around a kernel class when timing is on
struct TimedScope {
    hts_ctx ctx;
    hipStream_t st;
    int cls;
    hipEvent_t b = nullptr;
    TimedScope(hts_ctx c, hipStream_t s, int k);
    ~TimedScope();
};

// ---------------------------------------------------------------- launchers
template <typename T>
hts_status launch_prep_points(hts_ctx ctx, hipStream_t st, const T *Y, int64_t n, PointRec<T> *pts);

// What a tree build can also do for the Barnes-Hut gradient that follows it
// (the work of the gradient's preparation launch, which is then left out):
// the point records of Y in input order (pts), the criterion thresholds of
// the internal nodes for theta, and the clearing of the item-list counter.
template <typename T>
struct TreeExtras {
    PointRec<T> *pts;
    double theta;
    unsigned *dense_count;
};

template <typename T>
hts_status tree_build(hts_ctx ctx, hipStream_t st, const T *Y, int64_t n, hts_tree t,
                      const TreeExtras<T> *extras = nullptr);

// device tables of a one-job layout over n points (when n changed)
hts_status tree_single_job(hipStream_t st, hts_tree t, int64_t n);

inline Jobs jobs_of(hts_tree t) {
    return Jobs{t->job_off, t->job_qb, t->qb_job, t->pjob, t->J};
}

// Euclidean node records (centres of mass, thresholds for theta) of the last
// build, for the h-SNE term
template <typename T>
hts_status tree_euclid(hts_ctx ctx, hipStream_t st, hts_tree t, double theta);

// stable LSD radix sort of (key, value) pairs by the low `bits` key bits
size_t radix_sort_temp_bytes(int64_t n);
hts_status radix_sort_pairs(hipStream_t st, uint64_t *keys_io, uint32_t *vals_io,
                            uint64_t *keys_out, uint32_t *vals_out, int64_t n, int bits,
                            void *tmp);

// timed: bracket the launch with the context's timing events (when on)
template <typename T>
hts_status launch_attract(hts_ctx ctx, hipStream_t st, const PointRec<T> *pts, const int64_t *rp,
                          const int32_t *col, const T *val, int64_t n, T *fattr,
                          bool timed = true);

// What the launch that starts a traversal also does: the point records of Y
// into pts (points), the criterion thresholds of the tree's hyperbolic nodes
// for theta (thresholds) and the clearing of the item-list counter (clear;
// when none of the three is asked, the launch is left out).
template <typename T>
struct BhPrep {
    const T *Y;
    double theta;
    bool points;
    bool thresholds;
    bool clear = true;
};

// The item-list counter of a one-job traversal of n points on ctx (the
// workspace is allocated as the traversal will use it), for a tree build
// that clears it (TreeExtras).
template <typename T>
hts_status bh_item_counter(hts_ctx ctx, hts_tree t, int64_t n, unsigned **counter);

// Barnes-Hut repulsion over the tree and the combine g = 4 (a F_attr - F_rep / Z)
// ex_job: per-job exaggeration (device, [J]) or NULL for ex; z_dev receives
// Z of every job ([J]); with accumulate, grad + scale g is stored.
// MET 0: hyperbolic terms over the tree's nodes; MET 1: the Euclidean
// Student-t terms over the Euclidean records of tree_euclid.
// (the first launch also computes the attractive term into fattr)
template <typename T, int MET>
hts_status launch_bh_repulsion(hts_ctx ctx, hipStream_t st, hts_tree t, int64_t n,
                               BhPrep<T> prep, PointRec<T> *pts, const int64_t *rp,
                               const int32_t *col, const T *val, T *fattr, double ex,
                               const double *ex_job, bool accumulate, double scale, T *grad,
                               double *z_dev, uint64_t *stats);

// the exact repulsion's per-chunk partials: exact_part_bytes(n) bytes in part
size_t exact_part_bytes(int64_t n);
template <typename T>
hts_status launch_exact(hts_ctx ctx, hipStream_t st, const PointRec<T> *pts, int64_t n,
                        double *part, double *frep, double *zpart, int64_t *nz_out,
                        bool timed = true);

template <typename T, typename FR>
hts_status launch_finalize(hts_ctx ctx, hipStream_t st, const T *fattr, const FR *frep,
                           const double *zpart, int64_t nz, int64_t n, double ex, T *grad,
                           double *z_dev, bool timed = true);

// Device memory of one exact-gradient call: point records, attractive
// forces, repulsive forces, Z partials, the repulsion's chunk partials and the
// cost's block sums (klpart may be NULL when no cost is asked for).
struct ExactWs {
    void *pts;
    void *fattr;
    double *frep, *zpart, *part, *klpart;
};
// bytes of those pieces for n points (sizes[6], each rounded up to 256) and
// their total; exact_carve lays them out one after another from base
template <typename T>
size_t exact_ws_bytes(int64_t n, size_t sizes[6]);
template <typename T>
ExactWs exact_carve(char *base, int64_t n);
// the exact gradient (and the cost when kl_dev is not NULL) on workspace w;
// timed: the launches carry the context's timing events when timing is on
template <typename T>
hts_status exact_impl(hts_ctx c, hipStream_t st, const T *Y, int64_t n, const int64_t *rp,
                      const int32_t *col, const T *val, double ex, T *grad, double *z_dev,
                      double *kl_dev, const ExactWs &w, bool timed);

// the cost of eq. (3) into *kl_dev (after *z_dev holds Z); part holds
// kl_parts(n) doubles
int64_t kl_parts(int64_t n);
template <typename T>
hts_status launch_kl(hts_ctx ctx, hipStream_t st, const PointRec<T> *pts, const int64_t *rp,
                     const int32_t *col, const T *val, int64_t n, double ex, double *part,
                     const double *z_dev, double *kl_dev);

template <typename T>
hts_status launch_cosne(hts_ctx ctx, hipStream_t st, const T *Y, int64_t n, const double *xnorm2,
                        double lambda1, double lambda2, T *grad);

// eta_job / mu_job: per-job values (device, indexed through pjob) or NULL
template <typename T>
hts_status launch_step(hts_ctx ctx, hipStream_t st, T *Y, T *U, T *G, const T *grad, int64_t n,
                       double eta, double mu, const int32_t *pjob, const double *eta_job,
                       const double *mu_job, double min_gain, double eps, int metric_power);

hts_status affinities(hts_ctx ctx, hipStream_t st, const void *X, int64_t n, int32_t d,
                      int32_t x_dtype, double perplexity, int32_t k, int32_t *knn_idx,
                      int64_t *row_ptr, int32_t *col_idx, void *p_val, int32_t p_dtype,
                      int64_t cap_nnz, int64_t *nnz_out);

}  // namespace hts
