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
constexpr int kNextBits = 26;
constexpr uint32_t kNextMask = (1u << kNextBits) - 1u;
constexpr int64_t kMaxNodes = (int64_t)1 << kNextBits;

// double-double triple used for the prefix sums of the midpoint summands
struct DD3 { double hi[3]; double lo[3]; };

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
};

}  // namespace hts

struct hts_ctx_s {
    int device = 0;
    uint32_t *d_err = nullptr;
    hts::Buffer pts, fattr, frep, zpart, part, spare;
    hts::Buffer aff[8];
    hts::Timing timing;
};

struct hts_tree_s {
    hts_ctx ctx = nullptr;
    int64_t n_max = 0;
    int32_t max_depth = 20;
    int64_t cap_nodes = 0;
    int64_t n = 0;            // points of the last build
    int32_t dtype = -1;       // dtype of the last build
    int64_t nb = 0;           // blocks over n_max
    double *r = nullptr, *phi = nullptr;
    double *mm = nullptr;     // per-block (min r, max r)
    double *root = nullptr;   // (r_min, r_max)
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
    int32_t *parent = nullptr;     // [cap_nodes] parent node (-1 for the root)
    int32_t *frontier = nullptr;   // [4^fdepth] node of each frontier cell, or -1
    int32_t fdepth = 0;            // depth of the frontier cells that split the traversal
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

template <typename T>
hts_status tree_build(hts_ctx ctx, hipStream_t st, const T *Y, int64_t n, hts_tree t);

hts_status tree_thresholds(hts_ctx ctx, hipStream_t st, hts_tree t, int dtype, double theta);

template <typename T>
hts_status launch_attract(hts_ctx ctx, hipStream_t st, const PointRec<T> *pts, const int64_t *rp,
                          const int32_t *col, const T *val, int64_t n, T *fattr);

// Barnes-Hut repulsion over the tree and the combine g = 4 (a F_attr - F_rep / Z)
template <typename T>
hts_status launch_bh_repulsion(hts_ctx ctx, hipStream_t st, hts_tree t, int64_t n, const T *fattr,
                               double ex, T *grad, double *z_dev, uint64_t *stats);

template <typename T>
hts_status launch_exact(hts_ctx ctx, hipStream_t st, const PointRec<T> *pts, int64_t n,
                        double *frep, double *zpart, int64_t *nz_out);

template <typename T, typename FR>
hts_status launch_finalize(hts_ctx ctx, hipStream_t st, const T *fattr, const FR *frep,
                           const double *zpart, int64_t nz, int64_t n, double ex, T *grad,
                           double *z_dev);

template <typename T>
hts_status launch_step(hts_ctx ctx, hipStream_t st, T *Y, T *U, T *G, const T *grad, int64_t n,
                       double eta, double mu, double min_gain, double eps, int metric_power);

hts_status affinities(hts_ctx ctx, hipStream_t st, const void *X, int64_t n, int32_t d,
                      int32_t x_dtype, double perplexity, int32_t k, int32_t *knn_idx,
                      int64_t *row_ptr, int32_t *col_idx, void *p_val, int32_t p_dtype,
                      int64_t cap_nnz, int64_t *nnz_out);

}  // namespace hts
