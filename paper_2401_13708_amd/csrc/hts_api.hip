// hts_api.hip -- the C ABI declared in include/hts.h: argument validation,
// handles, workspaces and kernel dispatch.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>

#include "hts_impl.hpp"

namespace hts {

static thread_local char g_err[512] = "";

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}

hts_status fail(hts_status s, const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return s;
}

hts_status hip_fail(hipError_t e, const char *what) {
    set_error("HIP error %d (%s) in %s", (int)e, hipGetErrorString(e), what);
    return e == hipErrorOutOfMemory ? HTS_ENOMEM : HTS_EDEVICE;
}

hts_status ensure(Buffer &b, size_t bytes) {
    if (b.bytes >= bytes && b.p) return HTS_OK;
    if (b.p) {
        HTS_HIP(hipFree(b.p));
        b.p = nullptr;
        b.bytes = 0;
    }
    size_t want = bytes < 256 ? 256 : bytes;
    if (b.gen) ++*b.gen;  // pointers to the old allocation are stale from here on
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) return hip_fail(e, "hipMalloc(workspace)");
    b.bytes = want;
    return HTS_OK;
}

TimedScope::TimedScope(hts_ctx c, hipStream_t s, int k) : ctx(c), st(s), cls(k) {
    if (!ctx || !ctx->timing.on) return;
    Timing &tm = ctx->timing;
    if (tm.used + 2 > tm.pool.size()) {
        for (int a = 0; a < 64; ++a) {
            hipEvent_t e;
            if (hipEventCreate(&e) != hipSuccess) return;
            tm.pool.push_back(e);
        }
    }
    b = tm.pool[tm.used++];
    (void)hipEventRecord(b, st);
}

TimedScope::~TimedScope() {
    if (!b) return;
    Timing &tm = ctx->timing;
    hipEvent_t e = tm.pool[tm.used++];
    (void)hipEventRecord(e, st);
    tm.recs.push_back({cls, b, e});
}

extern hts_status tree_sort_bytes(int64_t n_max, int L, size_t *bytes);

static bool dtype_ok(int32_t d) { return d == HTS_F32 || d == HTS_F64; }

}  // namespace hts

using namespace hts;

extern "C" {

const char *hts_last_error(void) { return hts::g_err; }

const char *hts_version(void) { return "hts 0.1 (gfx950)"; }

hts_status hts_create(int32_t device, hts_ctx *out) {
    if (!out) return fail(HTS_EINVAL, "hts_create: out is NULL");
    *out = nullptr;
    int ndev = 0;
    HTS_HIP(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev)
        return fail(HTS_EINVAL, "hts_create: device %d not in [0, %d)", device, ndev);
    HTS_HIP(hipSetDevice(device));
    hts_ctx c = new hts_ctx_s();
    c->device = device;
    for (Buffer *b : {&c->pts, &c->fattr, &c->frep, &c->zpart, &c->part, &c->spare}) b->gen = &c->gen;
    for (Buffer &b : c->aff) b.gen = &c->gen;
    hipError_t e = hipMalloc(&c->d_err, 64);
    if (e != hipSuccess) {
        delete c;
        return hip_fail(e, "hipMalloc(error word)");
    }
    e = hipMemset(c->d_err, 0, 64);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(c->d_err);
        delete c;
        return hip_fail(e, "hipMemset(error word)");
    }
    *out = c;
    return HTS_OK;
}

hts_status hts_destroy(hts_ctx c) {
    if (!c) return fail(HTS_EINVAL, "hts_destroy: ctx is NULL");
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    Buffer *bufs[] = {&c->pts, &c->fattr, &c->frep, &c->zpart, &c->part, &c->spare};
    for (Buffer *b : bufs)
        if (b->p) (void)hipFree(b->p);
    for (Buffer &b : c->aff)
        if (b.p) (void)hipFree(b.p);
    for (hipEvent_t e : c->timing.pool) (void)hipEventDestroy(e);
    (void)hipFree(c->d_err);
    delete c;
    return HTS_OK;
}

hts_status hts_check(hts_ctx c, hts_stream stream, uint32_t *bits_out) {
    if (!c) return fail(HTS_EINVAL, "hts_check: ctx is NULL");
    hipStream_t st = (hipStream_t)stream;
    uint32_t bits = 0;
    HTS_HIP(hipStreamSynchronize(st));
    HTS_HIP(hipMemcpy(&bits, c->d_err, sizeof(bits), hipMemcpyDeviceToHost));
    if (bits_out) *bits_out = bits;
    if (bits) {
        HTS_HIP(hipMemset(c->d_err, 0, sizeof(uint32_t)));
        return fail(HTS_ENUMERIC, "device error word 0x%x (1: non-finite gradient, 2: point outside the disk, 4: non-finite point)", bits);
    }
    return HTS_OK;
}

// ---------------------------------------------------------------- affinities
hts_status hts_build_affinities(hts_ctx c, hts_stream stream, const void *X, int64_t n, int32_t d,
                                int32_t x_dtype, double perplexity, int32_t k, int32_t *knn_idx,
                                int64_t *row_ptr, int32_t *col_idx, void *p_val, int32_t p_dtype,
                                int64_t cap_nnz, int64_t *nnz_out) {
    if (n < 2) return fail(HTS_EINVAL, "hts_build_affinities: n = %lld < 2", (long long)n);
    if (n > 0x7fffffff) return fail(HTS_EINVAL, "hts_build_affinities: n too large");
    if (d < 1) return fail(HTS_EINVAL, "hts_build_affinities: d = %d < 1", d);
    if (k < 1 || k >= n) return fail(HTS_EINVAL, "hts_build_affinities: k = %d not in [1, n)", k);
    if (k > 128) return fail(HTS_EINVAL, "hts_build_affinities: k = %d > 128", k);
    if (!(perplexity > 0.0) || !(perplexity < (double)k))
        return fail(HTS_EINVAL, "hts_build_affinities: perplexity %g not in (0, k)", perplexity);
    if (!dtype_ok(x_dtype) || !dtype_ok(p_dtype))
        return fail(HTS_EINVAL, "hts_build_affinities: bad dtype");
    if (!X || !row_ptr || !col_idx || !p_val || !nnz_out)
        return fail(HTS_EINVAL, "hts_build_affinities: NULL pointer argument");
    if (cap_nnz < 0) return fail(HTS_EINVAL, "hts_build_affinities: cap_nnz < 0");
    if (!c) return fail(HTS_EINVAL, "hts_build_affinities: ctx is NULL");
    HTS_HIP(hipSetDevice(c->device));
    return affinities(c, (hipStream_t)stream, X, n, d, x_dtype, perplexity, k, knn_idx, row_ptr,
                      col_idx, p_val, p_dtype, cap_nnz, nnz_out);
}

// ---------------------------------------------------------------- tree
hts_status hts_tree_create(hts_ctx c, int64_t n_max, int32_t max_depth, hts_tree *out) {
    if (!out) return fail(HTS_EINVAL, "hts_tree_create: out is NULL");
    *out = nullptr;
    if (n_max < 2) return fail(HTS_EINVAL, "hts_tree_create: n_max < 2");
    if (max_depth < 1 || max_depth > 24)
        return fail(HTS_EINVAL, "hts_tree_create: max_depth %d not in [1, 24]", max_depth);
    int64_t cap = n_max * (int64_t)(max_depth + 1) + 1;
    if (cap >= kMaxNodes)
        return fail(HTS_EINVAL, "hts_tree_create: n_max * (max_depth + 1) must stay below 2^26");
    if (!c) return fail(HTS_EINVAL, "hts_tree_create: ctx is NULL");
    HTS_HIP(hipSetDevice(c->device));
    hts_tree t = new hts_tree_s();
    t->ctx = c;
    t->device = c->device;
    t->n_max = n_max;
    t->max_depth = max_depth;
    t->cap_nodes = cap;
    t->nb = cdiv(n_max, kBlock);
    size_t nm = (size_t)n_max;
    const size_t nqb_max = (size_t)cdiv(n_max, kWave);
    struct A { void **p; size_t bytes; } allocs[] = {
        {(void **)&t->job_off, 2 * 8},
        {(void **)&t->job_qb, 2 * 4},
        {(void **)&t->qb_job, nqb_max * 4},
        {(void **)&t->pjob, nm * 4},
        {(void **)&t->root, 2 * 8},
        {(void **)&t->r, nm * 8},
        {(void **)&t->mm, (size_t)t->nb * 32},
        {(void **)&t->keys_in, nm * 8},
        {(void **)&t->keys, nm * 8},
        {(void **)&t->idx_in, nm * 4},
        {(void **)&t->perm, nm * 4},
        {(void **)&t->ncnt_part, (size_t)t->nb * 4},
        {(void **)&t->q_part, (size_t)t->nb * sizeof(DD3)},
        {(void **)&t->node_start, (nm + 1) * 4},
        {(void **)&t->psum, (nm + 1) * sizeof(DD3)},
        {(void **)&t->d_m, 64},
        {(void **)&t->spts, nm * sizeof(PointRec<double>)},
        {(void **)&t->nodes, (size_t)cap * sizeof(NodeRec<double>)},
        {(void **)&t->r_cell, (size_t)cap * 8},
        {(void **)&t->node_first, (size_t)cap * 4},
        {(void **)&t->sinhalf, 32 * 8},
    };
    hts_status s = HTS_OK;
    for (auto &a : allocs) {
        hipError_t e = hipMalloc(a.p, a.bytes);
        if (e != hipSuccess) {
            s = hip_fail(e, "hipMalloc(tree)");
            break;
        }
    }
    if (s == HTS_OK) s = tree_sort_bytes(n_max, max_depth, &t->sort_tmp_bytes);
    if (s == HTS_OK) {
        hipError_t e = hipMalloc(&t->sort_tmp, t->sort_tmp_bytes ? t->sort_tmp_bytes : 256);
        if (e != hipSuccess) s = hip_fail(e, "hipMalloc(sort)");
    }
    if (s == HTS_OK) {
        // sine of half the angular width of a depth-l cell, capped at 1 for
        // the two top levels (widths 2 pi and pi)
        double sh[32];
        for (int l = 0; l < 32; ++l) sh[l] = l <= 1 ? 1.0 : std::sin(M_PI / std::ldexp(1.0, l));
        hipError_t e = hipMemcpy(t->sinhalf, sh, sizeof(sh), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(t->d_m, 0, 64);
        // one job: every point and every query block belongs to job 0
        if (e == hipSuccess) e = hipMemset(t->pjob, 0, nm * 4);
        if (e == hipSuccess) e = hipMemset(t->qb_job, 0, nqb_max * 4);
        if (e == hipSuccess) e = hipDeviceSynchronize();
        if (e != hipSuccess) s = hip_fail(e, "tree init");
    }

    if (s != HTS_OK) {
        hts_tree_destroy(t);
        return s;
    }
    *out = t;
    return HTS_OK;
}

hts_status hts_tree_destroy(hts_tree t) {
    if (!t) return fail(HTS_EINVAL, "hts_tree_destroy: tree is NULL");
    (void)hipSetDevice(t->device);  // not through ctx, which may be destroyed already
    (void)hipDeviceSynchronize();
    void *ptrs[] = {t->job_off, t->job_qb, t->qb_job, t->pjob, t->root, t->r, t->mm,
                    t->keys_in, t->keys, t->idx_in, t->perm, t->sort_tmp, t->ncnt_part,
                    t->q_part, t->node_start, t->psum, t->d_m, t->spts, t->nodes, t->r_cell,
                    t->node_first, t->sinhalf, t->enodes, t->epsum, t->epart};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete t;
    return HTS_OK;
}

hts_status hts_tree_set_jobs(hts_tree t, int32_t n_jobs, const int64_t *n_per_job) {
    if (!t) return fail(HTS_EINVAL, "hts_tree_set_jobs: tree is NULL");
    if (n_jobs < 1 || n_jobs > (1 << 24))
        return fail(HTS_EINVAL, "hts_tree_set_jobs: n_jobs = %d not in [1, 2^24]", n_jobs);
    if (!n_per_job) return fail(HTS_EINVAL, "hts_tree_set_jobs: n_per_job is NULL");
    std::vector<int64_t> off((size_t)n_jobs + 1, 0);
    std::vector<int32_t> jqb((size_t)n_jobs + 1, 0);
    for (int32_t j = 0; j < n_jobs; ++j) {
        if (n_per_job[j] < 2)
            return fail(HTS_EINVAL, "hts_tree_set_jobs: job %d has %lld < 2 points", j,
                        (long long)n_per_job[j]);
        off[j + 1] = off[j] + n_per_job[j];
        if (off[j + 1] > t->n_max)
            return fail(HTS_EINVAL, "hts_tree_set_jobs: %lld points in all exceed n_max = %lld",
                        (long long)off[j + 1], (long long)t->n_max);
        jqb[j + 1] = jqb[j] + (int32_t)cdiv(n_per_job[j], kWave);
    }
    const int64_t n = off[n_jobs];
    const int64_t nqb = jqb[n_jobs];
    if (nqb > cdiv(t->n_max, kWave) + n_jobs)
        return fail(HTS_EINVAL, "hts_tree_set_jobs: too many query blocks");
    // the job index sits above the 2 max_depth cell bits of a 64-bit key
    int bits = 0;
    while ((1 << bits) < n_jobs) ++bits;
    if (bits + 2 * t->max_depth > 64)
        return fail(HTS_EINVAL,
                    "hts_tree_set_jobs: %d jobs need %d key bits above the %d cell bits of "
                    "max_depth %d; at most 64 in all",
                    n_jobs, bits, 2 * t->max_depth, t->max_depth);
    std::vector<int32_t> pj((size_t)n), qj((size_t)nqb);
    for (int32_t j = 0; j < n_jobs; ++j) {
        for (int64_t i = off[j]; i < off[j + 1]; ++i) pj[(size_t)i] = j;
        for (int32_t b = jqb[j]; b < jqb[j + 1]; ++b) qj[(size_t)b] = j;
    }
    HTS_HIP(hipSetDevice(t->ctx->device));
    HTS_HIP(hipDeviceSynchronize());
    void **tabs[] = {(void **)&t->job_off, (void **)&t->job_qb, (void **)&t->qb_job,
                     (void **)&t->root};
    const size_t bytes[] = {off.size() * 8, jqb.size() * 4,
                            (size_t)(nqb > cdiv(t->n_max, kWave) ? nqb : cdiv(t->n_max, kWave)) * 4,
                            (size_t)n_jobs * 16};
    ++t->ctx->gen;  // the tables below move
    for (int a = 0; a < 4; ++a) {
        HTS_HIP(hipFree(*tabs[a]));
        *tabs[a] = nullptr;
        HTS_HIP(hipMalloc(tabs[a], bytes[a]));
    }
    HTS_HIP(hipMemcpy(t->job_off, off.data(), off.size() * 8, hipMemcpyHostToDevice));
    HTS_HIP(hipMemcpy(t->job_qb, jqb.data(), jqb.size() * 4, hipMemcpyHostToDevice));
    HTS_HIP(hipMemcpy(t->qb_job, qj.data(), qj.size() * 4, hipMemcpyHostToDevice));
    HTS_HIP(hipMemcpy(t->pjob, pj.data(), pj.size() * 4, hipMemcpyHostToDevice));
    t->J = n_jobs;
    t->h_off = off;
    t->max_job = 0;
    for (int32_t j = 0; j < n_jobs; ++j)
        if (off[j + 1] - off[j] > t->max_job) t->max_job = off[j + 1] - off[j];
    t->nqb = nqb;
    t->jobs_set = true;
    t->tab_n = n;
    t->job_bits = bits;
    t->n = 0;  // nothing built for this layout yet
    return HTS_OK;
}

hts_status hts_tree_set_split(hts_tree t, int32_t split_rule) {
    if (!t) return fail(HTS_EINVAL, "hts_tree_set_split: tree is NULL");
    if (split_rule != 0 && split_rule != 1)
        return fail(HTS_EINVAL, "hts_tree_set_split: split_rule must be 0 or 1");
    t->split_rule = split_rule;
    t->n = 0;  // rebuild before the next traversal
    return HTS_OK;
}

hts_status hts_build_polar_tree(hts_ctx c, hts_stream stream, const void *Y, int64_t n,
                                int32_t y_dtype, hts_tree t) {
    if (!c || !t) return fail(HTS_EINVAL, "hts_build_polar_tree: NULL handle");
    if (t->ctx != c) return fail(HTS_EINVAL, "hts_build_polar_tree: tree belongs to another context");
    if (n < 2 || n > t->n_max)
        return fail(HTS_EINVAL, "hts_build_polar_tree: n = %lld not in [2, n_max = %lld]",
                    (long long)n, (long long)t->n_max);
    if (t->jobs_set && n != t->h_off.back())
        return fail(HTS_EINVAL, "hts_build_polar_tree: n = %lld, but the job layout holds %lld points",
                    (long long)n, (long long)t->h_off.back());
    if (!dtype_ok(y_dtype)) return fail(HTS_EINVAL, "hts_build_polar_tree: bad dtype");
    if (!Y) return fail(HTS_EINVAL, "hts_build_polar_tree: Y is NULL");
    HTS_HIP(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    if (y_dtype == HTS_F64) return tree_build<double>(c, st, (const double *)Y, n, t);
    return tree_build<float>(c, st, (const float *)Y, n, t);
}

}  // extern "C"
__global__ void k_export_nodes(const void *nodes, int dtype, const int32_t *d_m,
                               const double *r_cell, const int32_t *node_first, int64_t cap,
                               int32_t *count, int32_t *depth, int32_t *first, int32_t *next,
                               double *mid, double *rc) {
    int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int64_t M = *d_m;
    if (k >= M || k >= cap) return;
    int32_t cnt;
    uint32_t nxd;
    double mx, my;
    if (dtype == HTS_F64) {
        NodeRec<double> r = ((const NodeRec<double> *)nodes)[k];
        cnt = r.count; nxd = r.next_depth; mx = r.mx; my = r.my;
    } else {
        NodeRec<float> r = ((const NodeRec<float> *)nodes)[k];
        cnt = r.count; nxd = r.next_depth; mx = r.mx; my = r.my;
    }
    if (count) count[k] = cnt;
    if (depth) depth[k] = (int32_t)(nxd >> kNextBits);
    if (next) next[k] = (int32_t)(nxd & kNextMask);
    if (first) first[k] = node_first[k];
    if (mid) { mid[2 * k] = mx; mid[2 * k + 1] = my; }
    if (rc) rc[k] = r_cell[k];
}

__global__ void k_export_perm(const uint32_t *perm, int64_t n, int32_t *out) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = (int32_t)perm[i];
}

extern "C" hts_status hts_tree_export(hts_ctx c, hts_stream stream, hts_tree t, int64_t *n_nodes_out,
                           int64_t cap, int32_t *count, int32_t *depth, int32_t *first,
                           int32_t *next, double *mid, double *r_cell, int32_t *perm) {
    if (!c || !t || !n_nodes_out) return fail(HTS_EINVAL, "hts_tree_export: NULL argument");
    if (t->n < 2) return fail(HTS_EINVAL, "hts_tree_export: the tree has not been built");
    HTS_HIP(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    int32_t M = 0;
    HTS_HIP(hipMemcpyAsync(&M, t->d_m, sizeof(M), hipMemcpyDeviceToHost, st));
    HTS_HIP(hipStreamSynchronize(st));
    *n_nodes_out = M;
    bool any = count || depth || first || next || mid || r_cell;
    if (any && M > cap) return fail(HTS_ECAPACITY, "hts_tree_export: %d nodes > cap %lld", M, (long long)cap);
    if (any) {
        hipLaunchKernelGGL(k_export_nodes, dim3(cdiv(M, kBlock)), dim3(kBlock), 0, st, t->nodes,
                           t->dtype, t->d_m, t->r_cell, t->node_first, cap, count, depth, first,
                           next, mid, r_cell);
        HTS_HIP(hipGetLastError());
    }
    if (perm) {
        hipLaunchKernelGGL(k_export_perm, dim3(cdiv(t->n, kBlock)), dim3(kBlock), 0, st, t->perm,
                           t->n, perm);
        HTS_HIP(hipGetLastError());
    }
    HTS_HIP(hipStreamSynchronize(st));
    return HTS_OK;
}

// ---------------------------------------------------------------- gradients
static hts_status grad_args(const char *fn, hts_ctx c, const void *Y, int64_t n, int32_t dtype,
                            const int64_t *rp, const int32_t *col, const void *val, double ex,
                            void *grad, double *z_dev) {
    if (n < 2) return fail(HTS_EINVAL, "%s: n = %lld < 2", fn, (long long)n);
    if (n > 0x7fffffff) return fail(HTS_EINVAL, "%s: n too large", fn);
    if (!dtype_ok(dtype)) return fail(HTS_EINVAL, "%s: bad dtype %d", fn, dtype);
    if (!(ex > 0.0) || !std::isfinite(ex)) return fail(HTS_EINVAL, "%s: exaggeration %g must be > 0", fn, ex);
    if (!Y || !rp || !col || !val || !grad || !z_dev) return fail(HTS_EINVAL, "%s: NULL pointer argument", fn);
    if (!c) return fail(HTS_EINVAL, "%s: ctx is NULL", fn);
    return HTS_OK;
}

template <typename T>
static hts_status exact_ws_grow(hts_ctx c, int64_t n, bool kl, ExactWs &w) {
    HTS_OKR(ensure(c->pts, (size_t)n * sizeof(PointRec<T>)));
    HTS_OKR(ensure(c->fattr, (size_t)n * 2 * sizeof(T)));
    HTS_OKR(ensure(c->frep, (size_t)n * 2 * sizeof(double)));
    HTS_OKR(ensure(c->zpart, (size_t)(cdiv(n, kBlock) + 8) * sizeof(double)));
    HTS_OKR(ensure(c->part, exact_part_bytes(n)));
    if (kl) HTS_OKR(ensure(c->spare, (size_t)kl_parts(n) * sizeof(double)));
    w.pts = c->pts.p;
    w.fattr = c->fattr.p;
    w.frep = (double *)c->frep.p;
    w.zpart = (double *)c->zpart.p;
    w.part = (double *)c->part.p;
    w.klpart = kl ? (double *)c->spare.p : nullptr;
    return HTS_OK;
}

extern "C" hts_status hts_gradient_exact(hts_ctx c, hts_stream stream, const void *Y, int64_t n,
                              int32_t dtype, const int64_t *row_ptr, const int32_t *col_idx,
                              const void *p_val, double exaggeration, void *grad, double *z_dev,
                              double *kl_dev) {
    HTS_OKR(grad_args("hts_gradient_exact", c, Y, n, dtype, row_ptr, col_idx, p_val, exaggeration,
                      grad, z_dev));
    HTS_HIP(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    ExactWs w;
    if (dtype == HTS_F64) {
        HTS_OKR(exact_ws_grow<double>(c, n, kl_dev != nullptr, w));
        return exact_impl<double>(c, st, (const double *)Y, n, row_ptr, col_idx,
                                  (const double *)p_val, exaggeration, (double *)grad, z_dev,
                                  kl_dev, w, true);
    }
    HTS_OKR(exact_ws_grow<float>(c, n, kl_dev != nullptr, w));
    return exact_impl<float>(c, st, (const float *)Y, n, row_ptr, col_idx, (const float *)p_val,
                             exaggeration, (float *)grad, z_dev, kl_dev, w, true);
}

template <typename T>
static hts_status bh_impl(hts_ctx c, hipStream_t st, const T *Y, int64_t n, const int64_t *rp,
                          const int32_t *col, const T *val, double ex, const double *ex_job,
                          hts_tree t, double theta, T *grad, double *z_dev, uint64_t *stats) {
    HTS_OKR(ensure(c->pts, (size_t)n * sizeof(PointRec<T>)));
    HTS_OKR(ensure(c->fattr, (size_t)n * 2 * sizeof(T)));
    PointRec<T> *pts = (PointRec<T> *)c->pts.p;
    return launch_bh_repulsion<T, 0>(c, st, t, n, BhPrep<T>{Y, theta, true, true}, pts, rp, col,
                                     val, (T *)c->fattr.p, ex, ex_job, false, 1.0, grad, z_dev,
                                     stats);
}

static hts_status bh_tree_args(const char *fn, hts_ctx c, hts_tree t, int64_t n, int32_t dtype,
                               double theta) {
    if (!(theta >= 0.0) || !std::isfinite(theta))
        return fail(HTS_EINVAL, "%s: theta %g must be finite and >= 0", fn, theta);
    if (!t) return fail(HTS_EINVAL, "%s: tree is NULL", fn);
    if (t->ctx != c) return fail(HTS_EINVAL, "%s: tree belongs to another context", fn);
    if (t->n != n) return fail(HTS_EINVAL, "%s: tree was built for n = %lld, not %lld", fn,
                               (long long)t->n, (long long)n);
    if (t->dtype != dtype) return fail(HTS_EINVAL, "%s: tree built with another dtype", fn);
    return HTS_OK;
}

extern "C" {
hts_status hts_gradient_bh(hts_ctx c, hts_stream stream, const void *Y, int64_t n, int32_t dtype,
                           const int64_t *row_ptr, const int32_t *col_idx, const void *p_val,
                           double exaggeration, hts_tree t, double theta, void *grad,
                           double *z_dev, uint64_t *stats_dev) {
    HTS_OKR(grad_args("hts_gradient_bh", c, Y, n, dtype, row_ptr, col_idx, p_val, exaggeration,
                      grad, z_dev));
    HTS_OKR(bh_tree_args("hts_gradient_bh", c, t, n, dtype, theta));
    if (t->J != 1)
        return fail(HTS_EINVAL, "hts_gradient_bh: the tree holds %d jobs; use hts_gradient_bh_jobs", t->J);
    HTS_HIP(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    if (dtype == HTS_F64)
        return bh_impl<double>(c, st, (const double *)Y, n, row_ptr, col_idx, (const double *)p_val,
                               exaggeration, nullptr, t, theta, (double *)grad, z_dev, stats_dev);
    return bh_impl<float>(c, st, (const float *)Y, n, row_ptr, col_idx, (const float *)p_val,
                          exaggeration, nullptr, t, theta, (float *)grad, z_dev, stats_dev);
}

hts_status hts_gradient_bh_jobs(hts_ctx c, hts_stream stream, const void *Y, int64_t n,
                                int32_t dtype, const int64_t *row_ptr, const int32_t *col_idx,
                                const void *p_val, const double *exaggeration_dev, hts_tree t,
                                double theta, void *grad, double *z_dev, uint64_t *stats_dev) {
    HTS_OKR(grad_args("hts_gradient_bh_jobs", c, Y, n, dtype, row_ptr, col_idx, p_val, 1.0, grad,
                      z_dev));
    HTS_OKR(bh_tree_args("hts_gradient_bh_jobs", c, t, n, dtype, theta));
    if (!exaggeration_dev) return fail(HTS_EINVAL, "hts_gradient_bh_jobs: exaggeration_dev is NULL");
    HTS_HIP(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    if (dtype == HTS_F64)
        return bh_impl<double>(c, st, (const double *)Y, n, row_ptr, col_idx, (const double *)p_val,
                               1.0, exaggeration_dev, t, theta, (double *)grad, z_dev, stats_dev);
    return bh_impl<float>(c, st, (const float *)Y, n, row_ptr, col_idx, (const float *)p_val, 1.0,
                          exaggeration_dev, t, theta, (float *)grad, z_dev, stats_dev);
}

// ---------------------------------------------------------------- h-SNE
}  // extern "C"

static hts_status tree_euclid_alloc(hts_tree t) {
    if (t->enodes) return HTS_OK;
    struct A { void **p; size_t bytes; } allocs[] = {
        {(void **)&t->enodes, (size_t)t->cap_nodes * sizeof(NodeRec<double>)},
        {(void **)&t->epsum, ((size_t)t->n_max + 1) * sizeof(DD2)},
        {(void **)&t->epart, (size_t)t->nb * sizeof(DD2)},
    };
    for (auto &a : allocs) {
        hipError_t e = hipMalloc(a.p, a.bytes);
        if (e != hipSuccess) {
            for (auto &b : allocs)
                if (*b.p) {
                    (void)hipFree(*b.p);
                    *b.p = nullptr;
                }
            return hip_fail(e, "hipMalloc(euclidean nodes)");
        }
    }
    return HTS_OK;
}

template <typename T>
static hts_status hsne_impl(hts_ctx c, hipStream_t st, const T *Y, int64_t n, const int64_t *rp,
                            const int32_t *col, const T *val, double ex, double lambda,
                            hts_tree t, double theta, T *grad, double *z_dev, uint64_t *stats) {
    HTS_OKR(tree_euclid_alloc(t));
    HTS_OKR(ensure(c->pts, (size_t)n * sizeof(PointRec<T>)));
    HTS_OKR(ensure(c->fattr, (size_t)n * 2 * sizeof(T)));
    PointRec<T> *pts = (PointRec<T> *)c->pts.p;
    T *fattr = (T *)c->fattr.p;
    HTS_OKR(tree_euclid<T>(c, st, t, theta));
    // Euclidean part into grad (its launch writes the point records), then
    // grad + lambda (hyperbolic part) (its launch sets the node thresholds)
    HTS_OKR((launch_bh_repulsion<T, 1>(c, st, t, n, BhPrep<T>{Y, theta, true, false}, pts, rp, col,
                                       val, fattr, ex, nullptr, false, 1.0, grad, z_dev, stats)));
    return launch_bh_repulsion<T, 0>(c, st, t, n, BhPrep<T>{Y, theta, false, true}, pts, rp, col,
                                     val, fattr, ex, nullptr, true, lambda, grad, z_dev + 1,
                                     stats ? stats + 2 * kBhStats : nullptr);
}

extern "C" {
hts_status hts_gradient_hsne(hts_ctx c, hts_stream stream, const void *Y, int64_t n, int32_t dtype,
                             const int64_t *row_ptr, const int32_t *col_idx, const void *p_val,
                             double exaggeration, double lambda, hts_tree t, double theta,
                             void *grad, double *z_dev, uint64_t *stats_dev) {
    HTS_OKR(grad_args("hts_gradient_hsne", c, Y, n, dtype, row_ptr, col_idx, p_val, exaggeration,
                      grad, z_dev));
    HTS_OKR(bh_tree_args("hts_gradient_hsne", c, t, n, dtype, theta));
    if (t->J != 1)
        return fail(HTS_EINVAL, "hts_gradient_hsne: the tree holds %d jobs; one is supported", t->J);
    if (!(lambda >= 0.0) || !std::isfinite(lambda))
        return fail(HTS_EINVAL, "hts_gradient_hsne: lambda %g must be finite and >= 0", lambda);
    HTS_HIP(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    if (dtype == HTS_F64)
        return hsne_impl<double>(c, st, (const double *)Y, n, row_ptr, col_idx,
                                 (const double *)p_val, exaggeration, lambda, t, theta,
                                 (double *)grad, z_dev, stats_dev);
    return hsne_impl<float>(c, st, (const float *)Y, n, row_ptr, col_idx, (const float *)p_val,
                            exaggeration, lambda, t, theta, (float *)grad, z_dev, stats_dev);
}

// ---------------------------------------------------------------- CO-SNE
hts_status hts_cosne_terms(hts_ctx c, hts_stream stream, const void *Y, int64_t n, int32_t dtype,
                           const double *xnorm2, double lambda1, double lambda2, void *grad) {
    if (!c) return fail(HTS_EINVAL, "hts_cosne_terms: ctx is NULL");
    if (n < 1) return fail(HTS_EINVAL, "hts_cosne_terms: n < 1");
    if (!dtype_ok(dtype)) return fail(HTS_EINVAL, "hts_cosne_terms: bad dtype");
    if (!Y || !xnorm2 || !grad) return fail(HTS_EINVAL, "hts_cosne_terms: NULL pointer argument");
    if (!std::isfinite(lambda1) || !std::isfinite(lambda2) || lambda2 < 0.0)
        return fail(HTS_EINVAL, "hts_cosne_terms: lambda1 must be finite and lambda2 >= 0");
    HTS_HIP(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    if (dtype == HTS_F64)
        return launch_cosne<double>(c, st, (const double *)Y, n, xnorm2, lambda1, lambda2,
                                    (double *)grad);
    return launch_cosne<float>(c, st, (const float *)Y, n, xnorm2, lambda1, lambda2, (float *)grad);
}

// ---------------------------------------------------------------- iteration
}  // extern "C"

// One iteration: tree, gradient and step, as the three calls make them.
template <typename T>
static hts_status iteration_impl(hts_ctx c, hipStream_t st, T *Y, T *U, T *G, int64_t n,
                                 const int64_t *rp, const int32_t *col, const T *val, double ex,
                                 hts_tree t, double theta, T *grad, double *z_dev, double eta,
                                 double momentum, double min_gain, double boundary_eps,
                                 int32_t metric_power) {
    // the gradient's workspaces first, so that the tree build can do the work
    // of the gradient's preparation launch (point records, thresholds, the
    // item-list counter), which is then left out
    HTS_OKR(tree_single_job(st, t, n));
    HTS_OKR(ensure(c->pts, (size_t)n * sizeof(PointRec<T>)));
    HTS_OKR(ensure(c->fattr, (size_t)n * 2 * sizeof(T)));
    unsigned *counter = nullptr;
    HTS_OKR(bh_item_counter<T>(c, t, n, &counter));
    PointRec<T> *pts = (PointRec<T> *)c->pts.p;
    const TreeExtras<T> extras{pts, theta, counter};
    HTS_OKR(tree_build<T>(c, st, Y, n, t, &extras));
    HTS_OKR((launch_bh_repulsion<T, 0>(c, st, t, n, BhPrep<T>{Y, theta, false, false, false}, pts, rp,
                                       col, val, (T *)c->fattr.p, ex, nullptr, false, 1.0, grad,
                                       z_dev, nullptr)));
    return launch_step<T>(c, st, Y, U, G, grad, n, eta, momentum, nullptr, nullptr, nullptr,
                          min_gain, boundary_eps, metric_power);
}

extern "C" {
hts_status hts_iteration_bh(hts_ctx c, hts_stream stream, void *Y, void *update, void *gains,
                            int64_t n, int32_t dtype, const int64_t *row_ptr,
                            const int32_t *col_idx, const void *p_val, double exaggeration,
                            hts_tree t, double theta, void *grad, double *z_dev, double eta,
                            double momentum, double min_gain, double boundary_eps,
                            int32_t metric_power) {
    HTS_OKR(grad_args("hts_iteration_bh", c, Y, n, dtype, row_ptr, col_idx, p_val, exaggeration,
                      grad, z_dev));
    if (!(theta >= 0.0) || !std::isfinite(theta))
        return fail(HTS_EINVAL, "hts_iteration_bh: theta %g must be finite and >= 0", theta);
    if (!t) return fail(HTS_EINVAL, "hts_iteration_bh: tree is NULL");
    if (t->ctx != c) return fail(HTS_EINVAL, "hts_iteration_bh: tree belongs to another context");
    if (t->jobs_set && t->J != 1)
        return fail(HTS_EINVAL, "hts_iteration_bh: the tree holds a layout of %d jobs", t->J);
    if (n < 2 || n > t->n_max)
        return fail(HTS_EINVAL, "hts_iteration_bh: n = %lld not in [2, n_max = %lld]", (long long)n,
                    (long long)t->n_max);
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(HTS_EINVAL, "hts_iteration_bh: eta must be > 0");
    if (!(momentum >= 0.0) || !(momentum < 1.0))
        return fail(HTS_EINVAL, "hts_iteration_bh: momentum not in [0, 1)");
    if (!(min_gain >= 0.0)) return fail(HTS_EINVAL, "hts_iteration_bh: min_gain < 0");
    if (!(boundary_eps > 0.0) || !(boundary_eps < 1.0))
        return fail(HTS_EINVAL, "hts_iteration_bh: boundary_eps not in (0, 1)");
    if (metric_power != 1 && metric_power != 2)
        return fail(HTS_EINVAL, "hts_iteration_bh: metric_power must be 1 or 2");
    if (!update || !gains) return fail(HTS_EINVAL, "hts_iteration_bh: NULL pointer argument");
    HTS_HIP(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    if (dtype == HTS_F64)
        return iteration_impl<double>(c, st, (double *)Y, (double *)update, (double *)gains, n,
                                      row_ptr, col_idx, (const double *)p_val, exaggeration, t,
                                      theta, (double *)grad, z_dev, eta, momentum, min_gain,
                                      boundary_eps, metric_power);
    return iteration_impl<float>(c, st, (float *)Y, (float *)update, (float *)gains, n, row_ptr,
                                 col_idx, (const float *)p_val, exaggeration, t, theta,
                                 (float *)grad, z_dev, eta, momentum, min_gain, boundary_eps,
                                 metric_power);
}

// ---------------------------------------------------------------- step
hts_status hts_step(hts_ctx c, hts_stream stream, void *Y, void *update, void *gains,
                    const void *grad, int64_t n, int32_t dtype, double eta, double momentum,
                    double min_gain, double boundary_eps, int32_t metric_power) {
    if (n < 1) return fail(HTS_EINVAL, "hts_step: n < 1");
    if (!dtype_ok(dtype)) return fail(HTS_EINVAL, "hts_step: bad dtype");
    if (!(eta > 0.0) || !std::isfinite(eta)) return fail(HTS_EINVAL, "hts_step: eta must be > 0");
    if (!(momentum >= 0.0) || !(momentum < 1.0)) return fail(HTS_EINVAL, "hts_step: momentum not in [0, 1)");
    if (!(min_gain >= 0.0)) return fail(HTS_EINVAL, "hts_step: min_gain < 0");
    if (!(boundary_eps > 0.0) || !(boundary_eps < 1.0)) return fail(HTS_EINVAL, "hts_step: boundary_eps not in (0, 1)");
    if (metric_power != 1 && metric_power != 2) return fail(HTS_EINVAL, "hts_step: metric_power must be 1 or 2");
    if (!Y || !update || !gains || !grad) return fail(HTS_EINVAL, "hts_step: NULL pointer argument");
    if (!c) return fail(HTS_EINVAL, "hts_step: ctx is NULL");
    HTS_HIP(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    if (dtype == HTS_F64)
        return launch_step<double>(c, st, (double *)Y, (double *)update, (double *)gains,
                                   (const double *)grad, n, eta, momentum, nullptr, nullptr,
                                   nullptr, min_gain, boundary_eps, metric_power);
    return launch_step<float>(c, st, (float *)Y, (float *)update, (float *)gains,
                              (const float *)grad, n, eta, momentum, nullptr, nullptr, nullptr,
                              min_gain, boundary_eps, metric_power);
}

hts_status hts_step_jobs(hts_ctx c, hts_stream stream, hts_tree t, void *Y, void *update,
                         void *gains, const void *grad, int64_t n, int32_t dtype,
                         const double *eta_dev, const double *momentum_dev, double min_gain,
                         double boundary_eps, int32_t metric_power) {
    if (!t) return fail(HTS_EINVAL, "hts_step_jobs: tree is NULL");
    if (!dtype_ok(dtype)) return fail(HTS_EINVAL, "hts_step_jobs: bad dtype");
    if (t->h_off.empty() || !t->jobs_set || n != t->h_off.back())
        return fail(HTS_EINVAL, "hts_step_jobs: n = %lld does not match the tree's job layout",
                    (long long)n);
    if (!(min_gain >= 0.0)) return fail(HTS_EINVAL, "hts_step_jobs: min_gain < 0");
    if (!(boundary_eps > 0.0) || !(boundary_eps < 1.0)) return fail(HTS_EINVAL, "hts_step_jobs: boundary_eps not in (0, 1)");
    if (metric_power != 1 && metric_power != 2) return fail(HTS_EINVAL, "hts_step_jobs: metric_power must be 1 or 2");
    if (!Y || !update || !gains || !grad || !eta_dev || !momentum_dev)
        return fail(HTS_EINVAL, "hts_step_jobs: NULL pointer argument");
    if (!c) return fail(HTS_EINVAL, "hts_step_jobs: ctx is NULL");
    if (t->ctx != c) return fail(HTS_EINVAL, "hts_step_jobs: tree belongs to another context");
    HTS_HIP(hipSetDevice(c->device));
    hipStream_t st = (hipStream_t)stream;
    if (dtype == HTS_F64)
        return launch_step<double>(c, st, (double *)Y, (double *)update, (double *)gains,
                                   (const double *)grad, n, 0.0, 0.0, t->pjob, eta_dev,
                                   momentum_dev, min_gain, boundary_eps, metric_power);
    return launch_step<float>(c, st, (float *)Y, (float *)update, (float *)gains,
                              (const float *)grad, n, 0.0, 0.0, t->pjob, eta_dev, momentum_dev,
                              min_gain, boundary_eps, metric_power);
}

// ---------------------------------------------------------------- schedule
}  // extern "C"
__global__ void k_jobs_schedule(int32_t J, int32_t *__restrict__ it, int32_t ee_iters, double ex,
                                double mu_early, double mu_late, double *__restrict__ ex_out,
                                double *__restrict__ mu_out) {
    const int j = (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (j >= J) return;
    const int32_t k = it[j];
    const bool early = k < ee_iters;
    ex_out[j] = early ? ex : 1.0;
    mu_out[j] = early ? mu_early : mu_late;
    it[j] = k + 1;
}

extern "C" {
hts_status hts_jobs_schedule(hts_ctx c, hts_stream stream, int32_t n_jobs, int32_t *it_dev,
                             int32_t ee_iters, double exaggeration, double momentum_early,
                             double momentum_late, double *exaggeration_dev, double *momentum_dev) {
    if (!c) return fail(HTS_EINVAL, "hts_jobs_schedule: ctx is NULL");
    if (n_jobs < 1) return fail(HTS_EINVAL, "hts_jobs_schedule: n_jobs < 1");
    if (!it_dev || !exaggeration_dev || !momentum_dev)
        return fail(HTS_EINVAL, "hts_jobs_schedule: NULL pointer argument");
    if (!(exaggeration > 0.0)) return fail(HTS_EINVAL, "hts_jobs_schedule: exaggeration must be > 0");
    if (!(momentum_early >= 0.0 && momentum_early < 1.0 && momentum_late >= 0.0 && momentum_late < 1.0))
        return fail(HTS_EINVAL, "hts_jobs_schedule: momentum not in [0, 1)");
    HTS_HIP(hipSetDevice(c->device));
    hipLaunchKernelGGL(k_jobs_schedule, dim3(cdiv(n_jobs, kBlock)), dim3(kBlock), 0,
                       (hipStream_t)stream, n_jobs, it_dev, ee_iters, exaggeration, momentum_early,
                       momentum_late, exaggeration_dev, momentum_dev);
    HTS_HIP(hipGetLastError());
    return HTS_OK;
}

// ---------------------------------------------------------------- tuning
hts_status hts_set_item_points(hts_ctx c, int32_t item_points) {
    if (!c) return fail(HTS_EINVAL, "hts_set_item_points: ctx is NULL");
    if (item_points < 1) return fail(HTS_EINVAL, "hts_set_item_points: item_points must be >= 1");
    c->item_points = item_points;
    return HTS_OK;
}

hts_status hts_set_item_list(hts_ctx c, int32_t items_per_wave) {
    if (!c) return fail(HTS_EINVAL, "hts_set_item_list: ctx is NULL");
    if (items_per_wave < 0)
        return fail(HTS_EINVAL, "hts_set_item_list: items_per_wave must be >= 0");
    c->list_items = items_per_wave;
    return HTS_OK;
}

hts_status hts_set_traversal_launch(hts_ctx c, int32_t workgroups, int32_t waves_per_workgroup) {
    if (!c) return fail(HTS_EINVAL, "hts_set_traversal_launch: ctx is NULL");
    if (workgroups < 0)
        return fail(HTS_EINVAL, "hts_set_traversal_launch: workgroups must be >= 0 (0: automatic)");
    if (waves_per_workgroup != 1 && waves_per_workgroup != 2 && waves_per_workgroup != 4)
        return fail(HTS_EINVAL, "hts_set_traversal_launch: waves_per_workgroup must be 1, 2 or 4");
    c->items_grid = workgroups;
    c->items_waves = waves_per_workgroup;
    return HTS_OK;
}

hts_status hts_set_attract_launch(hts_ctx c, int32_t where) {
    if (!c) return fail(HTS_EINVAL, "hts_set_attract_launch: ctx is NULL");
    if (where < 0 || where > 2)
        return fail(HTS_EINVAL, "hts_set_attract_launch: where = %d not 0 (automatic), 1 or 2", where);
    c->attract_at = where;
    return HTS_OK;
}

hts_status hts_workspace_generation(hts_ctx c, uint64_t *gen_out) {
    if (!c || !gen_out) return fail(HTS_EINVAL, "hts_workspace_generation: NULL argument");
    *gen_out = c->gen;
    return HTS_OK;
}

// ---------------------------------------------------------------- timing
hts_status hts_timing_enable(hts_ctx c, int32_t on) {
    if (!c) return fail(HTS_EINVAL, "hts_timing_enable: ctx is NULL");
    c->timing.on = on != 0;
    return HTS_OK;
}

hts_status hts_timing_read(hts_ctx c, double *ms_out, int64_t *launches_out) {
    if (!c || !ms_out || !launches_out) return fail(HTS_EINVAL, "hts_timing_read: NULL argument");
    Timing &tm = c->timing;
    for (auto &r : tm.recs) {
        HTS_HIP(hipEventSynchronize(r.b));
        float ms = 0.f;
        HTS_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        if (r.cls >= 0 && r.cls < HTS_KCLASS_COUNT) {
            ms_out[r.cls] += ms;
            launches_out[r.cls] += 1;
        }
    }
    tm.recs.clear();
    tm.used = 0;
    return HTS_OK;
}

}  // extern "C"
