// k_grad.hip -- gradient kernels: point records, attractive CSR sum, exact
// repulsion, Z reduction + combine, and the Riemannian step.
#include "hts_impl.hpp"
#include "hts_math.hpp"

namespace hts {

// ---------------------------------------------------------------- points
// PointRec with ia = 1 / (1 - |y|^2) in double (the conformal factor of
// eq. (7) is lambda = 2 ia).  Flags points outside the open disk.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_prep_points(const T *__restrict__ Y, int64_t n,
                                                        PointRec<T> *__restrict__ pts,
                                                        uint32_t *__restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i < n) prep_point<T>(Y, i, pts, err);
}

template <typename T>
hts_status launch_prep_points(hts_ctx ctx, hipStream_t st, const T *Y, int64_t n, PointRec<T> *pts) {
    hipLaunchKernelGGL(k_prep_points<T>, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, Y, n, pts,
                       ctx->d_err);
    HTS_HIP(hipGetLastError());
    return HTS_OK;
}

// ---------------------------------------------------------------- attraction
// First sum of eq. (15) on its own (the exact path; the Barnes-Hut path runs
// the same rows inside the first traversal launch).
template <typename T, int G>
__global__ __launch_bounds__(kBlock) void k_attract(const PointRec<T> *__restrict__ pts,
                                                    const int64_t *__restrict__ rp,
                                                    const int32_t *__restrict__ col,
                                                    const T *__restrict__ val, int64_t n,
                                                    T *__restrict__ fattr,
                                                    uint32_t *__restrict__ err) {
    attract_rows<T, G>((int64_t)blockIdx.x * kBlock + threadIdx.x, pts, rp, col, val, n, fattr, err);
}

template <typename T>
hts_status launch_attract(hts_ctx ctx, hipStream_t st, const PointRec<T> *pts, const int64_t *rp,
                          const int32_t *col, const T *val, int64_t n, T *fattr, bool timed) {
    constexpr int G = 16;
    TimedScope ts(timed ? ctx : nullptr, st, HTS_K_ATTRACT);
    hipLaunchKernelGGL((k_attract<T, G>), dim3(cdiv(n * G, kBlock)), dim3(kBlock), 0, st, pts, rp,
                       col, val, n, fattr, ctx->d_err);
    HTS_HIP(hipGetLastError());
    return HTS_OK;
}

// ---------------------------------------------------------------- exact
// Second sum of eq. (15) and Z over all pairs.  A lane owns a query point;
// the j loop is uniform across the wave, so the other point's record comes
// through scalar loads.  Short runs of j accumulate in T, then in double.
// blockIdx.y selects a chunk of j so that enough waves exist to fill the chip.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_exact(const PointRec<T> *__restrict__ pts, int64_t n,
                                                  int64_t chunk_len, double *__restrict__ part) {
    constexpr int kRun = 256;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    bool valid = i < n;
    PointRec<T> q = pts[valid ? i : 0];
    int64_t j0 = (int64_t)blockIdx.y * chunk_len;
    int64_t j1 = j0 + chunk_len < n ? j0 + chunk_len : n;
    double Fx = 0.0, Fy = 0.0, Z = 0.0;
    for (int64_t jt = j0; jt < j1; jt += kRun) {
        int64_t je = jt + kRun < j1 ? jt + kRun : j1;
        T fx = 0, fy = 0;
        double z = 0.0;
        for (int64_t j = jt; j < je; ++j) {
            PointRec<T> o = pts[j];
            double dd;
            double t = dist_arg<T>(q.x, q.y, q.ia, o.x, o.y, o.ia, dd);
            PairTerm<T> r = pair_term<T>(q.x, q.y, q.ia, o.x, o.y, o.ia, t, dd);
            bool self = (j == i);
            T coef = self ? (T)0 : r.w * r.w * r.base;
            fx += coef * r.vx;
            fy += coef * r.vy;
            z += self ? 0.0 : (double)r.w;
        }
        Fx += (double)fx;
        Fy += (double)fy;
        Z += z;
    }
    if (valid) {
        int64_t o = ((int64_t)blockIdx.y * n + i) * 3;
        part[o] = Fx;
        part[o + 1] = Fy;
        part[o + 2] = Z;
    }
}

// per point: sum the chunks in order; per block: partial of Z
__global__ __launch_bounds__(kBlock) void k_exact_reduce(const double *__restrict__ part, int64_t n,
                                                         int nchunks, double *__restrict__ frep,
                                                         double *__restrict__ zpart) {
    __shared__ double sh[kBlock];
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    double z = 0.0;
    if (i < n) {
        double fx = 0.0, fy = 0.0;
        for (int c = 0; c < nchunks; ++c) {
            int64_t o = ((int64_t)c * n + i) * 3;
            fx += part[o];
            fy += part[o + 1];
            z += part[o + 2];
        }
        frep[2 * i] = fx;
        frep[2 * i + 1] = fy;
    }
    sh[threadIdx.x] = z;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) zpart[blockIdx.x] = sh[0];
}

// chunks of j per query block: about 8 waves per SIMD on 256 CUs x 4 SIMDs
static void exact_chunks(int64_t n, int64_t &nchunks, int64_t &chunk_len) {
    const int64_t qblocks = cdiv(n, kBlock);
    nchunks = cdiv(8192, qblocks * (kBlock / kWave));
    if (nchunks < 1) nchunks = 1;
    if (nchunks > 64) nchunks = 64;
    if (nchunks > n) nchunks = n;
    chunk_len = cdiv(n, nchunks);
    nchunks = cdiv(n, chunk_len);
}

size_t exact_part_bytes(int64_t n) {
    int64_t nchunks, chunk_len;
    exact_chunks(n, nchunks, chunk_len);
    return (size_t)(nchunks * n * 3) * sizeof(double);
}

template <typename T>
hts_status launch_exact(hts_ctx ctx, hipStream_t st, const PointRec<T> *pts, int64_t n,
                        double *part, double *frep, double *zpart, int64_t *nz_out, bool timed) {
    const int64_t qblocks = cdiv(n, kBlock);
    int64_t nchunks, chunk_len;
    exact_chunks(n, nchunks, chunk_len);
    {
        TimedScope ts(timed ? ctx : nullptr, st, HTS_K_EXACT);
        hipLaunchKernelGGL(k_exact<T>, dim3(qblocks, nchunks), dim3(kBlock), 0, st, pts, n,
                           chunk_len, part);
        HTS_HIP(hipGetLastError());
    }
    hipLaunchKernelGGL(k_exact_reduce, dim3(qblocks), dim3(kBlock), 0, st, part, n, (int)nchunks,
                       frep, zpart);
    HTS_HIP(hipGetLastError());
    *nz_out = qblocks;
    return HTS_OK;
}

// ---------------------------------------------------------------- combine
// Z = sum of the partials in a fixed order (every block repeats the same
// reduction, so no global synchronisation is needed), then
// g_i = 4 (a F_attr,i - F_rep,i / Z).
template <typename T, typename FR>
__global__ __launch_bounds__(kBlock) void k_finalize(const T *__restrict__ fattr,
                                                     const FR *__restrict__ frep,
                                                     const double *__restrict__ zpart, int64_t nz,
                                                     int64_t n, double ex, T *__restrict__ grad,
                                                     double *__restrict__ z_dev,
                                                     uint32_t *__restrict__ err) {
    __shared__ double sh[kBlock];
    double s = 0.0;
    for (int64_t a = threadIdx.x; a < nz; a += kBlock) s += zpart[a];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    double Z = sh[0];
    if (blockIdx.x == 0 && threadIdx.x == 0) *z_dev = Z;
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    double inv = 1.0 / Z;
    double gx = 4.0 * (ex * (double)fattr[2 * i] - (double)frep[2 * i] * inv);
    double gy = 4.0 * (ex * (double)fattr[2 * i + 1] - (double)frep[2 * i + 1] * inv);
    T ox = (T)gx, oy = (T)gy;
    if (!isfinite(ox) || !isfinite(oy)) atomicOr(err, HTS_ERR_NONFINITE_GRAD);
    grad[2 * i] = ox;
    grad[2 * i + 1] = oy;
}

template <typename T, typename FR>
hts_status launch_finalize(hts_ctx ctx, hipStream_t st, const T *fattr, const FR *frep,
                           const double *zpart, int64_t nz, int64_t n, double ex, T *grad,
                           double *z_dev, bool timed) {
    TimedScope ts(timed ? ctx : nullptr, st, HTS_K_FINALIZE);
    hipLaunchKernelGGL((k_finalize<T, FR>), dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, fattr, frep,
                       zpart, nz, n, ex, grad, z_dev, ctx->d_err);
    HTS_HIP(hipGetLastError());
    return HTS_OK;
}

// ---------------------------------------------------------------- cost
// The cost of eq. (3) with q_ij = w_ij / Z (eq. (12)), evaluated over the
// non-zeros of P:  C = sum_ij a p_ij (ln(a p_ij) - ln w_ij) + ln Z, which for
// exaggeration a = 1 is KL(P || Q) (sum P = 1) and in general the objective
// whose gradient the gradient calls return.  Every term is formed in double
// from the stored coordinates (ln w = -ln(1 + d^2), d from the double
// distance argument); 16 lanes share a row, their sums are combined in a
// fixed butterfly and the rows of a workgroup in row order, so the result is
// the same from run to run.
constexpr int kKlLanes = 16;

template <typename T>
__global__ __launch_bounds__(kBlock) void k_kl_rows(const PointRec<T> *__restrict__ pts,
                                                    const int64_t *__restrict__ rp,
                                                    const int32_t *__restrict__ col,
                                                    const T *__restrict__ val, int64_t n, double ex,
                                                    double *__restrict__ part,
                                                    uint32_t *__restrict__ err) {
    __shared__ double s_row[kBlock / kKlLanes];
    const int64_t gid = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int64_t row = gid / kKlLanes;
    const int sub = (int)(gid % kKlLanes);
    double c = 0.0;
    if (row < n) {
        const PointRec<T> q = pts[row];
        for (int64_t e = rp[row] + sub; e < rp[row + 1]; e += kKlLanes) {
            const int32_t j = col[e];
            if ((uint32_t)j >= (uint64_t)n) {
                atomicOr(err, HTS_ERR_BAD_INDEX);
                continue;
            }
            const double p = ex * (double)val[e];
            if (!(p > 0.0)) continue;
            const PointRec<T> o = pts[j];
            double dq, sh;
            const double t = dist_arg<T>(q.x, q.y, q.ia, o.x, o.y, o.ia, dq);
            const double d = acosh1p(t, sh);
            c += p * (log(p) + log1p(d * d));
        }
    }
    c = group_sum<kKlLanes>(c);
    if (sub == 0) s_row[threadIdx.x / kKlLanes] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        double b = 0.0;
        for (int r = 0; r < kBlock / kKlLanes; ++r) b += s_row[r];
        part[blockIdx.x] = b;
    }
}

// one workgroup: the block sums in a fixed order, plus ln Z
__global__ __launch_bounds__(kBlock) void k_kl_final(const double *__restrict__ part, int64_t nparts,
                                                     const double *__restrict__ z_dev,
                                                     double *__restrict__ kl_dev) {
    __shared__ double sh[kBlock];
    double s = 0.0;
    for (int64_t a = threadIdx.x; a < nparts; a += kBlock) s += part[a];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) *kl_dev = sh[0] + log(*z_dev);
}

int64_t kl_parts(int64_t n) { return cdiv(n * kKlLanes, kBlock); }

template <typename T>
hts_status launch_kl(hts_ctx ctx, hipStream_t st, const PointRec<T> *pts, const int64_t *rp,
                     const int32_t *col, const T *val, int64_t n, double ex, double *part,
                     const double *z_dev, double *kl_dev) {
    const int64_t nb = kl_parts(n);
    hipLaunchKernelGGL(k_kl_rows<T>, dim3(nb), dim3(kBlock), 0, st, pts, rp, col, val, n, ex, part,
                       ctx->d_err);
    hipLaunchKernelGGL(k_kl_final, dim3(1), dim3(kBlock), 0, st, part, nb, z_dev, kl_dev);
    HTS_HIP(hipGetLastError());
    return HTS_OK;
}

// ---------------------------------------------------------------- exact call
// Device memory of one exact-gradient call: point records, attractive
// forces, repulsive forces, Z partials, the repulsion's chunk partials and the
// cost's block sums.  Either the context's grow-on-demand workspaces or
// consecutive pieces of one fixed region (exact_carve).
static size_t ws_round(size_t b) { return (b + 255) & ~(size_t)255; }

// bytes of the pieces of an exact call on n points (each rounded to 256)
template <typename T>
size_t exact_ws_bytes(int64_t n, size_t sizes[6]) {
    sizes[0] = ws_round((size_t)n * sizeof(PointRec<T>));
    sizes[1] = ws_round((size_t)n * 2 * sizeof(T));
    sizes[2] = ws_round((size_t)n * 2 * sizeof(double));
    sizes[3] = ws_round((size_t)(cdiv(n, kBlock) + 8) * sizeof(double));
    sizes[4] = ws_round(exact_part_bytes(n));
    sizes[5] = ws_round((size_t)kl_parts(n) * sizeof(double));
    size_t tot = 0;
    for (int a = 0; a < 6; ++a) tot += sizes[a];
    return tot;
}

template <typename T>
ExactWs exact_carve(char *base, int64_t n) {
    size_t sz[6];
    exact_ws_bytes<T>(n, sz);
    ExactWs w;
    w.pts = base;
    w.fattr = base + sz[0];
    w.frep = (double *)(base + sz[0] + sz[1]);
    w.zpart = (double *)(base + sz[0] + sz[1] + sz[2]);
    w.part = (double *)(base + sz[0] + sz[1] + sz[2] + sz[3]);
    w.klpart = (double *)(base + sz[0] + sz[1] + sz[2] + sz[3] + sz[4]);
    return w;
}

// timed: the launches carry the context's timing events when timing is on
template <typename T>
hts_status exact_impl(hts_ctx c, hipStream_t st, const T *Y, int64_t n, const int64_t *rp,
                             const int32_t *col, const T *val, double ex, T *grad, double *z_dev,
                             double *kl_dev, const ExactWs &w, bool timed) {
    PointRec<T> *pts = (PointRec<T> *)w.pts;
    HTS_OKR(launch_prep_points<T>(c, st, Y, n, pts));
    HTS_OKR(launch_attract<T>(c, st, pts, rp, col, val, n, (T *)w.fattr, timed));
    int64_t nz = 0;
    HTS_OKR(launch_exact<T>(c, st, pts, n, w.part, w.frep, w.zpart, &nz, timed));
    HTS_OKR((launch_finalize<T, double>(c, st, (const T *)w.fattr, w.frep, w.zpart, nz, n, ex, grad,
                                        z_dev, timed)));
    if (kl_dev) HTS_OKR(launch_kl<T>(c, st, pts, rp, col, val, n, ex, w.klpart, z_dev, kl_dev));
    return HTS_OK;
}

// ---------------------------------------------------------------- step
// Riemannian step with momentum and gains (eqs. (7), (16)-(18), Sec. 5).
// State is stored in T; the exponential map, the Mobius addition and the
// projection run in double.
// Learning rate and momentum are per job when eta_job / mu_job are given.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_step(T *__restrict__ Y, T *__restrict__ U,
                                                 T *__restrict__ G, const T *__restrict__ grad,
                                                 int64_t n, double eta, double mu,
                                                 const int32_t *__restrict__ pjob,
                                                 const double *__restrict__ eta_job,
                                                 const double *__restrict__ mu_job,
                                                 double min_gain, double eps, int metric_power,
                                                 uint32_t *__restrict__ err) {
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    if (pjob) {
        const int job = pjob[i];
        eta = eta_job[job];
        mu = mu_job[job];
    }
    double y0 = (double)Y[2 * i], y1 = (double)Y[2 * i + 1];
    double a = 1.0 - (y0 * y0 + y1 * y1);
    double s = metric_power == 2 ? a * a * 0.25 : a * 0.5;
    double u[2];
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        double gh = s * (double)grad[2 * i + c];
        double uc = (double)U[2 * i + c];
        double g = (double)G[2 * i + c];
        g = ((gh > 0.0) != (uc > 0.0)) ? g + 0.2 : g * 0.8;
        if (g < min_gain) g = min_gain;
        T gs = (T)g;
        T us = (T)(mu * uc - eta * (double)gs * gh);
        G[2 * i + c] = gs;
        U[2 * i + c] = us;
        u[c] = (double)us;
        if (!isfinite(gh)) atomicOr(err, HTS_ERR_NONFINITE_GRAD);
    }
    double nv = sqrt(u[0] * u[0] + u[1] * u[1]);
    double o0 = y0, o1 = y1;
    if (nv > 0.0) {
        // exp_y(u) = y (+) tanh(lambda |u| / 2) u / |u|,  lambda = 2 / a
        double sc = tanh(nv / a) / nv;
        double b0 = sc * u[0], b1 = sc * u[1];
        double ab = y0 * b0 + y1 * b1;
        double aa = y0 * y0 + y1 * y1;
        double bb = b0 * b0 + b1 * b1;
        double na = 1.0 + 2.0 * ab + bb;
        double nb = 1.0 - aa;
        double den = 1.0 + 2.0 * ab + aa * bb;
        o0 = (na * y0 + nb * b0) / den;
        o1 = (na * y1 + nb * b1) / den;
    }
    // eq. (18) when |y| >= 1; |y|^2 within 2^-50 of 1 counts as on the circle,
    // so 1 - |y|^2 of a stored point never rounds to zero
    constexpr double kOnCircle = 1.0 - 0x1p-50;
    double q2 = o0 * o0 + o1 * o1;
    if (q2 >= kOnCircle) {
        double r = sqrt(q2);
        o0 = (1.0 - eps) * o0 / r;
        o1 = (1.0 - eps) * o1 / r;
    }
    T s0 = (T)o0, s1 = (T)o1;
    double r2 = (double)s0 * (double)s0 + (double)s1 * (double)s1;
    if (r2 >= kOnCircle) {  // the rounded point reached the circle: project the stored value
        double rr = sqrt(r2);
        s0 = (T)((1.0 - eps) * (double)s0 / rr);
        s1 = (T)((1.0 - eps) * (double)s1 / rr);
    }
    if (!isfinite(s0) || !isfinite(s1)) atomicOr(err, HTS_ERR_NONFINITE_Y);
    Y[2 * i] = s0;
    Y[2 * i + 1] = s1;
}

template <typename T>
hts_status launch_step(hts_ctx ctx, hipStream_t st, T *Y, T *U, T *G, const T *grad, int64_t n,
                       double eta, double mu, const int32_t *pjob, const double *eta_job,
                       const double *mu_job, double min_gain, double eps, int metric_power) {
    TimedScope ts(ctx, st, HTS_K_STEP);
    hipLaunchKernelGGL(k_step<T>, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, Y, U, G, grad, n, eta,
                       mu, pjob, eta_job, mu_job, min_gain, eps, metric_power, ctx->d_err);
    HTS_HIP(hipGetLastError());
    return HTS_OK;
}

// ---------------------------------------------------------------- CO-SNE
// Sec. 4-C: gradient of lambda1 KL + (lambda2 / n) sum (|x_i|^2 - |y_i|^2)^2
// from the KL gradient in grad, in place:
//   grad_i <- lambda1 grad_i - (4 lambda2 / n)(|x_i|^2 - |y_i|^2) y_i
template <typename T>
__global__ __launch_bounds__(kBlock) void k_cosne(const T *__restrict__ Y, int64_t n,
                                                  const double *__restrict__ xnorm2, double l1,
                                                  double c, T *__restrict__ grad,
                                                  uint32_t *__restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double y0 = (double)Y[2 * i], y1 = (double)Y[2 * i + 1];
    const double e = c * (xnorm2[i] - (y0 * y0 + y1 * y1));
    const T g0 = (T)(l1 * (double)grad[2 * i] - e * y0);
    const T g1 = (T)(l1 * (double)grad[2 * i + 1] - e * y1);
    if (!isfinite(g0) || !isfinite(g1)) atomicOr(err, HTS_ERR_NONFINITE_GRAD);
    grad[2 * i] = g0;
    grad[2 * i + 1] = g1;
}

template <typename T>
hts_status launch_cosne(hts_ctx ctx, hipStream_t st, const T *Y, int64_t n, const double *xnorm2,
                        double lambda1, double lambda2, T *grad) {
    TimedScope ts(ctx, st, HTS_K_FINALIZE);
    hipLaunchKernelGGL(k_cosne<T>, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, Y, n, xnorm2,
                       lambda1, 4.0 * lambda2 / (double)n, grad, ctx->d_err);
    HTS_HIP(hipGetLastError());
    return HTS_OK;
}

#define HTS_INST(T)                                                                              \
    template hts_status launch_prep_points<T>(hts_ctx, hipStream_t, const T *, int64_t,           \
                                              PointRec<T> *);                                    \
    template hts_status launch_attract<T>(hts_ctx, hipStream_t, const PointRec<T> *,              \
                                          const int64_t *, const int32_t *, const T *, int64_t,   \
                                          T *, bool);                                            \
    template hts_status launch_exact<T>(hts_ctx, hipStream_t, const PointRec<T> *, int64_t,       \
                                        double *, double *, double *, int64_t *, bool);          \
    template hts_status launch_finalize<T, T>(hts_ctx, hipStream_t, const T *, const T *,         \
                                              const double *, int64_t, int64_t, double, T *,      \
                                              double *, bool);                                   \
    template hts_status launch_kl<T>(hts_ctx, hipStream_t, const PointRec<T> *, const int64_t *,  \
                                     const int32_t *, const T *, int64_t, double, double *,       \
                                     const double *, double *);                                  \
    template hts_status launch_cosne<T>(hts_ctx, hipStream_t, const T *, int64_t,                \
                                        const double *, double, double, T *);                     \
    template hts_status launch_step<T>(hts_ctx, hipStream_t, T *, T *, T *, const T *, int64_t,   \
                                       double, double, const int32_t *, const double *,          \
                                       const double *, double, double, int);                     \
    template size_t exact_ws_bytes<T>(int64_t, size_t *);                                       \
    template ExactWs exact_carve<T>(char *, int64_t);                                           \
    template hts_status exact_impl<T>(hts_ctx, hipStream_t, const T *, int64_t, const int64_t *, \
                                      const int32_t *, const T *, double, T *, double *, double *, \
                                      const ExactWs &, bool);
HTS_INST(float)
HTS_INST(double)
template hts_status launch_finalize<float, double>(hts_ctx, hipStream_t, const float *,
                                                   const double *, const double *, int64_t,
                                                   int64_t, double, float *, double *, bool);

}  // namespace hts
