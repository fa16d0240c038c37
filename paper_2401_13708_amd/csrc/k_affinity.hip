// k_affinity.hip -- input affinities P (Sec. 2-A, eq. (1)), truncated to the
// k nearest neighbours and symmetrised.
//
//  1. exact k-NN: a block owns 64 queries and streams every candidate in
//     tiles of 128; each thread accumulates a 4 x 8 block of squared
//     distances in double precision, summing the dimensions in ascending order
//     with one fused multiply-add per term (a fixed, reproducible order).
//     The dimensions come through LDS in stages of 16; each thread's share of
//     the next stage is loaded into registers while the current one is summed
//     (twelve loads in flight, from clamped addresses).  A
//     running top-k list per query (ordered by distance, then index) is
//     merged with the candidates that beat its current k-th entry by a
//     one-wave bitonic sort in LDS; after the first tiles almost no
//     candidate passes, so the merges cost little next to the distances.
//  2. bandwidth per row: 100 bisection steps on beta = 1 / (2 sigma^2) so the
//     entropy of p_{j|i} equals ln(perplexity); one wave per row.
//  3. P = (P_c + P_c^T) / (2 n): both orientations of every (i, j, p_{j|i})
//     are sorted by (row, col) with the library's radix sort (keys with
//     their positions; the values follow by a gather), duplicates summed
//     (each appears at most twice: a + b = b + a, so the sum does not depend
//     on their order), and written as CSR at positions from an exclusive
//     scan of the first-copy flags.
#include <climits>

#include "hts_impl.hpp"
#include "hts_math.hpp"

namespace hts {

constexpr int kQ = 64;     // queries per block
constexpr int kC = 128;    // candidates per tile
constexpr int kD = 16;     // dimensions per LDS stage
constexpr int kMaxK = 128; // largest k this kernel keeps
constexpr int kSort = 256; // merge buffer per wave (>= kMaxK + kC)

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// ascending bitonic sort of P2 (power of two, <= kSort) (distance, index)
// pairs held in LDS, by the 64 lanes of one wave
__device__ void wave_bitonic(double *sd, int *sj, int P2, int lane) {
    for (int size = 2; size <= P2; size <<= 1) {
        for (int stride = size >> 1; stride > 0; stride >>= 1) {
            for (int t = lane; t < (P2 >> 1); t += kWave) {
                int i = 2 * t - (t & (stride - 1));
                int j = i + stride;
                bool up = (i & size) == 0;
                double di = sd[i], dj = sd[j];
                int ji = sj[i], jj = sj[j];
                bool gt = (di > dj) || (di == dj && ji > jj);
                if (gt == up) {
                    sd[i] = dj; sd[j] = di;
                    sj[i] = jj; sj[j] = ji;
                }
            }
            wave_sync();
        }
    }
}

template <typename XT>
__global__ __launch_bounds__(kBlock) void k_knn(const XT *__restrict__ X, int64_t n, int d, int k,
                                                double *__restrict__ ld, int32_t *__restrict__ lj) {
    __shared__ double Qs[kD][kQ];
    __shared__ double Cs[kD][kC];
    __shared__ double thr_d[kQ];
    __shared__ int thr_j[kQ];
    __shared__ int len[kQ];
    __shared__ double sd[kBlock / kWave][kSort];
    __shared__ int sj[kBlock / kWave][kSort];

    const int tid = threadIdx.x;
    const int lane = tid & (kWave - 1);
    const int w = tid / kWave;
    const int tq = tid >> 4, tc = tid & 15;
    const int64_t q0 = (int64_t)blockIdx.x * kQ;
    if (tid < kQ) {
        thr_d[tid] = __builtin_inf();
        thr_j[tid] = INT_MAX;
        len[tid] = 0;
    }
    __syncthreads();

    // the thread's share of a stage: dimension kk of 4 queries and 8
    // candidates, loaded from clamped (always valid) addresses so that all
    // twelve loads are in flight at once; entries outside the data are zeroed
    // when they are stored to LDS
    const int kk = tid & 15;
    XT qr[4], cr[8];
    auto load_stage = [&](int64_t c0, int k0) {
        const int64_t dim = k0 + kk < d ? k0 + kk : d - 1;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int64_t q = q0 + (tid >> 4) + 16 * r;
            qr[r] = X[(q < n ? q : n - 1) * d + dim];
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int64_t c = c0 + (tid >> 4) + 16 * r;
            cr[r] = X[(c < n ? c : n - 1) * d + dim];
        }
    };
    load_stage(0, 0);
    for (int64_t c0 = 0; c0 < n; c0 += kC) {
        double acc[4][8];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 8; ++b) acc[a][b] = 0.0;
        for (int k0 = 0; k0 < d; k0 += kD) {
            const bool din = k0 + kk < d;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int qq = (tid >> 4) + 16 * r;
                Qs[kk][qq] = (q0 + qq < n && din) ? (double)qr[r] : 0.0;
            }
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                int cc = (tid >> 4) + 16 * r;
                Cs[kk][cc] = (c0 + cc < n && din) ? (double)cr[r] : 0.0;
            }
            __syncthreads();
            // the next stage (of this tile, else the next tile's first) is
            // loaded while this one is summed
            if (k0 + kD < d) load_stage(c0, k0 + kD);
            else if (c0 + kC < n) load_stage(c0 + kC, 0);
            const int kmax = d - k0 < kD ? d - k0 : kD;
            for (int s = 0; s < kmax; ++s) {
                double qv[4], cv[8];
#pragma unroll
                for (int a = 0; a < 4; ++a) qv[a] = Qs[s][tq + 16 * a];
#pragma unroll
                for (int b = 0; b < 8; ++b) cv[b] = Cs[s][tc + 16 * b];
#pragma unroll
                for (int a = 0; a < 4; ++a)
#pragma unroll
                    for (int b = 0; b < 8; ++b) {
                        double dl = qv[a] - cv[b];
                        acc[a][b] = fma(dl, dl, acc[a][b]);
                    }
            }
            __syncthreads();
        }
        // merge the tile into the running lists of this wave's 16 queries
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            // one query at a time (not unrolled: the merge's registers then
            // fit two waves per SIMD beside the distance tile)
#pragma unroll 1
            for (int r = 0; r < 4; ++r) {
                const int qq = 4 * w + r + 16 * a;
                const int64_t q = q0 + qq;
                if (q >= n) continue;
                const double td = thr_d[qq];
                const int tj = thr_j[qq];
                const bool mine = (lane >> 4) == r;
                uint64_t masks[8];
                int tot = 0;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    int64_t c = c0 + tc + 16 * b;
                    double dv = acc[a][b];
                    bool p = mine && c < n && c != q && (dv < td || (dv == td && c < (int64_t)tj));
                    masks[b] = __ballot(p);
                    tot += __popcll(masks[b]);
                }
                if (tot == 0) continue;
                const int L = len[qq];
                double *wd = sd[w];
                int *wj = sj[w];
                for (int t = lane; t < L; t += kWave) {
                    // the list was written by this wave earlier: read it past the L1
                    wd[t] = __hip_atomic_load(&ld[q * k + t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    wj[t] = __hip_atomic_load(&lj[q * k + t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                }
                int off = L;
                const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
#pragma unroll
                for (int b = 0; b < 8; ++b) {
                    if ((masks[b] >> lane) & 1ull) {
                        int pos = off + __popcll(masks[b] & below);
                        wd[pos] = acc[a][b];
                        wj[pos] = (int)(c0 + tc + 16 * b);
                    }
                    off += __popcll(masks[b]);
                }
                const int total = L + tot;
                int P2 = kWave;
                while (P2 < total) P2 <<= 1;
                for (int t = total + lane; t < P2; t += kWave) {
                    wd[t] = __builtin_inf();
                    wj[t] = INT_MAX;
                }
                wave_sync();
                wave_bitonic(wd, wj, P2, lane);
                const int nl = total < k ? total : k;
                for (int t = lane; t < nl; t += kWave) {
                    ld[q * k + t] = wd[t];
                    lj[q * k + t] = wj[t];
                }
                if (lane == 0) {
                    len[qq] = nl;
                    if (nl == k) {
                        thr_d[qq] = wd[k - 1];
                        thr_j[qq] = wj[k - 1];
                    }
                }
                wave_sync();
            }
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- perplexity
// One wave per row; the k sorted squared distances of the row are spread over
// the lanes.  Same bisection as described in the header (start at 1, double or
// halve until bracketed, 100 steps).
__global__ __launch_bounds__(kBlock) void k_perplexity(const double *__restrict__ ld, int64_t n,
                                                       int k, double log_perp,
                                                       double *__restrict__ pc) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t row = ((int64_t)blockIdx.x * kBlock + threadIdx.x) / kWave;
    if (row >= n) return;
    const double *di = ld + row * k;
    double D[kMaxK / kWave];
    double dmin = __builtin_inf();
#pragma unroll
    for (int s = 0; s < kMaxK / kWave; ++s) {
        int t = lane + kWave * s;
        D[s] = t < k ? di[t] : 0.0;
        if (t < k) dmin = fmin(dmin, D[s]);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) dmin = fmin(dmin, __shfl_xor(dmin, o, 64));
    double beta = 1.0, lo = -__builtin_inf(), hi = __builtin_inf();
    double e[kMaxK / kWave];
    double s = 0.0;
    for (int it = 0; it <= 100; ++it) {
        double ls = 0.0, lsd = 0.0;
#pragma unroll
        for (int u = 0; u < kMaxK / kWave; ++u) {
            int t = lane + kWave * u;
            double Dt = D[u] - dmin;
            e[u] = t < k ? exp(-beta * Dt) : 0.0;
            ls += e[u];
            lsd += t < k ? Dt * e[u] : 0.0;
        }
        s = wave_sum(ls);
        if (it == 100) break;  // final pass: probabilities at the last beta
        double sdd = wave_sum(lsd);
        double H = log(s) + beta * sdd / s;
        if (H > log_perp) {
            lo = beta;
            beta = isinf(hi) ? beta * 2.0 : 0.5 * (beta + hi);
        } else {
            hi = beta;
            beta = isinf(lo) ? beta * 0.5 : 0.5 * (beta + lo);
        }
    }
#pragma unroll
    for (int u = 0; u < kMaxK / kWave; ++u) {
        int t = lane + kWave * u;
        if (t < k) pc[row * k + t] = e[u] / s;
    }
}

// ---------------------------------------------------------------- symmetrise
__global__ __launch_bounds__(kBlock) void k_coo(const int32_t *__restrict__ lj,
                                                const double *__restrict__ pc, int64_t n, int k,
                                                uint64_t *__restrict__ keys,
                                                double *__restrict__ vals,
                                                uint32_t *__restrict__ at,
                                                int32_t *__restrict__ knn_out) {
    int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= n * k) return;
    int64_t i = e / k;
    int64_t j = lj[e];
    double p = pc[e];
    keys[2 * e] = (uint64_t)(i * n + j);
    keys[2 * e + 1] = (uint64_t)(j * n + i);
    vals[2 * e] = p;
    vals[2 * e + 1] = p;
    at[2 * e] = (uint32_t)(2 * e);
    at[2 * e + 1] = (uint32_t)(2 * e + 1);
    if (knn_out) knn_out[e] = (int32_t)j;
}

// the values in sorted order: vout[t] = vin[at[t]]
__global__ __launch_bounds__(kBlock) void k_gather_vals(const uint32_t *__restrict__ at,
                                                        const double *__restrict__ vin, int64_t m,
                                                        double *__restrict__ vout) {
    const int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e < m) vout[e] = vin[at[e]];
}

// ---------------------------------------------------------------- int scan
// Exclusive prefix sum of m int32 values in three kernels: per 2048-value
// block its total, an exclusive scan of the totals in one workgroup, then
// each block's values from its offset (integers: exact in any order).
constexpr int kScanItems = 8;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ int block_excl_scan(int v, int *s) {
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const int u = t >= o ? s[t - o] : 0;
        __syncthreads();
        s[t] += u;
        __syncthreads();
    }
    const int incl = s[t];
    __syncthreads();
    return incl - v;
}

__global__ __launch_bounds__(kBlock) void k_iscan_reduce(const int32_t *__restrict__ in, int64_t m,
                                                         int32_t *__restrict__ part) {
    __shared__ int s[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int v = 0;
#pragma unroll
    for (int a = 0; a < kScanItems; ++a) v += base + a < m ? in[base + a] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int o = kBlock / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) s[threadIdx.x] += s[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(kBlock) void k_iscan_parts(int32_t *__restrict__ part, int64_t nb) {
    __shared__ int s[kBlock];
    const int64_t per = cdiv(nb, kBlock);
    const int64_t a0 = (int64_t)threadIdx.x * per, a1 = a0 + per < nb ? a0 + per : nb;
    int v = 0;
    for (int64_t a = a0; a < a1; ++a) v += part[a];
    int run = block_excl_scan(v, s);
    for (int64_t a = a0; a < a1; ++a) {
        const int c = part[a];
        part[a] = run;
        run += c;
    }
}

__global__ __launch_bounds__(kBlock) void k_iscan_apply(const int32_t *__restrict__ in, int64_t m,
                                                        const int32_t *__restrict__ part,
                                                        int32_t *__restrict__ out) {
    __shared__ int s[kBlock];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int x[kScanItems], v = 0;
#pragma unroll
    for (int a = 0; a < kScanItems; ++a) {
        x[a] = base + a < m ? in[base + a] : 0;
        v += x[a];
    }
    int run = part[blockIdx.x] + block_excl_scan(v, s);
#pragma unroll
    for (int a = 0; a < kScanItems; ++a) {
        if (base + a < m) out[base + a] = run;
        run += x[a];
    }
}

__global__ __launch_bounds__(kBlock) void k_uflags(const uint64_t *__restrict__ keys, int64_t m,
                                                   int32_t *__restrict__ flag) {
    int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    flag[e] = (e == 0 || keys[e] != keys[e - 1]) ? 1 : 0;
}

template <typename PT>
__global__ __launch_bounds__(kBlock) void k_csr(const uint64_t *__restrict__ keys,
                                                const double *__restrict__ vals,
                                                const int32_t *__restrict__ pos, int64_t m,
                                                int64_t n, int64_t nnz, int64_t *__restrict__ row_ptr,
                                                int32_t *__restrict__ col, PT *__restrict__ pval) {
    int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= m) return;
    uint64_t key = keys[e];
    if (e > 0 && keys[e - 1] == key) return;  // second copy of a pair: summed by the first
    int64_t u = pos[e];
    int64_t row = (int64_t)(key / (uint64_t)n);
    double v = vals[e];
    if (e + 1 < m && keys[e + 1] == key) v = v + vals[e + 1];
    col[u] = (int32_t)(key % (uint64_t)n);
    pval[u] = (PT)(v / (2.0 * (double)n));
    if (e == 0 || (int64_t)(keys[e - 1] / (uint64_t)n) != row) row_ptr[row] = u;
    if (u == nnz - 1) row_ptr[n] = nnz;
}

template <typename XT>
static hts_status knn_launch(hts_ctx ctx, hipStream_t st, const XT *X, int64_t n, int d, int k,
                             double *ld, int32_t *lj) {
    TimedScope ts(ctx, st, HTS_K_KNN);
    hipLaunchKernelGGL(k_knn<XT>, dim3(cdiv(n, kQ)), dim3(kBlock), 0, st, X, n, d, k, ld, lj);
    HTS_HIP(hipGetLastError());
    return HTS_OK;
}

hts_status affinities(hts_ctx ctx, hipStream_t st, const void *X, int64_t n, int32_t d,
                      int32_t x_dtype, double perplexity, int32_t k, int32_t *knn_idx,
                      int64_t *row_ptr, int32_t *col_idx, void *p_val, int32_t p_dtype,
                      int64_t cap_nnz, int64_t *nnz_out) {
    if (k > kMaxK) return fail(HTS_EINVAL, "hts_build_affinities: k = %d > %d", k, kMaxK);
    const int64_t nk = n * (int64_t)k, m = 2 * nk;
    HTS_OKR(ensure(ctx->aff[0], (size_t)nk * 8));    // list distances
    HTS_OKR(ensure(ctx->aff[1], (size_t)nk * 4));    // list indices
    HTS_OKR(ensure(ctx->aff[2], (size_t)nk * 8));    // conditional p
    HTS_OKR(ensure(ctx->aff[3], (size_t)m * 8 * 2)); // keys in / out
    HTS_OKR(ensure(ctx->aff[4], (size_t)m * 8 * 2)); // values in / out
    HTS_OKR(ensure(ctx->aff[5], (size_t)m * 4 * 2)); // flags, positions
    double *ld = (double *)ctx->aff[0].p;
    int32_t *lj = (int32_t *)ctx->aff[1].p;
    double *pc = (double *)ctx->aff[2].p;
    uint64_t *kin = (uint64_t *)ctx->aff[3].p, *kout = kin + m;
    double *vin = (double *)ctx->aff[4].p, *vout = vin + m;
    int32_t *flag = (int32_t *)ctx->aff[5].p, *pos = flag + m;

    if (x_dtype == HTS_F64)
        HTS_OKR(knn_launch<double>(ctx, st, (const double *)X, n, d, k, ld, lj));
    else
        HTS_OKR(knn_launch<float>(ctx, st, (const float *)X, n, d, k, ld, lj));
    hipLaunchKernelGGL(k_perplexity, dim3(cdiv(n * kWave, kBlock)), dim3(kBlock), 0, st, ld, n, k,
                       std::log(perplexity), pc);
    HTS_HIP(hipGetLastError());
    // the sort's values are the entries' positions (in the flag buffer, then
    // the position buffer), free until the flags and their scan are formed
    uint32_t *at_in = (uint32_t *)flag, *at_out = (uint32_t *)pos;
    hipLaunchKernelGGL(k_coo, dim3(cdiv(nk, kBlock)), dim3(kBlock), 0, st, lj, pc, n, k, kin, vin,
                       at_in, knn_idx);
    HTS_HIP(hipGetLastError());
    int bits = 1;
    while (bits < 64 && ((uint64_t)1 << bits) < (uint64_t)n * (uint64_t)n) ++bits;
    HTS_OKR(ensure(ctx->aff[6], radix_sort_temp_bytes(m)));
    HTS_OKR(radix_sort_pairs(st, kin, at_in, kout, at_out, m, bits, ctx->aff[6].p));
    hipLaunchKernelGGL(k_gather_vals, dim3(cdiv(m, kBlock)), dim3(kBlock), 0, st, at_out, vin, m,
                       vout);
    HTS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_uflags, dim3(cdiv(m, kBlock)), dim3(kBlock), 0, st, kout, m, flag);
    HTS_HIP(hipGetLastError());
    const int64_t nsb = cdiv(m, kScanTile);
    HTS_OKR(ensure(ctx->aff[7], (size_t)nsb * 4));
    int32_t *spart = (int32_t *)ctx->aff[7].p;
    hipLaunchKernelGGL(k_iscan_reduce, dim3(nsb), dim3(kBlock), 0, st, flag, m, spart);
    hipLaunchKernelGGL(k_iscan_parts, dim3(1), dim3(kBlock), 0, st, spart, nsb);
    hipLaunchKernelGGL(k_iscan_apply, dim3(nsb), dim3(kBlock), 0, st, flag, m, spart, pos);
    HTS_HIP(hipGetLastError());
    int32_t last[2] = {0, 0};
    HTS_HIP(hipMemcpyAsync(&last[0], pos + m - 1, 4, hipMemcpyDeviceToHost, st));
    HTS_HIP(hipMemcpyAsync(&last[1], flag + m - 1, 4, hipMemcpyDeviceToHost, st));
    HTS_HIP(hipStreamSynchronize(st));
    const int64_t nnz = (int64_t)last[0] + last[1];
    *nnz_out = nnz;
    if (nnz > cap_nnz)
        return fail(HTS_ECAPACITY, "hts_build_affinities: nnz = %lld > cap_nnz = %lld",
                    (long long)nnz, (long long)cap_nnz);
    if (p_dtype == HTS_F64)
        hipLaunchKernelGGL(k_csr<double>, dim3(cdiv(m, kBlock)), dim3(kBlock), 0, st, kout, vout,
                           pos, m, n, nnz, row_ptr, col_idx, (double *)p_val);
    else
        hipLaunchKernelGGL(k_csr<float>, dim3(cdiv(m, kBlock)), dim3(kBlock), 0, st, kout, vout,
                           pos, m, n, nnz, row_ptr, col_idx, (float *)p_val);
    HTS_HIP(hipGetLastError());
    HTS_HIP(hipStreamSynchronize(st));
    return HTS_OK;
}

}  // namespace hts
