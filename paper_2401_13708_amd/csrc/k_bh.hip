// k_bh.hip -- Barnes-Hut repulsion over the polar quadtree (eq. (19) and the
// depth-first traversal of Sec. 4-B).
//
// One wave owns 64 consecutive points of the key order (so its queries are
// spatial neighbours) and walks the union of their traversals in pre-order.
// The node index is uniform across the wave, so every node record arrives
// through scalar loads; each lane keeps its own criterion decision.  The set
// of lanes that still need a subtree is a 64-bit mask per depth, held in two
// VGPRs used as lane-indexed arrays (readlane with the depth, a lane select to write).
// At an internal node a lane in the mask either accepts the cell
// (r_cell / d(y_i, m) < theta, tested as t > cosh(r_cell/theta) - 1 with the
// distance argument t in double) and adds N_cell w^2 d dd/dy, or joins the
// mask of the children.  Leaves are evaluated exactly, skipping the query.
#include "hts_impl.hpp"
#include "hts_math.hpp"

namespace hts {

template <typename T, bool STATS>
__global__ __launch_bounds__(kBlock) void k_traverse(const NodeRec<T> *__restrict__ nodes,
                                                     const int32_t *__restrict__ d_m,
                                                     const PointRec<T> *__restrict__ spts,
                                                     const uint32_t *__restrict__ perm, int64_t n,
                                                     T *__restrict__ frep,
                                                     double *__restrict__ zpart,
                                                     unsigned long long *__restrict__ stats) {
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const bool valid = q < n;
    const PointRec<T> me = spts[valid ? q : 0];
    const int M = uniform(*d_m);

    T fx = 0, fy = 0;
    double z = 0.0;
    unsigned long long n_test = 0, n_acc = 0, n_pair = 0;

    uint64_t act = __ballot(valid);
    int mlo = lane == 0 ? (int)(uint32_t)act : 0;
    int mhi = lane == 0 ? (int)(uint32_t)(act >> 32) : 0;

    int k = 0;
    while (k < M) {
        const NodeRec<T> nd = nodes[k];
        const uint32_t nxd = (uint32_t)uniform((int)nd.next_depth);
        const int next = (int)(nxd & kNextMask);
        const int depth = (int)(nxd >> kNextBits);
        const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(mhi, depth) << 32) |
                           (uint64_t)(uint32_t)__builtin_amdgcn_readlane(mlo, depth);
        const bool in = (m >> lane) & 1ull;
        if (next == k + 1) {
            // leaf: exact terms with each of its points, skipping the query
            const int64_t first = (int64_t)__double_as_longlong(nd.c);
            const int cnt = uniform(nd.count);
            if (cnt == 1) {
                const bool use = in && first != q;
                if (use) {
                    double dd;
                    double t = dist_arg<T>(me.x, me.y, me.ia, nd.mx, nd.my, nd.ib, dd);
                    PairTerm<T> r = pair_term<T>(me.x, me.y, me.ia, nd.mx, nd.my, nd.ib, t, dd);
                    T coef = r.w * r.w * r.base;
                    fx += coef * r.vx;
                    fy += coef * r.vy;
                    z += (double)r.w;
                }
                if (STATS) n_pair += __popcll(__ballot(use));
            } else {
                for (int a = 0; a < cnt; ++a) {
                    const PointRec<T> o = spts[first + a];
                    const bool use = in && (first + a) != q;
                    if (use) {
                        double dd;
                        double t = dist_arg<T>(me.x, me.y, me.ia, o.x, o.y, o.ia, dd);
                        PairTerm<T> r = pair_term<T>(me.x, me.y, me.ia, o.x, o.y, o.ia, t, dd);
                        T coef = r.w * r.w * r.base;
                        fx += coef * r.vx;
                        fy += coef * r.vy;
                        z += (double)r.w;
                    }
                    if (STATS) n_pair += __popcll(__ballot(use));
                }
            }
            k = next;
        } else {
            bool acc = false;
            if (in) {
                double dd;
                double t = dist_arg<T>(me.x, me.y, me.ia, nd.mx, nd.my, nd.ib, dd);
                acc = t > nd.c;
                if (acc) {
                    PairTerm<T> r = pair_term<T>(me.x, me.y, me.ia, nd.mx, nd.my, nd.ib, t, dd);
                    T nc = (T)nd.count;
                    T coef = nc * r.w * r.w * r.base;
                    fx += coef * r.vx;
                    fy += coef * r.vy;
                    z += (double)(nc * r.w);
                }
            }
            const uint64_t rej = __ballot(in && !acc);
            if (STATS) {
                n_test += __popcll(m);
                n_acc += __popcll(__ballot(acc));
            }
            if (rej) {
                const bool here = lane == depth + 1;
                mlo = here ? (int)(uint32_t)rej : mlo;
                mhi = here ? (int)(uint32_t)(rej >> 32) : mhi;
                k = k + 1;
            } else {
                k = next;
            }
        }
    }
    if (valid) {
        uint32_t o = perm[q];
        frep[2 * (int64_t)o] = fx;
        frep[2 * (int64_t)o + 1] = fy;
    }
    double zs = wave_sum(z);
    if (lane == 0) {
        zpart[q / kWave] = zs;
        if (STATS) {
            atomicAdd(&stats[0], n_test);
            atomicAdd(&stats[1], n_acc);
            atomicAdd(&stats[2], n_pair);
        }
    }
}

template <typename T>
hts_status launch_traverse(hts_ctx ctx, hipStream_t st, hts_tree t, int64_t n, T *frep,
                           double *zpart, int64_t *nz_out, uint64_t *stats) {
    TimedScope ts(ctx, st, HTS_K_TRAVERSE);
    dim3 grid(cdiv(n, kBlock));
    const NodeRec<T> *nodes = (const NodeRec<T> *)t->nodes;
    const PointRec<T> *spts = (const PointRec<T> *)t->spts;
    if (stats)
        hipLaunchKernelGGL((k_traverse<T, true>), grid, dim3(kBlock), 0, st, nodes, t->d_m, spts,
                           t->perm, n, frep, zpart, (unsigned long long *)stats);
    else
        hipLaunchKernelGGL((k_traverse<T, false>), grid, dim3(kBlock), 0, st, nodes, t->d_m, spts,
                           t->perm, n, frep, zpart, (unsigned long long *)nullptr);
    HTS_HIP(hipGetLastError());
    *nz_out = (int64_t)grid.x * (kBlock / kWave);
    return HTS_OK;
}

template hts_status launch_traverse<float>(hts_ctx, hipStream_t, hts_tree, int64_t, float *,
                                           double *, int64_t *, uint64_t *);
template hts_status launch_traverse<double>(hts_ctx, hipStream_t, hts_tree, int64_t, double *,
                                            double *, int64_t *, uint64_t *);

}  // namespace hts
