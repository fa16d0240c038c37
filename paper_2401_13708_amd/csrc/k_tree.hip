// k_tree.hip -- GPU build of the polar quadtree (Sec. 2-D, Sec. 4-A).
//
// The tree is built from sorted (r, phi) keys instead of by insertion:
//  1. polar position of every point (double, from the single-precision
//     coordinates) and per-block min/max of r per job;
//  2. root annulus of every job (a job spanning blocks is reduced from the
//     block partials), then the key of every point: max_depth levels of the
//     split rule, two bits per
//     level (radial bit: r at or above the radial split of eq. (10), or of
//     eq. (9) when the tree is set to equal areas; angular bit: the point on
//     or counter-clockwise of the cell's split ray, an exact sign test),
//     most significant level first;
//  3. stable radix sort of (key, index) (k_sort.hip);
//  4. per sorted position: how many nodes start there (from the common
//     prefixes with both neighbours), the sorted point record and the
//     Einstein-midpoint summands, with block aggregates;
//  5. exclusive scans (node offsets; double-double summand sums), after
//     which every point records itself as the first point of the nodes it
//     starts;
//  6. node emission in depth-first pre-order, one thread per node: its
//     count, subtree end, leaf point or midpoint (eq. (11)) and cell
//     diameter.
// A cell becomes a node when its parent holds two or more points (the same
// set of cells the insertion build of Sec. 2-D produces), so no insertion
// order is involved.
//
// Several embeddings (jobs) are built in one pass: the job index sits in the
// key bits above the cell bits, so the sort groups each job's points, no cell
// spans two jobs, and the pre-order array is the concatenation of the jobs'
// trees.  Every job has its own root annulus.
#include "hts_impl.hpp"
#include "hts_math.hpp"

namespace hts {


// ---------------------------------------------------------------- 1. polar
// Radius of every point, and the radial range of every job: a job that lies
// inside one block is reduced here completely; for the others the block
// leaves the (min, max) of its first and of its last job's points in mm
// (segmented scan over the block, jobs being contiguous).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_polar(const T *__restrict__ Y, int64_t n,
                                                  const int32_t *__restrict__ pjob,
                                                  const int64_t *__restrict__ job_off,
                                                  double *__restrict__ r,
                                                  double *__restrict__ mm,
                                                  double *__restrict__ root) {
    __shared__ double smin[kBlock], smax[kBlock];
    __shared__ int sjob[kBlock];
    const int t = threadIdx.x;
    const int64_t b0 = (int64_t)blockIdx.x * kBlock;
    const int64_t i = b0 + t;
    double vmin = __builtin_inf(), vmax = -__builtin_inf();
    int job = -1;
    if (i < n) {
        // radius of the single-precision coordinates; products are exact
        double x = (double)(float)Y[2 * i], y = (double)(float)Y[2 * i + 1];
        double rr = __dsqrt_rn(__dadd_rn(__dmul_rn(x, x), __dmul_rn(y, y)));
        r[i] = rr;
        vmin = vmax = rr;
        job = pjob[i];
    }
    smin[t] = vmin;
    smax[t] = vmax;
    sjob[t] = job;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const bool take = t >= o && sjob[t - o] == job;
        const double pa = take ? smin[t - o] : __builtin_inf();
        const double pb = take ? smax[t - o] : -__builtin_inf();
        __syncthreads();
        smin[t] = fmin(smin[t], pa);
        smax[t] = fmax(smax[t], pb);
        __syncthreads();
    }
    if (job < 0) return;
    const bool last = t == kBlock - 1 || sjob[t + 1] != job;
    if (!last) return;
    const int64_t b1 = b0 + kBlock < n ? b0 + kBlock : n;
    const int64_t j0 = job_off[job], j1 = job_off[job + 1];
    if (j0 >= b0 && j1 <= b1) {
        root[2 * job] = smin[t];
        root[2 * job + 1] = smax[t];
        return;
    }
    if (j0 < b0) {  // the block's first job
        mm[4 * blockIdx.x] = smin[t];
        mm[4 * blockIdx.x + 1] = smax[t];
    }
    if (j1 > b1 || i == b1 - 1) {  // the block's last job
        mm[4 * blockIdx.x + 2] = smin[t];
        mm[4 * blockIdx.x + 3] = smax[t];
    }
}

// The (min, max) of r of a job that spans several blocks, from the partials
// k_polar leaves: the job is the last one of its first block and the first
// one of every later block (one wave; min and max are exact in any order).
__device__ __forceinline__ void job_range(const int64_t *__restrict__ job_off, int j,
                                          const double *__restrict__ mm, int lane, double &lo,
                                          double &hi) {
    const int64_t b0 = job_off[j] / kBlock, b1 = (job_off[j + 1] - 1) / kBlock;
    double vmin = __builtin_inf(), vmax = -__builtin_inf();
    for (int64_t b = b0 + lane; b <= b1; b += kWave) {
        const int h = b == b0 ? 2 : 0;
        vmin = fmin(vmin, mm[4 * b + h]);
        vmax = fmax(vmax, mm[4 * b + h + 1]);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        vmin = fmin(vmin, __shfl_xor(vmin, o, 64));
        vmax = fmax(vmax, __shfl_xor(vmax, o, 64));
    }
    lo = vmin;
    hi = vmax;
}

// Radial split point of a cell with embedding radii [lo, hi]: rule 0 halves
// the radial length (eq. (10)); rule 1 splits at the hyperbolic radius whose
// cosh is the mean of the two bounds' (eq. (9), equal hyperbolic areas),
// computed in the embedding radius through cosh(rho) = 1 + 2 r^2 / (1 - r^2):
// mid^2 = s / (2 + s), s = lo^2/(1-lo^2) + hi^2/(1-hi^2).  Every operation
// is rounded on its own (no fused multiply-add), so the split points are
// reproducible to the bit.
__device__ __forceinline__ double radial_mid(double lo, double hi, int rule) {
#pragma clang fp contract(off)
    if (rule == 0) return __dmul_rn(__dadd_rn(lo, hi), 0.5);
    const double l2 = __dmul_rn(lo, lo), h2 = __dmul_rn(hi, hi);
    const double s = __dadd_rn(__ddiv_rn(l2, __dsub_rn(1.0, l2)), __ddiv_rn(h2, __dsub_rn(1.0, h2)));
    return __dsqrt_rn(__ddiv_rn(s, __dadd_rn(2.0, s)));
}

// Angular split of a cell (Sec. 2-D: the angular range halved at
// (max_phi + min_phi) / 2), decided without the angle of the point, whose
// last bit would depend on the math library: the split ray is a direction
// built from those of the cell's bounds -- the negative x-axis at the root
// (the ray at pi), the lower bound turned by a right angle at depth 1 (widths
// pi), below that the normalised sum of the two bound directions, every
// operation rounded on its own in double -- and the point (x, y) is in the
// upper half iff c y - s x >= 0, (c, s) the ray rounded to single precision.
// With single-precision coordinates both products are exact in double and
// the one rounding of the difference keeps its sign: the decision is exact,
// and a point on the ray goes to the upper half.  At the root the upper half
// is y < 0, or y = 0 and x < 0.
__device__ __forceinline__ void ang_mid(int depth, const double *lo, const double *hi, double *mid) {
    if (depth == 0) {
        mid[0] = -1.0;
        mid[1] = 0.0;
    } else if (depth == 1) {
        mid[0] = -lo[1];
        mid[1] = lo[0];
    } else {
        const double sx = __dadd_rn(lo[0], hi[0]), sy = __dadd_rn(lo[1], hi[1]);
        const double h = __dsqrt_rn(__dadd_rn(__dmul_rn(sx, sx), __dmul_rn(sy, sy)));
        mid[0] = __ddiv_rn(sx, h);
        mid[1] = __ddiv_rn(sy, h);
    }
}

__device__ __forceinline__ int ang_bit(int depth, const double *mid, double xs, double ys) {
    if (depth == 0) return ys < 0.0 || (ys == 0.0 && xs < 0.0);
    const double c = (double)__double2float_rn(mid[0]), s = (double)__double2float_rn(mid[1]);
    return __dsub_rn(__dmul_rn(c, ys), __dmul_rn(s, xs)) >= 0.0;
}

// ---------------------------------------------------------------- 2. keys
// job index above max_depth levels of the split rule, two bits per level
// (radial bit: r at or above the radial split; angular bit: the upper half
// of the angular split above).  A job inside one block has its root annulus from
// k_polar; the block's first and last jobs may span other blocks, and their
// annuli are reduced here from k_polar's partials (the block holding a job's
// first point stores it for the later kernels).
template <typename T>
__global__ __launch_bounds__(kBlock) void k_keys(const double *__restrict__ r,
                                                 const T *__restrict__ Y, int64_t n,
                                                 const int32_t *__restrict__ pjob,
                                                 const int64_t *__restrict__ job_off,
                                                 const double *__restrict__ mm,
                                                 double *__restrict__ root, int L, int split,
                                                 uint64_t *__restrict__ keys,
                                                 uint32_t *__restrict__ idx) {
    __shared__ double s_range[2][2];
    const int64_t b0 = (int64_t)blockIdx.x * kBlock;
    const int64_t bl = (b0 + kBlock < n ? b0 + kBlock : n) - 1;
    const int jf = pjob[b0], jl = pjob[bl];
    const int wave = (int)(threadIdx.x / kWave), lane = (int)(threadIdx.x & (kWave - 1));
    if (wave < 2) {
        const int j = wave == 0 ? jf : jl;
        const bool spans = job_off[j] / kBlock != (job_off[j + 1] - 1) / kBlock;
        if (spans && (wave == 0 || jl != jf)) {
            double lo, hi;
            job_range(job_off, j, mm, lane, lo, hi);
            if (lane == 0) {
                s_range[wave][0] = lo;
                s_range[wave][1] = hi;
                if (job_off[j] >= b0 && job_off[j] <= bl) {
                    root[2 * j] = lo;
                    root[2 * j + 1] = hi;
                }
            }
        }
    }
    __syncthreads();
    const int64_t i = b0 + threadIdx.x;
    if (i >= n) return;
    const int job = pjob[i];
    double lo, hi;
    if (job_off[job] / kBlock == (job_off[job + 1] - 1) / kBlock) {
        lo = root[2 * job];
        hi = root[2 * job + 1];
    } else {
        const int w = job == jf ? 0 : 1;
        lo = s_range[w][0];
        hi = s_range[w][1];
    }
    const double rv = r[i];
    const double xs = (double)(float)Y[2 * i], ys = (double)(float)Y[2 * i + 1];
    double alo[2] = {1.0, 0.0}, ahi[2] = {1.0, 0.0};  // the root's bounds: angle 0 = 2 pi
    uint64_t key = (uint64_t)job;
    for (int l = 0; l < L; ++l) {
        const double mr = radial_mid(lo, hi, split);
        double am[2];
        ang_mid(l, alo, ahi, am);
        const int rb = rv >= mr, pb = ang_bit(l, am, xs, ys);
        key = (key << 2) | (uint64_t)(2 * rb + pb);
        if (rb) lo = mr; else hi = mr;
        double *bound = pb ? alo : ahi;
        bound[0] = am[0];
        bound[1] = am[1];
    }
    keys[i] = key;
    idx[i] = (uint32_t)i;
}

// number of equal leading levels of two keys
// (-1 for points of different jobs, which share no cell, not even a root)
__device__ __forceinline__ int lcp_levels(uint64_t a, uint64_t b, int L) {
    uint64_t x = a ^ b;
    if (x == 0) return L;
    if (x >> (2 * L)) return -1;
    return (__clzll((long long)x) - (64 - 2 * L)) >> 1;
}

// nodes starting at sorted position i: depths s..D with s = lcp(i-1, i) + 1
// (0 for a job's first point) and D = min(L, max(lcp with either neighbour) + 1), the depth
// at which the point's cell holds it alone (or the depth cap).
struct NodeSpan { int s, D; };
__device__ __forceinline__ NodeSpan node_span(const uint64_t *__restrict__ keys, int64_t i, int64_t n,
                                              int L) {
    uint64_t k = keys[i];
    int lcpl = i > 0 ? lcp_levels(keys[i - 1], k, L) : -1;
    int lcpr = i + 1 < n ? lcp_levels(k, keys[i + 1], L) : -1;
    int mx = lcpl > lcpr ? lcpl : lcpr;
    NodeSpan sp;
    sp.D = mx + 1 < L ? mx + 1 : L;
    sp.s = i > 0 ? lcpl + 1 : 0;
    return sp;
}

// ---------------------------------------------------------------- 4. sorted
template <typename T>
__global__ __launch_bounds__(kBlock) void k_sorted(const T *__restrict__ Y, int64_t n,
                                                   const uint64_t *__restrict__ keys,
                                                   const uint32_t *__restrict__ perm, int L,
                                                   PointRec<T> *__restrict__ spts,
                                                   int32_t *__restrict__ cnt,
                                                   DD3 *__restrict__ q,
                                                   int32_t *__restrict__ cnt_part,
                                                   DD3 *__restrict__ q_part,
                                                   PointRec<T> *__restrict__ pts_in,
                                                   uint32_t *__restrict__ err) {
    __shared__ int scnt[kBlock];
    __shared__ DD3 sq[kBlock];
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    int c = 0;
    DD3 v = dd_zero();
    if (i < n) {
        uint32_t p = perm[i];
        // for a gradient that follows: the input-order record of this point,
        // as its preparation launch writes it
        if (pts_in) prep_point<T>(Y, p, pts_in, err);
        T x = Y[2 * p], y = Y[2 * p + 1];
        double xd = (double)x, yd = (double)y;
        double r2 = xd * xd + yd * yd;
        double a = 1.0 - r2;
        PointRec<T> pr;
        pr.x = x;
        pr.y = y;
        pr.ia = 1.0 / a;
        if constexpr (sizeof(T) == 8) pr.pad = 0.0;
        spts[i] = pr;
        // Klein coordinates v = 2y / (1 + |y|^2) with gamma(v) = (1 + |y|^2) / (1 - |y|^2):
        // gamma v = lambda y, the summands of eq. (11)
        double lam = 2.0 / a;
        v.hi[0] = lam * xd;
        v.hi[1] = lam * yd;
        v.hi[2] = (1.0 + r2) / a;
        NodeSpan sp = node_span(keys, i, n, L);
        c = sp.D - sp.s + 1;
        if (c < 0) c = 0;
        cnt[i] = c;
        q[i] = v;
    }
    scnt[threadIdx.x] = c;
    sq[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            scnt[threadIdx.x] += scnt[threadIdx.x + s];
            sq[threadIdx.x] = dd_add(sq[threadIdx.x], sq[threadIdx.x + s]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cnt_part[blockIdx.x] = scnt[0];
        q_part[blockIdx.x] = sq[0];
    }
}

// ---------------------------------------------------------------- 5. scans
// The scan of the nb block aggregates as one workgroup takes it: thread t
// adds blocks [t per, (t + 1) per) in order, then an inclusive Hillis-Steele
// scan runs over the thread totals (left in scnt / sq).  Every caller gets
// the same sums to the bit.
__device__ __forceinline__ void parts_scan(const int32_t *__restrict__ cnt_part,
                                           const DD3 *__restrict__ q_part, int64_t nb, int *scnt,
                                           DD3 *sq, int64_t &b0, int64_t &b1) {
    const int64_t per = cdiv(nb, kBlock);
    b0 = threadIdx.x * per;
    b1 = b0 + per < nb ? b0 + per : nb;
    int c = 0;
    DD3 v = dd_zero();
    for (int64_t b = b0; b < b1; ++b) {
        c += cnt_part[b];
        v = dd_add(v, q_part[b]);
    }
    scnt[threadIdx.x] = c;
    sq[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        int ca = 0;
        DD3 va = dd_zero();
        bool take = (int)threadIdx.x >= o;
        if (take) {
            ca = scnt[threadIdx.x - o];
            va = sq[threadIdx.x - o];
        }
        __syncthreads();
        if (take) {
            scnt[threadIdx.x] += ca;
            sq[threadIdx.x] = dd_add(va, sq[threadIdx.x]);
        }
        __syncthreads();
    }
}

// the totals of all blocks: node count (checked against the node storage)
// and midpoint-summand sum
__device__ __forceinline__ void parts_totals(const int *scnt, const DD3 *sq,
                                             int32_t *__restrict__ node_start,
                                             DD3 *__restrict__ psum, int64_t n,
                                             int32_t *__restrict__ d_m, int64_t cap,
                                             uint32_t *__restrict__ err) {
    int m = scnt[kBlock - 1];
    if (m > cap) {
        atomicOr(err, HTS_ERR_TREE_OVERFLOW);
        m = (int)cap;
    }
    node_start[n] = m;
    psum[n] = sq[kBlock - 1];
    *d_m = m;
}

// one block: exclusive scan of the block aggregates in place; writes the totals
__global__ __launch_bounds__(kBlock) void k_scan_parts(int32_t *__restrict__ cnt_part,
                                                       DD3 *__restrict__ q_part, int64_t nb,
                                                       int32_t *__restrict__ node_start,
                                                       DD3 *__restrict__ psum, int64_t n,
                                                       int32_t *__restrict__ d_m, int64_t cap,
                                                       uint32_t *__restrict__ err) {
    __shared__ int scnt[kBlock];
    __shared__ DD3 sq[kBlock];
    int64_t b0, b1;
    parts_scan(cnt_part, q_part, nb, scnt, sq, b0, b1);
    int ex_c = threadIdx.x > 0 ? scnt[threadIdx.x - 1] : 0;
    DD3 ex_v = threadIdx.x > 0 ? sq[threadIdx.x - 1] : dd_zero();
    for (int64_t b = b0; b < b1; ++b) {
        int cb = cnt_part[b];
        DD3 vb = q_part[b];
        cnt_part[b] = ex_c;
        q_part[b] = ex_v;
        ex_c += cb;
        ex_v = dd_add(ex_v, vb);
    }
    if (threadIdx.x == kBlock - 1) parts_totals(scnt, sq, node_start, psum, n, d_m, cap, err);
}

// Applies the block offsets: node_start[i] (in place of the node counts) and
// the exclusive midpoint-summand sums; then every point records itself as the
// first point of the nodes it starts (node_first), which are stored
// consecutively from node_start[i].  With OWN, the aggregates are the raw
// ones k_sorted left and every workgroup scans them itself as k_scan_parts
// would (the same sums to the bit; one launch fewer, for inputs of few
// blocks); workgroup 0 then writes the totals.
template <bool OWN>
__global__ __launch_bounds__(kBlock) void k_scan_apply(int32_t *__restrict__ cnt,
                                                       DD3 *__restrict__ q, int64_t n,
                                                       const int32_t *__restrict__ cnt_part,
                                                       const DD3 *__restrict__ q_part, int64_t nb,
                                                       int32_t *__restrict__ node_first,
                                                       int32_t *__restrict__ d_m,
                                                       int64_t cap, uint32_t *__restrict__ err) {
    __shared__ int scnt[kBlock];
    __shared__ DD3 sq[kBlock];
    __shared__ int s_bc;
    __shared__ DD3 s_bq;
    int32_t block_c;
    DD3 block_q;
    if (OWN) {
        int64_t b0, b1;
        parts_scan(cnt_part, q_part, nb, scnt, sq, b0, b1);
        const int64_t me = blockIdx.x;
        if (me >= b0 && me < b1) {  // the thread whose range holds this block
            int c = threadIdx.x > 0 ? scnt[threadIdx.x - 1] : 0;
            DD3 v = threadIdx.x > 0 ? sq[threadIdx.x - 1] : dd_zero();
            for (int64_t b = b0; b < me; ++b) {
                c += cnt_part[b];
                v = dd_add(v, q_part[b]);
            }
            s_bc = c;
            s_bq = v;
        }
        if (me == 0 && threadIdx.x == kBlock - 1)
            parts_totals(scnt, sq, cnt, q, n, d_m, cap, err);  // entry n: the totals
        __syncthreads();
        block_c = s_bc;
        block_q = s_bq;
        __syncthreads();
    } else {
        block_c = cnt_part[blockIdx.x];
        block_q = q_part[blockIdx.x];
    }
    int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    scnt[threadIdx.x] = i < n ? cnt[i] : 0;
    sq[threadIdx.x] = i < n ? q[i] : dd_zero();
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        int ca = 0;
        DD3 va = dd_zero();
        bool take = (int)threadIdx.x >= o;
        if (take) {
            ca = scnt[threadIdx.x - o];
            va = sq[threadIdx.x - o];
        }
        __syncthreads();
        if (take) {
            scnt[threadIdx.x] += ca;
            sq[threadIdx.x] = dd_add(va, sq[threadIdx.x]);
        }
        __syncthreads();
    }
    if (i < n) {
        const int ex_c = threadIdx.x > 0 ? scnt[threadIdx.x - 1] : 0;
        const DD3 ex_v = threadIdx.x > 0 ? sq[threadIdx.x - 1] : dd_zero();
        const int c = scnt[threadIdx.x] - ex_c;  // nodes starting at i
        const int32_t base = block_c + ex_c;
        cnt[i] = base;
        q[i] = dd_add(block_q, ex_v);
        for (int a = 0; a < c; ++a) {
            const int64_t k = (int64_t)base + a;
            if (k >= cap) {  // cannot happen for a consistent scan; never write past the storage
                atomicOr(err, HTS_ERR_TREE_OVERFLOW);
                break;
            }
            node_first[k] = (int32_t)i;
        }
    }
}

// ---------------------------------------------------------------- 6. nodes
// radial bounds [lo, hi] of the depth-l cell holding a key (the same
// arithmetic as the keys)
__device__ __forceinline__ void cell_radii(uint64_t key, int l, int L,
                                           const double *__restrict__ root, int split,
                                           double &lo, double &hi) {
    const int64_t job = (int64_t)(key >> (2 * L));
    lo = root[2 * job];
    hi = root[2 * job + 1];
    for (int lev = 0; lev < l; ++lev) {
        const int rb = (int)((key >> (2 * (L - 1 - lev) + 1)) & 1u);
        const double mr = radial_mid(lo, hi, split);
        if (rb) lo = mr; else hi = mr;
    }
}

__device__ __forceinline__ double dd_diff(const DD3 &a, const DD3 &b, int c) {
    double s, e;
    two_sum(a.hi[c], -b.hi[c], s, e);
    e += a.lo[c] - b.lo[c];
    return s + e;
}

// first position j > i whose key differs from keys[i] in the first l levels
// (a cell is a contiguous range of the sorted keys): gallop from i with
// doubling steps, then bisect, so a cell of c points costs about 2 log2(c)
// loads rather than log2(n)
__device__ __forceinline__ int64_t cell_end(const uint64_t *__restrict__ keys, int64_t i, int64_t n,
                                            int l, int L) {
    const int sh = 2 * (L - l);  // the prefix keeps the job bits
    const uint64_t pre = keys[i] >> sh;
    int64_t a = i, b = n, step = 1;  // keys[a] is inside; b is outside (or n)
    for (;;) {
        const int64_t probe = a + step;
        if (probe >= n) break;
        if ((keys[probe] >> sh) != pre) {
            b = probe;
            break;
        }
        a = probe;
        step *= 2;
    }
    int64_t lo = a + 1, hi = b;  // the answer lies in [lo, hi]
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((keys[mid] >> sh) == pre) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// 6. one thread per node: count, subtree end, leaf point or Einstein
// midpoint, and cell diameter (threads of a wave do equal work, whatever the
// length of their points' chains of nodes)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_emit(const uint64_t *__restrict__ keys, int64_t n, int L,
                                                 const PointRec<T> *__restrict__ spts,
                                                 const int32_t *__restrict__ node_start,
                                                 const DD3 *__restrict__ psum,
                                                 const double *__restrict__ root,
                                                 const double *__restrict__ sinhalf,
                                                 NodeRec<T> *__restrict__ nodes,
                                                 double *__restrict__ r_cell,
                                                 const int32_t *__restrict__ node_first,
                                                 const int32_t *__restrict__ d_m, int split,
                                                 double theta, unsigned *__restrict__ dense_count) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    const int32_t M = *d_m;
    if (k >= M) return;
    if (k == 0 && dense_count) *dense_count = 0u;  // for a traversal that follows
    const int64_t i = node_first[k];
    const NodeSpan sp = node_span(keys, i, n, L);
    const int l = sp.s + (int)(k - node_start[i]);
    const uint64_t key = keys[i];
    const bool leaf = (l == sp.D);
    const int64_t end = (leaf && l < L) ? i + 1 : cell_end(keys, i, n, l, L);
    const int32_t count = (int32_t)(end - i);
    const int32_t next = end < n ? node_start[end] : M;
    NodeRec<T> rec;
    rec.count = count;
    rec.next_depth = (uint32_t)next | ((uint32_t)l << kNextBits);
    if constexpr (sizeof(T) == 8) rec.pad = 0.0;
    if (leaf && count == 1) {
        const PointRec<T> p = spts[i];
        rec.mx = p.x;
        rec.my = p.y;
        rec.ib = p.ia;
    } else {
        // Einstein midpoint, eq. (11): Klein average then back to the disk
        const DD3 se = psum[end], si = psum[i];
        const double sx = dd_diff(se, si, 0), sy = dd_diff(se, si, 1), sg = dd_diff(se, si, 2);
        const double kx = sx / sg, ky = sy / sg;
        const double den = 1.0 + sqrt(fmax(0.0, 1.0 - (kx * kx + ky * ky)));
        const T mx = (T)(kx / den), my = (T)(ky / den);
        rec.mx = mx;
        rec.my = my;
        rec.ib = 1.0 / (1.0 - ((double)mx * (double)mx + (double)my * (double)my));
    }
    double lo, hi;
    cell_radii(key, l, L, root, split, lo, hi);
    // hyperbolic diameter: the larger of the outer-arc chord and the
    // diagonal (the radial edge is never longer than the diagonal); the
    // angular half-width is capped at pi/2 for the two top levels
    const double s = sinhalf[l];
    const double ahi = 1.0 - hi * hi, alo = 1.0 - lo * lo;
    const double t_outer = 8.0 * hi * hi * s * s / (ahi * ahi);
    const double dr = hi - lo;
    const double t_diag = 2.0 * (dr * dr + 4.0 * lo * hi * s * s) / (alo * ahi);
    const double t = fmax(t_outer, t_diag);
    const double rc = log1p(t + sqrt(t * (t + 2.0)));
    r_cell[k] = rc;
    // a leaf keeps its first point; an internal node gets its criterion
    // threshold when a gradient that follows gave theta (theta < 0: later)
    rec.c = leaf ? __longlong_as_double((long long)i) : theta >= 0.0 ? node_threshold(rc, theta) : 0.0;
    nodes[k] = rec;
}

__global__ void k_single_job(int64_t *__restrict__ job_off, int32_t *__restrict__ job_qb,
                             int64_t n) {
    if (threadIdx.x == 0) {
        job_off[0] = 0;
        job_off[1] = n;
        job_qb[0] = 0;
        job_qb[1] = (int32_t)cdiv(n, kWave);
    }
}

hts_status tree_single_job(hipStream_t st, hts_tree t, int64_t n) {
    if (t->jobs_set || t->tab_n == n) return HTS_OK;
    hipLaunchKernelGGL(k_single_job, dim3(1), dim3(kWave), 0, st, t->job_off, t->job_qb, n);
    HTS_HIP(hipGetLastError());
    t->tab_n = n;
    t->nqb = cdiv(n, kWave);
    return HTS_OK;
}

// up to this many blocks (points / 256) every workgroup of the apply scans
// the block aggregates itself
constexpr int64_t kOwnScanBlocks = 1024;

template <typename T>
hts_status tree_build(hts_ctx ctx, hipStream_t st, const T *Y, int64_t n, hts_tree t,
                      const TreeExtras<T> *extras) {
    TimedScope ts(ctx, st, HTS_K_TREE);
    HTS_OKR(tree_single_job(st, t, n));
    const int L = t->max_depth;
    const int64_t nb = cdiv(n, kBlock);
    hipLaunchKernelGGL(k_polar<T>, dim3(nb), dim3(kBlock), 0, st, Y, n, t->pjob, t->job_off, t->r,
                       t->mm, t->root);
    HTS_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_keys<T>, dim3(nb), dim3(kBlock), 0, st, t->r, Y, n, t->pjob, t->job_off,
                       t->mm, t->root, L, t->split_rule, t->keys_in, t->idx_in);
    HTS_HIP(hipGetLastError());
    HTS_OKR(radix_sort_pairs(st, t->keys_in, t->idx_in, t->keys, t->perm, n, 2 * L + t->job_bits,
                             t->sort_tmp));
    hipLaunchKernelGGL(k_sorted<T>, dim3(nb), dim3(kBlock), 0, st, Y, n, t->keys, t->perm, L,
                       (PointRec<T> *)t->spts, t->node_start, t->psum, t->ncnt_part, t->q_part,
                       extras ? extras->pts : nullptr, ctx->d_err);
    HTS_HIP(hipGetLastError());
    if (nb <= kOwnScanBlocks) {
        hipLaunchKernelGGL(k_scan_apply<true>, dim3(nb), dim3(kBlock), 0, st, t->node_start, t->psum,
                           n, t->ncnt_part, t->q_part, nb, t->node_first, t->d_m, t->cap_nodes,
                           ctx->d_err);
    } else {
        hipLaunchKernelGGL(k_scan_parts, dim3(1), dim3(kBlock), 0, st, t->ncnt_part, t->q_part, nb,
                           t->node_start, t->psum, n, t->d_m, t->cap_nodes, ctx->d_err);
        HTS_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_scan_apply<false>, dim3(nb), dim3(kBlock), 0, st, t->node_start,
                           t->psum, n, t->ncnt_part, t->q_part, nb, t->node_first, t->d_m,
                           t->cap_nodes, ctx->d_err);
    }
    HTS_HIP(hipGetLastError());
    // over the node capacity for n points; the kernel reads the live count
    int64_t nbm = cdiv(n * (int64_t)(L + 1) + 1, kBlock);
    if (nbm > cdiv(t->cap_nodes, kBlock)) nbm = cdiv(t->cap_nodes, kBlock);
    hipLaunchKernelGGL(k_emit<T>, dim3(nbm), dim3(kBlock), 0, st, t->keys, n, L,
                       (const PointRec<T> *)t->spts, t->node_start, t->psum, t->root, t->sinhalf,
                       (NodeRec<T> *)t->nodes, t->r_cell, t->node_first, t->d_m, t->split_rule,
                       extras ? extras->theta : -1.0, extras ? extras->dense_count : nullptr);
    HTS_HIP(hipGetLastError());
    t->n = n;
    t->dtype = sizeof(T) == 8 ? HTS_F64 : HTS_F32;
    return HTS_OK;
}

// temporary storage of the sort
hts_status tree_sort_bytes(int64_t n_max, int L, size_t *bytes) {
    (void)L;
    *bytes = radix_sort_temp_bytes(n_max);
    return HTS_OK;
}

// ---------------------------------------------------------------- Euclidean summaries
// For the Euclidean Student-t term of h-SNE (Sec. 4-C) the same tree is walked
// with Euclidean cell summaries: the centre of mass of a cell's points (from
// double-double prefix sums of the sorted coordinates) and the criterion
// ediam / |y - c| < theta, tested as |y - c|^2 > (ediam / theta)^2 with the
// Euclidean diameter ediam = max(2 r_hi s, sqrt((r_hi - r_lo)^2 + 4 r_lo r_hi s^2)),
// s the sine of half the (capped) angular width: the larger of the outer
// chord and the diagonal, the farthest pair of corners of a polar cell.

__device__ __forceinline__ DD2 dd2_add(const DD2 &a, const DD2 &b) {
    DD2 r;
#pragma unroll
    for (int c = 0; c < 2; ++c) {
        double s, e;
        two_sum(a.hi[c], b.hi[c], s, e);
        e += a.lo[c] + b.lo[c];
        const double h = s + e;
        r.lo[c] = e - (h - s);
        r.hi[c] = h;
    }
    return r;
}
__device__ __forceinline__ DD2 dd2_zero() {
    DD2 r;
    r.hi[0] = r.hi[1] = r.lo[0] = r.lo[1] = 0.0;
    return r;
}

// block aggregates of the sorted coordinates
template <typename T>
__global__ __launch_bounds__(kBlock) void k_esum(const PointRec<T> *__restrict__ spts, int64_t n,
                                                 DD2 *__restrict__ part) {
    __shared__ DD2 sq[kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    DD2 v = dd2_zero();
    if (i < n) {
        v.hi[0] = (double)spts[i].x;
        v.hi[1] = (double)spts[i].y;
    }
    sq[threadIdx.x] = v;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) sq[threadIdx.x] = dd2_add(sq[threadIdx.x], sq[threadIdx.x + s]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sq[0];
}

// one block: exclusive scan of the block aggregates in place
__global__ __launch_bounds__(kBlock) void k_escan_parts(DD2 *__restrict__ part, int64_t nb) {
    __shared__ DD2 sq[kBlock];
    const int64_t per = cdiv(nb, kBlock);
    const int64_t b0 = threadIdx.x * per, b1 = b0 + per < nb ? b0 + per : nb;
    DD2 v = dd2_zero();
    for (int64_t b = b0; b < b1; ++b) v = dd2_add(v, part[b]);
    sq[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const bool take = (int)threadIdx.x >= o;
        const DD2 va = take ? sq[threadIdx.x - o] : dd2_zero();
        __syncthreads();
        if (take) sq[threadIdx.x] = dd2_add(va, sq[threadIdx.x]);
        __syncthreads();
    }
    DD2 ex = threadIdx.x > 0 ? sq[threadIdx.x - 1] : dd2_zero();
    for (int64_t b = b0; b < b1; ++b) {
        const DD2 vb = part[b];
        part[b] = ex;
        ex = dd2_add(ex, vb);
    }
}

// exclusive prefix sums psum[0..n] of the sorted coordinates
template <typename T>
__global__ __launch_bounds__(kBlock) void k_escan_apply(const PointRec<T> *__restrict__ spts,
                                                        int64_t n, const DD2 *__restrict__ part,
                                                        DD2 *__restrict__ psum) {
    __shared__ DD2 sq[kBlock];
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    DD2 v = dd2_zero();
    if (i < n) {
        v.hi[0] = (double)spts[i].x;
        v.hi[1] = (double)spts[i].y;
    }
    sq[threadIdx.x] = v;
    __syncthreads();
    for (int o = 1; o < kBlock; o <<= 1) {
        const bool take = (int)threadIdx.x >= o;
        const DD2 va = take ? sq[threadIdx.x - o] : dd2_zero();
        __syncthreads();
        if (take) sq[threadIdx.x] = dd2_add(va, sq[threadIdx.x]);
        __syncthreads();
    }
    if (i < n) {
        const DD2 ex = threadIdx.x > 0 ? sq[threadIdx.x - 1] : dd2_zero();
        psum[i] = dd2_add(part[blockIdx.x], ex);
        if (i == n - 1) psum[n] = dd2_add(part[blockIdx.x], sq[threadIdx.x]);
    }
}

// one thread per node: the Euclidean record (count and links as the
// hyperbolic record; leaves unchanged, internal nodes with their centre of
// mass and Euclidean threshold)
template <typename T>
__global__ __launch_bounds__(kBlock) void k_emit_euclid(const NodeRec<T> *__restrict__ nodes,
                                                        const int32_t *__restrict__ d_m,
                                                        const int32_t *__restrict__ node_first,
                                                        const uint64_t *__restrict__ keys, int L,
                                                        const double *__restrict__ root, int split,
                                                        const double *__restrict__ sinhalf,
                                                        const DD2 *__restrict__ psum, double theta,
                                                        NodeRec<T> *__restrict__ enodes) {
    const int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= *d_m) return;
    NodeRec<T> rec = nodes[k];
    const uint32_t next = rec.next_depth & kNextMask;
    if ((int64_t)next != k + 1) {
        const int l = (int)(rec.next_depth >> kNextBits);
        const int64_t i = node_first[k];
        const int64_t end = i + rec.count;
        const DD2 se = psum[end], si = psum[i];
        double c[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            double sm, e;
            two_sum(se.hi[a], -si.hi[a], sm, e);
            e += se.lo[a] - si.lo[a];
            c[a] = (sm + e) / (double)rec.count;
        }
        rec.mx = (T)c[0];
        rec.my = (T)c[1];
        rec.ib = 0.0;
        double lo, hi;
        cell_radii(keys[i], l, L, root, split, lo, hi);
        const double s = sinhalf[l];
        const double outer = 2.0 * hi * s;
        const double dr = hi - lo;
        const double diag = sqrt(dr * dr + 4.0 * lo * hi * s * s);
        const double diam = fmax(outer, diag);
        if (theta > 0.0) {
            const double q = diam / theta;
            rec.c = q * q;
        } else {
            rec.c = __builtin_inf();
        }
    }
    enodes[k] = rec;
}

template <typename T>
hts_status tree_euclid(hts_ctx ctx, hipStream_t st, hts_tree t, double theta) {
    TimedScope ts(ctx, st, HTS_K_TREE);
    const int64_t n = t->n;
    const int64_t nb = cdiv(n, kBlock);
    const PointRec<T> *spts = (const PointRec<T> *)t->spts;
    hipLaunchKernelGGL(k_esum<T>, dim3(nb), dim3(kBlock), 0, st, spts, n, t->epart);
    hipLaunchKernelGGL(k_escan_parts, dim3(1), dim3(kBlock), 0, st, t->epart, nb);
    hipLaunchKernelGGL(k_escan_apply<T>, dim3(nb), dim3(kBlock), 0, st, spts, n, t->epart,
                       t->epsum);
    int64_t nbm = cdiv(n * (int64_t)(t->max_depth + 1) + 1, kBlock);
    if (nbm > cdiv(t->cap_nodes, kBlock)) nbm = cdiv(t->cap_nodes, kBlock);
    hipLaunchKernelGGL(k_emit_euclid<T>, dim3(nbm), dim3(kBlock), 0, st,
                       (const NodeRec<T> *)t->nodes, t->d_m, t->node_first, t->keys, t->max_depth,
                       t->root, t->split_rule, t->sinhalf, t->epsum, theta,
                       (NodeRec<T> *)t->enodes);
    HTS_HIP(hipGetLastError());
    return HTS_OK;
}

template hts_status tree_euclid<float>(hts_ctx, hipStream_t, hts_tree, double);
template hts_status tree_euclid<double>(hts_ctx, hipStream_t, hts_tree, double);

template hts_status tree_build<float>(hts_ctx, hipStream_t, const float *, int64_t, hts_tree,
                                     const TreeExtras<float> *);
template hts_status tree_build<double>(hts_ctx, hipStream_t, const double *, int64_t, hts_tree,
                                      const TreeExtras<double> *);

}  // namespace hts
