// k_bh.hip -- Barnes-Hut repulsion over the polar quadtree (eq. (19) and the
// depth-first traversal of Sec. 4-B).
//
// A query block is 64 consecutive points of the key order (spatial
// neighbours), one per lane of a wave.  The block walks the tree depth-first;
// the node index is uniform across the wave and each lane keeps its own
// criterion decision: at an internal node a lane either accepts the cell
// (r_cell / d(y_i, m) < theta, tested as t > cosh(r_cell / theta) - 1 with the
// distance argument t in double) and adds N_cell w^2 d dd/dy, or joins the
// set of lanes that need the children.  Leaves are evaluated exactly, skipping
// the query.  The lanes that need a subtree form a 64-bit mask per depth, kept
// in two VGPRs used as lane-indexed arrays (readlane with the depth to read,
// a lane select to write), and a mask serves directly as the lane predicate
// of the masked term.  Node records are read with scalar loads; the next
// sibling's is in flight while a node is evaluated, and so is the first
// child's in the walks of the work items (phase A loads it when it descends);
// enough waves per SIMD hide most of the latency.
//
// One wave walking the whole tree for its block is a long serial chain, so the
// walk is split in two phases:
//  A. four waves per query block, one per subtree below the root, walk the
//     nodes that hold more than S points; when some lanes reject a smaller
//     cell, the cell and their mask become a work item instead of being
//     descended;
//  B. waves walk the work items, each a short independent chain; an item
//     record is self-contained (subtree, lane mask, query block).  The grid
//     holds several times the waves that fit on the chip, so the hardware
//     hands the next waves (and their items) to whichever SIMD frees up.
// Every item writes its own partial force per lane and partial Z; the items
// of a phase-A wave occupy one contiguous run of the item list, and the
// combine adds, per query block, its waves' partials and runs in a fixed
// order, so the result does not depend on scheduling.
//
// The walk is written once over a metric (Geo<MET>): the Poincare disk for
// the hyperbolic gradient, and the Euclidean Student-t kernel of the disk
// coordinates for the first part of the h-SNE gradient (Sec. 4-C), which walks
// the same tree with Euclidean node records.
#include "hts_impl.hpp"
#include "hts_math.hpp"

namespace hts {

constexpr int kStats = kBhStats;
constexpr int kAttractLanes = 16;  // lanes per CSR row of the attractive term
constexpr int64_t kAttractWithTopAt = 131072;  // automatic placement threshold (points of a job)
constexpr int kItemCap = 256;  // items one phase-A wave can hand to phase B
// The item list holds ctx->list_items items per phase-A wave (kItemCap by
// default: every item a wave records); a wave hands over at most that many
// and walks the rest itself (see k_bh_top).
constexpr int kTopDepth = 1;   // phase A splits each query block's walk at this depth ...
constexpr int kTopSlots = 1 << (2 * kTopDepth);  // ... over this many waves

// work item as phase A records it (in LDS) ...
struct LdsItem {
    int32_t node;      // pre-order index of the rejected cell
    uint32_t nd;       // its next | depth word
    uint64_t mask;     // lanes that rejected it
};
// ... and as phase B reads it (one 32-byte scalar load)
struct alignas(16) ItemRec {
    int32_t node;
    uint32_t nd;
    int32_t q0;        // first query point (sorted position) of the block
    int32_t cnt;       // query points in the block
    uint64_t mask;
    uint64_t pad;
};

struct Counters {
    unsigned long long test = 0, acc = 0, pair = 0, step = 0, work = 0, cover = 0;
};

// Depth-first walk of the pre-order range [k, kend), which starts at a node
// of depth d0 and holds its subtree, for the lanes in mask0.  With EMIT, an
// internal node of at most S points that some lanes reject is appended to the
// wave's item list (while there is room) instead of being descended.  The
// walk's Z terms are summed in T and added to z once at the end.
// Node records are read with scalar loads (the node index is uniform).
// Internal nodes are walked in an inner loop and each leaf in the outer one,
// so the accumulators keep their registers across the masked terms.  A
// successor index is at most M, and the node arrays hold more than M records
// (their capacity n_max (depth cap + 1) + 1 exceeds any node count), so the
// successor of the last node is a readable record that is never used.
// THRU marks the walks of phase B, which run among many waves and are bound
// by instruction issue: there scalar branches that save vector instructions
// pay (the term's wave-uniform branch choice, and the mask of the current
// depth kept in scalar registers and read from the stack only when the walk
// moves up); in phase A, a chain of dependent steps, they would lengthen it.
template <typename T, int MET, bool STATS, bool EMIT, bool THRU = false>
__device__ __forceinline__ void walk(const NodeRec<T> *__restrict__ nodes, int M,
                                     const PointRec<T> *__restrict__ spts, const PointRec<T> &me,
                                     int64_t q, int lane, int k, int kend, int d0, uint64_t mask0,
                                     int S, LdsItem *items, int &nitems, T &fx, T &fy, double &z,
                                     Counters &c) {
    T zw = 0;  // this walk's Z terms, added to z once at the end
    int mlo = lane == d0 ? (int)(uint32_t)mask0 : 0;
    int mhi = lane == d0 ? (int)(uint32_t)(mask0 >> 32) : 0;
    // with THRU, the mask of depth mdep (equal to its stack entry)
    uint64_t mc = mask0;
    int mdep = d0;
    auto mask_at = [&](int depth) -> uint64_t {
        if (THRU && depth == mdep) return mc;
        const uint64_t m = ((uint64_t)(uint32_t)__builtin_amdgcn_readlane(mhi, depth) << 32) |
                           (uint64_t)(uint32_t)__builtin_amdgcn_readlane(mlo, depth);
        if (THRU) {
            mc = m;
            mdep = depth;
        }
        return m;
    };
    NodeRec<T> nrec = nodes[k < M ? k : M - 1];
    while (k < kend) {
        NodeRec<T> cur = nrec;
        uint32_t nxd = (uint32_t)uniform((int)cur.next_depth);
        int next = (int)(nxd & kNextMask);
        // internal nodes, until the walk meets a leaf or leaves its range
        // (one exit test per pass; past the range the record read is the
        // unused one after it)
        bool inner = next != k + 1;
        while (inner) {
            const int depth = (int)(nxd >> kNextBits);
            const uint64_t m = mask_at(depth);
            // the next sibling's record is loaded before the test and the term
            // (the compiler barrier keeps the load from sinking to its use);
            // the first child's too in the walks that emit no items, and only
            // on descent in those that do (phase A)
            const NodeRec<T> over = nodes[(uint32_t)next];
            NodeRec<T> first_child;
            if (!EMIT) first_child = nodes[(uint32_t)(k + 1)];
            asm volatile("" ::: "memory");
            if (STATS) c.step += 1;
            // the test costs the same for every lane (some lane of the wave
            // is always in the mask here); only the term is masked, by the
            // lanes of m that accept (the masks serve as lane predicates
            // directly, with no vector work)
            double dd;
            const double t = Geo<MET>::arg(me, cur.mx, cur.my, cur.ib, dd);
            const uint64_t am = __builtin_amdgcn_ballot_w64(t > cur.c) & m;
            if (__builtin_amdgcn_inverse_ballot_w64(am))
                Geo<MET>::template repel<THRU>(me, cur.mx, cur.my, cur.ib, t, dd, (T)cur.count, fx, fy, zw);
            const uint64_t rej = m & ~am;
            if (STATS) {
                c.test += __popcll(m);
                c.acc += __popcll(am);
                c.work += am != 0;
                c.cover += (unsigned long long)__popcll(am) * (unsigned)cur.count;
            }
            if (EMIT && rej && cur.count <= S && nitems < kItemCap) {
                if (lane == 0) items[nitems] = LdsItem{k, nxd, rej};
                ++nitems;
                k = next;
                nrec = over;
            } else if (rej) {
                const bool here = lane == depth + 1;
                mlo = here ? (int)(uint32_t)rej : mlo;
                mhi = here ? (int)(uint32_t)(rej >> 32) : mhi;
                if (THRU) {
                    mc = rej;
                    mdep = depth + 1;
                }
                nrec = !EMIT ? first_child : nodes[(uint32_t)(k + 1)];
                k = k + 1;
            } else {
                k = next;
                nrec = over;
            }
            cur = nrec;
            nxd = (uint32_t)uniform((int)cur.next_depth);
            next = (int)(nxd & kNextMask);
            inner = (k < kend) & (next != k + 1);
        }
        if (k >= kend) break;
        // leaf: exact terms with each of its points, skipping the query
        const int depth = (int)(nxd >> kNextBits);
        const uint64_t m = mask_at(depth);
        const bool in = __builtin_amdgcn_inverse_ballot_w64(m);
        const NodeRec<T> over = nodes[(uint32_t)next];
        if (STATS) c.step += 1;
        const int64_t first = (int64_t)__double_as_longlong(cur.c);
        const int cnt = uniform(cur.count);
        if (cnt == 1) {
            const bool use = in && first != q;
            if (use) {
                double dd;
                double t = Geo<MET>::arg(me, cur.mx, cur.my, cur.ib, dd);
                Geo<MET>::template repel<THRU>(me, cur.mx, cur.my, cur.ib, t, dd, (T)1, fx, fy, zw);
            }
            if (STATS) {
                const uint64_t um = __ballot(use);
                c.pair += __popcll(um);
                c.cover += __popcll(um);
                c.work += um != 0;
            }
        } else {
            for (int a = 0; a < cnt; ++a) {
                const PointRec<T> o = spts[first + a];
                const bool use = in && (first + a) != q;
                if (use) {
                    double dd;
                    double t = Geo<MET>::arg(me, o.x, o.y, o.ia, dd);
                    Geo<MET>::template repel<THRU>(me, o.x, o.y, o.ia, t, dd, (T)1, fx, fy, zw);
                }
                if (STATS) {
                    const int u = __popcll(__ballot(use));
                    c.pair += u;
                    c.cover += u;
                }
            }
        }
        k = next;
        nrec = over;
    }
    z += (double)zw;
}

template <bool STATS>
__device__ __forceinline__ void put_stats(uint32_t *__restrict__ sp, const Counters &c) {
    if (!STATS) return;
    sp[0] = (uint32_t)c.test;
    sp[1] = (uint32_t)c.acc;
    sp[2] = (uint32_t)c.pair;
    sp[3] = (uint32_t)c.step;
    sp[4] = (uint32_t)c.work;
    sp[5] = (uint32_t)c.cover;
}

// Phase A: the walk of a query block over the nodes of more than S points,
// split over kTopSlots = 4^kTopDepth waves.  Slot s owns one node f of the
// frontier at depth kTopDepth (its base-4 digits pick the child at each level
// below the root; a leaf above that depth belongs to the slot whose remaining
// digits are 0; a slot naming a missing child is idle).  The wave first tests
// the ancestors of f for its lanes -- a lane that accepts one, or whose
// rejected ancestor becomes a work item, leaves the walk -- then walks f's
// subtree.  An ancestor's term, item and counters belong to the one slot whose
// digits below it are all 0, so every lane meets every cell exactly as in a
// single depth-first walk.  These waves are latency-bound chains.  The
// attractive term (first sum of eq. (15)) runs either in this launch, in the
// workgroups from top_blocks on, where its waves compete with the chains for
// issue and are hidden when the chains are long, or in the last workgroups of
// phase B's launch (hts_set_attract_launch).
template <typename T, int MET, bool STATS>
__global__ __launch_bounds__(kBlock) void k_bh_top(
    const NodeRec<T> *__restrict__ nodes, const int32_t *__restrict__ d_m,
    const int32_t *__restrict__ node_start, Jobs jb, const PointRec<T> *__restrict__ spts,
    int64_t nqb, int S, int *__restrict__ item_base, int *__restrict__ nitems_out,
    T *__restrict__ part0, double *__restrict__ ztop, uint32_t *__restrict__ stats_top,
    unsigned *__restrict__ dense_count, ItemRec *__restrict__ dense, int share, int64_t n,
    int64_t top_blocks, const PointRec<T> *__restrict__ pts, const int64_t *__restrict__ rp,
    const int32_t *__restrict__ col, const T *__restrict__ val, T *__restrict__ fattr,
    uint32_t *__restrict__ err) {
    __shared__ LdsItem s_items[kBlock / kWave][kItemCap];
    if ((int64_t)blockIdx.x >= top_blocks) {
        attract_rows<T, kAttractLanes, MET>(((int64_t)blockIdx.x - top_blocks) * kBlock + threadIdx.x,
                                            pts, rp, col, val, n, fattr, err);
        return;
    }
    const int64_t g = (int64_t)blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    const int64_t qb = g / kTopSlots;
    const int slot = (int)(g % kTopSlots);
    if (qb >= nqb) return;
    const int lane = (int)(threadIdx.x & (kWave - 1));
    LdsItem *items = s_items[threadIdx.x / kWave];
    int64_t q0;
    int cnt, job;
    jb.block(qb, q0, cnt, job);
    q0 = uniform((int)q0);
    cnt = uniform(cnt);
    job = uniform(job);
    const int64_t q = q0 + lane;
    const bool valid = lane < cnt;
    const PointRec<T> me = spts[valid ? q : q0];
    const int M = uniform(*d_m);
    // the job's tree: the pre-order range from its root
    int a = uniform(node_start[jb.off[job]]);
    T fx = 0, fy = 0;
    double z = 0.0;
    Counters c;
    int nitems = 0;
    uint64_t m = __ballot(valid);
    bool live = true;
    for (int d = 0; d < kTopDepth; ++d) {
        const NodeRec<T> A = nodes[a];
        const uint32_t nxd = (uint32_t)uniform((int)A.next_depth);
        const int nx = (int)(nxd & kNextMask);
        // this slot owns node a when its digits below depth d are all 0
        const bool owner = (slot & ((1 << (2 * (kTopDepth - d))) - 1)) == 0;
        if (nx == a + 1) {  // a leaf above the frontier depth: its owner walks it
            live = owner;
            break;
        }
        const bool in = (m >> lane) & 1ull;
        bool acc = false;
        if (in) {
            double dd;
            const double t = Geo<MET>::arg(me, A.mx, A.my, A.ib, dd);
            acc = t > A.c;
            if (acc && owner) Geo<MET>::repel(me, A.mx, A.my, A.ib, t, dd, (T)A.count, fx, fy, z);
        }
        const uint64_t rej = __ballot(in && !acc);
        if (STATS && owner) {
            const uint64_t am = __ballot(acc);
            c.test += __popcll(m);
            c.acc += __popcll(am);
            c.step += 1;
            c.work += am != 0;
            c.cover += (unsigned long long)__popcll(am) * (unsigned)A.count;
        }
        if (rej && A.count <= S) {  // the rejecting lanes take the cell as one work item
            if (owner) {
                if (lane == 0) items[nitems] = LdsItem{a, nxd, rej};
                ++nitems;
            }
            m = 0;
        } else {
            m = rej;
        }
        if (!m) break;
        // the child picked by this slot's digit at depth d + 1
        const int digit = (slot >> (2 * (kTopDepth - 1 - d))) & 3;
        int ch = a + 1;
        for (int i = 0; i < digit && ch < nx; ++i)
            ch = (int)((uint32_t)uniform((int)nodes[ch].next_depth) & kNextMask);
        if (ch >= nx) {
            live = false;
            break;
        }
        a = ch;
    }
    if (live && m) {
        const int nxa = (int)((uint32_t)uniform((int)nodes[a].next_depth) & kNextMask);
        const int da = (int)((uint32_t)uniform((int)nodes[a].next_depth) >> kNextBits);
        walk<T, MET, STATS, true>(nodes, M, spts, me, q, lane, a, nxa, da, m, S, items, nitems,
                                   fx, fy, z, c);
    }
    // hand over at most this wave's share of the item list (the share depends
    // on nothing but the wave, so neither does the result); reserve a
    // contiguous run for it (one atomic per wave; the runs of different waves
    // may come in any order)
    const int hand = nitems < share ? nitems : share;
    int base = 0;
    if (lane == 0 && hand > 0) base = (int)atomicAdd(dense_count, (unsigned)hand);
    base = __shfl(base, 0, 64);
    // the records were written to LDS by lane 0 of this wave
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
    for (int j = lane; j < hand; j += kWave) {
        const LdsItem it = items[j];
        dense[base + j] = ItemRec{it.node, it.nd, (int32_t)q0, cnt, it.mask, 0};
    }
    // items beyond the share: this wave makes the walks phase B would have made
    // (same cells, same lanes, nothing more handed over)
    int none = 0;
    for (int j = hand; j < nitems; ++j) {
        const LdsItem it = items[j];
        const int node = uniform(it.node);
        const uint32_t nd = (uint32_t)uniform((int)it.nd);
        const uint64_t im = ((uint64_t)(uint32_t)uniform((int)(it.mask >> 32)) << 32) |
                            (uint64_t)(uint32_t)uniform((int)it.mask);
        walk<T, MET, STATS, false>(nodes, M, spts, me, q, lane, node + 1, (int)(nd & kNextMask),
                                    (int)(nd >> kNextBits) + 1, im, 0, nullptr, none, fx, fy, z, c);
    }
    if (valid) {
        part0[((int64_t)slot * n + q) * 2] = fx;
        part0[((int64_t)slot * n + q) * 2 + 1] = fy;
    }
    const double zs = wave_sum(z);
    if (lane == 0) {
        ztop[g] = zs;
        item_base[g] = base;
        nitems_out[g] = hand;
        put_stats<STATS>(stats_top + g * kStats, c);
    }
}

// Before a traversal: clears the item-list counter (a kernel, not a memset,
// so the sequence can be captured in a graph), and as asked writes the point
// records of Y and the criterion thresholds of the internal nodes.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bh_prepare(const T *__restrict__ Y, int64_t n,
                                                       PointRec<T> *__restrict__ pts, bool points,
                                                       NodeRec<T> *__restrict__ nodes,
                                                       const double *__restrict__ r_cell,
                                                       const int32_t *__restrict__ d_m,
                                                       double theta, bool thresholds,
                                                       unsigned *__restrict__ dense_count,
                                                       uint32_t *__restrict__ err) {
    const int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (i == 0 && dense_count) *dense_count = 0u;
    if (points && i < n) prep_point<T>(Y, i, pts, err);
    if (thresholds) {
        const int64_t M = *d_m;
        const int64_t G = (int64_t)gridDim.x * kBlock;
        for (int64_t k = i; k < M; k += G) {
            const uint32_t next = nodes[k].next_depth & kNextMask;
            if ((int64_t)next != k + 1) nodes[k].c = node_threshold(r_cell[k], theta);
        }
    }
}

// one item record in scalar registers
__device__ __forceinline__ ItemRec load_item(const ItemRec *__restrict__ dense, int64_t i) {
    const ItemRec r = dense[i];
    ItemRec u;
    u.node = uniform(r.node);
    u.nd = (uint32_t)uniform((int)r.nd);
    u.q0 = uniform(r.q0);
    u.cnt = uniform(r.cnt);
    u.mask = ((uint64_t)(uint32_t)uniform((int)(r.mask >> 32)) << 32) |
             (uint64_t)(uint32_t)uniform((int)r.mask);
    u.pad = 0;
    return u;
}

// Phase B: wave w walks items w, w + G, ... of the item list (G waves in the
// grid; a workgroup holds 1, 2 or 4 waves).
template <typename T, int MET, bool STATS>
__global__ __launch_bounds__(kBlock) void k_bh_items(
    const NodeRec<T> *__restrict__ nodes, const int32_t *__restrict__ d_m,
    const PointRec<T> *__restrict__ spts, const unsigned *__restrict__ dense_count,
    const ItemRec *__restrict__ dense, int64_t cap, T *__restrict__ part,
    double *__restrict__ zitem, uint32_t *__restrict__ stats_items, int64_t item_blocks,
    const PointRec<T> *__restrict__ pts, const int64_t *__restrict__ rp,
    const int32_t *__restrict__ col, const T *__restrict__ val, int64_t n, T *__restrict__ fattr,
    uint32_t *__restrict__ err) {
    // the workgroups past the items' compute the attractive rows when they
    // run here: they start last, and fill the chip while the longest walks
    // finish
    if ((int64_t)blockIdx.x >= item_blocks) {
        attract_rows<T, kAttractLanes, MET>(((int64_t)blockIdx.x - item_blocks) * blockDim.x +
                                                threadIdx.x, pts, rp, col, val, n, fattr, err);
        return;
    }
    const int lane = (int)(threadIdx.x & (kWave - 1));
    const int M = uniform(*d_m);
    const int64_t reserved = (int64_t)(uint32_t)uniform((int)*dense_count);
    const int64_t total = reserved < cap ? reserved : cap;  // never more, by the shares
    const int wpb = (int)(blockDim.x / kWave);
    const int64_t G = item_blocks * wpb;
    int dummy = 0;
    for (int64_t i = (int64_t)blockIdx.x * wpb + threadIdx.x / kWave; i < total; i += G) {
        const ItemRec rec = load_item(dense, i);
        const PointRec<T> me = spts[lane < rec.cnt ? rec.q0 + lane : rec.q0];
        const int64_t q = (int64_t)rec.q0 + lane;
        const bool valid = lane < rec.cnt;
        T fx = 0, fy = 0;
        double z = 0.0;
        Counters c;
        walk<T, MET, STATS, false, true>(nodes, M, spts, me, q, lane, rec.node + 1,
                                   (int)(rec.nd & kNextMask), (int)(rec.nd >> kNextBits) + 1,
                                   rec.mask, 0, nullptr, dummy, fx, fy, z, c);
        if (valid) {
            T *o = part + (i * kWave + lane) * 2;
            o[0] = fx;
            o[1] = fy;
        }
        const double zs = wave_sum(z);
        if (lane == 0) {
            zitem[i] = zs;
            put_stats<STATS>(stats_items + i * kStats, c);
        }
    }
}

// Combine, stage 1: one workgroup per query block, one wave per phase-A slot.
// Wave s adds its slot's phase-A partial and then its items' partials in item
// order (eight loads in flight at a time); the first wave then adds the four
// slot sums in slot order and applies the query's common factor of the terms.
// The order of every sum is fixed, so the result does not depend on
// scheduling.  The counters of the block are added to the caller's totals.
static_assert(kTopSlots == kBlock / kWave, "one wave per phase-A slot");
template <typename T, int MET, bool STATS>
__global__ __launch_bounds__(kBlock) void k_bh_gather(
    const PointRec<T> *__restrict__ spts,
    const T *__restrict__ part0, const double *__restrict__ ztop, const T *__restrict__ part,
    const double *__restrict__ zitem, const int *__restrict__ item_base,
    const int *__restrict__ nitems_in, Jobs jb, int64_t nqb, int64_t n, T *__restrict__ frep,
    double *__restrict__ zq, const uint32_t *__restrict__ stats_top,
    const uint32_t *__restrict__ stats_items, unsigned long long *__restrict__ stats) {
    __shared__ T s_f[kTopSlots][2][kWave];
    __shared__ double s_z[kTopSlots];
    const int64_t qb = blockIdx.x;
    if (qb >= nqb) return;  // the whole workgroup
    const int sl = (int)(threadIdx.x / kWave);
    const int lane = (int)(threadIdx.x & (kWave - 1));
    int64_t q0;
    int cnt, job;
    jb.block(qb, q0, cnt, job);
    const int64_t q = q0 + lane;
    const bool valid = lane < cnt;
    T fx = 0, fy = 0;
    const int64_t g = qb * kTopSlots + sl;
    const int64_t b0 = uniform(item_base[g]);
    const int ni = uniform(nitems_in[g]);
    if (valid) {
        fx = part0[((int64_t)sl * n + q) * 2];
        fy = part0[((int64_t)sl * n + q) * 2 + 1];
        constexpr int U = 8;
        int j = 0;
        for (; j + U <= ni; j += U) {
            T px[U], py[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const T *p = part + ((b0 + j + u) * kWave + lane) * 2;
                px[u] = p[0];
                py[u] = p[1];
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                fx += px[u];
                fy += py[u];
            }
        }
        for (; j < ni; ++j) {
            const T *p = part + ((b0 + j) * kWave + lane) * 2;
            fx += p[0];
            fy += p[1];
        }
    }
    double zl = 0.0;
    for (int j = lane; j < ni; j += kWave) zl += zitem[b0 + j];
    const double zs = ztop[g] + wave_sum(zl);
    s_f[sl][0][lane] = fx;
    s_f[sl][1][lane] = fy;
    if (lane == 0) s_z[sl] = zs;
    if (STATS) {
        unsigned long long s_it[kStats], s_all[kStats];
#pragma unroll
        for (int a = 0; a < kStats; ++a) s_it[a] = s_all[a] = 0;
        for (int j = lane; j < ni; j += kWave)
#pragma unroll
            for (int a = 0; a < kStats; ++a) s_it[a] += stats_items[(b0 + j) * kStats + a];
        if (lane == 0)
#pragma unroll
            for (int a = 0; a < kStats; ++a) s_all[a] = stats_top[g * kStats + a];
#pragma unroll
        for (int a = 0; a < kStats; ++a) {
            unsigned long long v = s_it[a], w = s_all[a];
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                v += __shfl_xor(v, o, 64);
                w += __shfl_xor(w, o, 64);
            }
            if (lane == 0) {
                atomicAdd(&stats[a], v + w);
                atomicAdd(&stats[kStats + a], v);
            }
        }
    }
    __syncthreads();
    if (sl != 0) return;
    double zb = s_z[0];
#pragma unroll
    for (int a = 1; a < kTopSlots; ++a) zb += s_z[a];
    if (valid) {
        T sx = s_f[0][0][lane], sy = s_f[0][1][lane];
#pragma unroll
        for (int a = 1; a < kTopSlots; ++a) {
            sx += s_f[a][0][lane];
            sy += s_f[a][1][lane];
        }
        // the query's common factor of the repulsive terms, once
        const T f = Geo<MET>::qfactor(spts[q]);
        frep[2 * q] = sx * f;
        frep[2 * q + 1] = sy * f;
    }
    if (lane == 0) zq[qb] = zb;
}

// Combine, stage 2: g_i = 4 (a F_attr,i - F_rep,i / Z) scattered to input
// order; with `accumulate`, grad_i + scale g_i is stored instead (the second
// term of a sum of gradients).  Z of a job is the sum of its query blocks'
// totals, formed by every workgroup that holds points of the job the same way
// (one wave: four lane-strided partial sums per lane, then a fixed butterfly), so
// all of them use the same value; the workgroup holding the job's first point
// writes it to z_dev.
template <typename T>
__global__ __launch_bounds__(kBlock) void k_bh_finalize(
    const T *__restrict__ fattr, const T *__restrict__ frep, const double *__restrict__ zq,
    Jobs jb, const uint32_t *__restrict__ perm, int64_t n, double ex,
    const double *__restrict__ ex_job, bool accumulate, double scale, T *__restrict__ grad,
    double *__restrict__ z_dev, uint32_t *__restrict__ err) {
    __shared__ double s_z[kBlock];  // a job holds at least one point of the workgroup
    const int64_t b0 = (int64_t)blockIdx.x * kBlock;
    const int64_t bl = (b0 + kBlock < n ? b0 + kBlock : n) - 1;
    const int j0 = jb.pjob[b0], j1 = jb.pjob[bl];
    const int wave = (int)(threadIdx.x / kWave), lane = (int)(threadIdx.x & (kWave - 1));
    for (int j = j0 + wave; j <= j1; j += kBlock / kWave) {
        const int64_t a0 = jb.job_qb[j], a1 = jb.job_qb[j + 1];
        // four partial sums per lane keep four loads in flight
        double z0 = 0.0, z1 = 0.0, z2 = 0.0, z3 = 0.0;
        int64_t a = a0 + lane;
        for (; a + 3 * kWave < a1; a += 4 * kWave) {
            z0 += zq[a];
            z1 += zq[a + kWave];
            z2 += zq[a + 2 * kWave];
            z3 += zq[a + 3 * kWave];
        }
        for (; a < a1; a += kWave) z0 += zq[a];
        const double zs = wave_sum((z0 + z1) + (z2 + z3));
        if (lane == 0) {
            s_z[j - j0] = zs;
            const int64_t f = jb.off[j];
            if (f >= b0 && f <= bl) z_dev[j] = zs;
        }
    }
    __syncthreads();
    const int64_t q = b0 + threadIdx.x;
    if (q >= n) return;
    // sorted positions of a job cover the same range as its input points
    const int job = jb.pjob[q];
    const double a = ex_job ? ex_job[job] : ex;
    const uint32_t i = perm[q];
    const double inv = 1.0 / s_z[job - j0];
    double gx = 4.0 * (a * (double)fattr[2 * (int64_t)i] - (double)frep[2 * q] * inv);
    double gy = 4.0 * (a * (double)fattr[2 * (int64_t)i + 1] - (double)frep[2 * q + 1] * inv);
    if (accumulate) {
        gx = (double)grad[2 * (int64_t)i] + scale * gx;
        gy = (double)grad[2 * (int64_t)i + 1] + scale * gy;
    }
    const T ox = (T)gx, oy = (T)gy;
    if (!isfinite(ox) || !isfinite(oy)) atomicOr(err, HTS_ERR_NONFINITE_GRAD);
    grad[2 * (int64_t)i] = ox;
    grad[2 * (int64_t)i + 1] = oy;
}

// The traversal's workspace (item list, partials, per-block sums) in ctx->part:
// the offsets of its 11 regions and the total, for nqb query blocks and n
// points (with the counters' region when stats are asked).
struct BhLayout {
    static constexpr int R = 11;
    size_t off[R];
    size_t tot;
};
template <typename T>
static BhLayout bh_layout(hts_ctx ctx, int64_t nqb, int64_t n, bool stats) {
    const int64_t nw = nqb * kTopSlots;
    const int share = ctx->list_items < kItemCap ? ctx->list_items : kItemCap;
    const int64_t slots = nw * share;
    const size_t b_base = (size_t)nw * 4, b_nit = (size_t)nw * 4;
    const size_t b_part0 = (size_t)kTopSlots * n * 2 * sizeof(T), b_ztop = (size_t)nw * 8;
    const size_t b_part = (size_t)slots * kWave * 2 * sizeof(T), b_zitem = (size_t)slots * 8;
    const size_t b_frep = (size_t)n * 2 * sizeof(T), b_zq = (size_t)nqb * 8;
    const size_t b_st = stats ? (size_t)(slots + nw) * kStats * 4 : 0;
    const size_t b_cnt = 256, b_dense = (size_t)slots * sizeof(ItemRec);
    const size_t sizes[BhLayout::R] = {b_base, b_nit, b_part0, b_ztop, b_part, b_zitem,
                                       b_frep, b_zq, b_st, b_cnt, b_dense};
    BhLayout L;
    L.tot = 0;
    for (int a = 0; a < BhLayout::R; ++a) {
        L.off[a] = L.tot;
        L.tot += (sizes[a] + 255) & ~(size_t)255;
    }
    return L;
}

template <typename T>
hts_status bh_item_counter(hts_ctx ctx, hts_tree t, int64_t n, unsigned **counter) {
    const BhLayout L = bh_layout<T>(ctx, t->nqb, n, false);
    HTS_OKR(ensure(ctx->part, L.tot));
    *counter = (unsigned *)((char *)ctx->part.p + L.off[9]);
    return HTS_OK;
}
template hts_status bh_item_counter<float>(hts_ctx, hts_tree, int64_t, unsigned **);
template hts_status bh_item_counter<double>(hts_ctx, hts_tree, int64_t, unsigned **);

template <typename T, int MET>
hts_status launch_bh_repulsion(hts_ctx ctx, hipStream_t st, hts_tree t, int64_t n,
                               BhPrep<T> prep, PointRec<T> *pts, const int64_t *rp,
                               const int32_t *col, const T *val, T *fattr, double ex,
                               const double *ex_job, bool accumulate, double scale, T *grad,
                               double *z_dev, uint64_t *stats) {
    const int64_t nqb = t->nqb;
    const Jobs jb = jobs_of(t);
    const int64_t nw = nqb * kTopSlots;  // phase-A waves
    const int share = ctx->list_items < kItemCap ? ctx->list_items : kItemCap;
    const int64_t slots = nw * share;
    const int S = ctx->item_points;
    // workspace: item list, partials, per-block sums
    const BhLayout L = bh_layout<T>(ctx, nqb, n, stats != nullptr);
    const size_t *off = L.off;
    HTS_OKR(ensure(ctx->part, L.tot));
    char *base = (char *)ctx->part.p;
    int *item_base = (int *)(base + off[0]);
    int *nitems = (int *)(base + off[1]);
    T *part0 = (T *)(base + off[2]);
    double *ztop = (double *)(base + off[3]);
    T *part = (T *)(base + off[4]);
    double *zitem = (double *)(base + off[5]);
    T *frep = (T *)(base + off[6]);
    double *zq = (double *)(base + off[7]);
    uint32_t *st_items = stats ? (uint32_t *)(base + off[8]) : nullptr;
    uint32_t *st_top = stats ? st_items + (size_t)slots * kStats : nullptr;
    unsigned *dense_count = (unsigned *)(base + off[9]);
    ItemRec *dense = (ItemRec *)(base + off[10]);

    const NodeRec<T> *nodes = (const NodeRec<T> *)(MET == 0 ? t->nodes : t->enodes);
    const PointRec<T> *spts = (const PointRec<T> *)t->spts;
    const dim3 gq(nqb);  // the combine: one workgroup per query block
    // phase B: items_grid workgroups of items_waves waves, by default 32
    // waves per phase-A wave (about one per item: the hardware hands each
    // freed wave slot the next item), never more than the list holds
    const int wpb = ctx->items_waves;
    // the attractive rows beside phase A (long chains hide them) or at the end
    // of phase B; automatic: beside phase A for a job of 131072 points or more
    const int64_t largest = t->jobs_set ? t->max_job : n;
    const bool attract_a = ctx->attract_at == 1 || (ctx->attract_at == 0 && largest >= kAttractWithTopAt);
    int64_t gi = ctx->items_grid > 0 ? (int64_t)ctx->items_grid : cdiv(32 * nw, wpb);
    if (gi > cdiv(slots, wpb)) gi = cdiv(slots, wpb);
    if (gi < 1) gi = 1;          // an empty list (no items can be handed over)
    // one thread per point, and the node thresholds strided over the same grid
    const int64_t gp = cdiv(n, kBlock) > 64 ? cdiv(n, kBlock) : 64;
    if (prep.points || prep.thresholds || prep.clear)
        hipLaunchKernelGGL(k_bh_prepare<T>, dim3(gp), dim3(kBlock), 0, st, prep.Y, n, pts,
                           prep.points, (NodeRec<T> *)t->nodes, t->r_cell, t->d_m, prep.theta,
                           prep.thresholds, prep.clear ? dense_count : nullptr, ctx->d_err);
    {
        TimedScope ts(ctx, st, HTS_K_TRAVERSE);
        const int64_t top_blocks = cdiv(nw, kBlock / kWave);
        const dim3 ga(top_blocks + (attract_a ? cdiv(n * kAttractLanes, kBlock) : 0));
        if (stats)
            hipLaunchKernelGGL((k_bh_top<T, MET, true>), ga, dim3(kBlock), 0, st, nodes, t->d_m,
                               t->node_start, jb, spts, nqb, S, item_base, nitems, part0, ztop,
                               st_top, dense_count, dense, share, n, top_blocks, pts, rp, col,
                               val, fattr, ctx->d_err);
        else
            hipLaunchKernelGGL((k_bh_top<T, MET, false>), ga, dim3(kBlock), 0, st, nodes, t->d_m,
                               t->node_start, jb, spts, nqb, S, item_base, nitems, part0, ztop,
                               nullptr, dense_count, dense, share, n, top_blocks, pts, rp, col,
                               val, fattr, ctx->d_err);
    }
    {
        TimedScope ts(ctx, st, HTS_K_ITEMS);
        const dim3 gb(gi + (attract_a ? 0 : cdiv(n * kAttractLanes, wpb * kWave)));
        if (stats)
            hipLaunchKernelGGL((k_bh_items<T, MET, true>), gb, dim3(wpb * kWave), 0, st, nodes, t->d_m,
                               spts, dense_count, dense, slots, part, zitem, st_items, gi, pts, rp,
                               col, val, n, fattr, ctx->d_err);
        else
            hipLaunchKernelGGL((k_bh_items<T, MET, false>), gb, dim3(wpb * kWave), 0, st, nodes,
                               t->d_m, spts, dense_count, dense, slots, part, zitem, nullptr, gi, pts,
                               rp, col, val, n, fattr, ctx->d_err);
    }
    HTS_HIP(hipGetLastError());
    TimedScope ts(ctx, st, HTS_K_FINALIZE);
    if (stats)
        hipLaunchKernelGGL((k_bh_gather<T, MET, true>), gq, dim3(kBlock), 0, st, spts, part0, ztop, part,
                           zitem, item_base, nitems, jb, nqb, n, frep, zq, st_top, st_items,
                           (unsigned long long *)stats);
    else
        hipLaunchKernelGGL((k_bh_gather<T, MET, false>), gq, dim3(kBlock), 0, st, spts, part0, ztop, part,
                           zitem, item_base, nitems, jb, nqb, n, frep, zq, nullptr, nullptr,
                           nullptr);
    hipLaunchKernelGGL(k_bh_finalize<T>, dim3(cdiv(n, kBlock)), dim3(kBlock), 0, st, fattr, frep,
                       zq, jb, t->perm, n, ex, ex_job, accumulate, scale, grad, z_dev,
                       ctx->d_err);
    HTS_HIP(hipGetLastError());
    return HTS_OK;
}

template hts_status launch_bh_repulsion<float, 0>(hts_ctx, hipStream_t, hts_tree, int64_t,
                                                   BhPrep<float>, PointRec<float> *, const int64_t *,
                                                   const int32_t *, const float *, float *, double,
                                                   const double *, bool, double, float *, double *,
                                                   uint64_t *);
template hts_status launch_bh_repulsion<float, 1>(hts_ctx, hipStream_t, hts_tree, int64_t,
                                                   BhPrep<float>, PointRec<float> *, const int64_t *,
                                                   const int32_t *, const float *, float *, double,
                                                   const double *, bool, double, float *, double *,
                                                   uint64_t *);
template hts_status launch_bh_repulsion<double, 0>(hts_ctx, hipStream_t, hts_tree, int64_t,
                                                   BhPrep<double>, PointRec<double> *, const int64_t *,
                                                   const int32_t *, const double *, double *, double,
                                                   const double *, bool, double, double *, double *,
                                                   uint64_t *);
template hts_status launch_bh_repulsion<double, 1>(hts_ctx, hipStream_t, hts_tree, int64_t,
                                                   BhPrep<double>, PointRec<double> *, const int64_t *,
                                                   const int32_t *, const double *, double *, double,
                                                   const double *, bool, double, double *, double *,
                                                   uint64_t *);

}  // namespace hts
