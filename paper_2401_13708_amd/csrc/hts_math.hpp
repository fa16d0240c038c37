// hts_math.hpp -- device arithmetic shared by the gradient kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "hts_impl.hpp"

namespace hts {

// acosh(1 + t) = log1p(t + sqrt(t (t + 2))) with full relative accuracy for
// small t (eq. (8) with the argument carried as t = gamma - 1, never gamma).
__device__ __forceinline__ float acosh1p(float t, float &sh) {
    sh = __builtin_sqrtf(t * (t + 2.0f));
    return log1pf(t + sh);
}
__device__ __forceinline__ double acosh1p(double t, double &sh) {
    sh = sqrt(t * (t + 2.0));
    return log1p(t + sh);
}

// One pair (query q, other point or cell midpoint o):
//   t   = 2 |q - o|^2 ia_q ib_o        (double: the eq. (8) argument minus 1)
//   d   = acosh(1 + t),  sinh d = sqrt(t (t + 2))
//   w   = (1 + d^2)^-1
//   d dd/dq = (d / sinh d) 4 ia_q ib_o ((q - o) + |q - o|^2 ia_q q)   (eq. (13))
// The caller multiplies `base` by the weight it needs: p w (attraction) or
// N w^2 (repulsion).
template <typename T>
struct PairTerm {
    T w;      // (1 + d^2)^-1
    T base;   // (d / sinh d) 4 ia ib
    T vx, vy; // (q - o) + |q - o|^2 ia_q q
};

// distance argument in double from coordinates in T.  dq = dd (2 qia) rounds
// to the same value as (2 dd) qia (the factor 2 is exact), and 2 qia is the
// same for every node a query meets, so it is formed once per walk; dq / 2 is
// |q - o|^2 ia_q exactly, the factor of q in eq. (13).
template <typename T>
__device__ __forceinline__ double dist_arg(T qx, T qy, double qia, T ox, T oy, double oib, double &dq) {
    double dx = (double)qx - (double)ox;
    double dy = (double)qy - (double)oy;
    const double dd = dx * dx + dy * dy;
    dq = dd * (2.0 * qia);
    return dq * oib;
}

// double precision: library functions throughout.  With QF = false the
// query's own factor 4 ia_q is left out of `base` (a caller that sums many
// terms of one query applies it once to the sum).
template <typename T, bool QF = true>
__device__ __forceinline__ PairTerm<T> pair_term(T qx, T qy, double qia, T ox, T oy, double oib,
                                                 double t, double dq) {
    PairTerm<T> r;
    T tf = (T)t;
    T sh;
    T d = acosh1p(tf, sh);
    r.w = (T)1 / ((T)1 + d * d);
    T ratio = sh > (T)0 ? d / sh : (T)1;
    r.base = QF ? ratio * (T)(4.0 * qia * oib) : ratio * (T)oib;
    T c = (T)(0.5 * dq);
    r.vx = (qx - ox) + c * qx;
    r.vy = (qy - oy) + c * qy;
    return r;
}

// single precision at hardware rate.  With cosh d = 1 + t:
//   d / sinh d = sum_n n! / (3/2)_n (-t/2)^n = 1 - t/3 + 2t^2/15 - 2t^3/35 + ...
// (a hypergeometric series, converging for t < 2); below t = 1/8 the terms
// up to t^6 leave a truncation error under 2e-9, and d = (d / sinh d) sinh d.
// Above it, d = ln(1 + t + sinh d) is well conditioned (the argument exceeds
// 1.6), so the hardware log2 / reciprocal / square root suffice.
// With UNI, when every active lane takes the same branch the other one is
// not evaluated (a wave-uniform choice; each lane's value is the same).  It
// pays where waves are many and instruction issue bounds the kernel, and
// costs a little where a wave's chain of dependent steps does.
template <bool QF, bool UNI = false>
__device__ __forceinline__ PairTerm<float> pair_term_f32(float qx, float qy, double qia, float ox,
                                                         float oy, double oib, double t,
                                                         double dq) {
    PairTerm<float> r;
    const float tf = (float)t;
    // one reciprocal square root gives 1 / sinh d, and sinh d = x / sqrt(x).
    // The argument is kept >= 1e-30 so that x = 0 gives sinh d = 0; below
    // 1e-30, sinh d < 1e-15 either way and d^2 vanishes next to 1.
    const float x = tf * (tf + 2.0f);
    const float rs = __builtin_amdgcn_rsqf(__builtin_fmaxf(x, 1e-30f));
    const float sh = x * rs;
    auto series = [&]() {
        float qs = 16.0f / 3003.0f;
        qs = __builtin_fmaf(qs, tf, -8.0f / 693.0f);
        qs = __builtin_fmaf(qs, tf, 8.0f / 315.0f);
        qs = __builtin_fmaf(qs, tf, -2.0f / 35.0f);
        qs = __builtin_fmaf(qs, tf, 2.0f / 15.0f);
        qs = __builtin_fmaf(qs, tf, -1.0f / 3.0f);
        return __builtin_fmaf(qs, tf, 1.0f);
    };
    auto logd = [&]() { return __builtin_amdgcn_logf(1.0f + tf + sh) * 0.6931471805599453f; };
    const bool small = tf < 0.125f;
    const uint64_t act = UNI ? __builtin_amdgcn_read_exec() : 1;
    const uint64_t sm = UNI ? __builtin_amdgcn_ballot_w64(small) : 2;
    float ratio, d;
    if (sm == act) {
        const float qs = series();
        ratio = qs;
        d = qs * sh;
    } else if (sm == 0) {
        const float dl = logd();
        ratio = dl * rs;
        d = dl;
    } else {
        const float qs = series();
        const float dl = logd();
        ratio = small ? qs : dl * rs;
        d = small ? qs * sh : dl;
    }
    r.w = __builtin_amdgcn_rcpf(__builtin_fmaf(d, d, 1.0f));
    r.base = QF ? ratio * (float)(4.0 * qia * oib) : ratio * (float)oib;
    // (float)(dq / 2) q = (float)dq (q / 2) exactly; q / 2 is the same for
    // every term of a query
    const float c = (float)dq;
    r.vx = (qx - ox) + c * (0.5f * qx);
    r.vy = (qy - oy) + c * (0.5f * qy);
    return r;
}
template <>
__device__ __forceinline__ PairTerm<float> pair_term<float, true>(float qx, float qy, double qia,
                                                                  float ox, float oy, double oib,
                                                                  double t, double dq) {
    return pair_term_f32<true>(qx, qy, qia, ox, oy, oib, t, dq);
}
template <>
__device__ __forceinline__ PairTerm<float> pair_term<float, false>(float qx, float qy, double qia,
                                                                   float ox, float oy, double oib,
                                                                   double t, double dq) {
    return pair_term_f32<false>(qx, qy, qia, ox, oy, oib, t, dq);
}

// ---------------------------------------------------------------- metrics
// The traversal and the attractive rows are written once over a metric:
//  Geo<0>: the Poincare disk (eqs. (8), (13)), terms w^m d dd/dy as above;
//  Geo<1>: the Euclidean Student-t kernel of the disk coordinates (the first
//          part of the h-SNE gradient, Sec. 4-C): w = (1 + |y - o|^2)^-1, terms
//          w^m (y - o); the criterion argument is |y - o|^2 itself.
// arg() returns the quantity compared with a node's threshold; attract() and
// repel() add p w (...) and N w^2 (...) to the force and N w to Z, except
// that repel() leaves out a factor common to all terms of the query,
// qfactor(), which the caller applies once to the query's summed repulsion.
// The arguments dd of repel() and of arg() are what arg() hands back.
template <int MET> struct Geo;

// the repulsive term's pair: no query factor, and for single precision the
// wave-uniform branch choice as asked
template <typename T, bool UNI>
__device__ __forceinline__ PairTerm<T> rep_term(T qx, T qy, double qia, T ox, T oy, double oib,
                                                double t, double dq) {
    if constexpr (sizeof(T) == 4)
        return pair_term_f32<false, UNI>(qx, qy, qia, ox, oy, oib, t, dq);
    else
        return pair_term<T, false>(qx, qy, qia, ox, oy, oib, t, dq);
}

template <> struct Geo<0> {
    template <typename T>
    static __device__ __forceinline__ double arg(const PointRec<T> &me, T ox, T oy, double oib,
                                                 double &dd) {
        return dist_arg<T>(me.x, me.y, me.ia, ox, oy, oib, dd);
    }
    template <bool UNI = false, typename T, typename Z>
    static __device__ __forceinline__ void repel(const PointRec<T> &me, T ox, T oy, double oib,
                                                 double t, double dd, T weight, T &fx, T &fy,
                                                 Z &z) {
        const PairTerm<T> r = rep_term<T, UNI>(me.x, me.y, me.ia, ox, oy, oib, t, dd);
        const T coef = weight * r.w * r.w * r.base;
        fx += coef * r.vx;
        fy += coef * r.vy;
        z += (Z)(weight * r.w);
    }
    // 4 ia_q of eq. (13)
    template <typename T>
    static __device__ __forceinline__ T qfactor(const PointRec<T> &me) {
        return (T)(4.0 * me.ia);
    }
    template <typename T>
    static __device__ __forceinline__ T attract(const PointRec<T> &q, const PointRec<T> &o, T p,
                                                T &vx, T &vy) {
        double dd;
        const double t = dist_arg<T>(q.x, q.y, q.ia, o.x, o.y, o.ia, dd);
        const PairTerm<T> r = pair_term<T>(q.x, q.y, q.ia, o.x, o.y, o.ia, t, dd);
        vx = r.vx;
        vy = r.vy;
        return p * r.w * r.base;
    }
};

template <typename T> __device__ __forceinline__ T recip(T x) { return (T)1 / x; }
template <> __device__ __forceinline__ float recip<float>(float x) {
    return __builtin_amdgcn_rcpf(x);
}

template <> struct Geo<1> {
    template <typename T>
    static __device__ __forceinline__ double arg(const PointRec<T> &me, T ox, T oy, double oib,
                                                 double &dd) {
        (void)oib;
        const double dx = (double)me.x - (double)ox;
        const double dy = (double)me.y - (double)oy;
        dd = dx * dx + dy * dy;
        return dd;
    }
    template <bool UNI = false, typename T, typename Z>
    static __device__ __forceinline__ void repel(const PointRec<T> &me, T ox, T oy, double oib,
                                                 double t, double dd, T weight, T &fx, T &fy,
                                                 Z &z) {
        (void)oib;
        (void)t;
        const T w = recip<T>((T)1 + (T)dd);
        const T coef = weight * w * w;
        fx += coef * (me.x - ox);
        fy += coef * (me.y - oy);
        z += (Z)(weight * w);
    }
    template <typename T>
    static __device__ __forceinline__ T qfactor(const PointRec<T> &) {
        return (T)1;
    }
    template <typename T>
    static __device__ __forceinline__ T attract(const PointRec<T> &q, const PointRec<T> &o, T p,
                                                T &vx, T &vy) {
        const double dx = (double)q.x - (double)o.x;
        const double dy = (double)q.y - (double)o.y;
        vx = q.x - o.x;
        vy = q.y - o.y;
        return p * recip<T>((T)1 + (T)(dx * dx + dy * dy));
    }
};

// ---------------------------------------------------------------- set-up
// Point record of Y[i] (coordinates and 1 / (1 - |y|^2) in double); a point
// outside the open disk or not finite sets the error word.
template <typename T>
__device__ __forceinline__ void prep_point(const T *__restrict__ Y, int64_t i,
                                           PointRec<T> *__restrict__ pts,
                                           uint32_t *__restrict__ err) {
    const T x = Y[2 * i], y = Y[2 * i + 1];
    const double a = 1.0 - ((double)x * (double)x + (double)y * (double)y);
    PointRec<T> p;
    p.x = x;
    p.y = y;
    p.ia = 1.0 / a;
    if constexpr (sizeof(T) == 8) p.pad = 0.0;
    if (!(a > 0.0)) atomicOr(err, (a == a) ? HTS_ERR_OUTSIDE_DISK : HTS_ERR_NONFINITE_Y);
    pts[i] = p;
}

// Criterion threshold of an internal node: r_cell / d < theta  <=>
// t > cosh(r_cell / theta) - 1 = 2 sinh^2(r_cell / (2 theta)) (the sinh form
// keeps small thresholds accurate); theta = 0 never accepts.
__device__ __forceinline__ double node_threshold(double r_cell, double theta) {
    if (theta > 0.0) {
        const double sh = sinh(r_cell / (2.0 * theta));
        return 2.0 * sh * sh;
    }
    return __builtin_inf();
}

// ---------------------------------------------------------------- wave ops
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
template <int G, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
    for (int o = G / 2; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

// double-double (Dekker/Knuth two-sum) for the prefix sums of the midpoint
// summands: the difference of two prefix sums keeps the node's own digits.
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
    s = a + b;
    double bb = s - a;
    e = (a - (s - bb)) + (b - bb);
}
__device__ __forceinline__ DD3 dd_add(const DD3 &a, const DD3 &b) {
    DD3 r;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double s, e;
        two_sum(a.hi[c], b.hi[c], s, e);
        e += a.lo[c] + b.lo[c];
        double h = s + e;
        r.lo[c] = e - (h - s);
        r.hi[c] = h;
    }
    return r;
}
__device__ __forceinline__ DD3 dd_zero() {
    DD3 r;
#pragma unroll
    for (int c = 0; c < 3; ++c) r.hi[c] = r.lo[c] = 0.0;
    return r;
}

// ---------------------------------------------------------------- attraction
// First sum of eq. (15), F_attr,i = sum_{j in row i} p_ij w_ij d_ij dd_ij/dy_i,
// by thread gid of a grid of G threads per row (groups of G lanes aligned in
// a wave): column/value reads are contiguous per row, the point records of
// the columns are gathered (they stay in L2).
template <typename T, int G, int MET = 0>
__device__ __forceinline__ void attract_rows(int64_t gid, const PointRec<T> *__restrict__ pts,
                                             const int64_t *__restrict__ rp,
                                             const int32_t *__restrict__ col,
                                             const T *__restrict__ val, int64_t n,
                                             T *__restrict__ fattr, uint32_t *__restrict__ err) {
    const int64_t row = gid / G;
    const int sub = (int)(gid % G);
    T fx = 0, fy = 0;
    if (row < n) {
        const PointRec<T> q = pts[row];
        const int64_t e1 = rp[row + 1];
        for (int64_t e = rp[row] + sub; e < e1; e += G) {
            const int32_t j = col[e];
            const T p = val[e];
            if ((uint32_t)j >= (uint64_t)n) {  // malformed CSR: flag it, never read outside
                atomicOr(err, HTS_ERR_BAD_INDEX);
                continue;
            }
            const PointRec<T> o = pts[j];
            T vx, vy;
            const T a = Geo<MET>::attract(q, o, p, vx, vy);
            const T coef = (j == row) ? (T)0 : a;
            fx += coef * vx;
            fy += coef * vy;
        }
    }
    fx = group_sum<G>(fx);
    fy = group_sum<G>(fy);
    if (row < n && sub == 0) {
        fattr[2 * row] = fx;
        fattr[2 * row + 1] = fy;
    }
}


}  // namespace hts
