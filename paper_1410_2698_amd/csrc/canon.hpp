// The canonical FP64 evaluation of one (query, entry) pair, shared by every
// search kernel of the library (temporal/spatial index search, self-join,
// fixed spatial grid) and by the host search that serves small requests.  Compiled without FP contraction (-ffp-contract=off),
// so the operations below are performed exactly in the order written.
#pragma once

#include <hip/hip_runtime.h>

namespace tds {

__host__ __device__ inline double dmax(double a, double b) { return a > b ? a : b; }
__host__ __device__ inline double dmin(double a, double b) { return a < b ? a : b; }

// Query side of the canonical evaluation.  aq = max(ts_q, t_start) and
// bq = min(te_q, t_end) are exact, so max(aq, ts_l) is the common start of
// the pair whatever order the maxima are taken in.
struct QCanon {
    double x, y, z, vx, vy, vz, ts, aq, bq, d;
};

// Membership and interval of one (query, entry) pair in the fixed FP64
// operation order: positions at the ends of the common extent, squared
// distances minus d^2 there (C0, C1), relative velocity W, A = |W|^2,
// B = D(a).W; member iff C0 <= 0, C1 <= 0 or the vertex of the convex
// quadratic lies strictly inside with a non-negative discriminant; the roots
// in cancellation-free form (Higham, Accuracy and Stability of Numerical
// Algorithms, Sec. 1.8).  Compiled without FP contraction.
template <bool kInterval>
__host__ __device__ __forceinline__ bool canon_eval(const QCanon& q, double lx, double ly, double lz,
                                           double lvx, double lvy, double lvz, double lts,
                                           double lte, double* t_lo, double* t_hi) {
    const double a = dmax(q.aq, lts);
    const double b = dmin(q.bq, lte);
    if (!(a < b)) return false;
    const double T = b - a;
    const double dqa = a - q.ts, dla = a - lts;
    const double dqb = b - q.ts, dlb = b - lts;
    const double dax = (q.x + q.vx * dqa) - (lx + lvx * dla);
    const double day = (q.y + q.vy * dqa) - (ly + lvy * dla);
    const double daz = (q.z + q.vz * dqa) - (lz + lvz * dla);
    const double dbx = (q.x + q.vx * dqb) - (lx + lvx * dlb);
    const double dby = (q.y + q.vy * dqb) - (ly + lvy * dlb);
    const double dbz = (q.z + q.vz * dqb) - (lz + lvz * dlb);
    const double wx = q.vx - lvx, wy = q.vy - lvy, wz = q.vz - lvz;
    const double dd = q.d * q.d;
    const double C0 = ((dax * dax + day * day) + daz * daz) - dd;
    const double C1 = ((dbx * dbx + dby * dby) + dbz * dbz) - dd;
    const double A = (wx * wx + wy * wy) + wz * wz;
    const double B = (dax * wx + day * wy) + daz * wz;
    const bool member = (C0 <= 0.0) || (C1 <= 0.0) ||
                        (A > 0.0 && B < 0.0 && -B < A * T && B * B - A * C0 >= 0.0);
    if (!kInterval || !member) return member;
    if (A == 0.0) {
        *t_lo = a;
        *t_hi = b;
        return true;
    }
    const double disc = B * B - A * C0;
    const double s = sqrt(dmax(disc, 0.0));
    const double qq = (B >= 0.0) ? (-B - s) : (-B + s);
    const double r1 = qq / A;
    const double r2 = (qq != 0.0) ? C0 / qq : 0.0;
    double lo = (C0 <= 0.0) ? a : a + dmin(dmax(dmin(r1, r2), 0.0), T);
    double hi = (C1 <= 0.0) ? b : a + dmin(dmax(dmax(r1, r2), 0.0), T);
    if (lo > hi) {
        const double tv = a + dmin(dmax(-B / A, 0.0), T);
        lo = tv;
        hi = tv;
    }
    *t_lo = lo;
    *t_hi = hi;
    return true;
}

}  // namespace tds
