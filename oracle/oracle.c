/*
 * Plain FP64 CPU oracle for the distance threshold search.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark do.  It shares no code with the GPU path.
 *
 * What it computes (problem definition, Sec. 3.1 of the paper): for every
 * query segment q and every entry segment l, the set of times in the common
 * temporal extent of q, l and the search window [t_start, t_end] at which the
 * Euclidean distance (Sec. 4.1) between the two linearly moving points is at
 * most d.  One record (q, l, [t_lo, t_hi]) is emitted per pair whose set is not
 * empty.  No index: every (q, l) pair is visited; the time-overlap filter is
 * the plain definition.
 *
 * Readings of what the paper leaves open (the paper never writes out its
 * compare() routine, Algorithms 1-3):
 *   - time overlap is strict: max(ts) < min(te) after clipping to the window;
 *     pairs that only touch at one instant are not results;
 *   - "within d" is inclusive (<= d); a tangent pair gives [t*, t*];
 *   - records are per segment pair, carrying both trajectory ids; intervals are
 *     not merged across consecutive segments;
 *   - the window [t_start, t_end] clips the common extent.
 *
 * Canonical FP64 evaluation (the operation order is part of the definition so
 * that a GPU implementation can reproduce every decision bit for bit; build
 * with -ffp-contract=off, no fast-math):
 *   V  = (P_end - P_start) / (t_end - t_start)                per segment
 *   a  = max(ts_q, t_start, ts_l), b = min(te_q, t_end, te_l); need a < b
 *   Dx(t) = (xs_q + vx_q*(t - ts_q)) - (xs_l + vx_l*(t - ts_l))   (x, y, z)
 *   C0 = ((Dx(a)^2 + Dy(a)^2) + Dz(a)^2) - d*d,  C1 the same at b
 *   W  = V_q - V_l,  A = (Wx^2 + Wy^2) + Wz^2,  B = (Dx(a)Wx + Dy(a)Wy) + Dz(a)Wz
 *   member = C0 <= 0  or  C1 <= 0  or  (A > 0 and B < 0 and -B < A*T and
 *            B*B - A*C0 >= 0),   T = b - a
 *   f(a + tau) = |D(a)|^2 + 2 B tau + A tau^2 is convex; the roots of
 *   f - d^2 come from the cancellation-free form (Higham, Accuracy and
 *   Stability of Numerical Algorithms, Sec. 1.8): s = sqrt(max(B*B - A*C0, 0)),
 *   qq = -B - s if B >= 0 else -B + s, r1 = qq / A, r2 = C0 / qq (0 if qq = 0).
 *   t_lo = a if C0 <= 0 else a + clamp(min(r1, r2), 0, T)
 *   t_hi = b if C1 <= 0 else a + clamp(max(r1, r2), 0, T)
 *   if A == 0 the interval is [a, b]; if rounding leaves t_lo > t_hi both
 *   become a + clamp(-B / A, 0, T).
 *
 * Temporal bins (Sec. 4.2.1): entries sorted by t_start (ties by input
 * position), m bins of width b = (t_max - t_min) / m, entry i in bin
 * floor((ts_i - t_min) / b) clamped to [0, m-1]; per bin B^start = t_min + j*b,
 * B^end = max(t_min + (j+1)*b, max te in bin), B^first / B^last the sorted
 * positions of its first and last entry.
 *
 * Schedule (Sec. 4.2.2): for a query segment clipped to the window,
 * [a_q, b_q], the candidate range E_k = [B^first, B^last] spans the bins from
 * the first bin whose entries reach past a_q (running maximum of te over
 * bins > a_q) to the last non-empty bin whose first entry starts before b_q,
 * taken as one contiguous span of sorted entries.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    uint32_t q_seg, e_seg, q_traj, e_traj;
    double t_lo, t_hi;
} orc_result;

static double dmax(double x, double y) { return x > y ? x : y; }
static double dmin(double x, double y) { return x < y ? x : y; }
static double clampd(double x, double lo, double hi) { return dmin(dmax(x, lo), hi); }

/* Per-segment velocity V = (P_end - P_start) / (t_end - t_start). */
void orc_velocity(int64_t n, const double* xs, const double* ys, const double* zs,
                  const double* ts, const double* xe, const double* ye,
                  const double* ze, const double* te,
                  double* vx, double* vy, double* vz) {
    for (int64_t i = 0; i < n; ++i) {
        double dt = te[i] - ts[i];
        vx[i] = (xe[i] - xs[i]) / dt;
        vy[i] = (ye[i] - ys[i]) / dt;
        vz[i] = (ze[i] - zs[i]) / dt;
    }
}

/*
 * One (query, entry) comparison.  Each segment is given as
 * {xs, ys, zs, vx, vy, vz, ts, te}.  Returns 1 and writes the interval when the
 * pair is a result, else 0.
 */
int orc_pair(const double* q, const double* l, double d, double t_start,
             double t_end, double* t_lo, double* t_hi) {
    double a = dmax(dmax(q[6], t_start), l[6]);
    double b = dmin(dmin(q[7], t_end), l[7]);
    if (!(a < b)) return 0;
    double T = b - a;
    double dqa = a - q[6], dla = a - l[6];
    double dqb = b - q[6], dlb = b - l[6];
    double Da[3], Db[3], W[3];
    for (int c = 0; c < 3; ++c) {
        double pqa = q[c] + q[3 + c] * dqa;
        double pla = l[c] + l[3 + c] * dla;
        Da[c] = pqa - pla;
        double pqb = q[c] + q[3 + c] * dqb;
        double plb = l[c] + l[3 + c] * dlb;
        Db[c] = pqb - plb;
        W[c] = q[3 + c] - l[3 + c];
    }
    double dd = d * d;
    double C0 = ((Da[0] * Da[0] + Da[1] * Da[1]) + Da[2] * Da[2]) - dd;
    double C1 = ((Db[0] * Db[0] + Db[1] * Db[1]) + Db[2] * Db[2]) - dd;
    double A = (W[0] * W[0] + W[1] * W[1]) + W[2] * W[2];
    double B = (Da[0] * W[0] + Da[1] * W[1]) + Da[2] * W[2];
    int member = (C0 <= 0.0) || (C1 <= 0.0) ||
                 (A > 0.0 && B < 0.0 && -B < A * T && B * B - A * C0 >= 0.0);
    if (!member) return 0;
    if (A == 0.0) {
        *t_lo = a;
        *t_hi = b;
        return 1;
    }
    double disc = B * B - A * C0;
    double s = sqrt(dmax(disc, 0.0));
    double qq = (B >= 0.0) ? (-B - s) : (-B + s);
    double r1 = qq / A;
    double r2 = (qq != 0.0) ? C0 / qq : 0.0;
    double lo = (C0 <= 0.0) ? a : a + clampd(dmin(r1, r2), 0.0, T);
    double hi = (C1 <= 0.0) ? b : a + clampd(dmax(r1, r2), 0.0, T);
    if (lo > hi) {
        double tv = a + clampd(-B / A, 0.0, T);
        lo = tv;
        hi = tv;
    }
    *t_lo = lo;
    *t_hi = hi;
    return 1;
}

typedef struct {
    orc_result* v;
    int64_t n, cap;
} orc_vec;

static int vec_push(orc_vec* a, orc_result r) {
    if (a->n == a->cap) {
        int64_t nc = a->cap ? 2 * a->cap : 1024;
        orc_result* nv = (orc_result*)realloc(a->v, (size_t)nc * sizeof(orc_result));
        if (!nv) return -1;
        a->v = nv;
        a->cap = nc;
    }
    a->v[a->n++] = r;
    return 0;
}

/*
 * Brute-force search over all (query, entry) pairs.  Segment arrays are SoA;
 * traj arrays may be NULL (id 0).  On success *out holds n records (caller
 * frees with orc_free) in unspecified order; returns n, or -1 on allocation
 * failure.  threads <= 0 uses the OpenMP default.
 */
int64_t orc_search(int64_t nq, const double* qxs, const double* qys, const double* qzs,
                   const double* qts, const double* qxe, const double* qye,
                   const double* qze, const double* qte, const uint32_t* qtraj,
                   int64_t nd, const double* dxs, const double* dys, const double* dzs,
                   const double* dts, const double* dxe, const double* dye,
                   const double* dze, const double* dte, const uint32_t* dtraj,
                   double d, double t_start, double t_end, int threads,
                   orc_result** out) {
    double* dv = (double*)malloc((size_t)(nd > 0 ? nd : 1) * 3 * sizeof(double));
    double* qv = (double*)malloc((size_t)(nq > 0 ? nq : 1) * 3 * sizeof(double));
    if (!dv || !qv) { free(dv); free(qv); return -1; }
    orc_velocity(nd, dxs, dys, dzs, dts, dxe, dye, dze, dte, dv, dv + nd, dv + 2 * nd);
    orc_velocity(nq, qxs, qys, qzs, qts, qxe, qye, qze, qte, qv, qv + nq, qv + 2 * nq);

    int nthreads = 1;
#ifdef _OPENMP
    if (threads > 0) omp_set_num_threads(threads);
    nthreads = omp_get_max_threads();
#endif
    orc_vec* per = (orc_vec*)calloc((size_t)nthreads, sizeof(orc_vec));
    int failed = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 16)
#endif
    for (int64_t k = 0; k < nq; ++k) {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double q[8] = {qxs[k], qys[k], qzs[k], qv[k], qv[nq + k], qv[2 * nq + k], qts[k], qte[k]};
        for (int64_t i = 0; i < nd; ++i) {
            /* time-overlap filter: the plain definition, no index */
            if (!(dmax(dmax(q[6], t_start), dts[i]) < dmin(dmin(q[7], t_end), dte[i]))) continue;
            double l[8] = {dxs[i], dys[i], dzs[i], dv[i], dv[nd + i], dv[2 * nd + i], dts[i], dte[i]};
            double lo, hi;
            if (orc_pair(q, l, d, t_start, t_end, &lo, &hi)) {
                orc_result r;
                r.q_seg = (uint32_t)k;
                r.e_seg = (uint32_t)i;
                r.q_traj = qtraj ? qtraj[k] : 0u;
                r.e_traj = dtraj ? dtraj[i] : 0u;
                r.t_lo = lo;
                r.t_hi = hi;
                if (vec_push(&per[tid], r)) failed = 1;
            }
        }
    }
    free(dv);
    free(qv);
    int64_t total = 0;
    for (int t = 0; t < nthreads; ++t) total += per[t].n;
    orc_result* res = (orc_result*)malloc((size_t)(total > 0 ? total : 1) * sizeof(orc_result));
    if (!res) failed = 1;
    int64_t pos = 0;
    for (int t = 0; t < nthreads; ++t) {
        if (res && per[t].n) memcpy(res + pos, per[t].v, (size_t)per[t].n * sizeof(orc_result));
        pos += per[t].n;
        free(per[t].v);
    }
    free(per);
    if (failed) { free(res); return -1; }
    *out = res;
    return total;
}

void orc_free(void* p) { free(p); }

/* Stable order of entries by t_start (ties keep input order). */
static const double* g_sort_ts;
static int cmp_ts(const void* x, const void* y) {
    int64_t i = *(const int64_t*)x, j = *(const int64_t*)y;
    double a = g_sort_ts[i], b = g_sort_ts[j];
    if (a < b) return -1;
    if (a > b) return 1;
    return (i > j) - (i < j);
}

/*
 * Temporal bins of Sec. 4.2.1.  Outputs (sorted positions are 0-based):
 *   order[n]        input position of the i-th entry in t_start order
 *   bin[n]          bin of the i-th sorted entry
 *   first[m], last[m]  sorted positions of the first / last entry of each bin
 *                   (an empty bin has last = first - 1, first = next position)
 *   bstart[m], bend[m]  B^start = t_min + j*b, B^end = max(t_min + (j+1)*b, max te)
 *   min_ts[m], max_te[m]  data extents of each bin (+inf / -inf when empty)
 *   cmax_te[m]      running maximum of max_te over bins 0..j
 *   t_range[2]      t_min, t_max
 * Returns 0, or -1 on bad arguments.
 */
int orc_bins(int64_t n, const double* ts, const double* te, int64_t m,
             int64_t* order, int32_t* bin, int64_t* first, int64_t* last,
             double* bstart, double* bend, double* min_ts, double* max_te,
             double* cmax_te, double* t_range) {
    if (n <= 0 || m <= 0) return -1;
    for (int64_t i = 0; i < n; ++i) order[i] = i;
    g_sort_ts = ts;
    qsort(order, (size_t)n, sizeof(int64_t), cmp_ts);
    double tmin = ts[0], tmax = te[0];
    for (int64_t i = 1; i < n; ++i) {
        tmin = dmin(tmin, ts[i]);
        tmax = dmax(tmax, te[i]);
    }
    double bw = (tmax - tmin) / (double)m;
    for (int64_t i = 0; i < n; ++i) {
        double u = floor((ts[order[i]] - tmin) / bw);
        int64_t j = (int64_t)u;
        if (j < 0) j = 0;
        if (j > m - 1) j = m - 1;
        bin[i] = (int32_t)j;
    }
    int64_t pos = 0;
    double run = -INFINITY;
    for (int64_t j = 0; j < m; ++j) {
        int64_t f = pos;
        double mx = -INFINITY, mn = INFINITY;
        while (pos < n && bin[pos] == j) {
            mn = dmin(mn, ts[order[pos]]);
            mx = dmax(mx, te[order[pos]]);
            ++pos;
        }
        first[j] = f;
        last[j] = pos - 1;
        bstart[j] = tmin + (double)j * bw;
        bend[j] = dmax(tmin + (double)(j + 1) * bw, mx);
        min_ts[j] = mn;
        max_te[j] = mx;
        run = dmax(run, mx);
        cmax_te[j] = run;
    }
    t_range[0] = tmin;
    t_range[1] = tmax;
    return 0;
}

/*
 * Schedule of Sec. 4.2.2 for nq query segments: lo[k] = B^first of the first
 * bin whose running max te exceeds a_q; hi[k] = B^last + 1 of the last
 * non-empty bin whose minimum ts is below b_q (exclusive end).
 * a_q = max(qts, t_start), b_q = min(qte, t_end).  An empty window or range
 * gives lo = hi = 0.
 */
void orc_schedule(int64_t m, const int64_t* first, const int64_t* last,
                  const double* min_ts, const double* cmax_te, int64_t nq,
                  const double* qts, const double* qte, double t_start,
                  double t_end, int64_t* lo, int64_t* hi) {
    for (int64_t k = 0; k < nq; ++k) {
        double aq = dmax(qts[k], t_start), bq = dmin(qte[k], t_end);
        int64_t l = 0, h = 0;
        int found = 0;
        if (aq < bq) {
            for (int64_t j = 0; j < m; ++j) {
                if (cmax_te[j] > aq) { l = first[j]; found = 1; break; }
            }
            for (int64_t j = 0; j < m; ++j)
                if (last[j] >= first[j] && min_ts[j] < bq) h = last[j] + 1;
        }
        if (!found || l >= h) { l = 0; h = 0; }
        lo[k] = l;
        hi[k] = h;
    }
}
