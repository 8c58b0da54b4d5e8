// Host search over a host copy of an index: the serving loop's route for
// requests too small to be worth a GPU batch (the hybrid CPU + GPU search the
// paper leaves for future work, Sec. 6; its measurements show the CPU ahead
// for small, sparse searches, Sec. 5.3-5.5).  It runs the same steps as the
// GPU search for one query segment: clip to the window, the candidate range
// E_k of Sec. 4.2.2 from the bin tables, the FP32 filter (block boxes of the
// spatial layout, then the bounding spheres and time extents: seg_box32,
// box_overlap, sphere32 and sphere_pass, the code the kernels use) and the
// canonical FP64 evaluation of every pair it passes (canon.hpp), so its
// records are bit-identical to the GPU's.
#include <algorithm>
#include <cmath>

#include "canon.hpp"
#include "tds_internal.hpp"

namespace tds {

int host_index_load(const tds_index* idx, HostIndex* h) {
    const uint64_t n = idx->n;
    const uint32_t m = idx->m;
    h->n = n;
    h->m = m;
    h->e64.resize(n);
    h->seg_id.resize(n);
    h->traj.resize(n);
    h->bin_first.resize((size_t)m + 1);
    h->cmax_te.resize(m);
    h->lo_ts.resize(m);
    h->e32.resize(n);
    const uint64_t nblk = (n + (1u << kBoxShift) - 1) >> kBoxShift;
    h->bbox.resize(idx->bbox ? nblk : 0);
    DeviceGuard g(idx->device);
    if (!g.ok) return TDS_E_DEVICE;
    TDS_HIP(hipMemcpy(h->e64.data(), idx->e64, n * sizeof(EntryF64), hipMemcpyDeviceToHost));
    TDS_HIP(hipMemcpy(h->e32.data(), idx->e32, n * sizeof(EntryF32), hipMemcpyDeviceToHost));
    if (idx->bbox)
        TDS_HIP(hipMemcpy(h->bbox.data(), idx->bbox, nblk * sizeof(BlockBox),
                          hipMemcpyDeviceToHost));
    TDS_HIP(hipMemcpy(h->seg_id.data(), idx->seg_id, n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    TDS_HIP(hipMemcpy(h->traj.data(), idx->traj, n * sizeof(uint32_t), hipMemcpyDeviceToHost));
    TDS_HIP(hipMemcpy(h->bin_first.data(), idx->bin_first, ((size_t)m + 1) * sizeof(uint32_t),
                      hipMemcpyDeviceToHost));
    TDS_HIP(hipMemcpy(h->cmax_te.data(), idx->cmax_te, m * sizeof(double), hipMemcpyDeviceToHost));
    TDS_HIP(hipMemcpy(h->lo_ts.data(), idx->lo_ts, m * sizeof(double), hipMemcpyDeviceToHost));
    return TDS_OK;
}

namespace {

// Candidate range [lo, hi) of a clipped query [aq, bq]: from the first entry
// of the first bin whose running maximum of t_end exceeds aq to the end of the
// last bin whose smallest t_start (over it and the bins after it) is below
// bq.  Both tables are non-decreasing, so each bound is one bisection.
void host_range(const HostIndex& h, double aq, double bq, uint32_t* lo, uint32_t* hi) {
    const auto j0 = (uint32_t)(std::upper_bound(h.cmax_te.begin(), h.cmax_te.end(), aq,
                                                [](double v, double e) { return v < e; }) -
                               h.cmax_te.begin());
    const auto L = (uint32_t)(std::lower_bound(h.lo_ts.begin(), h.lo_ts.end(), bq) -
                              h.lo_ts.begin());
    *lo = (j0 < h.m) ? h.bin_first[j0] : (uint32_t)h.n;
    *hi = h.bin_first[L];
}

// One query segment k of Q (8 arrays of L values, xs .. te) prepared as the
// GPU prepares it: canonical data, candidate range, FP32 filter record.
struct HostQuery {
    QCanon c;
    uint32_t lo, hi;
    float cx, cy, cz, R, a32, b32;
    Box32 box;  // box of the clipped segment grown by d (block culling)
};

bool host_query(const HostIndex& h, const double* q, uint64_t L, uint64_t k, double d, double t0,
                double t1, HostQuery* hq) {
    const double xs = q[k], ys = q[L + k], zs = q[2 * L + k], ts = q[3 * L + k];
    const double xe = q[4 * L + k], ye = q[5 * L + k], ze = q[6 * L + k], te = q[7 * L + k];
    QCanon& c = hq->c;
    c.aq = dmax(ts, t0);
    c.bq = dmin(te, t1);
    if (!(c.aq < c.bq)) return false;
    host_range(h, c.aq, c.bq, &hq->lo, &hq->hi);
    if (hq->lo >= hq->hi) return false;
    // canonical query data: the velocity as every search form computes it
    const double dt = te - ts;
    c.x = xs;
    c.y = ys;
    c.z = zs;
    c.vx = (xe - xs) / dt;
    c.vy = (ye - ys) / dt;
    c.vz = (ze - zs) / dt;
    c.ts = ts;
    c.d = d;
    // sphere of the clipped segment, from its end points at aq and bq
    const double pax = c.x + c.vx * (c.aq - ts), pay = c.y + c.vy * (c.aq - ts),
                 paz = c.z + c.vz * (c.aq - ts);
    const double pbx = c.x + c.vx * (c.bq - ts), pby = c.y + c.vy * (c.bq - ts),
                 pbz = c.z + c.vz * (c.bq - ts);
    sphere32(pax, pay, paz, pbx, pby, pbz, d, hq->cx, hq->cy, hq->cz, hq->R);
    hq->box = seg_box32(pax, pay, paz, pbx, pby, pbz, d);
    hq->a32 = f32_rd(c.aq);
    hq->b32 = f32_ru(c.bq);
    return true;
}

// Calls f(i) for every candidate i of the query that passes the FP32 filter;
// returns the pair tests made (candidates of blocks that pass their box test).
template <class F>
uint64_t host_filter(const HostIndex& h, const HostQuery& hq, F&& f) {
    uint64_t tests = 0;
    const uint32_t b0 = hq.lo >> kBoxShift, b1 = (hq.hi - 1) >> kBoxShift;
    for (uint32_t b = b0; b <= b1; ++b) {
        if (!h.bbox.empty() && !box_overlap(h.bbox[b].b, hq.box)) continue;
        const uint32_t i0 = std::max(hq.lo, b << kBoxShift);
        const uint32_t i1 = std::min<uint64_t>(hq.hi, (uint64_t)(b + 1) << kBoxShift);
        tests += i1 - i0;
        for (uint32_t i = i0; i < i1; ++i) {
            const EntryF32& e = h.e32[i];
            if (sphere_pass(hq.cx, hq.cy, hq.cz, hq.R, e.cx, e.cy, e.cz, e.r) &&
                hq.a32 < e.te && e.ts < hq.b32)
                f(i);
        }
    }
    return tests;
}

}  // namespace

uint64_t host_candidates(const HostIndex& h, const double* q, uint64_t L, double t0, double t1,
                         uint64_t limit) {
    uint64_t total = 0;
    for (uint64_t k = 0; k < L && total <= limit; ++k) {
        const double aq = dmax(q[3 * L + k], t0), bq = dmin(q[7 * L + k], t1);
        if (!(aq < bq)) continue;
        uint32_t lo, hi;
        host_range(h, aq, bq, &lo, &hi);
        if (lo < hi) total += hi - lo;
    }
    return total;
}

void host_search(const HostIndex& h, const double* q, const uint32_t* qtraj, uint64_t L,
                 double d, double t0, double t1, std::vector<tds_result>* out) {
    out->clear();
    for (uint64_t k = 0; k < L; ++k) {
        HostQuery hq;
        if (!host_query(h, q, L, k, d, t0, t1, &hq)) continue;
        host_filter(h, hq, [&](uint32_t i) {
            const EntryF64& e = h.e64[i];
            double t_lo, t_hi;
            if (!canon_eval<true>(hq.c, e.x, e.y, e.z, e.vx, e.vy, e.vz, e.ts, e.te, &t_lo,
                                  &t_hi))
                return;
            tds_result r;
            r.q_seg = (uint32_t)k;
            r.e_seg = h.seg_id[i];
            r.q_traj = qtraj ? qtraj[k] : 0u;
            r.e_traj = h.traj[i];
            r.t_lo = t_lo;
            r.t_hi = t_hi;
            out->push_back(r);
        });
    }
}

}  // namespace tds
