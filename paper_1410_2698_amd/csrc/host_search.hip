// Host search over a host copy of an index: the serving loop's route for
// requests too small to be worth a GPU batch (the hybrid CPU + GPU search the
// paper leaves for future work, Sec. 6; its measurements show the CPU ahead
// for small, sparse searches, Sec. 5.3-5.5).  It runs the same steps as the
// GPU search for one query segment: clip to the window, the candidate range
// E_k of Sec. 4.2.2 from the bin tables, and the canonical FP64 evaluation of
// every candidate (canon.hpp, the code the kernels use), so its records are
// bit-identical to the GPU's.
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
    DeviceGuard g(idx->device);
    if (!g.ok) return TDS_E_DEVICE;
    TDS_HIP(hipMemcpy(h->e64.data(), idx->e64, n * sizeof(EntryF64), hipMemcpyDeviceToHost));
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

// Clipped extent of query segment k of Q (8 arrays of L values, xs .. te).
bool host_clip(const double* q, uint64_t L, uint64_t k, double t0, double t1, double* aq,
               double* bq) {
    *aq = dmax(q[3 * L + k], t0);
    *bq = dmin(q[7 * L + k], t1);
    return *aq < *bq;
}

}  // namespace

uint64_t host_candidates(const HostIndex& h, const double* q, uint64_t L, double t0, double t1) {
    uint64_t total = 0;
    for (uint64_t k = 0; k < L; ++k) {
        double aq, bq;
        if (!host_clip(q, L, k, t0, t1, &aq, &bq)) continue;
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
        double aq, bq;
        if (!host_clip(q, L, k, t0, t1, &aq, &bq)) continue;
        uint32_t lo, hi;
        host_range(h, aq, bq, &lo, &hi);
        // canonical query data: the velocity as every search form computes it
        const double xs = q[k], ys = q[L + k], zs = q[2 * L + k], ts = q[3 * L + k];
        const double xe = q[4 * L + k], ye = q[5 * L + k], ze = q[6 * L + k], te = q[7 * L + k];
        const double dt = te - ts;
        QCanon c;
        c.x = xs;
        c.y = ys;
        c.z = zs;
        c.vx = (xe - xs) / dt;
        c.vy = (ye - ys) / dt;
        c.vz = (ze - zs) / dt;
        c.ts = ts;
        c.aq = aq;
        c.bq = bq;
        c.d = d;
        for (uint32_t i = lo; i < hi; ++i) {
            const EntryF64& e = h.e64[i];
            double t_lo, t_hi;
            if (!canon_eval<true>(c, e.x, e.y, e.z, e.vx, e.vy, e.vz, e.ts, e.te, &t_lo, &t_hi))
                continue;
            tds_result r;
            r.q_seg = (uint32_t)k;
            r.e_seg = h.seg_id[i];
            r.q_traj = qtraj ? qtraj[k] : 0u;
            r.e_traj = h.traj[i];
            r.t_lo = t_lo;
            r.t_hi = t_hi;
            out->push_back(r);
        }
    }
}

}  // namespace tds
