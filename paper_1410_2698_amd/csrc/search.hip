// Distance threshold search on the GPU (Sec. 3.1 problem, Sec. 4.2.2 search).
//
// Per search, on one stream:
//   k_zero       clear the header, bucket counters and request counters;
//   k_qprep      one thread per query segment: validate, velocity, clip to the
//                window, candidate range [lo, hi) by bisection of the bin
//                tables (the schedule S of Sec. 4.2.2, computed on the GPU),
//                FP32 filter sphere, bucket key = (first bin, bin span);
//   k_bucket_scan  one block: bucket offsets, 64-segment groups per bucket,
//                candidate chunks per bucket and the work-item table;
//   k_scatter    order the query segments by bucket, and fill the work-item
//                table (item -> bucket);
//   k_distance   persistent waves take work items round-robin (64 query
//                segments of one bucket x one chunk of their common candidate
//                range).  FP32 form: the lanes hold the chunk's candidates
//                (coalesced loads) and the boxes of its 64-entry blocks; each
//                block's box is tested against every query of the group (one
//                lane per query) and only the surviving queries are tested
//                against the block's candidates.  FP64 plain form: one query
//                segment per lane, candidates streamed through wave-uniform
//                scalar loads.  Pairs that pass are queued in LDS and
//                evaluated 64 at a time by the canonical FP64 code; results
//                are appended with one atomic per request per 64 evaluations.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>

#include <hip/hip_ext.h>

#include "canon.hpp"
#include "tds_internal.hpp"

namespace tds {

namespace {

constexpr uint32_t kInactive = 0xFFFFFFFFu;

// The bucket slot counters are split into parts: about 1,500 returning
// atomics on one address serialize for ≈ 25 µs; 16 parts are the best
// balance between that and the bucket scan's work of adding up the parts
// (8 and 32 were slower).  Part p counts for the query-preparation workgroups
// [p * bpp, (p + 1) * bpp) (bpp = workgroups per part): the parts are laid
// out one after the other in each bucket, so its segments stay close to
// their input order, and the segments of one request (one d) stay together
// in the 64-segment groups.  The counters are stored part by part (bucket b
// of part p at p * buckets + b): the 64 lanes of a wave, whose keys are
// often consecutive, then hit a few cache lines, which the atomics of one
// instruction share (stored bucket by bucket, the same atomics took as long
// as without parts).  1 or kCountParts parts: kCountParts when parts *
// buckets fits the kMaxBuckets-entry tables.
constexpr uint32_t kCountParts = 16;

uint32_t count_parts(uint32_t nb) {
    return (uint64_t)nb * kCountParts <= kMaxBuckets ? kCountParts : 1u;
}

constexpr uint32_t kPartedBuckets = kMaxBuckets / kCountParts;  // most buckets with parts

// Maximum over the kCountParts parts of bucket b (nb buckets).
__device__ __forceinline__ uint32_t parts_max(const uint32_t* c, uint32_t b, uint32_t nb) {
    uint32_t v[kCountParts];
#pragma unroll
    for (uint32_t p = 0; p < kCountParts; ++p) v[p] = c[p * nb + b];
    uint32_t m = 0;
#pragma unroll
    for (uint32_t p = 0; p < kCountParts; ++p) m = max(m, v[p]);
    return m;
}

// Candidates held per lane by the FP32 form: a wave works on tiles of
// kCpl * 64 candidates, so each query record fetched by a scalar load feeds
// kCpl * 64 pair tests.  kCpl is a launch choice (2 or 4, the autotuner's tile
// size); chunks are rounded to whole tiles of the larger one.
constexpr int kCplMax = 4;
constexpr uint32_t kTile = kCplMax * kWave;

// FP64 entry records are read through the constant address space with a
// wave-uniform index, so the compiler fetches them with scalar loads into
// SGPRs: one load serves the 64 lanes (query segments) of the wave.
typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef const __attribute__((address_space(4))) f64x4* ConstE64;

struct IndexView {
    const EntryF64* e64;
    const EntryF32* e32;
    const uint32_t* seg_id;
    const uint32_t* traj;
    const uint32_t* bin_first;
    const double* cmax_te;
    const double* lo_ts;
    const EntryV32* ev32;  // FP32 motion of the entries (filter refinement)
    const BlockBox* bbox;  // block boxes (spatial layout) or nullptr
    double t_min, bw;      // bin origin and width (search starting points)
    uint32_t n, m;
};

struct QueryView {
    const double* a[8];  // xs, ys, zs, ts, xe, ye, ze, te
    const uint32_t* traj;
    uint64_t n;
    // self-join: query segment k is index entry k (its FP64 record, input id
    // and trajectory); each unordered pair of entries of different
    // trajectories is then tested once, from its entry of lower position
    const EntryF64* ent;
    const uint32_t* ent_id;
    const uint32_t* ent_traj;
};

IndexView view_of(const tds_index* idx) {
    IndexView v;
    v.e64 = idx->e64;
    v.e32 = idx->e32;
    v.seg_id = idx->seg_id;
    v.traj = idx->traj;
    v.bin_first = idx->bin_first;
    v.cmax_te = idx->cmax_te;
    v.lo_ts = idx->lo_ts;
    v.ev32 = idx->ev32;
    v.bbox = idx->bbox;
    v.t_min = idx->t_min;
    v.bw = idx->bw;
    v.n = (uint32_t)idx->n;
    v.m = idx->m;
    return v;
}


__device__ inline uint64_t lanemask_lt() {
    const uint32_t lane = __lane_id();
    return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

// Keeps LDS traffic of one wave in program order around cross-lane exchange.
__device__ inline void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ inline uint32_t uniform(uint32_t v) { return __builtin_amdgcn_readfirstlane(v); }

// Lane 0's 64-bit value in every lane (the value need not be uniform).
__device__ inline uint64_t lane0_64(uint64_t v) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 0);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 0);
    return ((uint64_t)hi << 32) | lo;
}

// ------------------------------------------------------------ schedule

// Smallest j in [0, m] with pred(j), for a predicate that is monotone
// (false ... false true ... true) with pred(m) true.  The bins have equal
// widths, so the caller's guess g (the bin of the time searched for) is
// usually within one of the answer: four neighbouring values are loaded at
// once, and only if the answer lies outside them does the search gallop
// away from g and bisect the bracket found.
template <class Pred>
__device__ inline uint32_t first_true(Pred pred, uint32_t m, uint32_t g) {
    g = min(g, m);
    const uint32_t a = (g > 0) ? g - 1 : 0;
    bool w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = (a + k >= m) ? true : pred(a + k);
    uint32_t l, h;  // the answer lies in [l, h] and pred(h) holds
    if (w[0]) {
        if (a == 0) return 0;
        // answer <= a: gallop down from a
        h = a;
        uint32_t step = 1;
        for (;;) {
            if (h < step) {
                l = 0;
                break;
            }
            const uint32_t c = h - step;
            if (!pred(c)) {
                l = c + 1;
                break;
            }
            h = c;
            step *= 2;
        }
    } else {
#pragma unroll
        for (int k = 1; k < 4; ++k)
            if (w[k] && !w[k - 1]) return a + k;
        // answer > a + 3: gallop up
        l = a + 4;
        uint32_t step = 1;
        for (;;) {
            const uint32_t c = l - 1 + step;
            if (c >= m) {
                h = m;
                break;
            }
            if (pred(c)) {
                h = c;
                break;
            }
            l = c + 1;
            step *= 2;
        }
    }
    while (l < h) {
        const uint32_t mid = l + (h - l) / 2;
        if (pred(mid)) h = mid;
        else l = mid + 1;
    }
    return l;
}

// Two independent first_true searches whose first windows are loaded together.
template <class P1, class P2>
__device__ inline void first_true2(P1 p1, uint32_t g1, P2 p2, uint32_t g2, uint32_t m,
                                   uint32_t* r1, uint32_t* r2) {
    g1 = min(g1, m);
    g2 = min(g2, m);
    const uint32_t a1 = (g1 > 0) ? g1 - 1 : 0, a2 = (g2 > 0) ? g2 - 1 : 0;
    bool w1[4], w2[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        w1[k] = (a1 + k >= m) ? true : p1(a1 + k);
        w2[k] = (a2 + k >= m) ? true : p2(a2 + k);
    }
    // answer inside a window: the first true after a false (or a true at 0)
    auto inside = [](const bool (&w)[4], uint32_t a, uint32_t* r) {
        if (w[0]) {
            if (a == 0) {
                *r = 0;
                return true;
            }
            return false;
        }
#pragma unroll
        for (int k = 1; k < 4; ++k)
            if (w[k] && !w[k - 1]) {
                *r = a + k;
                return true;
            }
        return false;
    };
    if (!inside(w1, a1, r1)) *r1 = first_true(p1, m, g1);
    if (!inside(w2, a2, r2)) *r2 = first_true(p2, m, g2);
}

// Bin of time t for a search starting point (any value is correct).
__device__ inline uint32_t guess_bin(const IndexView& I, double t) {
    const double u = floor((t - I.t_min) / I.bw);
    if (!(u > 0.0)) return 0u;
    if (u >= (double)I.m) return I.m;
    return (uint32_t)u;
}

// Candidate range E_k of a clipped query [aq, bq] (Sec. 4.2.2): from the
// first entry of the first bin whose running max t_end exceeds aq (bin j0)
// to the last entry of the last non-empty bin whose smallest t_start is below
// bq (bin j1), as one contiguous span [lo, hi) of index positions.
__device__ inline void cand_range(const IndexView& I, double aq, double bq, uint32_t* lo,
                                  uint32_t* hi, uint32_t* j0o, uint32_t* j1o) {
    // j0 = first j with cmax_te[j] > aq (m if none); L = number of bins j for
    // which some entry of a bin >= j has t_start < bq (lo_ts, the minimum
    // t_start over bins >= j, is non-decreasing), i.e. the first j with
    // lo_ts[j] >= bq; entries before bin_first[L] are those of bins < L.
    // Both searches read their first windows before either decides.
    uint32_t j0, L;
    first_true2([&](uint32_t j) { return I.cmax_te[j] > aq; }, guess_bin(I, aq),
                [&](uint32_t j) { return I.lo_ts[j] >= bq; }, guess_bin(I, bq) + 1u, I.m, &j0, &L);
    *lo = (j0 < I.m) ? I.bin_first[j0] : I.n;
    *hi = I.bin_first[L];
    *j0o = j0;
    *j1o = (L > 0) ? L - 1 : 0;
}

__device__ inline bool finite(double v) { return isfinite(v); }

// Request of query segment k: requests hold contiguous, ascending slices.
__device__ inline uint32_t request_of(const Request* req, uint32_t nreq, uint64_t k) {
    uint32_t l = 0, h = nreq;
    while (h - l > 1) {
        uint32_t mid = (l + h) >> 1;
        if (req[mid].q_begin <= k) l = mid;
        else h = mid;
    }
    return l;
}

// ------------------------------------------------------------ kernels

__global__ __launch_bounds__(kBlock) void k_zero(SearchHeader* hdr, uint32_t* b_count,
                                                 uint32_t* b_hi, uint32_t nb,
                                                 uint32_t nparts, ReqCounter* rc, uint32_t nreq,
                                                 unsigned long long* dyn_ctr) {
    // nreq: capacity of the request counters (all of them are cleared);
    // b_count and b_hi hold nparts parts for each of the nb buckets
    const uint32_t i = blockIdx.x * kBlock + threadIdx.x;
    if (i == 0) {
        SearchHeader h = {};
        *hdr = h;
    }
    if (i < nb * nparts) {
        b_count[i] = 0;
        b_hi[i] = 0;
    }
    if (i < nreq) {
        rc[i].count = 0;
        rc[i].pad = 0;
    }
    if (i < kCtrSlots * kCtrStride) dyn_ctr[i] = 0;
}

// Canonical FP64 data of query segment k of request r, from the query
// arrays (the same operations wherever it is needed, so bit-identical).
// Canonical query data from the segment's end points (the velocity of the
// segment as every search form computes it).
__device__ inline void query_canon_pts(double xs, double ys, double zs, double ts, double xe,
                                       double ye, double ze, double te, const Request& R,
                                       QCanon& q) {
    const double dt = te - ts;
    q.x = xs;
    q.y = ys;
    q.z = zs;
    q.vx = (xe - xs) / dt;
    q.vy = (ye - ys) / dt;
    q.vz = (ze - zs) / dt;
    q.ts = ts;
    q.aq = dmax(ts, R.t_start);
    q.bq = dmin(te, R.t_end);
    q.d = R.d;
}

__device__ inline void query_canon(const QueryView& Q, const Request& R, uint64_t k, QCanon& q) {
    if (!Q.ent) {
        query_canon_pts(Q.a[0][k], Q.a[1][k], Q.a[2][k], Q.a[3][k], Q.a[4][k], Q.a[5][k],
                        Q.a[6][k], Q.a[7][k], R, q);
        return;
    }
    double ts, te;
    {
        // the entry record holds the same velocity, computed the same way
        const EntryF64 e = Q.ent[k];
        q.x = e.x;
        q.y = e.y;
        q.z = e.z;
        q.vx = e.vx;
        q.vy = e.vy;
        q.vz = e.vz;
        ts = e.ts;
        te = e.te;
    }
    q.ts = ts;
    q.aq = dmax(ts, R.t_start);
    q.bq = dmin(te, R.t_end);
    q.d = R.d;
}

__global__ __launch_bounds__(kBlock) void k_qprep(QueryView Q, const BatchDesc* __restrict__ desc,
                                                  const Request* __restrict__ req, IndexView I,
                                                  QF32* __restrict__ qfu,
                                                  uint32_t* __restrict__ qreq,
                                                  uint32_t* __restrict__ qkey,
                                                  uint32_t* __restrict__ qslot, uint32_t* b_count,
                                                  uint32_t* b_hi, uint32_t shift, uint32_t nb,
                                                  uint32_t bpp, SearchHeader* hdr) {
    // the first requests' starts in LDS: the request of a query segment is
    // then found without a chain of dependent global loads
    __shared__ uint64_t s_begin[kBlock];
    const uint32_t nreq = desc->nreq;
    if (threadIdx.x < nreq) s_begin[threadIdx.x] = req[threadIdx.x].q_begin;
    __syncthreads();
    const uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    // this workgroup's part of the bucket counters (k_scatter finds it the
    // same way)
    const uint32_t part = blockIdx.x / bpp;
    bool act = false;  // the segment gets a bucket slot
    uint32_t key = 0;
    if (k < desc->nq) {
        uint32_t r;
        if (nreq <= kBlock) {
            uint32_t l = 0, h = nreq;
            while (h - l > 1) {
                const uint32_t mid = (l + h) >> 1;
                if (s_begin[mid] <= k) l = mid;
                else h = mid;
            }
            r = l;
        } else {
            r = request_of(req, nreq, k);
        }
        bool ok = true;  // index entries were validated when the index was built
        QCanon p;
        if (Q.ent) {
            query_canon(Q, req[r], k, p);
        } else {
            // the end points are read once, for the validation and the
            // canonical data
            const double xs = Q.a[0][k], ys = Q.a[1][k], zs = Q.a[2][k], ts = Q.a[3][k];
            const double xe = Q.a[4][k], ye = Q.a[5][k], ze = Q.a[6][k], te = Q.a[7][k];
            ok = finite(xs) && finite(ys) && finite(zs) && finite(ts) && finite(xe) &&
                 finite(ye) && finite(ze) && finite(te) && te > ts;
            if (ok) query_canon_pts(xs, ys, zs, ts, xe, ye, ze, te, req[r], p);
        }
        if (!ok) {
            atomicOr(&hdr->err, 1u);
        } else {
            const double ts = p.ts;
            if (p.aq < p.bq) {
                uint32_t lo, hi, j0, j1;
                cand_range(I, p.aq, p.bq, &lo, &hi, &j0, &j1);
                if (Q.ent) lo = max(lo, (uint32_t)k + 1u);  // self-join: entries after k
                if (lo < hi) {
                    const double pax = p.x + p.vx * (p.aq - ts), pay = p.y + p.vy * (p.aq - ts),
                                 paz = p.z + p.vz * (p.aq - ts);
                    const double pbx = p.x + p.vx * (p.bq - ts), pby = p.y + p.vy * (p.bq - ts),
                                 pbz = p.z + p.vz * (p.bq - ts);
                    QF32 f;
                    sphere32(pax, pay, paz, pbx, pby, pbz, p.d, f.cx, f.cy, f.cz, f.R);
                    f.box = seg_box32(pax, pay, paz, pbx, pby, pbz, p.d);
                    f.pad[0] = f.pad[1] = 0.f;
                    f.a32 = __double2float_rd(p.aq);
                    f.b32 = __double2float_ru(p.bq);
                    f.lo = lo;
                    f.hi = hi;
                    const uint32_t span = min(j1 - j0, kSpanClasses - 1);
                    key = (j0 * kSpanClasses + span) >> shift;
                    act = true;
                    qkey[k] = key;
                    // the bucket's range follows from its key unless it merges
                    // several first bins or spans an open number of bins
                    if (shift || span == kSpanClasses - 1) atomicMax(&b_hi[part * nb + key], hi);
                    qfu[k] = f;
                    qreq[k] = r;
                }
            }
        }
    }
    // bucket slots: one atomic per run of equal keys in consecutive lanes
    // (neighbouring query segments often share a bucket, e.g. in the
    // self-join, where a wave's segments are neighbours in one bin)
    const uint32_t lane = __lane_id();
    const uint32_t ke = act ? key : 0xFFFFFFFFu;
    const uint32_t prev = __shfl_up(ke, 1);
    const uint64_t bnd = __ballot(lane == 0 || prev != ke || !act);
    const uint64_t upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
    const uint32_t start = 63u - (uint32_t)__clzll(bnd & upto);
    const uint64_t above = bnd & ~upto;
    const uint32_t next = above ? (uint32_t)__ffsll((unsigned long long)above) - 1u : 64u;
    uint32_t base = 0;
    if (act && lane == start) base = atomicAdd(&b_count[part * nb + key], next - start);
    base = __shfl(base, start);
    if (k < desc->nq) qslot[k] = act ? base + (lane - start) : kInactive;
}

// Schedule only (tds_schedule): candidate range per query segment.
__global__ __launch_bounds__(kBlock) void k_schedule(QueryView Q, double t_start, double t_end,
                                                     IndexView I, uint32_t* __restrict__ lo_out,
                                                     uint32_t* __restrict__ hi_out,
                                                     uint32_t* err) {
    const uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
    if (k >= Q.n) return;
    bool ok = true;
    for (int c = 0; c < 8; ++c) ok = ok && finite(Q.a[c][k]);
    const double ts = Q.a[3][k], te = Q.a[7][k];
    ok = ok && te > ts;
    uint32_t lo = 0, hi = 0;
    if (!ok) {
        atomicOr(err, 1u);
    } else {
        const double aq = dmax(ts, t_start), bq = dmin(te, t_end);
        if (aq < bq) {
            uint32_t j0, j1;
            cand_range(I, aq, bq, &lo, &hi, &j0, &j1);
            if (lo >= hi) lo = hi = 0;
        }
    }
    lo_out[k] = lo;
    hi_out[k] = hi;
}

// Bucket offsets, groups and the work-item table, one block.  The parts of
// each bucket's slot counter become the parts' offsets within the bucket.
__global__ __launch_bounds__(1024) void k_bucket_scan(uint32_t* __restrict__ b_count,
                                                      const uint32_t* __restrict__ b_hi,
                                                      const uint32_t* __restrict__ bin_first,
                                                      const double* __restrict__ min_te,
                                                      const double* __restrict__ max_ts,
                                                      uint32_t m, uint32_t shift,
                                                      uint32_t nb, uint32_t nparts, uint32_t chunk,
                                                      uint32_t* __restrict__ b_start,
                                                      uint32_t* __restrict__ b_nch,
                                                      BucketInfo* __restrict__ binfo,
                                                      SearchHeader* hdr) {
    __shared__ uint32_t pc[1024], pi[1024];
    __shared__ uint32_t s_cnt[kPartedBuckets], s_hi[kPartedBuckets];
    const uint32_t tid = threadIdx.x;
    if (nparts == kCountParts) {
        // bucket totals and range maxima of the parts (nb <= kPartedBuckets),
        // each part's count replaced by its first slot in the bucket;
        // consecutive threads take consecutive buckets (coalesced)
        for (uint32_t b = tid; b < nb; b += 1024) {
            uint32_t v[kCountParts];
#pragma unroll
            for (uint32_t p = 0; p < kCountParts; ++p) v[p] = b_count[p * nb + b];
            uint32_t cnt = 0;
#pragma unroll
            for (uint32_t p = 0; p < kCountParts; ++p) {
                b_count[p * nb + b] = cnt;
                cnt += v[p];
            }
            s_cnt[b] = cnt;
            const uint32_t code = b << shift;
            s_hi[b] = (cnt && (shift || code % kSpanClasses == kSpanClasses - 1))
                          ? parts_max(b_hi, b, nb)
                          : 0u;
        }
        __syncthreads();
    }
    // each thread's consecutive buckets: the record of each (all but its
    // offsets), then the offsets after the scan.  Items per bucket are kept
    // in s_hi (parts) or b_nch for the second pass.
    const uint32_t per = (nb + 1023) / 1024;
    const uint32_t b0 = tid * per, b1 = min(nb, b0 + per);
    uint32_t sc = 0, si = 0;
    for (uint32_t b = b0; b < b1; ++b) {
        const uint32_t cnt = nparts == kCountParts ? s_cnt[b] : b_count[b];
        BucketInfo bi;
        bi.lo = 0xFFFFFFFFu;
        bi.hi = 0;
        bi.nch = 0;
        bi.clen = 0;
        bi.count = cnt;
        bi.start = 0;
        bi.item0 = 0;
        bi.pad = 0;
        bi.tmin_te = -INFINITY;  // unknown: the kernel keeps the per-pair time test
        bi.tmax_ts = INFINITY;
        bi.pad2[0] = bi.pad2[1] = 0.0;
        if (cnt) {
            // range of the bucket: first entry of its smallest first bin to
            // the end of its last bin (from the key, or the members' maximum)
            const uint32_t code = b << shift;  // smallest (j0 * classes + span) of the bucket
            const uint32_t j0 = code / kSpanClasses, span = code % kSpanClasses;
            const uint32_t lo = bin_first[j0];
            uint32_t hi;
            if (shift == 0 && span < kSpanClasses - 1)
                hi = bin_first[min(j0 + span + 1, m)];
            else
                hi = nparts == kCountParts ? s_hi[b] : b_hi[b];
            if (shift == 0 && span < kSpanClasses - 1) {
                // time bounds of the bins the bucket's range covers
                const uint32_t j1 = min(j0 + span, m - 1);
                double mn = INFINITY, mx = -INFINITY;
                for (uint32_t j = j0; j <= j1; ++j) {
                    mn = fmin(mn, min_te[j]);
                    mx = fmax(mx, max_ts[j]);
                }
                bi.tmin_te = mn;
                bi.tmax_ts = mx;
            }
            // balanced chunks of at most `chunk` candidates counted from the
            // 64-entry block of lo (chunk c covers [base + c clen, base +
            // (c + 1) clen) clipped to [lo, hi)), whole 64-candidate tiles
            // where possible, none empty
            const uint32_t len = hi - (lo & ~(uint32_t)(kWave - 1));
            const uint32_t n0 = (len + chunk - 1) / chunk;
            uint32_t clen = (len + n0 - 1) / n0;
            clen = (clen + kWave - 1) / kWave * kWave;
            if (clen > 2 * kTile) clen = (clen + kTile - 1) / kTile * kTile;
            bi.lo = lo;
            bi.hi = hi;
            bi.clen = clen;
            bi.nch = (len + clen - 1) / clen;
        }
        binfo[b] = bi;
        const uint32_t items = ((cnt + kWave - 1) / kWave) * bi.nch;
        if (nparts == kCountParts) s_hi[b] = items;
        else b_nch[b] = items;
        sc += cnt;
        si += items;
    }
    pc[tid] = sc;
    pi[tid] = si;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const uint32_t tc = (tid >= off) ? pc[tid - off] : 0u;
        const uint32_t ti = (tid >= off) ? pi[tid - off] : 0u;
        __syncthreads();
        pc[tid] += tc;
        pi[tid] += ti;
        __syncthreads();
    }
    uint32_t rc = pc[tid] - sc, ri = pi[tid] - si;
    for (uint32_t b = b0; b < b1; ++b) {
        uint32_t cnt, items;
        if (nparts == kCountParts) {
            cnt = s_cnt[b];
            items = s_hi[b];
        } else {
            cnt = b_count[b];
            items = b_nch[b];
            b_count[b] = 0;  // the one part's first slot
        }
        b_start[b] = rc;
        binfo[b].start = rc;
        binfo[b].item0 = ri;
        rc += cnt;
        ri += items;
    }
    if (tid == 1023) {
        hdr->n_items = pi[1023];
        hdr->n_buckets = nb;
        hdr->active = pc[1023];  // every active query segment has a bucket slot
    }
}

// Workgroups [0, qblocks): one thread per query segment, which goes to its
// bucket position (bucket start + its counter part's offset + its slot in
// the part).  Workgroups [qblocks, qblocks + nb): item_bucket[i] = bucket of
// work item i, one workgroup per bucket.
__global__ __launch_bounds__(kBlock) void k_scatter(const BatchDesc* __restrict__ desc,
                                                    const uint32_t* __restrict__ qkey,
                                                    const uint32_t* __restrict__ qslot,
                                                    const uint32_t* __restrict__ b_start,
                                                    const uint32_t* __restrict__ b_part,
                                                    uint32_t nb, uint32_t bpp, uint32_t qblocks,
                                                    const QF32* __restrict__ qfu,
                                                    uint32_t* __restrict__ qsorted,
                                                    QF32* __restrict__ qf,
                                                    const BucketInfo* __restrict__ binfo,
                                                    uint32_t* __restrict__ item_bucket,
                                                    SearchHeader* hdr) {
    if (blockIdx.x < qblocks) {
        const uint64_t k = (uint64_t)blockIdx.x * kBlock + threadIdx.x;
        if (k >= desc->nq) return;
        const uint32_t s = qslot[k];
        if (s == kInactive) return;
        const uint32_t key = qkey[k];
        const uint32_t pos = b_start[key] + b_part[(blockIdx.x / bpp) * nb + key] + s;
        qsorted[pos] = (uint32_t)k;
        qf[pos] = qfu[k];
        return;
    }
    const uint32_t b = blockIdx.x - qblocks;
    const BucketInfo bi = binfo[b];
    const uint32_t n = ((bi.count + kWave - 1) / kWave) * bi.nch;
    const uint32_t cap = desc->item_cap;
    if (threadIdx.x == 0 && n && (uint64_t)bi.item0 + n > cap) atomicOr(&hdr->err, 2u);
    for (uint32_t i = threadIdx.x; i < n; i += kBlock)
        if (bi.item0 + i < cap) item_bucket[bi.item0 + i] = b;
}

// Resets the per-pass request counters and the dynamic item counters of the
// distance kernel.
__global__ void k_reset_pass(ReqCounter* rc, uint32_t nreq, unsigned long long* dyn_ctr) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nreq) rc[i].count = 0;
    if (i < kCtrSlots * kCtrStride) dyn_ctr[i] = 0;
}

// Adds the per-workgroup counters of one distance-kernel launch to the
// header (one block).
__global__ __launch_bounds__(256) void k_stats_fold(const BlockStats* __restrict__ bs, uint32_t nb,
                                                    SearchHeader* hdr) {
    __shared__ uint64_t red[5][256];
    uint64_t v[5] = {0, 0, 0, 0, 0};
    for (uint32_t i = threadIdx.x; i < nb; i += 256) {
        const BlockStats b = bs[i];
        v[0] += b.tests;
        v[1] += b.evals;
        v[2] += b.ftests;
        v[3] += b.btests;
        v[4] += b.flushes;
    }
    for (int k = 0; k < 5; ++k) red[k][threadIdx.x] = v[k];
    __syncthreads();
    for (uint32_t off = 128; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int k = 0; k < 5; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        hdr->tests += red[0][0];
        hdr->evals += red[1][0];
        hdr->ftests += red[2][0];
        hdr->btests += red[3][0];
        hdr->flushes += (uint32_t)red[4][0];
    }
}

// Waves of a distance-kernel launch that may use direct output (the fill
// plan keeps one 16-bit entry per chunk it looks at, at most one more than
// the waves, in LDS).
constexpr uint32_t kMaxDirectWaves = 16384;

// Exclusive prefix sums of f(0..n-1) into out[0..n] (out[n] = total) by one
// workgroup of 1024 threads, 1024 values per round.
template <class F>
__device__ void block_scan_1024(uint32_t n, F f, uint64_t* __restrict__ out) {
    __shared__ uint64_t wsum[1024 / kWave];
    __shared__ uint64_t carry_s;
    const uint32_t t = threadIdx.x, lane = t % kWave, wv = t / kWave;
    if (t == 0) carry_s = 0;
    __syncthreads();
    for (uint32_t r0 = 0; r0 < n; r0 += 1024) {
        const uint32_t i = r0 + t;
        const uint64_t v = i < n ? f(i) : 0;
        uint64_t x = v;
        for (uint32_t o = 1; o < kWave; o <<= 1) {
            const uint64_t y = __shfl_up(x, o);
            if (lane >= o) x += y;
        }
        if (lane == kWave - 1) wsum[wv] = x;
        __syncthreads();
        uint64_t before = carry_s;
        for (uint32_t k = 0; k < wv; ++k) before += wsum[k];
        if (i < n) out[i] = before + x - v;
        __syncthreads();
        if (t == 1023) carry_s = before + x;
        __syncthreads();
    }
    if (t == 0) out[n] = carry_s;
}

// Direct output, after the distance kernel (one workgroup): the plan of the
// fill.  T = min(count, capacity) is the end of the dense output.  The
// holes are the unused tails of the waves' last chunks below T (at most one
// per wave); the sources are the results at positions at or past T, in
// position order, of which the first (total hole size) are moved.  Those lie
// within W (C - 1) positions of T (every hole is shorter than C), so the
// chunks c0 = T / C .. c0 + W are enough, and positions past the capacity
// within W C of it are in the scratch buffer.  Writes the source prefix sums
// per chunk, the hole prefix sums and starts per wave, and (T, c0, chunks).
__global__ __launch_bounds__(1024) void k_fill_plan(const Request* __restrict__ req,
                                                    const ReqCounter* __restrict__ rc,
                                                    const unsigned long long* __restrict__ dir_ctr,
                                                    const uint64_t* __restrict__ dlast, uint32_t nw,
                                                    uint32_t C, uint64_t* __restrict__ s_pre,
                                                    uint64_t* __restrict__ d_pre,
                                                    uint64_t* __restrict__ d_start,
                                                    uint64_t* __restrict__ plan) {
    __shared__ uint16_t used[kMaxDirectWaves + 1];  // positions used of chunk c0 + i
    const uint32_t t = threadIdx.x;
    const uint64_t count = rc[0].count, cap = req[0].out_capacity, R = *dir_ctr;
    const uint64_t T = min(count, cap);
    const uint64_t c0 = T / C, nch = R / C;
    const uint32_t ns = nch > c0 ? (uint32_t)min(nch - c0, (uint64_t)nw + 1) : 0u;
    for (uint32_t i = t; i < ns; i += 1024) used[i] = (uint16_t)C;  // full unless a last chunk
    __syncthreads();
    for (uint32_t w = t; w < nw; w += 1024) {
        const uint64_t v = dlast[w];
        if (v == ~0ull) continue;
        const uint64_t k = v >> 16;
        if (k >= c0 && k - c0 < ns) used[k - c0] = (uint16_t)(v & 0xFFFFu);
    }
    __syncthreads();
    block_scan_1024(
        ns,
        [&](uint32_t i) -> uint64_t {
            const uint64_t cb = (c0 + i) * C, a = max(cb, T), e = cb + used[i];
            return e > a ? e - a : 0;
        },
        s_pre);
    block_scan_1024(
        nw,
        [&](uint32_t w) -> uint64_t {
            const uint64_t v = dlast[w];
            if (v == ~0ull) return 0;
            const uint64_t cb = (v >> 16) * C, a = cb + (v & 0xFFFFu), e = min(cb + C, T);
            d_start[w] = a;
            return e > a ? e - a : 0;
        },
        d_pre);
    if (t == 0) {
        plan[0] = T;
        plan[1] = c0;
        plan[2] = ns;
    }
}

// Direct output: moves source t of the plan to hole position t (any pairing
// of the two lists makes the output dense; a source is never a hole below T).
__global__ __launch_bounds__(256) void k_fill_copy(const uint64_t* __restrict__ plan,
                                                   const uint64_t* __restrict__ s_pre,
                                                   const uint64_t* __restrict__ d_pre,
                                                   const uint64_t* __restrict__ d_start,
                                                   uint32_t nw, uint32_t C,
                                                   const Request* __restrict__ req,
                                                   tds_result* __restrict__ out,
                                                   const tds_result* __restrict__ scratch) {
    const uint64_t T = plan[0], c0 = plan[1];
    const uint32_t ns = (uint32_t)plan[2];
    const uint64_t total = d_pre[nw];
    const Request R = req[0];
    for (uint64_t t = (uint64_t)blockIdx.x * 256 + threadIdx.x; t < total;
         t += (uint64_t)gridDim.x * 256) {
        uint32_t lo = 0, hi = nw;  // last hole with d_pre <= t
        while (hi - lo > 1) {
            const uint32_t m = (lo + hi) >> 1;
            if (d_pre[m] <= t) lo = m;
            else hi = m;
        }
        const uint64_t dst = d_start[lo] + (t - d_pre[lo]);
        uint32_t a = 0, b = ns;  // last source chunk with s_pre <= t
        while (b - a > 1) {
            const uint32_t m = (a + b) >> 1;
            if (s_pre[m] <= t) a = m;
            else b = m;
        }
        const uint64_t src = max((c0 + a) * C, T) + (t - s_pre[a]);
        const tds_result v =
            src < R.out_capacity ? out[R.out_offset + src] : scratch[src - R.out_capacity];
        out[R.out_offset + dst] = v;
    }
}

struct DistArgs {
    IndexView I;
    QueryView Q;             // query arrays (FP64 data of rechecked pairs)
    const uint32_t* qreq;    // request of each query segment
    const QF32* qf;
    const uint32_t* qsorted;
    const BucketInfo* binfo;
    const uint32_t* item_bucket;
    const BatchDesc* desc;
    SearchHeader* hdr;
    BlockStats* bstats;
    const Request* req;
    ReqCounter* rc;
    tds_result* out;
    uint64_t win_lo;        // first request-local result position kept
    unsigned long long* dyn_ctr;  // per-XCD dynamic item counters (kCtrStride apart)
    uint32_t item_begin;    // work items [item_begin, item_end)
    uint32_t item_end;      // 0xFFFFFFFF: every item of the search
    uint32_t* item_count;   // results per work item, or nullptr
    tds_result* stage;      // per-wave result stages, stage_cap records each
    uint32_t* stage_meta;   // group lane | index among the slot's staged results << 6
    uint32_t stage_cap;     // records per wave (a multiple of 64)
    uint32_t by_order;      // 1: a single-request item run whose results go to
                            // their order in the item (minus win_lo), no stage
    uint32_t cpl;           // FP32 form: candidates per lane per tile (2 or 4)
    uint32_t inline_refine; // FP32 form: refinement in the filter walk, not the queue
    uint32_t deal;          // TDS_DEAL_STATIC or TDS_DEAL_DYNAMIC
    // direct output (one request, not by_order): results go straight to the
    // request's output through per-wave reservations of dir_chunk positions
    uint32_t direct;
    uint32_t dir_chunk;
    unsigned long long* dir_ctr;  // next free position (reservation counter)
    tds_result* dscratch;   // positions [cap, cap + dscratch_cap) (the stage buffer)
    uint64_t dscratch_cap;
    uint64_t* dlast;        // per wave: last reservation (chunk << 16 | used), ~0: none
};

// FP32 data of a query segment for the closest-approach refinement (one per
// group lane): its velocity and the time of its sphere centre (the mid time
// of its clipped extent), each rounded to nearest; d rounded up; and the
// query's parts of the refinement's error scale.
struct QRef {
    float vx, vy, vz, tq;
    float d;
    float sc;  // |cx| + |cy| + |cz| of the sphere centre
    float sv;  // |vx| + |vy| + |vz|
    float st;  // |a| + |b| + |tq| + 1, [a, b] the clipped extent rounded outwards
};
static_assert(sizeof(QRef) == 32, "QRef layout");

// Results go through a stage of stage_cap records per wave in device memory
// and get their output positions when the stage is flushed (when the next
// batch of evaluations might not fit, and at the end of every work item):
// one device-scope atomic per request present in the item's query group
// reserves exactly the staged results of that request.  A returning atomic
// that every wave directs at its request's counter serialises across the
// chip; one per 64 evaluations cost a search with 10^8 results most of its
// time.  Positions within a request are unique and dense, in no fixed order.
//
// With by_order set (one request, one work item, re-run to fill successive
// windows of the host's buffer), a result's position is instead its order
// among the item's results, which a wave computes the same way on every run.
//
// Direct output (a one-request search's first pass): a wave reserves
// dir_chunk consecutive positions of the request at a time (one atomic per
// reservation, aligned chunks since every reservation has that size) and
// writes its results straight to them, keeping its last reservation open from
// one item to the next.  At the end each wave's last chunk may be partly
// used; positions at or past the output capacity go to a scratch buffer.  A
// fill pass (k_fill_plan, k_fill_copy) then moves the results found past the
// final count (or the capacity) into the unused tails below it, so that the
// output is dense again.  No result takes the round trip through a stage.
// Filter record of a query segment as the wave keeps it in LDS: the sphere
// and the clipped extent of its QF32 record (the candidate range stays in the
// registers of the query's lane).
struct QF24 {
    float cx, cy, cz, R;
    float a32, b32;
};
static_assert(sizeof(QF24) == 24, "QF24 layout");

// The wave's LDS: 10,240 bytes, so that four workgroups of four waves fit in a
// compute unit's 160 KB.  Per-lane values of the group (the request of query
// j, its request slot, the staged results of a slot) live in the registers of
// lane j (ItemState) and are read across lanes by shuffles.
struct alignas(64) WaveLDS {
    uint32_t queue[2 * kWave];  // < 64 left over + one pair per lane
    uint32_t rq[2 * kWave];     // FP32 form: refined pairs awaiting the FP64 evaluation
    QF24 qrec[kWave];           // filter records of the item's query group
    QRef qref[kWave];           // FP32 form: refinement data of the group's queries
    QCanon qc[kWave];           // canonical FP64 data of the group's queries
    uint32_t qid[kWave];        // group lane j -> q_seg of its records
    uint32_t qtraj[kWave];      // group lane j -> its trajectory
};
static_assert(sizeof(WaveLDS) == 10240, "WaveLDS size");

struct ItemState {
    uint32_t c0, c1, qbase, nq;
    uint32_t qn, evals;
    uint32_t rqn;     // pairs in the refined queue (FP32 form)
    bool refine;      // FP32 form: queued pairs go through the refinement first
    uint32_t found;   // results of the item so far (their order in the item)
    uint32_t nst;     // results in the wave's stage
    uint64_t sbase;   // the wave's stage: records [sbase, sbase + stage_cap)
    uint64_t ftests, btests;
    // direct output: the wave's open reservation [dpos, dend) (kept across
    // items) and its reservations so far
    uint64_t dpos, dend;
    uint32_t nres;
    // per lane j of the group
    uint32_t qr;      // request of query j
    uint32_t rslot;   // its request slot: the first lane with the same request
    uint32_t rcnt;    // staged results of request slot j (slot lanes only)
};

// Wave-wide ordering of device-memory accesses: stores of one lane are
// visible to loads of the other lanes after it (the stage is written by the
// lane that found a result and read back by the lane that copies it).
__device__ inline void wave_sync_mem() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
}

// Staged records each lane copies per round of a flush (their loads in
// flight together).
constexpr int kFlushUnroll = 4;

// Reserves the staged results of every request slot (one atomic each) and
// copies them from the stage to their positions; the stage is then empty.
// Slot lane s learns where its request's results go: staged result k of the
// slot has request position base + k and is kept when that position falls
// in the window [win_lo, win_lo + out_capacity), at out[dst + k].  The copy
// then reads kFlushUnroll records per lane before it writes any, so a flush
// waits for about one memory round trip per 256 records.
__device__ __forceinline__ void stage_flush(WaveLDS& L, const DistArgs& A, ItemState& S) {
    const uint32_t lane = __lane_id();
    wave_sync_mem();
    int64_t dst = 0;
    uint32_t klo = 0, khi = 0;  // kept staged results of slot `lane`: [klo, khi)
    if (S.rcnt) {
        const uint64_t base =
            (uint64_t)atomicAdd(&A.rc[S.qr].count, (unsigned long long)S.rcnt);
        const Request& R = A.req[S.qr];
        const uint64_t w0 = A.win_lo, w1 = A.win_lo + R.out_capacity, n = S.rcnt;
        klo = (uint32_t)min(max(w0, base) - base, n);
        khi = (uint32_t)min(max(w1, base) - base, n);
        dst = (int64_t)R.out_offset + (int64_t)base - (int64_t)A.win_lo;
    }
    S.rcnt = 0;
    for (uint32_t p0 = 0; p0 < S.nst; p0 += kFlushUnroll * kWave) {
        uint32_t meta[kFlushUnroll];
        uint4 ra[kFlushUnroll], rb[kFlushUnroll];
#pragma unroll
        for (int u = 0; u < kFlushUnroll; ++u) {
            const uint32_t p = p0 + u * kWave + lane;
            meta[u] = 0xFFFFFFFFu;  // no record (a real one is below 2^17)
            ra[u] = rb[u] = make_uint4(0u, 0u, 0u, 0u);
            if (p < S.nst) {
                meta[u] = A.stage_meta[S.sbase + p];
                const uint4* src = reinterpret_cast<const uint4*>(A.stage + S.sbase + p);
                ra[u] = src[0];
                rb[u] = src[1];
            }
        }
#pragma unroll
        for (int u = 0; u < kFlushUnroll; ++u) {
            // every lane takes part in the shuffles
            const uint32_t ql = meta[u] & (kWave - 1);
            const uint32_t k = (meta[u] >> 6) & 0x3FFFFFFu;
            const uint32_t slot = (uint32_t)__shfl((int)S.rslot, (int)ql);
            const int64_t d = __shfl((long long)dst, (int)slot);
            const uint32_t lo = (uint32_t)__shfl((int)klo, (int)slot);
            const uint32_t hi = (uint32_t)__shfl((int)khi, (int)slot);
            if (meta[u] != 0xFFFFFFFFu && k >= lo && k < hi) {
                uint4* o = reinterpret_cast<uint4*>(A.out + (d + (int64_t)k));
                o[0] = ra[u];
                o[1] = rb[u];
            }
        }
    }
    S.nst = 0;
    wave_sync_mem();
}

// Evaluates `cnt` <= 64 queued pairs from position `head` (one per lane) with
// the canonical FP64 code and stages the results (or, by order, writes them).
__device__ __forceinline__ void drain(WaveLDS& L, const uint32_t* queue, uint32_t head,
                                      uint32_t cnt, ItemState& S, const DistArgs& A) {
    const uint32_t lane = __lane_id();
    const bool act = lane < cnt;
    const uint32_t pk = act ? queue[head + lane] : 0u;
    const uint32_t ql = pk & (kWave - 1);
    const uint32_t i = S.c0 + (pk >> 6);
    const uint32_t slot = (uint32_t)__shfl((int)S.rslot, (int)ql);  // every lane takes part
    double t_lo = 0.0, t_hi = 0.0;
    bool hit = false;
    uint32_t qid = 0, qtraj = 0, eid = 0, etraj = 0;
    if (act) {
        const EntryF64 e = A.I.e64[i];
        eid = A.I.seg_id[i];
        etraj = A.I.traj[i];
        const QCanon q = L.qc[ql];
        qid = L.qid[ql];
        qtraj = L.qtraj[ql];
        hit = canon_eval<true>(q, e.x, e.y, e.z, e.vx, e.vy, e.vz, e.ts, e.te, &t_lo, &t_hi);
        if (A.Q.ent) {
            // self-join: pairs of one trajectory are not results, and a record
            // names the lower segment id first (its interval is symmetric)
            hit = hit && qtraj != etraj;
            if (qid > eid) {
                const uint32_t t0 = qid, t1 = qtraj;
                qid = eid;
                qtraj = etraj;
                eid = t0;
                etraj = t1;
            }
        }
    }
    tds_result rec;
    rec.q_seg = qid;
    rec.e_seg = eid;
    rec.q_traj = qtraj;
    rec.e_traj = etraj;
    rec.t_lo = t_lo;
    rec.t_hi = t_hi;
    const uint64_t hm = ballot(hit);
    const uint32_t nhit = (uint32_t)__popcll(hm);
    const uint32_t rank = (uint32_t)__popcll(hm & lanemask_lt());
    S.evals += cnt;
    if (A.by_order) {
        const uint64_t pos = (uint64_t)S.found + rank;
        const Request& R = A.req[0];
        if (hit && pos >= A.win_lo && pos - A.win_lo < R.out_capacity)
            A.out[R.out_offset + (pos - A.win_lo)] = rec;
        S.found += nhit;
        return;
    }
    if (A.direct) {
        if (!nhit) return;
        // nhit <= 64 <= dir_chunk: at most one new reservation
        const uint64_t room = S.dend - S.dpos;
        uint64_t pos = S.dpos + rank;
        if (nhit > room) {
            unsigned long long nb = 0;
            if (lane == 0) nb = atomicAdd(A.dir_ctr, (unsigned long long)A.dir_chunk);
            const uint64_t b = lane0_64(nb);
            if (rank >= room) pos = b + (rank - room);
            S.dpos = b + (nhit - room);
            S.dend = b + A.dir_chunk;
            ++S.nres;
        } else {
            S.dpos += nhit;
        }
        if (hit) {
            const Request& R = A.req[0];
            if (pos < R.out_capacity) A.out[R.out_offset + pos] = rec;
            else if (pos - R.out_capacity < A.dscratch_cap) A.dscratch[pos - R.out_capacity] = rec;
        }
        S.found += nhit;
        return;
    }
    if (!nhit) return;
    if (S.nst + nhit > A.stage_cap) stage_flush(L, A, S);
    // index of each result among the staged results of its request slot
    uint32_t idx = 0;
    uint64_t rem = hm;
    while (rem) {
        const uint32_t leader = (uint32_t)__ffsll((unsigned long long)rem) - 1u;
        const uint32_t sl = uniform((uint32_t)__shfl((int)slot, (int)leader));
        const uint64_t mm = ballot(hit && slot == sl);
        const uint32_t c = uniform((uint32_t)__builtin_amdgcn_readlane((int)S.rcnt, (int)sl));
        if (hit && slot == sl) idx = c + (uint32_t)__popcll(mm & lanemask_lt());
        if (lane == sl) S.rcnt = c + (uint32_t)__popcll(mm);
        rem &= ~mm;
    }
    if (hit) {
        A.stage[S.sbase + S.nst + rank] = rec;
        A.stage_meta[S.sbase + S.nst + rank] = ql | (idx << 6);
    }
    S.nst += nhit;
    S.found += nhit;
}

// Appends the lanes of mask m (candidate i) to the wave's pair queue.
__device__ __forceinline__ void enqueue(WaveLDS& L, uint64_t m, bool pass, uint32_t i, uint32_t c0,
                                        uint32_t& qn) {
    if (pass) L.queue[qn + (uint32_t)__popcll(m & lanemask_lt())] = ((i - c0) << 6) | __lane_id();
    qn += (uint32_t)__popcll(m);
}

// Closest-approach refinement of the FP32 filter, for a pair that passed the
// sphere and time tests: lower bounds, in FP32, on the smallest distance of
// the two moving points over their common extent.  The pair is dropped only
// when one of them exceeds d by more than the FP32 data and arithmetic can
// account for, so every pair the canonical FP64 evaluation accepts is kept.
//
// Query: centre cq = its position at tq (mid time of its clipped extent),
// velocity vq, clipped extent [qa, qb] rounded outwards; entry likewise (cl,
// vl, tl, [la, lb]).  On the common extent [a, b] (rounded outwards, so it
// contains the exact one), with tm = (a + b) / 2 and h = (b - a) / 2, the
// relative position is D(tau) = Dm + W tau for |tau| <= h, Dm = (cq - cl) +
// (vq (tm - tq) - vl (tm - tl)), W = vq - vl.  Its distance from the origin is
// at least
//   (1) |Dm| - h |W|                    (triangle inequality),
//   (2) |Dm x W| / |W|                  (distance to the line of motion),
//   (3) min(|Dm - h W|, |Dm + h W|)     when the vertex -Dm.W / |W|^2 lies
//                                       outside [-h, h] for certain.
// Error budget (u = 2^-24): rounding of the FP32 data to nearest and the
// operations forming Dm and W move D(tau) by at most about 10 u S0, S0 =
// |cq|1 + |cl|1 + (|vq|1 + |vl|1)(|a| + |b| + |tq| + |tl| + 1) (L1 norms; this
// also covers the FP64 rounding of the canonical evaluation, about 1e-15 S0).
// The scale used is S = (sc_q + sc_l) + (sv_q + sv_l)(st_q + st_l) >= S0 (the
// parts of each side are precomputed, QRef and the candidate's registers;
// |a| + |b| <= |qa| + |qb| + |la| + |lb| since a is qa or la and b is qb or
// lb), and E = 2^-17 S.  The squared forms below are evaluated with errors
// below 10 u (|Dm|1 + h|W|1)^2 and 20 u |Dm|1^2 |W|1^2, bounded by 2^-17 and
// 2^-16 times those magnitudes.  |W| comes from the hardware square root
// (within 1 ulp; its operand is kept normal by adding 2^-100, which only
// raises it) and is inflated by 2^-18.  Every test is "value > bound", so
// overflow to infinity or NaN never drops a pair.
__device__ __forceinline__ bool refine32(const QF24& f, const QRef& r, float clx, float cly,
                                         float clz, float vlx, float vly, float vlz, float tl,
                                         float la, float lb, float scl, float svl, float stl) {
    // sums of products are fused (fmaf): each has at most the rounding error
    // of the separate multiply and add it replaces
    const float a = fmaxf(f.a32, la), b = fminf(f.b32, lb);
    const float tm = 0.5f * (a + b), h = 0.5f * (b - a);
    const float dq = tm - r.tq, dl = tm - tl;
    const float dx = (f.cx - clx) + fmaf(r.vx, dq, -(vlx * dl));
    const float dy = (f.cy - cly) + fmaf(r.vy, dq, -(vly * dl));
    const float dz = (f.cz - clz) + fmaf(r.vz, dq, -(vlz * dl));
    const float wx = r.vx - vlx, wy = r.vy - vly, wz = r.vz - vlz;
    const float S = fmaf(r.sv + svl, r.st + stl, r.sc + scl);
    const float R = fmaf(0x1p-17f, S, r.d) * (1.0f + 0x1p-20f);
    const float R2 = (R * R) * (1.0f + 0x1p-20f);
    const float dm1 = fabsf(dx) + fabsf(dy) + fabsf(dz);
    const float w1 = fabsf(wx) + fabsf(wy) + fabsf(wz);
    const float Dm2 = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float WW = fmaf(wz, wz, fmaf(wy, wy, wx * wx));
    const float DW = fmaf(dz, wz, fmaf(dy, wy, dx * wx));
    const float span = fmaf(h, w1, dm1);
    const float errA = 0x1p-17f * (span * span);
    // (1)
    const float hw = (h * __builtin_amdgcn_sqrtf(WW + 0x1p-100f)) * (1.0f + 0x1p-18f);
    const float Rh = R + hw;
    if (Dm2 - errA > (Rh * Rh) * (1.0f + 0x1p-20f)) return false;
    // (2), multiplied through by |W|^2
    const float cross = dm1 * w1;
    if (fmaf(-DW, DW, Dm2 * WW) - 0x1p-16f * (cross * cross) > (R2 * WW) * (1.0f + 0x1p-18f))
        return false;
    // (3)
    if (fabsf(DW) > fmaf(h, WW, 0x1p-17f * fmaf(h, w1 * w1, cross))) {
        const float ax = fmaf(-h, wx, dx), ay = fmaf(-h, wy, dy), az = fmaf(-h, wz, dz);
        const float bx = fmaf(h, wx, dx), by = fmaf(h, wy, dy), bz = fmaf(h, wz, dz);
        const float D0 = fmaf(az, az, fmaf(ay, ay, ax * ax));
        const float D1 = fmaf(bz, bz, fmaf(by, by, bx * bx));
        if (fminf(D0, D1) - errA > R2) return false;
    }
    return true;
}

// The query's refinement data, from its canonical data and filter record.
__device__ __forceinline__ QRef qref_of(const QCanon& q, const QF32& f) {
    QRef r;
    r.vx = __double2float_rn(q.vx);
    r.vy = __double2float_rn(q.vy);
    r.vz = __double2float_rn(q.vz);
    r.tq = __double2float_rn(0.5 * (q.aq + q.bq));
    r.d = __double2float_ru(q.d);
    r.sc = (fabsf(f.cx) + fabsf(f.cy)) + fabsf(f.cz);
    r.sv = (fabsf(r.vx) + fabsf(r.vy)) + fabsf(r.vz);
    r.st = ((fabsf(f.a32) + fabsf(f.b32)) + fabsf(r.tq)) + 1.0f;
    return r;
}

// The candidate's parts of the refinement's error scale (see refine32).
struct ERef {
    float sc, sv, st;
};
__device__ __forceinline__ ERef eref_of(float cx, float cy, float cz, const EntryV32& v, float ts,
                                        float te) {
    ERef e;
    e.sc = (fabsf(cx) + fabsf(cy)) + fabsf(cz);
    e.sv = (fabsf(v.vx) + fabsf(v.vy)) + fabsf(v.vz);
    e.st = (fabsf(ts) + fabsf(te)) + fabsf(v.tm);
    return e;
}

// FP32 form: the closest-approach refinement (refine32) of `cnt` <= 64 queued
// sphere survivors from position `head`, one per lane; the pairs it keeps go
// to the refined queue.  A stage of its own, so that its registers are not
// held across the filter's walk and searches with few survivors seldom run it.
__device__ __forceinline__ void refine_step(WaveLDS& L, uint32_t head, uint32_t cnt,
                                            ItemState& S, const DistArgs& A) {
    const uint32_t lane = __lane_id();
    const bool act = lane < cnt;
    const uint32_t pk = act ? L.queue[head + lane] : 0u;
    bool keep = false;
    if (act) {
        const uint32_t ql = pk & (kWave - 1);
        const uint32_t i = S.c0 + (pk >> 6);
        const EntryF32 e = A.I.e32[i];
        const EntryV32 v = A.I.ev32[i];
        const QF24 f = L.qrec[ql];
        keep = true;
        // an unbounded sphere (stored centre 0) passes unrefined
        if (e.r < INFINITY && f.R < INFINITY) {
            const ERef x = eref_of(e.cx, e.cy, e.cz, v, e.ts, e.te);
            keep = refine32(f, L.qref[ql], e.cx, e.cy, e.cz, v.vx, v.vy, v.vz, v.tm, e.ts, e.te,
                            x.sc, x.sv, x.st);
        }
    }
    const uint64_t m = ballot(keep);
    if (keep) L.rq[S.rqn + (uint32_t)__popcll(m & lanemask_lt())] = pk;
    S.rqn += (uint32_t)__popcll(m);
    wave_sync();
}

// Moves entries [from, n) of a queue to its front.
__device__ __forceinline__ void queue_shift(uint32_t* queue, uint32_t from, uint32_t n) {
    const uint32_t lane = __lane_id();
    const uint32_t rest = n - from;  // < 64
    wave_sync();
    uint32_t v = 0;
    if (lane < rest) v = queue[from + lane];
    wave_sync();
    if (lane < rest) queue[lane] = v;
    wave_sync();
}

// Evaluates full batches of 64 queued pairs (FP32 form: refined first, then
// evaluated 64 refined pairs at a time); keeps the remainders queued.
__device__ __forceinline__ void drain_full(WaveLDS& L, ItemState& S, const DistArgs& A) {
    uint32_t head = 0;
    wave_sync();
    while (S.qn - head >= kWave) {
        if (S.refine) {
            refine_step(L, head, kWave, S, A);
            if (S.rqn >= kWave) {
                drain(L, L.rq, 0, kWave, S, A);
                queue_shift(L.rq, kWave, S.rqn);
                S.rqn -= kWave;
            }
        } else {
            drain(L, L.queue, head, kWave, S, A);
        }
        head += kWave;
    }
    if (head) {
        queue_shift(L.queue, head, S.qn);
        S.qn -= head;
    }
    wave_sync();
}

// Evaluates everything still queued (end of a work item).
__device__ __forceinline__ void drain_rest(WaveLDS& L, ItemState& S, const DistArgs& A) {
    wave_sync();
    if (S.qn) {
        if (S.refine) refine_step(L, 0, S.qn, S, A);
        else drain(L, L.queue, 0, S.qn, S, A);
        S.qn = 0;
    }
    uint32_t head = 0;
    while (S.rqn - head > 0) {
        const uint32_t c = min(S.rqn - head, (uint32_t)kWave);
        drain(L, L.rq, head, c, S, A);
        head += c;
    }
    S.rqn = 0;
    wave_sync();
}

// Start of a work item: the canonical data, record ids and request of each
// query segment of the group, and its request slot (the first lane of the
// group with the same request).
__device__ __forceinline__ void item_begin(WaveLDS& L, const DistArgs& A, ItemState& S) {
    const uint32_t lane = __lane_id();
    const bool has = lane < S.nq;
    uint32_t r = 0;
    QCanon q = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0};  // empty window: never a member
    uint32_t qid = 0, qtraj = 0;
    if (has) {
        const uint32_t k = A.qsorted[S.qbase + lane];
        r = A.qreq[k];
        const Request& R = A.req[r];
        query_canon(A.Q, R, k, q);
        if (A.Q.ent) {
            qid = A.Q.ent_id[k];
            qtraj = A.Q.ent_traj[k];
        } else {
            qid = (uint32_t)(k - R.q_begin);
            qtraj = A.Q.traj ? A.Q.traj[k] : 0u;
        }
    }
    uint32_t slot = lane;
    uint64_t rem = ballot(has);
    while (rem) {
        const uint32_t leader = (uint32_t)__ffsll((unsigned long long)rem) - 1u;
        const uint32_t rr = uniform((uint32_t)__shfl((int)r, (int)leader));
        const uint64_t mm = ballot(has && r == rr);
        if ((mm >> lane) & 1ull) slot = leader;
        rem &= ~mm;
    }
    wave_sync();
    L.qc[lane] = q;
    L.qid[lane] = qid;
    L.qtraj[lane] = qtraj;
    S.qr = r;
    S.rslot = slot;
    S.rcnt = 0;
    wave_sync();
}

// FP32 filter record of the query segment held by a lane (its QF32 record).
struct QReg {
    Box32 box;        // box of the clipped segment grown by d (seg_box32)
    float a, b;       // clipped window rounded outwards
    uint32_t lo, hi;  // candidate range
};

// Value of v in lane j (wave-uniform j): a register read, no memory access.
__device__ __forceinline__ float lane_val(float v, uint32_t j) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), (int)j));
}

// FP32 filter of one query (its record q, read from LDS at a wave-uniform
// address, i.e. broadcast to every lane) against the candidate held in this
// lane.  A pair can only be a result if the two bounding spheres come within
// d (the error margins are folded into R and r) and the outward-rounded time
// extents overlap strictly.  With kTime false the caller has established
// that every pair of the slot overlaps in time.
template <bool kTime>
__device__ __forceinline__ bool pass32(const QF24& q, float ecx, float ecy, float ecz, float er,
                                       float ets, float ete) {
    bool p = sphere_pass(q.cx, q.cy, q.cz, q.R, ecx, ecy, ecz, er);
    if (kTime) p = p & (q.a32 < ete) & (ets < q.b32);
    return p;
}

// One 64-candidate slot (candidate `cand` in the lane) against the queries of
// mask mk, in ascending order.  For each query, the sphere and time test of
// every lane's candidate, then, with kInline, the closest-approach refinement
// of the pairs that passed (the candidate's motion is loaded at the slot's
// first survivor); the pairs kept are queued, and full batches of 64 go on to
// the FP64 evaluation.  Without kInline the sphere survivors are queued and
// the refinement is a stage of the queue (refine_step).  mk is wave uniform:
// the walk over its bits is scalar, and the query records are read from LDS
// at wave-uniform addresses.  With kUniform false, the queries of `part`
// have candidate ranges that cover the slot only in part: their bounds are
// read from the registers of their lanes (qlo, qhi) and checked per pair.
template <bool kUniform, bool kTime, bool kInline>
__device__ __forceinline__ void slot_fp32(WaveLDS& L, const DistArgs& A, ItemState& S,
                                          uint64_t mk, uint64_t part, uint32_t qlo, uint32_t qhi,
                                          uint32_t cand, float ecx, float ecy, float ecz,
                                          float er, float ets, float ete) {
    const uint32_t code = (cand - S.c0) << 6;  // used in lanes whose candidate is in the chunk
    bool motion = false;
    EntryV32 ev = {0.f, 0.f, 0.f, 0.f};
    ERef ex = {0.f, 0.f, 0.f};
    while (mk) {
        const uint32_t j = (uint32_t)__builtin_ctzll(mk);
        mk &= mk - 1u;
        const QF24 q = L.qrec[j];
        bool p = pass32<kTime>(q, ecx, ecy, ecz, er, ets, ete);
        if (!kUniform && ((part >> j) & 1ull)) {
            const uint32_t lo = uniform((uint32_t)__builtin_amdgcn_readlane((int)qlo, (int)j));
            const uint32_t hi = uniform((uint32_t)__builtin_amdgcn_readlane((int)qhi, (int)j));
            p = p & (cand >= lo) & (cand < hi);
        }
        uint64_t m = ballot(p);
        if (!m) continue;
        if (kInline) {
            if (!motion) {
                motion = true;
                // lanes outside the chunk load its last entry (they never pass)
                const uint32_t i = (cand >= S.c0 && cand < S.c1) ? cand : S.c1 - 1u;
                ev = A.I.ev32[i];
                ex = eref_of(ecx, ecy, ecz, ev, ets, ete);
            }
            // an unbounded sphere (stored centre 0) passes unrefined
            if (p && er < INFINITY && q.R < INFINITY)
                p = refine32(q, L.qref[j], ecx, ecy, ecz, ev.vx, ev.vy, ev.vz, ev.tm, ets, ete,
                             ex.sc, ex.sv, ex.st);
            m = ballot(p);
        }
        if (p) L.queue[S.qn + (uint32_t)__popcll(m & lanemask_lt())] = code | j;
        S.qn += (uint32_t)__popcll(m);
        if (S.qn >= kWave) drain_full(L, S, A);
    }
}

// FP32 form: the wave takes the chunk kCpl * 64 candidates at a time (kCpl
// per lane, coalesced vector loads, tiles aligned to the 64-entry blocks).
// Lane j holds query j of the group and, with the spatial layout, the box of
// one of the next 64 blocks (broadcast from its registers by readlane, so the
// loop over blocks makes no memory access).  Each block's box is first tested
// against every query (one lane per query), and only the queries that pass
// are tested against the block's entries, their records read from the wave's
// LDS copy of the group.  When every
// candidate of the bucket overlaps every query of the group in time, the
// per-pair time test is skipped: exact, since the outward-rounded FP32 times
// then overlap as well.
template <bool kUniform, int kCpl, bool kInline>
__device__ __forceinline__ void scan_chunk_fp32(WaveLDS& L, const DistArgs& A, ItemState& S,
                                                const BucketInfo& bi) {
    constexpr uint32_t kStep = kCpl * kWave;  // candidates per tile
    const uint32_t lane = __lane_id();
    const bool has = lane < S.nq;
    const bool cull = A.I.bbox != nullptr;
    // a lane without a query: an empty box (it never passes a block) and an
    // unbounded window (it never blocks the whole-overlap shortcut)
    QReg q = {{INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY},
              -INFINITY, INFINITY, 0u, 0u};
    if (has) {
        const QF32 f = A.qf[S.qbase + lane];
        q.box = f.box;
        q.a = f.a32;
        q.b = f.b32;
        q.lo = f.lo;
        q.hi = f.hi;
        L.qrec[lane] = QF24{f.cx, f.cy, f.cz, f.R, f.a32, f.b32};
        if (kInline || S.refine) L.qref[lane] = qref_of(L.qc[lane], f);
    }
    wave_sync();
    const bool all_overlap =
        ballot(((double)q.a < bi.tmin_te) && (bi.tmax_ts < (double)q.b)) == ~0ull;
    const uint64_t has_mask = ballot(has);
    const uint32_t last_blk = (S.c1 - 1) >> kBoxShift;
    uint32_t wb = 0xFFFFFFFFu;  // first block of the box window held in the lanes
    Box32 wbox;
    for (uint32_t tile = S.c0 & ~(uint32_t)(kWave - 1); tile < S.c1; tile += kStep) {
        uint32_t cand[kCpl];
        float ecx[kCpl], ecy[kCpl], ecz[kCpl], er[kCpl], ets[kCpl], ete[kCpl];
        bool valid[kCpl];
#pragma unroll
        for (int k = 0; k < kCpl; ++k) {
            cand[k] = tile + k * kWave + lane;
            valid[k] = cand[k] >= S.c0 && cand[k] < S.c1;
            const EntryF32 e = A.I.e32[valid[k] ? cand[k] : S.c1 - 1];
            ecx[k] = e.cx;
            ecy[k] = e.cy;
            ecz[k] = e.cz;
            er[k] = e.r;
            // a slot outside the chunk gets an empty time extent: it never passes
            ets[k] = valid[k] ? e.ts : INFINITY;
            ete[k] = valid[k] ? e.te : -INFINITY;
        }
        const uint32_t tb = tile >> kBoxShift;
        if (cull && (wb == 0xFFFFFFFFu || tb + kCpl > wb + kWave)) {
            // lane l takes the box of block wb + l (the last block of the
            // chunk repeated past the end)
            wb = tb;
            wbox = A.I.bbox[min(wb + lane, last_blk)].b;
        }
#pragma unroll
        for (int k = 0; k < kCpl; ++k) {
            const uint32_t b0 = tile + k * kWave;  // first entry of the block
            if (b0 >= S.c1) break;
            uint64_t mk = has_mask, part = 0;
            if (!kUniform) {
                mk &= ballot(q.lo < b0 + kWave && q.hi > b0);
                part = mk & ~ballot(q.lo <= b0 && q.hi >= b0 + kWave);
            }
            if (cull && mk) {
                const uint32_t bl = tb + k - wb;
                const Box32 box = {lane_val(wbox.lx, bl), lane_val(wbox.ly, bl),
                                   lane_val(wbox.lz, bl), lane_val(wbox.hx, bl),
                                   lane_val(wbox.hy, bl), lane_val(wbox.hz, bl)};
                mk &= ballot(box_overlap(box, q.box));
                S.btests += S.nq;
            }
            if (!mk) continue;
            const uint64_t vm = ballot(valid[k]);
            S.ftests += (uint64_t)__popcll(mk) * (uint64_t)__popcll(vm);
            // the time test can be dropped only on full slots
            if (all_overlap && vm == ~0ull)
                slot_fp32<kUniform, false, kInline>(L, A, S, mk, part, q.lo, q.hi, cand[k], ecx[k],
                                                    ecy[k], ecz[k], er[k], ets[k], ete[k]);
            else
                slot_fp32<kUniform, true, kInline>(L, A, S, mk, part, q.lo, q.hi, cand[k], ecx[k],
                                                   ecy[k], ecz[k], er[k], ets[k], ete[k]);
        }
    }
}

// Plain FP64 form: one query segment per lane, every candidate of the chunk
// streamed through scalar loads and tested with the canonical predicate.
template <bool kUniform>
__device__ __forceinline__ void scan_chunk_fp64(WaveLDS& L, const DistArgs& A, ItemState& S) {
    const uint32_t lane = __lane_id();
    const bool has = lane < S.nq;
    ConstE64 ce = (ConstE64)(A.I.e64);
    const QCanon q = L.qc[lane];  // an empty window past the group's end
    uint32_t qlo = 0, qhi = 0;
    if (has) {
        const QF32 f = A.qf[S.qbase + lane];
        qlo = f.lo;
        qhi = f.hi;
    }
    for (uint32_t i = S.c0; i < S.c1; ++i) {
        const f64x4 e0 = ce[2 * i], e1 = ce[2 * i + 1];  // x, y, z, vx | vy, vz, ts, te
        bool pass = canon_eval<false>(q, e0[0], e0[1], e0[2], e0[3], e1[0], e1[1], e1[2], e1[3],
                                      nullptr, nullptr);
        if (!kUniform) pass = pass & (i >= qlo) & (i < qhi);
        const uint64_t m = ballot(pass);
        if (!m) continue;
        enqueue(L, m, pass, i, S.c0, S.qn);
        if (S.qn >= kWave) drain_full(L, S, A);
    }
}

template <int kPrec, int kCplT, bool kInline>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4))) void k_distance(DistArgs A) {
    __shared__ WaveLDS wl[kWavesPerBlock];
    WaveLDS& L = wl[threadIdx.x / kWave];
    const uint32_t lane = __lane_id();
    uint64_t tests = 0, evals_total = 0, ftests = 0, btests = 0;
    uint32_t flushes = 0;  // stage flushes at the end of an item (direct output: reservations)
    uint64_t dpos = 0, dend = 0, found_total = 0;  // direct output (see DistArgs)
    // all items of the search, unless a range is given (incremental passes)
    const uint32_t item_end = (A.item_end == 0xFFFFFFFFu)
                                  ? uniform(min(A.hdr->n_items, A.desc->item_cap))
                                  : A.item_end;
    // Items [item_begin, item_end) are split into 8 contiguous parts, one
    // per XCD (workgroups are dispatched to the XCDs round-robin, so
    // workgroup b runs on XCD b mod 8; consecutive items share buckets, hence
    // candidate ranges, which then stay under one XCD's L2).  Each wave first
    // takes one item of its XCD's part statically (item p0 + its index among
    // the XCD's waves: no atomic on the critical path of light searches,
    // where this round covers every item).  Items beyond that round are
    // taken dynamically from the part's counter, and a wave whose part is
    // used up takes from the next parts: item costs vary by orders of
    // magnitude where results cluster (a static deal left some XCDs idle for
    // more than half of a galaxy search).  A part's counter is read before
    // it is incremented, so exhausted parts cost loads, not contended atomics.
    const uint64_t n_it = item_end > A.item_begin ? item_end - A.item_begin : 0u;
    // this wave's result stage
    const uint64_t sbase =
        (uint64_t)(blockIdx.x * kWavesPerBlock + threadIdx.x / kWave) * A.stage_cap;
    const uint32_t ng = min(gridDim.x, kXcds);
    const uint32_t grp = blockIdx.x % ng;
    const uint32_t gw = uniform((blockIdx.x / ng) * kWavesPerBlock + threadIdx.x / kWave);
    // waves of the workgroups on XCD x
    auto waves_of = [&](uint32_t x) {
        return ((gridDim.x - x + ng - 1) / ng) * (uint32_t)kWavesPerBlock;
    };
    auto part_lo = [&](uint32_t x) { return n_it * x / ng; };
    // static deal (chosen per launch): every item round-robin over the
    // XCD's waves, no counter at all
    const bool stat = A.deal == TDS_DEAL_STATIC;
    bool dyn = false;  // does any part hold more items than its XCD has waves?
    if (!stat)
        for (uint32_t x = 0; x < ng; ++x) dyn = dyn || part_lo(x + 1) - part_lo(x) > waves_of(x);
    uint64_t k = part_lo(grp) + gw;
    bool have = k < part_lo(grp + 1);
    uint32_t xs = grp;  // the part dynamic items are taken from
    for (;;) {
        if (!have) {
            if (!dyn) break;
            // the next dynamic item: the parts' counters are read at once,
            // one part per lane in rotation from part xs, and the first part
            // with items left past its static round is taken from; losing
            // the race for a part's last items exhausts that part, so this
            // ends after at most ng + 1 rounds
            for (uint32_t round = 0; round <= ng && !have; ++round) {
                bool avail = false;
                if (lane < ng) {
                    const uint32_t x = (xs + lane) % ng;
                    const uint64_t ps = part_lo(x) + waves_of(x), pe = part_lo(x + 1);
                    if (ps < pe) {
                        const uint64_t v = __hip_atomic_load(A.dyn_ctr + (size_t)x * kCtrStride,
                                                             __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                        avail = ps + v < pe;
                    }
                }
                const uint64_t am = ballot(avail);
                if (!am) break;  // every part is used up
                xs = (xs + (uint32_t)__ffsll((unsigned long long)am) - 1u) % ng;
                uint64_t v = 0;
                if (lane == 0) v = atomicAdd(A.dyn_ctr + (size_t)xs * kCtrStride, 1ull);
                v = lane0_64(v);
                const uint64_t ps = part_lo(xs) + waves_of(xs), pe = part_lo(xs + 1);
                if (ps + v < pe) {
                    k = ps + v;
                    have = true;
                }
            }
            if (!have) break;
        }
        have = false;
        const uint32_t it = A.item_begin + (uint32_t)k;
        const uint32_t b = uniform(A.item_bucket[it]);
        const BucketInfo bi = A.binfo[b];
        const uint32_t local = it - bi.item0;
        // chunk-major inside a bucket: the groups of one chunk are adjacent
        // items, so the waves of an XCD, which work through a contiguous
        // part of the item list, share the chunk's records in their L2
        const uint32_t ngr = (bi.count + kWave - 1) / kWave;
        const uint32_t c = local / ngr;
        const uint32_t g = local - c * ngr;
        ItemState S;
        S.sbase = sbase;
        S.nq = uniform(min((uint32_t)kWave, bi.count - g * kWave));
        const uint64_t base = (uint64_t)(bi.lo & ~(uint32_t)(kWave - 1)) + (uint64_t)c * bi.clen;
        S.c0 = uniform((uint32_t)max((uint64_t)bi.lo, base));
        S.c1 = uniform((uint32_t)min((uint64_t)bi.hi, base + bi.clen));
        S.qbase = uniform(bi.start + g * kWave);
        S.qn = 0;
        S.rqn = 0;
        S.refine = kPrec == TDS_PREC_FP32_RECHECK && !kInline;
        S.evals = 0;
        S.found = 0;
        S.nst = 0;
        S.ftests = 0;
        S.btests = 0;
        S.dpos = dpos;
        S.dend = dend;
        S.nres = 0;
        // does every query of the group cover the whole chunk?
        bool cover = true;
        if (lane < S.nq) {
            const QF32 f = A.qf[S.qbase + lane];
            cover = f.lo <= S.c0 && f.hi >= S.c1;
        }
        const bool all_cover = ballot(cover) == ~0ull;
        item_begin(L, A, S);
        if (kPrec == TDS_PREC_FP32_RECHECK) {
            if (all_cover) scan_chunk_fp32<true, kCplT, kInline>(L, A, S, bi);
            else scan_chunk_fp32<false, kCplT, kInline>(L, A, S, bi);
        } else {
            if (all_cover) scan_chunk_fp64<true>(L, A, S);
            else scan_chunk_fp64<false>(L, A, S);
        }
        drain_rest(L, S, A);
        // the item's results get their positions (the next item's group has
        // other request slots)
        if (S.nst) {
            stage_flush(L, A, S);
            ++flushes;
        }
        dpos = S.dpos;
        dend = S.dend;
        flushes += S.nres;
        found_total += S.found;
        tests += (uint64_t)(S.c1 - S.c0) * S.nq;
        ftests += (kPrec == TDS_PREC_FP64) ? (uint64_t)(S.c1 - S.c0) * S.nq : S.ftests;
        btests += S.btests;
        evals_total += S.evals;
        if (A.item_count && lane == 0) A.item_count[it] = S.found;
        if (stat) {
            // the wave's next item of its part
            k += waves_of(grp);
            have = k < part_lo(grp + 1);
        }
    }
    const uint32_t wid = threadIdx.x / kWave;
    if (A.direct && lane == 0) {
        // the wave's results and its last reservation (chunk, positions used)
        if (found_total) atomicAdd(&A.rc[0].count, (unsigned long long)found_total);
        A.dlast[blockIdx.x * kWavesPerBlock + wid] =
            dend ? ((dend / A.dir_chunk - 1) << 16) | (A.dir_chunk - (dend - dpos)) : ~0ull;
    }
    // per-workgroup counters (folded into the header by k_stats_fold), each
    // wave's in the front of its own LDS, which it no longer uses
    wave_sync();
    if (lane == 0) {
        BlockStats& w = *reinterpret_cast<BlockStats*>(wl[wid].queue);
        w.tests = tests;
        w.evals = evals_total;
        w.ftests = ftests;
        w.btests = btests;
        w.flushes = flushes;
        w.pad[0] = w.pad[1] = w.pad[2] = 0;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        BlockStats b = *reinterpret_cast<const BlockStats*>(wl[0].queue);
        for (int k = 1; k < kWavesPerBlock; ++k) {
            const BlockStats& w = *reinterpret_cast<const BlockStats*>(wl[k].queue);
            b.tests += w.tests;
            b.evals += w.evals;
            b.ftests += w.ftests;
            b.btests += w.btests;
            b.flushes += w.flushes;
        }
        A.bstats[blockIdx.x] = b;
    }
}

// ------------------------------------------------------------ host side

template <typename T>
int grow(T** p, size_t* cap, size_t need) {
    if (*cap >= need && *p) return TDS_OK;
    dfree(*p);
    *p = nullptr;
    *cap = 0;
    TDS_TRY(dmalloc(p, need));
    *cap = need;
    return TDS_OK;
}

}  // namespace

Workspace::~Workspace() {
    for (void* p : {(void*)qfu, (void*)qreq, (void*)qkey, (void*)qslot, (void*)qsorted, (void*)qf, (void*)qstage,
                    (void*)qtraj_stage, (void*)ctl, (void*)b_count,
                    (void*)b_hi, (void*)b_start, (void*)b_nch,
                    (void*)binfo, (void*)item_bucket, (void*)item_count, (void*)res,
                    (void*)bstats, (void*)stage, (void*)stage_meta, (void*)dyn_ctr,
                    (void*)dlast, (void*)fill_s, (void*)fill_d, (void*)fill_dstart,
                    (void*)fill_plan})
        dfree(p);
    if (ctl_host) (void)hipHostFree(ctl_host);
    if (ev0) (void)hipEventDestroy(ev0);
    if (ev1) (void)hipEventDestroy(ev1);
}

int ws_init(Workspace* w) {
    TDS_TRY(dmalloc(&w->b_count, kMaxBuckets));
    TDS_TRY(dmalloc(&w->b_hi, kMaxBuckets));
    TDS_TRY(dmalloc(&w->b_start, kMaxBuckets));
    TDS_TRY(dmalloc(&w->b_nch, kMaxBuckets));
    TDS_TRY(dmalloc(&w->binfo, kMaxBuckets));
    TDS_TRY(dmalloc(&w->bstats, kMaxDistBlocks));
    TDS_TRY(dmalloc(&w->dyn_ctr, (size_t)kCtrSlots * kCtrStride));
    TDS_HIP(hipEventCreate(&w->ev0));
    TDS_HIP(hipEventCreate(&w->ev1));
    return ws_reserve(w, 0, 1);
}

namespace {

// Byte offsets in the control block for r_cap requests (every part starts
// on a 64-B boundary: the four structures are multiples of 16 B, and
// BatchDesc and SearchHeader are 64-B aligned).
struct CtlLayout {
    size_t req, hdr, ctr, bytes;
};

CtlLayout ctl_layout(size_t r_cap) {
    auto up = [](size_t v) { return (v + 63) / 64 * 64; };
    CtlLayout L;
    L.req = up(sizeof(BatchDesc));
    L.hdr = up(L.req + r_cap * sizeof(Request));
    L.ctr = up(L.hdr + sizeof(SearchHeader));
    L.bytes = up(L.ctr + r_cap * sizeof(ReqCounter));
    return L;
}

}  // namespace

int ws_upload(Workspace* w, uint32_t nreq, hipStream_t s) {
    const CtlLayout L = ctl_layout(w->r_cap);
    TDS_HIP(hipMemcpyAsync(w->ctl, w->ctl_host, L.req + nreq * sizeof(Request),
                           hipMemcpyHostToDevice, s));
    return TDS_OK;
}

int ws_download(Workspace* w, uint32_t nreq, hipStream_t s) {
    const CtlLayout L = ctl_layout(w->r_cap);
    TDS_HIP(hipMemcpyAsync(w->ctl_host + L.hdr, w->ctl + L.hdr,
                           L.ctr - L.hdr + nreq * sizeof(ReqCounter), hipMemcpyDeviceToHost, s));
    return TDS_OK;
}

int ws_reserve(Workspace* w, size_t nq, size_t nreq) {
    if (w->q_cap < nq || !w->qfu) {
        for (void* p : {(void*)w->qfu, (void*)w->qreq, (void*)w->qkey, (void*)w->qslot,
                        (void*)w->qsorted, (void*)w->qf})
            dfree(p);
        w->qfu = nullptr;
        w->qreq = nullptr;
        w->qf = nullptr;
        w->qkey = w->qslot = w->qsorted = nullptr;
        w->q_cap = 0;
        TDS_TRY(dmalloc(&w->qfu, nq));
        TDS_TRY(dmalloc(&w->qreq, nq));
        TDS_TRY(dmalloc(&w->qkey, nq));
        TDS_TRY(dmalloc(&w->qslot, nq));
        TDS_TRY(dmalloc(&w->qsorted, nq));
        TDS_TRY(dmalloc(&w->qf, nq + kQfPad));
        w->q_cap = nq;
    }
    if (w->r_cap < nreq || !w->ctl) {
        dfree(w->ctl);
        if (w->ctl_host) (void)hipHostFree(w->ctl_host);
        w->ctl = w->ctl_host = nullptr;
        w->desc = w->desc_host = nullptr;
        w->req = w->req_host = nullptr;
        w->hdr = w->hdr_host = nullptr;
        w->req_ctr = w->rc_host = nullptr;
        w->r_cap = 0;
        const size_t r_cap = std::max<size_t>(nreq, 16);
        const CtlLayout L = ctl_layout(r_cap);
        TDS_TRY(dmalloc(&w->ctl, L.bytes));
        TDS_HIP(hipHostMalloc((void**)&w->ctl_host, L.bytes, hipHostMallocDefault));
        std::memset(w->ctl_host, 0, L.bytes);
        for (int side = 0; side < 2; ++side) {
            char* base = side ? w->ctl_host : w->ctl;
            BatchDesc* desc = reinterpret_cast<BatchDesc*>(base);
            Request* req = reinterpret_cast<Request*>(base + L.req);
            SearchHeader* hdr = reinterpret_cast<SearchHeader*>(base + L.hdr);
            ReqCounter* ctr = reinterpret_cast<ReqCounter*>(base + L.ctr);
            (side ? w->desc_host : w->desc) = desc;
            (side ? w->req_host : w->req) = req;
            (side ? w->hdr_host : w->hdr) = hdr;
            (side ? w->rc_host : w->req_ctr) = ctr;
        }
        w->r_cap = r_cap;
    }
    return TDS_OK;
}

namespace {
uint32_t launch_blocks(uint32_t grid_waves);
size_t stage_total(uint32_t grid_waves);
}  // namespace

int ws_reserve_stage(Workspace* w, uint32_t grid_waves) {
    const size_t need = stage_total(grid_waves);
    const uint32_t waves = launch_blocks(grid_waves) * kWavesPerBlock;
    if (w->stage_waves < waves || !w->dlast) {
        for (void* p : {(void*)w->dlast, (void*)w->fill_s, (void*)w->fill_d,
                        (void*)w->fill_dstart, (void*)w->fill_plan})
            dfree(p);
        w->dlast = w->fill_s = w->fill_d = w->fill_dstart = w->fill_plan = nullptr;
        w->stage_waves = 0;
        TDS_TRY(dmalloc(&w->dlast, waves));
        TDS_TRY(dmalloc(&w->fill_s, (size_t)waves + 2));
        TDS_TRY(dmalloc(&w->fill_d, (size_t)waves + 1));
        TDS_TRY(dmalloc(&w->fill_dstart, waves));
        TDS_TRY(dmalloc(&w->fill_plan, 4));
        w->stage_waves = waves;
    }
    if (w->stage_recs >= need && w->stage) return TDS_OK;
    dfree(w->stage);
    dfree(w->stage_meta);
    w->stage = nullptr;
    w->stage_meta = nullptr;
    w->stage_recs = 0;
    TDS_TRY(dmalloc(&w->stage, need));
    TDS_TRY(dmalloc(&w->stage_meta, need));
    w->stage_recs = need;
    return TDS_OK;
}

namespace {

uint32_t bucket_shift(uint32_t m) {
    uint32_t shift = 0;
    while ((((uint64_t)m * kSpanClasses - 1) >> shift) >= kMaxBuckets) ++shift;
    return shift;
}

uint32_t bucket_count(uint32_t m) {
    return (uint32_t)((((uint64_t)m * kSpanClasses - 1) >> bucket_shift(m)) + 1);
}

// Upper bound of the work items of a batch of nq query segments: every
// non-empty bucket contributes ceil(count / 64) groups, each split into at
// most ceil((n + 63) / chunk) chunks (chunks count from a 64-entry block).
uint64_t item_bound(uint64_t nq, uint32_t nb, uint64_t n, uint32_t chunk) {
    const uint64_t groups = (nq + kWave - 1) / kWave + std::min<uint64_t>(nq, nb);
    const uint64_t nch = std::max<uint64_t>((n + kWave - 1 + chunk - 1) / chunk, 1);
    return groups * nch;
}

constexpr uint64_t kMaxItemTable = 1ull << 26;  // entries (256 MiB) kept without an exact count

// Largest chunk: a queued pair packs its candidate's offset in the chunk
// (at most the chunk rounded up to whole tiles) above 6 bits of query lane,
// in 32 bits.
constexpr uint32_t kMaxChunk = 1u << 19;
static_assert((uint64_t)kMaxChunk + 2 * kTile < (1ull << 26), "packed queue entries");

uint32_t resolve_chunk(int prec, uint32_t chunk) {
    if (chunk) return std::min(std::max(chunk, 64u), kMaxChunk);
    return prec == TDS_PREC_FP64 ? 512u : 4096u;
}

// Default: 4 waves per SIMD on all 256 CUs (the occupancy the distance
// kernel's register use allows).
uint32_t resolve_grid(uint32_t grid_waves) {
    return std::min(grid_waves ? grid_waves : 256u * 4u * 4u, kMaxDistBlocks * kWavesPerBlock);
}

// Waves of a distance-kernel launch of grid_waves (whole workgroups).
uint32_t launch_blocks(uint32_t grid_waves) {
    return std::min(kMaxDistBlocks, std::max(1u, ceil_div(grid_waves, kWavesPerBlock)));
}

// Result stage of each wave: up to kStageMax records, within a workspace
// total of at most kStageTotal (the stages of one launch never exceed about
// 300 MB; at the default grid every wave gets kStageMax).
constexpr uint32_t kStageMax = 2048;
constexpr size_t kStageTotal = size_t(1) << 23;

size_t stage_total(uint32_t grid_waves) {
    const size_t waves = (size_t)launch_blocks(grid_waves) * kWavesPerBlock;
    return std::min(kStageTotal, waves * kStageMax);
}

uint32_t stage_per_wave(size_t recs, uint32_t blocks) {
    const size_t per = recs / ((size_t)blocks * kWavesPerBlock);
    return (uint32_t)std::min<size_t>(kStageMax, per / kWave * kWave);
}

// Kernel variant and dealing of a launch, packed: candidates per lane per
// tile of the FP32 form (0 selects 4; 2 and 4 are built) in the low byte,
// the place of the closest-approach refinement (TDS_REFINE_*, 0 selects the
// queue stage) in the next, the dealing of the work items (TDS_DEAL_*, 0
// selects the dynamic tail) above; 0 if any of them is unknown.
uint32_t resolve_tile(uint32_t t, uint32_t refine = 0, uint32_t deal = 0) {
    if (t == 0) t = 4;
    if (t != 2 && t != 4) return 0;
    if (refine == TDS_REFINE_DEFAULT) refine = TDS_REFINE_QUEUED;
    if (refine != TDS_REFINE_QUEUED && refine != TDS_REFINE_INLINE) return 0;
    if (deal == TDS_DEAL_DEFAULT) deal = TDS_DEAL_DYNAMIC;
    if (deal != TDS_DEAL_DYNAMIC && deal != TDS_DEAL_STATIC) return 0;
    return t | (refine << 8) | (deal << 16);
}

int resolve_prec(int p) {
    if (p == TDS_PREC_DEFAULT) return TDS_PREC_FP32_RECHECK;
    if (p != TDS_PREC_FP64 && p != TDS_PREC_FP32_RECHECK) return -1;
    return p;
}

// Device view of the query arrays; host arrays are copied into the staging
// buffers first.
int stage_queries(const tds_segments* Q, QueryView* V, hipStream_t s, double** stage_buf,
                  size_t* stage_cap, uint32_t** traj_buf, size_t* traj_cap, bool force_copy) {
    V->n = Q->n;
    const double* src[8] = {Q->xs, Q->ys, Q->zs, Q->ts, Q->xe, Q->ye, Q->ze, Q->te};
    if (Q->on_device && !force_copy) {
        for (int k = 0; k < 8; ++k) V->a[k] = src[k];
        V->traj = Q->traj_id;
        return TDS_OK;
    }
    const hipMemcpyKind kind = Q->on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
    TDS_TRY(grow(stage_buf, stage_cap, 8 * (size_t)Q->n));
    for (int k = 0; k < 8; ++k) {
        TDS_HIP(hipMemcpyAsync(*stage_buf + k * Q->n, src[k], Q->n * sizeof(double), kind, s));
        V->a[k] = *stage_buf + k * Q->n;
    }
    V->traj = nullptr;
    if (Q->traj_id) {
        TDS_TRY(grow(traj_buf, traj_cap, (size_t)Q->n));
        TDS_HIP(hipMemcpyAsync(*traj_buf, Q->traj_id, Q->n * sizeof(uint32_t), kind, s));
        V->traj = *traj_buf;
    }
    return TDS_OK;
}

DistArgs dist_args(const tds_index* idx, const Workspace* w, const QueryView& Q, tds_result* out,
                   uint64_t win_lo, uint32_t item_begin, uint32_t item_end, uint32_t* item_count,
                   uint32_t grid_waves, bool by_order, uint32_t cpl, bool direct = false) {
    DistArgs A;
    A.cpl = cpl & 0xFFu;
    A.inline_refine = ((cpl >> 8) & 0xFFu) == TDS_REFINE_INLINE ? 1u : 0u;
    A.deal = cpl >> 16;
    A.dyn_ctr = w->dyn_ctr;
    A.stage = w->stage;
    A.stage_meta = w->stage_meta;
    A.stage_cap = stage_per_wave(w->stage_recs, launch_blocks(grid_waves));
    A.by_order = by_order ? 1u : 0u;
    A.I = view_of(idx);
    A.Q = Q;
    A.qreq = w->qreq;
    A.qsorted = w->qsorted;
    A.qf = w->qf;
    A.binfo = w->binfo;
    A.item_bucket = w->item_bucket;
    A.desc = w->desc;
    A.hdr = w->hdr;
    A.bstats = w->bstats;
    A.req = w->req;
    A.rc = w->req_ctr;
    A.out = out;
    A.win_lo = win_lo;
    A.item_begin = item_begin;
    A.item_end = item_end;
    A.item_count = item_count;
    // direct output: chunks of a wave's stage size, the stage buffer as the
    // scratch for positions past the capacity (W C records, within it)
    const uint32_t waves = launch_blocks(grid_waves) * kWavesPerBlock;
    A.direct = (direct && !by_order && win_lo == 0 && waves <= kMaxDirectWaves &&
                waves <= w->stage_waves && A.stage_cap >= (uint32_t)kWave)
                   ? 1u
                   : 0u;
    A.dir_chunk = A.stage_cap;
    A.dir_ctr = w->dyn_ctr + (size_t)kXcds * kCtrStride;
    A.dscratch = w->stage;
    A.dscratch_cap = (uint64_t)waves * A.stage_cap;
    A.dlast = w->dlast;
    return A;
}

// The distance kernel, timed by the two events when both are given, then the
// fold of its per-workgroup counters into the header.
int launch_distance(int prec, const DistArgs& A, uint32_t grid_waves, hipStream_t s,
                    hipEvent_t ev_begin, hipEvent_t ev_end) {
    const uint32_t blocks = launch_blocks(grid_waves);
    // every wave must be able to stage a full batch of 64 evaluations
    if (!A.stage || A.stage_cap < (uint32_t)kWave) return TDS_E_DEVICE;
    void (*kern)(DistArgs);
    if (A.inline_refine)
        kern = (A.cpl == 2) ? k_distance<TDS_PREC_FP32_RECHECK, 2, true>
                            : k_distance<TDS_PREC_FP32_RECHECK, 4, true>;
    else
        kern = (A.cpl == 2) ? k_distance<TDS_PREC_FP32_RECHECK, 2, false>
                            : k_distance<TDS_PREC_FP32_RECHECK, 4, false>;
    if (prec == TDS_PREC_FP64) kern = k_distance<TDS_PREC_FP64, 4, false>;
    if (ev_begin && ev_end) {
        // the events take the dispatch's own start and end times (no marker
        // packets around the kernel, so no bubbles before and after it)
        hipExtLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, s, ev_begin, ev_end, 0u, A);
    } else {
        hipLaunchKernelGGL(kern, dim3(blocks), dim3(kBlock), 0, s, A);
    }
    hipLaunchKernelGGL(k_stats_fold, dim3(1), dim3(256), 0, s, A.bstats, blocks, A.hdr);
    TDS_HIP(hipGetLastError());
    return TDS_OK;
}

// Direct output: the fill of the holes left by the waves' last reservations.
int launch_fill(const DistArgs& A, const Workspace* w, uint32_t grid_waves, hipStream_t s) {
    const uint32_t nw = launch_blocks(grid_waves) * kWavesPerBlock;
    hipLaunchKernelGGL(k_fill_plan, dim3(1), dim3(1024), 0, s, A.req, A.rc, A.dir_ctr, A.dlast,
                       nw, A.dir_chunk, w->fill_s, w->fill_d, w->fill_dstart, w->fill_plan);
    hipLaunchKernelGGL(k_fill_copy, dim3(1024), dim3(256), 0, s, w->fill_plan, w->fill_s,
                       w->fill_d, w->fill_dstart, nw, A.dir_chunk, A.req, A.out, A.dscratch);
    TDS_HIP(hipGetLastError());
    return TDS_OK;
}

// The whole search for the batch described by w->desc / w->req, as a fixed
// sequence of fixed-shape launches (capturable in a graph): clear, prepare
// queries, bucket table, ordering, item table, distance kernel over every
// item.  q_grid and r_cap are the capacities the launches are shaped for.
int enqueue_pipeline(const tds_index* idx, Workspace* w, const QueryView& Q, size_t q_grid,
                     uint32_t r_cap, int prec, uint32_t chunk, uint32_t grid_waves, uint32_t cpl,
                     tds_result* out, uint32_t* item_count, hipStream_t s, hipEvent_t ev_begin,
                     hipEvent_t ev_end, bool direct = false) {
    const IndexView I = view_of(idx);
    const uint32_t shift = bucket_shift(idx->m);
    const uint32_t nb = bucket_count(idx->m);
    const uint32_t nparts = count_parts(nb);
    const uint32_t zn = std::max(std::max(nb * nparts, r_cap), kCtrSlots * kCtrStride);
    // k_zero also clears the request counters the distance kernel appends with
    hipLaunchKernelGGL(k_zero, dim3(ceil_div(zn, kBlock)), dim3(kBlock), 0, s, w->hdr, w->b_count,
                       w->b_hi, nb, nparts, w->req_ctr, r_cap, w->dyn_ctr);
    const uint32_t qblocks = std::max(1u, ceil_div(q_grid, kBlock));
    const uint32_t bpp = ceil_div(qblocks, nparts);  // workgroup b counts in part b / bpp < nparts
    hipLaunchKernelGGL(k_qprep, dim3(qblocks), dim3(kBlock), 0, s, Q, w->desc, w->req, I, w->qfu,
                       w->qreq, w->qkey, w->qslot, w->b_count, w->b_hi, shift, nb, bpp, w->hdr);
    hipLaunchKernelGGL(k_bucket_scan, dim3(1), dim3(1024), 0, s, w->b_count, w->b_hi,
                       idx->bin_first, idx->min_te, idx->max_ts, idx->m, shift, nb, nparts, chunk,
                       w->b_start, w->b_nch, w->binfo, w->hdr);
    hipLaunchKernelGGL(k_scatter, dim3(qblocks + nb), dim3(kBlock), 0, s, w->desc, w->qkey,
                       w->qslot, w->b_start, w->b_count, nb, bpp, qblocks, w->qfu, w->qsorted,
                       w->qf, w->binfo, w->item_bucket, w->hdr);
    TDS_HIP(hipGetLastError());
    const DistArgs A = dist_args(idx, w, Q, out, 0, 0, 0xFFFFFFFFu, item_count, grid_waves, false,
                                 cpl, direct);
    TDS_TRY(launch_distance(prec, A, grid_waves, s, ev_begin, ev_end));
    return A.direct ? launch_fill(A, w, grid_waves, s) : TDS_OK;
}

// Re-runs the distance kernel over work items [i0, i1) keeping result
// positions [win_lo, win_lo + capacity) (incremental processing).
// by_order: one item of a one-request search, its results placed by their
// order in the item (a window of an item larger than the device buffer).
int enqueue_range(const tds_index* idx, Workspace* w, const QueryView& Q, int prec, uint32_t r_cap,
                  tds_result* out, uint64_t win_lo, uint32_t i0, uint32_t i1, bool by_order,
                  uint32_t grid_waves, uint32_t cpl, hipStream_t s, hipEvent_t ev_begin,
                  hipEvent_t ev_end) {
    hipLaunchKernelGGL(k_reset_pass, dim3(ceil_div(std::max(r_cap, kCtrSlots * kCtrStride), 256)),
                       dim3(256), 0, s, w->req_ctr, r_cap, w->dyn_ctr);
    TDS_HIP(hipGetLastError());
    return launch_distance(prec,
                           dist_args(idx, w, Q, out, win_lo, i0, i1, nullptr, grid_waves, by_order,
                                     cpl),
                           grid_waves, s, ev_begin, ev_end);
}

Workspace* acquire(tds_index* idx) {
    {
        std::lock_guard<std::mutex> g(idx->mu);
        if (!idx->pool.empty()) {
            Workspace* w = idx->pool.back();
            idx->pool.pop_back();
            return w;
        }
    }
    Workspace* w = new (std::nothrow) Workspace();
    if (!w) return nullptr;
    w->device = idx->device;
    if (ws_init(w) != TDS_OK) {
        delete w;
        return nullptr;
    }
    return w;
}

void release(tds_index* idx, Workspace* w) {
    std::lock_guard<std::mutex> g(idx->mu);
    idx->pool.push_back(w);
}

struct WsGuard {
    tds_index* idx;
    Workspace* w;
    ~WsGuard() {
        if (w) release(idx, w);
    }
};

bool valid_window(double d, double t0, double t1) {
    return d >= 0.0 && !std::isinf(d) && t0 < t1;
}

// Sizes the item table for the batch: from the bound when it is small enough,
// else from the exact count after the preparation launches (one extra sync).
int reserve_items(const tds_index* idx, Workspace* w, uint64_t nq, uint32_t chunk,
                  uint64_t* cap_out) {
    const uint64_t bound = item_bound(nq, bucket_count(idx->m), idx->n, chunk);
    const uint64_t cap = std::min<uint64_t>(bound, kMaxItemTable);
    TDS_TRY(grow(&w->item_bucket, &w->item_bucket_cap, std::max<size_t>(cap, 1)));
    TDS_TRY(grow(&w->item_count, &w->item_cap, std::max<size_t>(cap, 1)));
    *cap_out = cap;
    return TDS_OK;
}

// Runs the pipeline once for the batch whose requests the caller staged in
// w->req_host (sent to the device here, with the descriptor), growing the
// item table and re-running if the bound was too small.
// One run of the pipeline for the batch whose requests the caller staged in
// w->req_host with an item table of `cap` entries: the descriptor and the
// requests go up, the launches are ordered on `s`, and the header and request
// counters come back into pinned memory.  Returns without waiting.
int enqueue_attempt(const tds_index* idx, Workspace* w, const QueryView& V, uint32_t nreq,
                    int prec, uint32_t chunk, uint32_t grid_waves, uint32_t cpl, uint32_t output,
                    tds_result* out, hipStream_t s, uint64_t cap) {
    w->desc_host->nq = V.n;
    w->desc_host->nreq = nreq;
    w->desc_host->item_cap = (uint32_t)std::min<uint64_t>(cap, 0xFFFFFFFFull);
    TDS_TRY(ws_upload(w, nreq, s));
    // one request: direct output unless staging is asked for
    TDS_TRY(enqueue_pipeline(idx, w, V, V.n, nreq, prec, chunk, grid_waves, cpl, out,
                             w->item_count, s, w->ev0, w->ev1,
                             nreq == 1 && output != TDS_OUTPUT_STAGED));
    return ws_download(w, nreq, s);
}

// After an attempt has completed: its header and kernel time; returns TDS_OK,
// TDS_E_INVALID, or 1 when the item table was too small (it is then sized
// exactly for another attempt).
int finish_attempt(Workspace* w, tds_stats* st, SearchHeader* h_out, uint64_t* cap) {
    *h_out = *w->hdr_host;
    float ms = 0.f;
    TDS_HIP(hipEventElapsedTime(&ms, w->ev0, w->ev1));
    st->kernel_ms += ms;
    st->passes += 1;
    if (h_out->err & 1u) return TDS_E_INVALID;
    if (!(h_out->err & 2u)) return TDS_OK;
    *cap = h_out->n_items;
    TDS_TRY(grow(&w->item_bucket, &w->item_bucket_cap, std::max<size_t>(*cap, 1)));
    TDS_TRY(grow(&w->item_count, &w->item_cap, std::max<size_t>(*cap, 1)));
    return 1;
}

// Runs the pipeline once for the batch whose requests the caller staged in
// w->req_host (sent to the device here, with the descriptor), growing the
// item table and re-running if the bound was too small.
int run_batch(const tds_index* idx, Workspace* w, const QueryView& V, uint32_t nreq, int prec,
              uint32_t chunk, uint32_t grid_waves, uint32_t cpl, uint32_t output, tds_result* out,
              hipStream_t s, tds_stats* st, SearchHeader* h_out) {
    uint64_t cap = 0;
    TDS_TRY(reserve_items(idx, w, V.n, chunk, &cap));
    TDS_TRY(ws_reserve_stage(w, grid_waves));
    for (int attempt = 0; attempt < 2; ++attempt) {
        TDS_TRY(enqueue_attempt(idx, w, V, nreq, prec, chunk, grid_waves, cpl, output, out, s,
                                cap));
        TDS_HIP(hipStreamSynchronize(s));
        const int r = finish_attempt(w, st, h_out, &cap);
        if (r != 1) return r;
    }
    return TDS_E_DEVICE;
}

}  // namespace

int resolve_config(const tds_search_params* params, PipelineConfig* cfg) {
    tds_search_params P;
    tds_search_params_default(&P);
    if (params) P = *params;
    cfg->prec = resolve_prec(P.precision);
    if (cfg->prec < 0) return TDS_E_INVALID;
    cfg->chunk = resolve_chunk(cfg->prec, P.chunk);
    cfg->grid_waves = resolve_grid(P.grid_waves);
    cfg->cpl = resolve_tile(P.tile, P.refine, P.deal);
    if (!cfg->cpl) return TDS_E_INVALID;
    if (P.output > TDS_OUTPUT_STAGED) return TDS_E_INVALID;  // batches always stage
    return TDS_OK;
}

uint64_t item_table_bound(const tds_index* idx, uint64_t nq, uint32_t chunk) {
    return item_bound(nq, bucket_count(idx->m), idx->n, chunk);
}

int enqueue_search(const tds_index* idx, Workspace* w, const double* const* qarrays,
                   const uint32_t* qtraj, size_t q_grid, uint32_t r_cap,
                   const PipelineConfig& cfg, tds_result* out, hipStream_t s) {
    QueryView V{};
    for (int k = 0; k < 8; ++k) V.a[k] = qarrays[k];
    V.traj = qtraj;
    V.n = q_grid;
    return enqueue_pipeline(idx, w, V, q_grid, r_cap, cfg.prec, cfg.chunk, cfg.grid_waves,
                            cfg.cpl, out, w->item_count, s, nullptr, nullptr);
}

int schedule_impl(tds_index* idx, const tds_segments* Q, double t_start, double t_end,
                  uint32_t* lo, uint32_t* hi, hipStream_t s) {
    if (!idx || !lo || !hi) return TDS_E_INVALID;
    TDS_TRY(validate_segments_args(Q));
    if (!(t_start < t_end)) return TDS_E_INVALID;
    const uint64_t nq = Q->n;
    double* stage = nullptr;
    size_t scap = 0;
    uint32_t* tstage = nullptr;
    size_t tcap = 0;
    uint32_t *dlo = nullptr, *dhi = nullptr, *err = nullptr;
    int st = TDS_OK;
    QueryView V{};
    do {
        if ((st = stage_queries(Q, &V, s, &stage, &scap, &tstage, &tcap, false))) break;
        if ((st = dmalloc(&dlo, nq))) break;
        if ((st = dmalloc(&dhi, nq))) break;
        if ((st = dmalloc(&err, 1))) break;
        if (hipMemsetAsync(err, 0, sizeof(uint32_t), s) != hipSuccess) { st = TDS_E_DEVICE; break; }
        hipLaunchKernelGGL(k_schedule, dim3(ceil_div(nq, kBlock)), dim3(kBlock), 0, s, V, t_start,
                           t_end, view_of(idx), dlo, dhi, err);
        uint32_t herr = 0;
        if (hipGetLastError() != hipSuccess ||
            hipMemcpyAsync(lo, dlo, nq * sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(hi, dhi, nq * sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipMemcpyAsync(&herr, err, sizeof(uint32_t), hipMemcpyDeviceToHost, s) != hipSuccess ||
            hipStreamSynchronize(s) != hipSuccess) {
            st = TDS_E_DEVICE;
            break;
        }
        if (herr) st = TDS_E_INVALID;
    } while (0);
    dfree(stage);
    dfree(tstage);
    dfree(dlo);
    dfree(dhi);
    dfree(err);
    return st;
}

namespace {
int search_core(tds_index* idx, const tds_segments* Q, bool self_join, double d, double t_start,
                double t_end, tds_result* out, uint64_t capacity, uint64_t* n_out,
                const tds_search_params* params, hipStream_t s, tds_stats* stats);
}  // namespace

int search_impl(tds_index* idx, const tds_segments* Q, double d, double t_start, double t_end,
                tds_result* out, uint64_t capacity, uint64_t* n_out,
                const tds_search_params* params, hipStream_t s, tds_stats* stats) {
    if (!idx || !n_out) return TDS_E_INVALID;
    *n_out = 0;
    TDS_TRY(validate_segments_args(Q));
    return search_core(idx, Q, false, d, t_start, t_end, out, capacity, n_out, params, s, stats);
}

int self_join_impl(tds_index* idx, double d, double t_start, double t_end, tds_result* out,
                   uint64_t capacity, uint64_t* n_out, const tds_search_params* params,
                   hipStream_t s, tds_stats* stats) {
    if (!idx || !n_out) return TDS_E_INVALID;
    *n_out = 0;
    return search_core(idx, nullptr, true, d, t_start, t_end, out, capacity, n_out, params, s,
                       stats);
}

namespace {
int search_core(tds_index* idx, const tds_segments* Q, bool self_join, double d, double t_start,
                double t_end, tds_result* out, uint64_t capacity, uint64_t* n_out,
                const tds_search_params* params, hipStream_t s, tds_stats* stats) {
    const auto t_begin = std::chrono::steady_clock::now();
    if (!valid_window(d, t_start, t_end)) return TDS_E_INVALID;
    if (capacity > 0 && !out) return TDS_E_INVALID;
    tds_search_params P;
    tds_search_params_default(&P);
    if (params) P = *params;
    const int prec = resolve_prec(P.precision);
    if (prec < 0) return TDS_E_INVALID;
    const uint32_t chunk = resolve_chunk(prec, P.chunk);
    const uint32_t grid_waves = resolve_grid(P.grid_waves);
    const uint32_t cpl = resolve_tile(P.tile, P.refine, P.deal);
    if (!cpl) return TDS_E_INVALID;
    if (P.output > TDS_OUTPUT_STAGED) return TDS_E_INVALID;
    const bool dev_out = P.out_on_device != 0;

    Workspace* w = acquire(idx);
    if (!w) return TDS_E_NOMEM;
    WsGuard guard{idx, w};
    const uint64_t nq = self_join ? idx->n : Q->n;
    TDS_TRY(ws_reserve(w, nq, 1));
    QueryView V{};
    if (self_join) {
        V.n = nq;
        V.ent = idx->e64;
        V.ent_id = idx->seg_id;
        V.ent_traj = idx->traj;
    } else {
        TDS_TRY(stage_queries(Q, &V, s, &w->qstage, &w->stage_cap, &w->qtraj_stage, &w->traj_cap,
                              false));
    }

    // result buffer
    uint64_t dev_cap;
    tds_result* res;
    if (dev_out) {
        dev_cap = capacity;
        res = out;
    } else {
        dev_cap = P.device_capacity ? P.device_capacity
                                    : std::min<uint64_t>(std::max<uint64_t>(capacity, 1), kDefaultDevCap);
        TDS_TRY(grow(&w->res, &w->res_cap, (size_t)std::max<uint64_t>(dev_cap, 1)));
        res = w->res;
    }
    Request R{};
    R.q_begin = 0;
    R.q_count = nq;
    R.d = d;
    R.t_start = t_start;
    R.t_end = t_end;
    R.out_offset = 0;
    R.out_capacity = dev_cap;
    *w->req_host = R;  // uploaded with the descriptor

    tds_stats st{};
    st.query_segments = nq;
    SearchHeader h{};
    // pass 1: every item, result window [0, dev_cap)
    TDS_TRY(run_batch(idx, w, V, 1, prec, chunk, grid_waves, cpl, P.output, res, s, &st, &h));
    const ReqCounter rc = w->rc_host[0];
    const uint32_t n_items = h.n_items;
    st.active_segments = h.active;
    st.work_items = n_items;
    st.candidate_tests = h.tests;
    st.filter_tests = h.ftests;
    st.block_tests = h.btests;
    st.fp64_evals = h.evals;
    st.stage_flushes = h.flushes;
    const uint64_t total = rc.count;
    float ms = 0.f;
    int status = TDS_OK;
    if (dev_out) {
        status = (total > capacity) ? TDS_E_OVERFLOW : TDS_OK;
    } else if (total <= dev_cap) {
        const uint64_t k = std::min(total, capacity);
        if (k) TDS_HIP(hipMemcpyAsync(out, res, k * sizeof(tds_result), hipMemcpyDeviceToHost, s));
        TDS_HIP(hipStreamSynchronize(s));
        status = (total > capacity) ? TDS_E_OVERFLOW : TDS_OK;
    } else if (total > capacity) {
        const uint64_t k = std::min(dev_cap, capacity);
        if (k) TDS_HIP(hipMemcpyAsync(out, res, k * sizeof(tds_result), hipMemcpyDeviceToHost, s));
        TDS_HIP(hipStreamSynchronize(s));
        status = TDS_E_OVERFLOW;
    } else {
        // incremental processing: re-run consecutive work items whose results
        // fit the device buffer; an item larger than the buffer is re-run
        // alone with a sliding window (one wave processes an item, in a fixed
        // order, so its result order is the same on every run)
        std::vector<uint32_t> cnt(n_items);
        TDS_HIP(hipMemcpyAsync(cnt.data(), w->item_count, n_items * sizeof(uint32_t),
                               hipMemcpyDeviceToHost, s));
        TDS_HIP(hipStreamSynchronize(s));
        uint64_t written = 0;
        uint32_t i0 = 0;
        while (i0 < n_items) {
            uint32_t i1 = i0;
            uint64_t sum = 0;
            while (i1 < n_items && sum + cnt[i1] <= dev_cap) sum += cnt[i1++];
            std::vector<std::pair<uint64_t, uint64_t>> windows;  // (win_lo, expected)
            const bool by_order = i1 == i0;  // one item larger than the buffer
            if (i1 == i0) {
                i1 = i0 + 1;
                for (uint64_t wl = 0; wl < cnt[i0]; wl += dev_cap)
                    windows.push_back({wl, std::min<uint64_t>(dev_cap, cnt[i0] - wl)});
            } else {
                windows.push_back({0, sum});
            }
            for (auto& win : windows) {
                if (win.second == 0) continue;
                TDS_TRY(enqueue_range(idx, w, V, prec, 1, res, win.first, i0, i1, by_order,
                                      std::min(grid_waves, i1 - i0), cpl, s, w->ev0, w->ev1));
                TDS_HIP(hipMemcpyAsync(out + written, res, win.second * sizeof(tds_result),
                                       hipMemcpyDeviceToHost, s));
                TDS_HIP(hipStreamSynchronize(s));
                TDS_HIP(hipEventElapsedTime(&ms, w->ev0, w->ev1));
                st.kernel_ms += ms;
                st.passes += 1;
                written += win.second;
            }
            i0 = i1;
        }
        if (written != total) return TDS_E_DEVICE;
    }
    *n_out = total;
    st.results = total;
    st.total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
    if (stats) *stats = st;
    {
        std::lock_guard<std::mutex> g(idx->mu);
        idx->last = st;
    }
    return status;
}
}  // namespace

// A search begun on a stream and not yet ended (tds_search_begin): it holds
// its workspace until tds_search_end.
struct PendingSearch {
    tds_index* idx = nullptr;
    Workspace* w = nullptr;
    hipStream_t s = nullptr;
    QueryView V{};
    tds_result* out = nullptr;
    uint64_t capacity = 0, cap_items = 0;
    int prec = 0;
    uint32_t chunk = 0, grid_waves = 0, cpl = 0, output = 0;
    hipEvent_t done = nullptr;
    std::chrono::steady_clock::time_point t0;
};

int search_begin_impl(tds_index* idx, const tds_segments* Q, double d, double t_start,
                      double t_end, tds_result* out, uint64_t capacity,
                      const tds_search_params* params, hipStream_t s, void** pending) {
    const auto t_begin = std::chrono::steady_clock::now();
    if (!idx || !pending) return TDS_E_INVALID;
    *pending = nullptr;
    TDS_TRY(validate_segments_args(Q));
    if (!valid_window(d, t_start, t_end)) return TDS_E_INVALID;
    if (capacity > 0 && !out) return TDS_E_INVALID;
    tds_search_params P;
    tds_search_params_default(&P);
    if (params) P = *params;
    if (!P.out_on_device) return TDS_E_INVALID;  // the output is device memory
    const int prec = resolve_prec(P.precision);
    if (prec < 0) return TDS_E_INVALID;
    const uint32_t cpl = resolve_tile(P.tile, P.refine, P.deal);
    if (!cpl || P.output > TDS_OUTPUT_STAGED) return TDS_E_INVALID;
    PendingSearch* ps = new (std::nothrow) PendingSearch();
    if (!ps) return TDS_E_NOMEM;
    ps->idx = idx;
    ps->s = s;
    ps->out = out;
    ps->capacity = capacity;
    ps->prec = prec;
    ps->chunk = resolve_chunk(prec, P.chunk);
    ps->grid_waves = resolve_grid(P.grid_waves);
    ps->cpl = cpl;
    ps->output = P.output;
    ps->t0 = t_begin;
    int st = TDS_OK;
    do {
        if (!(ps->w = acquire(idx))) { st = TDS_E_NOMEM; break; }
        Workspace* w = ps->w;
        if ((st = ws_reserve(w, Q->n, 1))) break;
        if ((st = stage_queries(Q, &ps->V, s, &w->qstage, &w->stage_cap, &w->qtraj_stage,
                                &w->traj_cap, false)))
            break;
        Request R{};
        R.q_begin = 0;
        R.q_count = Q->n;
        R.d = d;
        R.t_start = t_start;
        R.t_end = t_end;
        R.out_offset = 0;
        R.out_capacity = capacity;
        *w->req_host = R;
        if ((st = reserve_items(idx, w, Q->n, ps->chunk, &ps->cap_items))) break;
        if ((st = ws_reserve_stage(w, ps->grid_waves))) break;
        if (hipEventCreateWithFlags(&ps->done, hipEventDisableTiming) != hipSuccess) {
            ps->done = nullptr;
            st = TDS_E_DEVICE;
            break;
        }
        if ((st = enqueue_attempt(idx, w, ps->V, 1, prec, ps->chunk, ps->grid_waves, cpl,
                                  ps->output, out, s, ps->cap_items)))
            break;
        if (hipEventRecord(ps->done, s) != hipSuccess) { st = TDS_E_DEVICE; break; }
    } while (0);
    if (st != TDS_OK) {
        if (ps->done) {
            (void)hipStreamSynchronize(s);  // nothing of it may still run
            (void)hipEventDestroy(ps->done);
        }
        if (ps->w) release(idx, ps->w);
        delete ps;
        return st;
    }
    *pending = ps;
    return TDS_OK;
}

int search_end_impl(void* pending, uint64_t* n_out, tds_stats* stats) {
    PendingSearch* ps = static_cast<PendingSearch*>(pending);
    if (!ps) return TDS_E_INVALID;
    Workspace* w = ps->w;
    tds_stats st{};
    st.query_segments = ps->V.n;
    SearchHeader h{};
    int status = TDS_OK;
    if (hipEventSynchronize(ps->done) != hipSuccess) {
        status = TDS_E_DEVICE;
    } else {
        int r = finish_attempt(w, &st, &h, &ps->cap_items);
        if (r == 1) {
            // the item table was too small: the search runs again, sized exactly
            r = enqueue_attempt(ps->idx, w, ps->V, 1, ps->prec, ps->chunk, ps->grid_waves,
                                ps->cpl, ps->output, ps->out, ps->s, ps->cap_items);
            if (r == TDS_OK)
                r = hipStreamSynchronize(ps->s) == hipSuccess
                        ? finish_attempt(w, &st, &h, &ps->cap_items)
                        : TDS_E_DEVICE;
            if (r == 1) r = TDS_E_DEVICE;
        }
        status = r;
    }
    if (status == TDS_OK) {
        const uint64_t total = w->rc_host[0].count;
        if (n_out) *n_out = total;
        st.active_segments = h.active;
        st.work_items = h.n_items;
        st.candidate_tests = h.tests;
        st.filter_tests = h.ftests;
        st.block_tests = h.btests;
        st.fp64_evals = h.evals;
        st.stage_flushes = h.flushes;
        st.results = total;
        st.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                ps->t0)
                          .count();
        if (stats) *stats = st;
        status = total > ps->capacity ? TDS_E_OVERFLOW : TDS_OK;
    }
    (void)hipEventDestroy(ps->done);
    release(ps->idx, w);
    delete ps;
    return status;
}

// Checks that the requests tile [0, nq) in order and their output slices fit.
int validate_requests(const tds_request* reqs, uint32_t nreq, uint64_t nq, uint64_t out_cap) {
    if (!reqs || nreq == 0) return TDS_E_INVALID;
    uint64_t next = 0;
    for (uint32_t r = 0; r < nreq; ++r) {
        const tds_request& q = reqs[r];
        if (q.q_begin != next || q.q_count == 0) return TDS_E_INVALID;
        next += q.q_count;
        if (!valid_window(q.d, q.t_start, q.t_end)) return TDS_E_INVALID;
        if (q.out_offset > out_cap || q.out_capacity > out_cap - q.out_offset) return TDS_E_INVALID;
    }
    return next == nq ? TDS_OK : TDS_E_INVALID;
}

int batch_impl(tds_index* idx, const tds_segments* Q, const tds_request* reqs, uint32_t nreq,
               tds_result* out, uint64_t out_capacity, uint64_t* counts,
               const tds_search_params* params, hipStream_t s, tds_stats* stats) {
    const auto t_begin = std::chrono::steady_clock::now();
    if (!idx || !counts || (out_capacity && !out)) return TDS_E_INVALID;
    TDS_TRY(validate_segments_args(Q));
    TDS_TRY(validate_requests(reqs, nreq, Q->n, out_capacity));
    tds_search_params P;
    tds_search_params_default(&P);
    if (params) P = *params;
    const int prec = resolve_prec(P.precision);
    if (prec < 0) return TDS_E_INVALID;
    const uint32_t chunk = resolve_chunk(prec, P.chunk);
    const uint32_t grid_waves = resolve_grid(P.grid_waves);
    const uint32_t cpl = resolve_tile(P.tile, P.refine, P.deal);
    if (!cpl) return TDS_E_INVALID;
    if (P.output > TDS_OUTPUT_STAGED) return TDS_E_INVALID;
    const bool dev_out = P.out_on_device != 0;

    Workspace* w = acquire(idx);
    if (!w) return TDS_E_NOMEM;
    WsGuard guard{idx, w};
    TDS_TRY(ws_reserve(w, Q->n, nreq));
    QueryView V{};
    TDS_TRY(stage_queries(Q, &V, s, &w->qstage, &w->stage_cap, &w->qtraj_stage, &w->traj_cap, false));
    tds_result* res = out;
    if (!dev_out) {
        TDS_TRY(grow(&w->res, &w->res_cap, (size_t)std::max<uint64_t>(out_capacity, 1)));
        res = w->res;
    }
    Request* R = w->req_host;
    for (uint32_t r = 0; r < nreq; ++r) {
        R[r].q_begin = reqs[r].q_begin;
        R[r].q_count = reqs[r].q_count;
        R[r].d = reqs[r].d;
        R[r].t_start = reqs[r].t_start;
        R[r].t_end = reqs[r].t_end;
        R[r].out_offset = reqs[r].out_offset;
        R[r].out_capacity = reqs[r].out_capacity;
        R[r].pad = 0;
    }
    tds_stats st{};
    st.query_segments = Q->n;
    SearchHeader h{};
    TDS_TRY(run_batch(idx, w, V, nreq, prec, chunk, grid_waves, cpl, P.output, res, s, &st,
                      &h));
    const ReqCounter* rc = w->rc_host;
    int status = TDS_OK;
    uint64_t total = 0;
    for (uint32_t r = 0; r < nreq; ++r) {
        counts[r] = rc[r].count;
        total += rc[r].count;
        if (rc[r].count > reqs[r].out_capacity) status = TDS_E_OVERFLOW;
        if (!dev_out) {
            const uint64_t k = std::min<uint64_t>(rc[r].count, reqs[r].out_capacity);
            if (k)
                TDS_HIP(hipMemcpyAsync(out + reqs[r].out_offset, res + reqs[r].out_offset,
                                       k * sizeof(tds_result), hipMemcpyDeviceToHost, s));
        }
    }
    if (!dev_out) TDS_HIP(hipStreamSynchronize(s));
    st.active_segments = h.active;
    st.work_items = h.n_items;
    st.candidate_tests = h.tests;
    st.filter_tests = h.ftests;
    st.block_tests = h.btests;
    st.fp64_evals = h.evals;
    st.stage_flushes = h.flushes;
    st.results = total;
    st.total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
    if (stats) *stats = st;
    {
        std::lock_guard<std::mutex> g(idx->mu);
        idx->last = st;
    }
    return status;
}

}  // namespace tds
