// Fixed spatial grid (FSG) index and search: the spatial method of Sec. 4.1
// (Alg. 1), built over the entries of a temporal index.
//
// Build: the entries' boxes (start and canonical end position, grown by a
// relative 1e-9) are reduced to the grid extent; each entry's cell range is
// counted, the counts scanned, and one (cell, entry position) listing written
// per overlapped cell; a radix sort by cell groups the listings, and a dense
// table gives each cell's first listing (cells are few enough, at most 2^24,
// for a dense table instead of the paper's searched array of non-empty cells).
//
// Search: one wave per query segment (persistent over the query set).  The
// wave walks the cells overlapped by the query's box grown by d (scalar
// loops); the lanes take the cell's listings 64 at a time, skip entries that
// do not overlap the query in time, and evaluate the rest with the canonical
// FP64 code.  A pair listed in several of the visited cells is reported only
// from the lowest cell of the intersection of the two cell ranges, so no
// duplicates are produced (the paper removed them on the host afterwards).
#include <algorithm>
#include <chrono>
#include <cmath>

#include <hip/hip_ext.h>

#include "canon.hpp"
#include "tds_internal.hpp"

namespace tds {

namespace {

constexpr int kFT = 256;

struct Grid {
    uint32_t g[3];
    double lo[3], cw[3];
};

// Bounding box of an entry: its start point and its canonical end position,
// grown by a relative 1e-9 (covers the rounding of every position the
// canonical evaluation forms along the segment).
__device__ inline void entry_box(const EntryF64& e, double* lo, double* hi) {
    const double dt = e.te - e.ts;
    const double p0[3] = {e.x, e.y, e.z};
    const double p1[3] = {e.x + e.vx * dt, e.y + e.vy * dt, e.z + e.vz * dt};
    for (int a = 0; a < 3; ++a) {
        const double l = dmin(p0[a], p1[a]), h = dmax(p0[a], p1[a]);
        const double m = 1e-9 * (fabs(l) + fabs(h) + 1.0);
        lo[a] = l - m;
        hi[a] = h + m;
    }
}

__device__ inline uint32_t cell_of(double v, double lo, double cw, uint32_t g) {
    if (!(cw > 0.0)) return 0u;
    const double u = floor((v - lo) / cw);
    if (!(u > 0.0)) return 0u;
    if (u >= (double)(g - 1)) return g - 1;
    return (uint32_t)u;
}

// Cell range of a box; a NaN bound (a position formed from an infinite
// velocity times zero) widens the range to the edge of the grid.
__device__ inline void cell_range(const Grid& G, const double* lo, const double* hi, uint32_t* c0,
                                  uint32_t* c1) {
    for (int a = 0; a < 3; ++a) {
        c0[a] = isnan(lo[a]) ? 0u : cell_of(lo[a], G.lo[a], G.cw[a], G.g[a]);
        c1[a] = isnan(hi[a]) ? G.g[a] - 1 : cell_of(hi[a], G.lo[a], G.cw[a], G.g[a]);
    }
}

// Per-block partial extents of the entry boxes (min lo, max hi per axis).
__global__ __launch_bounds__(kFT) void k_fsg_extent(const EntryF64* __restrict__ e64, uint32_t n,
                                                    double* __restrict__ part) {
    __shared__ double sp[6][kFT];
    const uint32_t i = blockIdx.x * kFT + threadIdx.x;
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    if (i < n) entry_box(e64[i], lo, hi);
    for (int a = 0; a < 3; ++a) {
        sp[a][threadIdx.x] = lo[a];
        sp[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (uint32_t off = kFT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off)
            for (int a = 0; a < 3; ++a) {
                sp[a][threadIdx.x] = fmin(sp[a][threadIdx.x], sp[a][threadIdx.x + off]);
                sp[3 + a][threadIdx.x] = fmax(sp[3 + a][threadIdx.x], sp[3 + a][threadIdx.x + off]);
            }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = sp[threadIdx.x][0];
}

// Number of cells each entry is listed in (kEmit false), or its listings
// written from its offset (kEmit true).
template <bool kEmit>
__global__ __launch_bounds__(kFT) void k_fsg_list(const EntryF64* __restrict__ e64, uint32_t n,
                                                  Grid G, uint32_t* __restrict__ cnt,
                                                  uint64_t* __restrict__ keys,
                                                  uint32_t* __restrict__ vals) {
    const uint32_t i = blockIdx.x * kFT + threadIdx.x;
    if (i >= n) return;
    double lo[3], hi[3];
    entry_box(e64[i], lo, hi);
    uint32_t c0[3], c1[3];
    cell_range(G, lo, hi, c0, c1);
    if (!kEmit) {
        cnt[i] = (c1[0] - c0[0] + 1) * (c1[1] - c0[1] + 1) * (c1[2] - c0[2] + 1);
        return;
    }
    uint32_t o = cnt[i];
    for (uint32_t z = c0[2]; z <= c1[2]; ++z)
        for (uint32_t y = c0[1]; y <= c1[1]; ++y)
            for (uint32_t x = c0[0]; x <= c1[0]; ++x) {
                keys[o] = ((uint64_t)z * G.g[1] + y) * G.g[0] + x;
                vals[o] = i;
                ++o;
            }
}

// first[c] = number of listings with a cell below c (c = 0..ncells): one
// thread per cell, a binary search of the sorted cell keys.
__global__ __launch_bounds__(kFT) void k_fsg_cell_first(const uint64_t* __restrict__ keys,
                                                        uint32_t nl, uint32_t ncells,
                                                        uint32_t* __restrict__ first) {
    const uint32_t c = blockIdx.x * kFT + threadIdx.x;
    if (c > ncells) return;
    uint32_t l = 0, h = nl;
    while (l < h) {
        const uint32_t mid = l + (h - l) / 2;
        if (keys[mid] < c) l = mid + 1;
        else h = mid;
    }
    first[c] = l;
}

struct FsgArgs {
    Grid G;
    const EntryF64* e64;
    const uint32_t* seg_id;
    const uint32_t* traj;
    const uint32_t* cell_first;
    const uint32_t* list;
    const double* q[8];  // xs, ys, zs, ts, xe, ye, ze, te (device)
    const uint32_t* qtraj;
    uint32_t nq;
    double d, t_start, t_end;
    tds_result* out;
    uint64_t capacity;
    unsigned long long* counters;  // [0] results, [1] listings compared, [2] invalid input
};

__device__ inline uint64_t lanemask_below() {
    const uint32_t lane = __lane_id();
    return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

__global__ __launch_bounds__(kFT) void k_fsg_search(FsgArgs A) {
    const uint32_t lane = __lane_id();
    const uint32_t wave = blockIdx.x * (kFT / kWave) + threadIdx.x / kWave;
    const uint32_t nwaves = gridDim.x * (kFT / kWave);
    unsigned long long tested = 0;
    for (uint32_t k = wave; k < A.nq; k += nwaves) {
        const double xs = A.q[0][k], ys = A.q[1][k], zs = A.q[2][k], ts = A.q[3][k];
        const double xe = A.q[4][k], ye = A.q[5][k], ze = A.q[6][k], te = A.q[7][k];
        if (!(isfinite(xs) && isfinite(ys) && isfinite(zs) && isfinite(ts) && isfinite(xe) &&
              isfinite(ye) && isfinite(ze) && isfinite(te) && te > ts)) {
            if (lane == 0) atomicAdd(&A.counters[2], 1ull);
            continue;
        }
        // the canonical query data (the same operations as every search form)
        const double dt = te - ts;
        QCanon q;
        q.x = xs;
        q.y = ys;
        q.z = zs;
        q.vx = (xe - xs) / dt;
        q.vy = (ye - ys) / dt;
        q.vz = (ze - zs) / dt;
        q.ts = ts;
        q.aq = dmax(ts, A.t_start);
        q.bq = dmin(te, A.t_end);
        q.d = A.d;
        if (!(q.aq < q.bq)) continue;
        const uint32_t qid = k;
        const uint32_t qt = A.qtraj ? A.qtraj[k] : 0u;
        // the query's box over its clipped extent, grown by d (+ rounding room)
        double lo[3], hi[3];
        {
            const double pa[3] = {q.x + q.vx * (q.aq - ts), q.y + q.vy * (q.aq - ts),
                                  q.z + q.vz * (q.aq - ts)};
            const double pb[3] = {q.x + q.vx * (q.bq - ts), q.y + q.vy * (q.bq - ts),
                                  q.z + q.vz * (q.bq - ts)};
            for (int a = 0; a < 3; ++a) {
                const double l = dmin(pa[a], pb[a]), h = dmax(pa[a], pb[a]);
                const double m = q.d + 1e-9 * (fabs(l) + fabs(h) + q.d + 1.0);
                lo[a] = l - m;
                hi[a] = h + m;
            }
        }
        uint32_t q0[3], q1[3];
        cell_range(A.G, lo, hi, q0, q1);
        for (uint32_t cz = q0[2]; cz <= q1[2]; ++cz)
            for (uint32_t cy = q0[1]; cy <= q1[1]; ++cy)
                for (uint32_t cx = q0[0]; cx <= q1[0]; ++cx) {
                    const uint32_t c = (cz * A.G.g[1] + cy) * A.G.g[0] + cx;
                    const uint32_t s = A.cell_first[c], e = A.cell_first[c + 1];
                    for (uint32_t i0 = s; i0 < e; i0 += kWave) {
                        const uint32_t i = i0 + lane;
                        bool hit = false;
                        double t_lo = 0.0, t_hi = 0.0;
                        uint32_t pos = 0;
                        if (i < e) {
                            ++tested;
                            pos = A.list[i];
                            const EntryF64 E = A.e64[pos];
                            if (E.ts < q.bq && E.te > q.aq) {
                                // report the pair only from the lowest cell of
                                // the intersection of the two cell ranges
                                double el[3], eh[3];
                                entry_box(E, el, eh);
                                uint32_t e0[3], e1[3];
                                cell_range(A.G, el, eh, e0, e1);
                                const bool first = max(q0[0], e0[0]) == cx &&
                                                   max(q0[1], e0[1]) == cy &&
                                                   max(q0[2], e0[2]) == cz;
                                hit = first && canon_eval<true>(q, E.x, E.y, E.z, E.vx, E.vy,
                                                                E.vz, E.ts, E.te, &t_lo, &t_hi);
                            }
                        }
                        const uint64_t hm = __ballot(hit);
                        if (!hm) continue;
                        unsigned long long base = 0;
                        if (lane == 0) base = atomicAdd(&A.counters[0], (unsigned long long)__popcll(hm));
                        base = __shfl(base, 0);
                        if (hit) {
                            const uint64_t p = base + (uint64_t)__popcll(hm & lanemask_below());
                            if (p < A.capacity) {
                                tds_result r;
                                r.q_seg = qid;
                                r.e_seg = A.seg_id[pos];
                                r.q_traj = qt;
                                r.e_traj = A.traj[pos];
                                r.t_lo = t_lo;
                                r.t_hi = t_hi;
                                A.out[p] = r;
                            }
                        }
                    }
                }
    }
    // listings compared, summed over the wave
    for (int off = kWave / 2; off > 0; off >>= 1) tested += __shfl_xor(tested, off);
    if (lane == 0 && tested) atomicAdd(&A.counters[1], tested);
}

struct Bufs {
    void* p[8] = {};
    ~Bufs() {
        for (void* q : p) dfree(q);
    }
};

}  // namespace

int fsg_build(const tds_index* idx, uint32_t gx, uint32_t gy, uint32_t gz, hipStream_t s,
              tds_fsg** out) {
    if (!idx || !out) return TDS_E_INVALID;
    *out = nullptr;
    const uint32_t g[3] = {gx ? gx : 50u, gy ? gy : 50u, gz ? gz : 50u};
    for (uint32_t v : g)
        if (v > 1024) return TDS_E_INVALID;
    const uint64_t ncells = (uint64_t)g[0] * g[1] * g[2];
    if (ncells > (1ull << 24)) return TDS_E_INVALID;
    const uint32_t n = (uint32_t)idx->n;
    const uint32_t nb = ceil_div(n, kFT);
    Bufs B;
    double* part = nullptr;
    TDS_TRY(dmalloc(&part, 6 * (size_t)nb));
    B.p[0] = part;
    hipLaunchKernelGGL(k_fsg_extent, dim3(nb), dim3(kFT), 0, s, idx->e64, n, part);
    TDS_HIP(hipGetLastError());
    std::vector<double> hp(6 * (size_t)nb);
    TDS_HIP(hipMemcpyAsync(hp.data(), part, hp.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    TDS_HIP(hipStreamSynchronize(s));
    Grid G;
    for (int a = 0; a < 3; ++a) {
        double lo = INFINITY, hi = -INFINITY;
        for (uint32_t b = 0; b < nb; ++b) {
            lo = std::fmin(lo, hp[6 * b + a]);
            hi = std::fmax(hi, hp[6 * b + 3 + a]);
        }
        G.g[a] = g[a];
        G.lo[a] = lo;
        const double w = (hi - lo) / (double)g[a];
        G.cw[a] = (std::isfinite(w) && w > 0.0) ? w : 0.0;
    }
    uint32_t* cnt = nullptr;
    TDS_TRY(dmalloc(&cnt, n));
    B.p[1] = cnt;
    hipLaunchKernelGGL(k_fsg_list<false>, dim3(nb), dim3(kFT), 0, s, idx->e64, n, G, cnt, nullptr,
                       nullptr);
    TDS_HIP(hipGetLastError());
    // the listing total must fit 32 bits: check with a 64-bit host sum
    {
        std::vector<uint32_t> hc(n);
        TDS_HIP(hipMemcpyAsync(hc.data(), cnt, n * sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        TDS_HIP(hipStreamSynchronize(s));
        uint64_t tot = 0;
        for (uint32_t c : hc) tot += c;
        if (tot >= 0xFFFFFFFFull) return TDS_E_NOMEM;
    }
    uint32_t nl = 0;
    TDS_TRY(exclusive_scan_u32(cnt, n, &nl, s));
    uint64_t *keys = nullptr, *keys2 = nullptr;
    uint32_t *vals = nullptr, *vals2 = nullptr;
    TDS_TRY(dmalloc(&keys, std::max<uint32_t>(nl, 1)));
    B.p[2] = keys;
    TDS_TRY(dmalloc(&keys2, std::max<uint32_t>(nl, 1)));
    B.p[3] = keys2;
    TDS_TRY(dmalloc(&vals2, std::max<uint32_t>(nl, 1)));
    B.p[4] = vals2;
    TDS_TRY(dmalloc(&vals, std::max<uint32_t>(nl, 1)));  // becomes the grid's list
    hipLaunchKernelGGL(k_fsg_list<true>, dim3(nb), dim3(kFT), 0, s, idx->e64, n, G, cnt, keys, vals);
    int bits = 1;
    while ((1ull << bits) < ncells) ++bits;
    int st = radix_sort_u64(keys, vals, keys2, vals2, nl, bits, s);
    uint32_t* first = nullptr;
    if (st == TDS_OK) st = dmalloc(&first, ncells + 1);
    if (st == TDS_OK) {
        hipLaunchKernelGGL(k_fsg_cell_first, dim3(ceil_div(ncells + 1, kFT)), dim3(kFT), 0, s, keys,
                           nl, (uint32_t)ncells, first);
        if (hipGetLastError() != hipSuccess || hipStreamSynchronize(s) != hipSuccess)
            st = TDS_E_DEVICE;
    }
    tds_fsg* f = (st == TDS_OK) ? new (std::nothrow) tds_fsg() : nullptr;
    if (!f) {
        dfree(vals);
        dfree(first);
        return st == TDS_OK ? TDS_E_NOMEM : st;
    }
    f->idx = idx;
    f->device = idx->device;
    for (int a = 0; a < 3; ++a) {
        f->g[a] = G.g[a];
        f->lo[a] = G.lo[a];
        f->cw[a] = G.cw[a];
    }
    f->cell_first = first;
    f->list = vals;
    f->nlist = nl;
    *out = f;
    return TDS_OK;
}

void fsg_destroy(tds_fsg* f) {
    if (!f) return;
    dfree(f->cell_first);
    dfree(f->list);
    delete f;
}

int fsg_search(const tds_fsg* f, const tds_segments* Q, double d, double t_start, double t_end,
               tds_result* out, uint64_t capacity, uint64_t* n_out, const tds_search_params* params,
               hipStream_t s, tds_stats* stats) {
    const auto t_begin = std::chrono::steady_clock::now();
    if (!f || !n_out) return TDS_E_INVALID;
    *n_out = 0;
    TDS_TRY(validate_segments_args(Q));
    if (!(d >= 0.0) || std::isinf(d) || !(t_start < t_end)) return TDS_E_INVALID;
    if (capacity > 0 && !out) return TDS_E_INVALID;
    tds_search_params P;
    tds_search_params_default(&P);
    if (params) P = *params;
    const bool dev_out = P.out_on_device != 0;
    const uint64_t nq = Q->n;
    Bufs B;
    FsgArgs A{};
    A.G.g[0] = f->g[0];
    A.G.g[1] = f->g[1];
    A.G.g[2] = f->g[2];
    for (int a = 0; a < 3; ++a) {
        A.G.lo[a] = f->lo[a];
        A.G.cw[a] = f->cw[a];
    }
    A.e64 = f->idx->e64;
    A.seg_id = f->idx->seg_id;
    A.traj = f->idx->traj;
    A.cell_first = f->cell_first;
    A.list = f->list;
    const double* src[8] = {Q->xs, Q->ys, Q->zs, Q->ts, Q->xe, Q->ye, Q->ze, Q->te};
    if (Q->on_device) {
        for (int k = 0; k < 8; ++k) A.q[k] = src[k];
        A.qtraj = Q->traj_id;
    } else {
        double* stage = nullptr;
        TDS_TRY(dmalloc(&stage, 8 * nq));
        B.p[0] = stage;
        for (int k = 0; k < 8; ++k) {
            TDS_HIP(hipMemcpyAsync(stage + k * nq, src[k], nq * sizeof(double),
                                   hipMemcpyHostToDevice, s));
            A.q[k] = stage + k * nq;
        }
        A.qtraj = nullptr;
        if (Q->traj_id) {
            uint32_t* tr = nullptr;
            TDS_TRY(dmalloc(&tr, nq));
            B.p[1] = tr;
            TDS_HIP(hipMemcpyAsync(tr, Q->traj_id, nq * sizeof(uint32_t), hipMemcpyHostToDevice, s));
            A.qtraj = tr;
        }
    }
    A.nq = (uint32_t)nq;
    A.d = d;
    A.t_start = t_start;
    A.t_end = t_end;
    A.capacity = capacity;
    if (dev_out) {
        A.out = out;
    } else {
        tds_result* res = nullptr;
        TDS_TRY(dmalloc(&res, std::max<uint64_t>(capacity, 1)));
        B.p[2] = res;
        A.out = res;
    }
    unsigned long long* ctr = nullptr;
    TDS_TRY(dmalloc(&ctr, 4));
    B.p[3] = ctr;
    A.counters = ctr;
    TDS_HIP(hipMemsetAsync(ctr, 0, 4 * sizeof(unsigned long long), s));
    hipEvent_t e0 = nullptr, e1 = nullptr;
    TDS_HIP(hipEventCreate(&e0));
    TDS_HIP(hipEventCreate(&e1));
    const uint32_t blocks = std::max(1u, std::min(ceil_div(nq, kFT / kWave), 4096u));
    hipExtLaunchKernelGGL(k_fsg_search, dim3(blocks), dim3(kFT), 0, s, e0, e1, 0u, A);
    unsigned long long h[4] = {0, 0, 0, 0};
    int st = (hipGetLastError() == hipSuccess) ? TDS_OK : TDS_E_DEVICE;
    if (st == TDS_OK &&
        hipMemcpyAsync(h, ctr, sizeof(h), hipMemcpyDeviceToHost, s) != hipSuccess)
        st = TDS_E_DEVICE;
    if (st == TDS_OK && hipStreamSynchronize(s) != hipSuccess) st = TDS_E_DEVICE;
    float ms = 0.f;
    if (st == TDS_OK) (void)hipEventElapsedTime(&ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    TDS_TRY(st);
    if (h[2]) return TDS_E_INVALID;
    *n_out = h[0];
    if (!dev_out) {
        const uint64_t k = std::min<uint64_t>(h[0], capacity);
        if (k) {
            TDS_HIP(hipMemcpyAsync(out, A.out, k * sizeof(tds_result), hipMemcpyDeviceToHost, s));
            TDS_HIP(hipStreamSynchronize(s));
        }
    }
    if (stats) {
        tds_stats st2{};
        st2.query_segments = nq;
        st2.candidate_tests = h[1];
        st2.filter_tests = h[1];
        st2.results = h[0];
        st2.passes = 1;
        st2.kernel_ms = ms;
        st2.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                 t_begin)
                           .count();
        *stats = st2;
    }
    return h[0] > capacity ? TDS_E_OVERFLOW : TDS_OK;
}

}  // namespace tds
