// Index build on the GPU: the temporal index of Sec. 4.2.1.
//
//   k_seg_prep    validate every segment, compute its velocity (IEEE FP64
//                 division), its FP32 bounding-sphere record, its sort key
//                 (order-preserving bits of t_start) and per-block partial
//                 min t_start / max t_end / sum of durations;
//   radix sort    stable, by t_start (radix_sort.hip);
//   k_gather      write the sorted AoS records, ids and trajectory ids;
//   k_bin_first   first sorted position of every bin (boundary detection);
//   k_bin_stats   per-bin data extents (min t_start, max t_end);
//   k_bin_cummax  running maximum of max t_end over bins, which makes the
//                 bins overlapping a query one contiguous, bisectable span.
#include <cmath>
#include <utility>

#include "tds_internal.hpp"

namespace tds {

namespace {

constexpr int kBT = 256;

__device__ inline uint64_t order_key(double t) {
    // order-preserving map of a finite double to u64 (-0 and +0 are equal)
    uint64_t u = (t == 0.0) ? 0ull : (uint64_t)__double_as_longlong(t);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ inline bool finite(double v) { return isfinite(v); }

__global__ __launch_bounds__(kBT) void k_seg_prep(SegView S, EntryF64* __restrict__ tmp64,
                                                  EntryF32* __restrict__ tmp32,
                                                  uint64_t* __restrict__ keys,
                                                  uint32_t* __restrict__ vals,
                                                  double* __restrict__ part, uint32_t* err) {
    __shared__ double smin[kBT], smax[kBT], ssum[kBT];
    const uint32_t tid = threadIdx.x;
    const uint64_t i = (uint64_t)blockIdx.x * kBT + tid;
    double lmin = INFINITY, lmax = -INFINITY, lsum = 0.0;
    if (i < S.n) {
        double xs = S.a[0][i], ys = S.a[1][i], zs = S.a[2][i], ts = S.a[3][i];
        double xe = S.a[4][i], ye = S.a[5][i], ze = S.a[6][i], te = S.a[7][i];
        bool ok = finite(xs) && finite(ys) && finite(zs) && finite(ts) && finite(xe) &&
                  finite(ye) && finite(ze) && finite(te) && te > ts;
        if (!ok) {
            atomicOr(err, 1u);
            ts = 0.0;
            te = 1.0;
        }
        double dt = te - ts;
        EntryF64 e;
        e.x = xs;
        e.y = ys;
        e.z = zs;
        e.vx = (xe - xs) / dt;
        e.vy = (ye - ys) / dt;
        e.vz = (ze - zs) / dt;
        e.ts = ts;
        e.te = te;
        tmp64[i] = e;
        EntryF32 f;
        sphere32(xs, ys, zs, xe, ye, ze, 0.0, f.cx, f.cy, f.cz, f.r);
        f.ts = __double2float_rd(ts);
        f.te = __double2float_ru(te);
        f.pad0 = 0.f;
        f.pad1 = 0.f;
        tmp32[i] = f;
        keys[i] = order_key(ts);
        vals[i] = (uint32_t)i;
        lmin = ts;
        lmax = te;
        lsum = dt;
    }
    smin[tid] = lmin;
    smax[tid] = lmax;
    ssum[tid] = lsum;
    __syncthreads();
    for (uint32_t off = kBT / 2; off > 0; off >>= 1) {
        if (tid < off) {
            smin[tid] = fmin(smin[tid], smin[tid + off]);
            smax[tid] = fmax(smax[tid], smax[tid + off]);
            ssum[tid] = ssum[tid] + ssum[tid + off];
        }
        __syncthreads();
    }
    if (tid == 0) {
        part[3 * blockIdx.x + 0] = smin[0];
        part[3 * blockIdx.x + 1] = smax[0];
        part[3 * blockIdx.x + 2] = ssum[0];
    }
}

// Bin of a t_start: floor((ts - t_min) / b) clamped to [0, m-1].
__device__ inline uint32_t bin_of(double ts, double tmin, double bw, uint32_t m) {
    double u = floor((ts - tmin) / bw);
    if (!(u > 0.0)) return 0u;
    if (u >= (double)(m - 1)) return m - 1;
    return (uint32_t)u;
}

__global__ __launch_bounds__(kBT) void k_gather(uint64_t n, const uint32_t* __restrict__ perm,
                                                const EntryF64* __restrict__ tmp64,
                                                const EntryF32* __restrict__ tmp32,
                                                const uint32_t* __restrict__ traj_in,
                                                EntryF64* __restrict__ e64,
                                                EntryF32* __restrict__ e32,
                                                uint32_t* __restrict__ seg_id,
                                                uint32_t* __restrict__ traj) {
    const uint64_t i = (uint64_t)blockIdx.x * kBT + threadIdx.x;
    if (i >= n) return;
    const uint32_t src = perm[i];
    e64[i] = tmp64[src];
    e32[i] = tmp32[src];
    seg_id[i] = src;
    traj[i] = traj_in ? traj_in[src] : 0u;
}

__global__ __launch_bounds__(kBT) void k_bin_first(uint64_t n, const EntryF64* __restrict__ e64,
                                                   double tmin, double bw, uint32_t m,
                                                   uint32_t* __restrict__ bin_first) {
    const uint64_t i = (uint64_t)blockIdx.x * kBT + threadIdx.x;
    if (i >= n) return;
    const uint32_t j = bin_of(e64[i].ts, tmin, bw, m);
    const int64_t jp = (i == 0) ? -1 : (int64_t)bin_of(e64[i - 1].ts, tmin, bw, m);
    for (int64_t k = jp + 1; k <= (int64_t)j; ++k) bin_first[k] = (uint32_t)i;
    if (i == n - 1)
        for (uint32_t k = j + 1; k <= m; ++k) bin_first[k] = (uint32_t)n;
}

__global__ __launch_bounds__(kBT) void k_bin_stats(uint64_t n, const EntryF64* __restrict__ e64,
                                                   const uint32_t* __restrict__ bin_first,
                                                   double* __restrict__ min_ts,
                                                   double* __restrict__ max_te,
                                                   double* __restrict__ min_te,
                                                   double* __restrict__ lo_ts) {
    __shared__ double smax[kBT], smin[kBT];
    const uint32_t j = blockIdx.x;
    const uint32_t f = bin_first[j], e = bin_first[j + 1];
    double mx = -INFINITY, mn = INFINITY;
    for (uint32_t i = f + threadIdx.x; i < e; i += kBT) {
        mx = fmax(mx, e64[i].te);
        mn = fmin(mn, e64[i].te);
    }
    smax[threadIdx.x] = mx;
    smin[threadIdx.x] = mn;
    __syncthreads();
    for (uint32_t off = kBT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        min_ts[j] = (f < e) ? e64[f].ts : INFINITY;
        max_te[j] = smax[0];
        min_te[j] = smin[0];
        lo_ts[j] = (f < n) ? e64[f].ts : INFINITY;
    }
}

// Running maximum over m values with one block of 1024 threads.
__global__ __launch_bounds__(1024) void k_bin_cummax(const double* __restrict__ v,
                                                     double* __restrict__ out, uint32_t len) {
    __shared__ double part[1024];
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (len + 1023) / 1024;
    const uint32_t b = tid * per, e = min(len, b + per);
    double mx = -INFINITY;
    for (uint32_t i = b; i < e; ++i) mx = fmax(mx, v[i]);
    part[tid] = mx;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        double t = (tid >= off) ? part[tid - off] : -INFINITY;
        __syncthreads();
        part[tid] = fmax(part[tid], t);
        __syncthreads();
    }
    double run = (tid > 0) ? part[tid - 1] : -INFINITY;
    for (uint32_t i = b; i < e; ++i) {
        run = fmax(run, v[i]);
        out[i] = run;
    }
}

struct Scratch {
    void* p[12] = {};
    ~Scratch() {
        for (void* q : p) dfree(q);
    }
};

}  // namespace

int validate_segments_args(const tds_segments* S) {
    if (!S) return TDS_E_INVALID;
    if (S->n == 0 || S->n >= 0xFFFFFFFFull) return TDS_E_INVALID;
    if (!S->xs || !S->ys || !S->zs || !S->ts || !S->xe || !S->ye || !S->ze || !S->te)
        return TDS_E_INVALID;
    return TDS_OK;
}

void destroy_index(tds_index* idx) {
    if (!idx) return;
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(idx->device);
    for (Workspace* w : idx->pool) delete w;
    idx->pool.clear();
    dfree(idx->e64);
    dfree(idx->e32);
    dfree(idx->seg_id);
    dfree(idx->traj);
    dfree(idx->bin_first);
    dfree(idx->min_ts);
    dfree(idx->max_te);
    dfree(idx->min_te);
    dfree(idx->cmax_te);
    dfree(idx->lo_ts);
    (void)hipSetDevice(cur);
    delete idx;
}

int build_impl(const tds_segments* D, const tds_build_params* p, hipStream_t stream,
               tds_index** out) {
    if (!out) return TDS_E_INVALID;
    *out = nullptr;
    TDS_TRY(validate_segments_args(D));
    const uint64_t n = D->n;
    const uint32_t req_bins = p ? p->num_bins : 0u;
    if (req_bins > kMaxBins) return TDS_E_INVALID;

    int dev = 0;
    TDS_HIP(hipGetDevice(&dev));
    Scratch sc;
    // ---- stage the input on the device
    SegView S{};
    S.n = n;
    const double* src[8] = {D->xs, D->ys, D->zs, D->ts, D->xe, D->ye, D->ze, D->te};
    if (D->on_device) {
        for (int k = 0; k < 8; ++k) S.a[k] = src[k];
        S.traj = D->traj_id;
    } else {
        double* stage = nullptr;
        TDS_TRY(dmalloc(&stage, 8 * n));
        sc.p[0] = stage;
        for (int k = 0; k < 8; ++k) {
            TDS_HIP(hipMemcpyAsync(stage + k * n, src[k], n * sizeof(double), hipMemcpyHostToDevice,
                                   stream));
            S.a[k] = stage + k * n;
        }
        S.traj = nullptr;
        if (D->traj_id) {
            uint32_t* tr = nullptr;
            TDS_TRY(dmalloc(&tr, n));
            sc.p[1] = tr;
            TDS_HIP(hipMemcpyAsync(tr, D->traj_id, n * sizeof(uint32_t), hipMemcpyHostToDevice,
                                   stream));
            S.traj = tr;
        }
    }
    // ---- per-segment preparation
    const uint32_t nb = ceil_div(n, kBT);
    EntryF64* tmp64 = nullptr;
    EntryF32* tmp32 = nullptr;
    uint64_t *keys = nullptr, *keys2 = nullptr;
    uint32_t *vals = nullptr, *vals2 = nullptr, *err = nullptr;
    double* part = nullptr;
    TDS_TRY(dmalloc(&tmp64, n));
    sc.p[2] = tmp64;
    TDS_TRY(dmalloc(&tmp32, n));
    sc.p[3] = tmp32;
    TDS_TRY(dmalloc(&keys, n));
    sc.p[4] = keys;
    TDS_TRY(dmalloc(&keys2, n));
    sc.p[5] = keys2;
    TDS_TRY(dmalloc(&vals, n));
    sc.p[6] = vals;
    TDS_TRY(dmalloc(&vals2, n));
    sc.p[7] = vals2;
    TDS_TRY(dmalloc(&part, 3 * (size_t)nb));
    sc.p[8] = part;
    TDS_TRY(dmalloc(&err, 1));
    sc.p[9] = err;
    TDS_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), stream));
    hipLaunchKernelGGL(k_seg_prep, dim3(nb), dim3(kBT), 0, stream, S, tmp64, tmp32, keys, vals,
                       part, err);
    TDS_HIP(hipGetLastError());
    std::vector<double> hpart(3 * (size_t)nb);
    uint32_t herr = 0;
    TDS_HIP(hipMemcpyAsync(hpart.data(), part, hpart.size() * sizeof(double), hipMemcpyDeviceToHost,
                           stream));
    TDS_HIP(hipMemcpyAsync(&herr, err, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    TDS_HIP(hipStreamSynchronize(stream));
    if (herr) return TDS_E_INVALID;
    double tmin = INFINITY, tmax = -INFINITY, dsum = 0.0;
    for (uint32_t b = 0; b < nb; ++b) {
        tmin = std::fmin(tmin, hpart[3 * b]);
        tmax = std::fmax(tmax, hpart[3 * b + 1]);
        dsum += hpart[3 * b + 2];
    }
    uint32_t m = req_bins;
    if (m == 0) {
        const double mean = dsum / (double)n;
        double mm = std::nearbyint((tmax - tmin) / mean);
        if (!(mm >= 1.0)) mm = 1.0;
        if (mm > (double)kMaxBins) mm = (double)kMaxBins;
        m = (uint32_t)mm;
    }
    const double bw = (tmax - tmin) / (double)m;

    // ---- sort by t_start
    TDS_TRY(radix_sort_u64(keys, vals, keys2, vals2, (uint32_t)n, 64, stream));

    // ---- the index object
    tds_index* idx = new (std::nothrow) tds_index();
    if (!idx) return TDS_E_NOMEM;
    idx->device = dev;
    idx->n = n;
    idx->m = m;
    idx->t_min = tmin;
    idx->t_max = tmax;
    idx->bw = bw;
    int st = TDS_OK;
    do {
        if ((st = dmalloc(&idx->e64, n))) break;
        if ((st = dmalloc(&idx->e32, n))) break;
        if ((st = dmalloc(&idx->seg_id, n))) break;
        if ((st = dmalloc(&idx->traj, n))) break;
        if ((st = dmalloc(&idx->bin_first, (size_t)m + 1))) break;
        if ((st = dmalloc(&idx->min_ts, m))) break;
        if ((st = dmalloc(&idx->max_te, m))) break;
        if ((st = dmalloc(&idx->min_te, m))) break;
        if ((st = dmalloc(&idx->cmax_te, m))) break;
        if ((st = dmalloc(&idx->lo_ts, m))) break;
    } while (0);
    if (st != TDS_OK) {
        destroy_index(idx);
        return st;
    }
    idx->device_bytes = n * (sizeof(EntryF64) + sizeof(EntryF32) + 8) + (size_t)m * 44 + 4;
    hipLaunchKernelGGL(k_gather, dim3(nb), dim3(kBT), 0, stream, n, vals, tmp64, tmp32, S.traj,
                       idx->e64, idx->e32, idx->seg_id, idx->traj);
    hipLaunchKernelGGL(k_bin_first, dim3(nb), dim3(kBT), 0, stream, n, idx->e64, tmin, bw, m,
                       idx->bin_first);
    hipLaunchKernelGGL(k_bin_stats, dim3(m), dim3(kBT), 0, stream, n, idx->e64, idx->bin_first,
                       idx->min_ts, idx->max_te, idx->min_te, idx->lo_ts);
    hipLaunchKernelGGL(k_bin_cummax, dim3(1), dim3(1024), 0, stream, idx->max_te, idx->cmax_te, m);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess) {
        destroy_index(idx);
        return TDS_E_DEVICE;
    }
    *out = idx;
    return TDS_OK;
}

}  // namespace tds
