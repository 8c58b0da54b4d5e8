// Index build on the GPU: the temporal index of Sec. 4.2.1, optionally with
// every temporal bin subdivided in space (the idea of Sec. 4.3).
//
//   k_seg_prep    validate every segment, compute its velocity (IEEE FP64
//                 division), its FP32 bounding-sphere record, its sort key
//                 (order-preserving bits of t_start) and per-block partial
//                 min t_start / max t_end / sum of durations / extent of the
//                 sphere centres;
//   k_spatial_key (spatial layout) replace the key by (bin, Hilbert index of
//                 the sphere centre on a 1024^3 grid over the centres' extent);
//   radix sort    stable, by the key (radix_sort.hip);
//   k_gather      write the ordered AoS records, ids and trajectory ids;
//   k_bin_first   first position of every bin (boundary detection);
//   k_bin_stats   per-bin data extents (min/max t_start, min/max t_end);
//   k_bin_scan    running maximum of max t_end over bins, which makes the
//                 bins overlapping a query one contiguous, bisectable span,
//                 and the minimum t_start over the bins from j on;
//   k_block_box   (spatial layout) box of the segments of every aligned
//                 block of 64 entries.
#include <cmath>
#include <utility>

#include "hilbert.hpp"
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

// Per-block partials written by k_seg_prep: min t_start, max t_end, sum of
// durations, then min and max of the sphere centres per axis.
constexpr int kPart = 9;

__global__ __launch_bounds__(kBT) void k_seg_prep(SegView S, EntryF64* __restrict__ tmp64,
                                                  EntryF32* __restrict__ tmp32,
                                                  uint64_t* __restrict__ keys,
                                                  uint32_t* __restrict__ vals,
                                                  double* __restrict__ part, uint32_t* err) {
    __shared__ double sp[kPart][kBT];
    const uint32_t tid = threadIdx.x;
    const uint64_t i = (uint64_t)blockIdx.x * kBT + tid;
    double v[kPart] = {INFINITY, -INFINITY, 0.0, INFINITY, -INFINITY,
                       INFINITY, -INFINITY, INFINITY, -INFINITY};
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
        v[0] = ts;
        v[1] = te;
        v[2] = dt;
        v[3] = v[4] = f.cx;
        v[5] = v[6] = f.cy;
        v[7] = v[8] = f.cz;
    }
    for (int k = 0; k < kPart; ++k) sp[k][tid] = v[k];
    __syncthreads();
    for (uint32_t off = kBT / 2; off > 0; off >>= 1) {
        if (tid < off) {
            sp[0][tid] = fmin(sp[0][tid], sp[0][tid + off]);
            sp[1][tid] = fmax(sp[1][tid], sp[1][tid + off]);
            sp[2][tid] = sp[2][tid] + sp[2][tid + off];
            for (int k = 3; k < kPart; k += 2) {
                sp[k][tid] = fmin(sp[k][tid], sp[k][tid + off]);
                sp[k + 1][tid] = fmax(sp[k + 1][tid], sp[k + 1][tid + off]);
            }
        }
        __syncthreads();
    }
    if (tid < kPart) part[kPart * blockIdx.x + tid] = sp[tid][0];
}

// Bin of a t_start: floor((ts - t_min) / b) clamped to [0, m-1].
__device__ inline uint32_t bin_of(double ts, double tmin, double bw, uint32_t m) {
    double u = floor((ts - tmin) / bw);
    if (!(u > 0.0)) return 0u;
    if (u >= (double)(m - 1)) return m - 1;
    return (uint32_t)u;
}

__device__ inline uint32_t cell10(float c, float lo, float scale) {
    const float u = (c - lo) * scale;
    if (!(u > 0.f)) return 0u;
    if (u >= 1023.f) return 1023u;
    return (uint32_t)u;
}

// Spatial layout key: bin in the high bits, then the Hilbert index of the
// sphere centre's cell.  Only the order inside a bin depends on the cell, so
// the bins, and every table derived from them, are those of the temporal
// layout.
__global__ __launch_bounds__(kBT) void k_spatial_key(uint64_t n, const EntryF64* __restrict__ tmp64,
                                                     const EntryF32* __restrict__ tmp32,
                                                     double tmin, double bw, uint32_t m,
                                                     float lx, float ly, float lz, float sx,
                                                     float sy, float sz,
                                                     uint64_t* __restrict__ keys) {
    const uint64_t i = (uint64_t)blockIdx.x * kBT + threadIdx.x;
    if (i >= n) return;
    const EntryF32 f = tmp32[i];
    const uint32_t h =
        hilbert3<10>(cell10(f.cx, lx, sx), cell10(f.cy, ly, sy), cell10(f.cz, lz, sz));
    keys[i] = ((uint64_t)bin_of(tmp64[i].ts, tmin, bw, m) << 30) | h;
}

__global__ __launch_bounds__(kBT) void k_gather(uint64_t n, const uint32_t* __restrict__ perm,
                                                const EntryF64* __restrict__ tmp64,
                                                const EntryF32* __restrict__ tmp32,
                                                const uint32_t* __restrict__ traj_in,
                                                EntryF64* __restrict__ e64,
                                                EntryF32* __restrict__ e32,
                                                EntryV32* __restrict__ ev32,
                                                uint32_t* __restrict__ seg_id,
                                                uint32_t* __restrict__ traj) {
    const uint64_t i = (uint64_t)blockIdx.x * kBT + threadIdx.x;
    if (i >= n) return;
    const uint32_t src = perm[i];
    const EntryF64 e = tmp64[src];
    e64[i] = e;
    e32[i] = tmp32[src];
    EntryV32 v;
    v.vx = __double2float_rn(e.vx);
    v.vy = __double2float_rn(e.vy);
    v.vz = __double2float_rn(e.vz);
    v.tm = __double2float_rn(0.5 * (e.ts + e.te));
    ev32[i] = v;
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

// Per-bin extents: min and max of t_start and of t_end over the bin's
// entries (+inf / -inf when the bin is empty); one block per bin.
__global__ __launch_bounds__(kBT) void k_bin_stats(const EntryF64* __restrict__ e64,
                                                   const uint32_t* __restrict__ bin_first,
                                                   double* __restrict__ min_ts,
                                                   double* __restrict__ max_ts,
                                                   double* __restrict__ min_te,
                                                   double* __restrict__ max_te) {
    __shared__ double sp[4][kBT];
    const uint32_t j = blockIdx.x;
    const uint32_t f = bin_first[j], e = bin_first[j + 1];
    double v[4] = {INFINITY, -INFINITY, INFINITY, -INFINITY};
    for (uint32_t i = f + threadIdx.x; i < e; i += kBT) {
        const double ts = e64[i].ts, te = e64[i].te;
        v[0] = fmin(v[0], ts);
        v[1] = fmax(v[1], ts);
        v[2] = fmin(v[2], te);
        v[3] = fmax(v[3], te);
    }
    for (int k = 0; k < 4; ++k) sp[k][threadIdx.x] = v[k];
    __syncthreads();
    for (uint32_t off = kBT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            for (int k = 0; k < 4; k += 2) {
                sp[k][threadIdx.x] = fmin(sp[k][threadIdx.x], sp[k][threadIdx.x + off]);
                sp[k + 1][threadIdx.x] = fmax(sp[k + 1][threadIdx.x], sp[k + 1][threadIdx.x + off]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        min_ts[j] = sp[0][0];
        max_ts[j] = sp[1][0];
        min_te[j] = sp[2][0];
        max_te[j] = sp[3][0];
    }
}

// Running extreme over len values with one block of 1024 threads: the
// maximum of v[0..i] (kMax, forward) or the minimum of v[i..len) (reverse).
template <bool kMax>
__global__ __launch_bounds__(1024) void k_bin_scan(const double* __restrict__ v,
                                                   double* __restrict__ out, uint32_t len) {
    __shared__ double part[1024];
    const double id = kMax ? -INFINITY : INFINITY;
    auto op = [](double a, double b) { return kMax ? fmax(a, b) : fmin(a, b); };
    // element k of the scan order: i = k (forward) or len - 1 - k (reverse)
    auto at = [&](uint32_t k) { return kMax ? k : len - 1 - k; };
    const uint32_t tid = threadIdx.x;
    const uint32_t per = (len + 1023) / 1024;
    const uint32_t b = tid * per, e = min(len, b + per);
    double acc = id;
    for (uint32_t k = b; k < e; ++k) acc = op(acc, v[at(k)]);
    part[tid] = acc;
    __syncthreads();
    for (uint32_t off = 1; off < 1024; off <<= 1) {
        const double t = (tid >= off) ? part[tid - off] : id;
        __syncthreads();
        part[tid] = op(part[tid], t);
        __syncthreads();
    }
    double run = (tid > 0) ? part[tid - 1] : id;
    for (uint32_t k = b; k < e; ++k) {
        run = op(run, v[at(k)]);
        out[at(k)] = run;
    }
}

// Box of each aligned block of 64 entries: the union of the entries' segment
// boxes (seg_box32 of the end points the canonical evaluation computes from
// the FP64 record), one wave per block (lanes past n contribute nothing).
__global__ __launch_bounds__(kBT) void k_block_box(uint64_t n, const EntryF64* __restrict__ e64,
                                                   BlockBox* __restrict__ box, uint32_t nblk) {
    const uint32_t blk = blockIdx.x * (kBT / kWave) + threadIdx.x / kWave;
    if (blk >= nblk) return;
    const uint64_t i = ((uint64_t)blk << kBoxShift) + __lane_id();
    Box32 v = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    if (i < n) {
        const EntryF64 e = e64[i];
        const double dt = e.te - e.ts;
        v = seg_box32(e.x, e.y, e.z, e.x + e.vx * dt, e.y + e.vy * dt, e.z + e.vz * dt, 0.0);
    }
    for (int off = kWave / 2; off > 0; off >>= 1) {
        v.lx = fminf(v.lx, __shfl_xor(v.lx, off));
        v.ly = fminf(v.ly, __shfl_xor(v.ly, off));
        v.lz = fminf(v.lz, __shfl_xor(v.lz, off));
        v.hx = fmaxf(v.hx, __shfl_xor(v.hx, off));
        v.hy = fmaxf(v.hy, __shfl_xor(v.hy, off));
        v.hz = fmaxf(v.hz, __shfl_xor(v.hz, off));
    }
    if (__lane_id() == 0) {
        BlockBox b;
        b.b = v;
        b.pad0 = 0.f;
        b.pad1 = 0.f;
        box[blk] = b;
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
    dfree(idx->ev32);
    dfree(idx->seg_id);
    dfree(idx->traj);
    dfree(idx->bin_first);
    dfree(idx->min_ts);
    dfree(idx->max_te);
    dfree(idx->min_te);
    dfree(idx->cmax_te);
    dfree(idx->lo_ts);
    dfree(idx->max_ts);
    dfree(idx->bbox);
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
    uint32_t layout = p ? p->layout : (uint32_t)TDS_LAYOUT_DEFAULT;
    if (layout == TDS_LAYOUT_DEFAULT) layout = TDS_LAYOUT_SPATIAL;
    if (layout != TDS_LAYOUT_TEMPORAL && layout != TDS_LAYOUT_SPATIAL) return TDS_E_INVALID;

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
    TDS_TRY(dmalloc(&part, kPart * (size_t)nb));
    sc.p[8] = part;
    TDS_TRY(dmalloc(&err, 1));
    sc.p[9] = err;
    TDS_HIP(hipMemsetAsync(err, 0, sizeof(uint32_t), stream));
    hipLaunchKernelGGL(k_seg_prep, dim3(nb), dim3(kBT), 0, stream, S, tmp64, tmp32, keys, vals,
                       part, err);
    TDS_HIP(hipGetLastError());
    std::vector<double> hpart(kPart * (size_t)nb);
    uint32_t herr = 0;
    TDS_HIP(hipMemcpyAsync(hpart.data(), part, hpart.size() * sizeof(double), hipMemcpyDeviceToHost,
                           stream));
    TDS_HIP(hipMemcpyAsync(&herr, err, sizeof(uint32_t), hipMemcpyDeviceToHost, stream));
    TDS_HIP(hipStreamSynchronize(stream));
    if (herr) return TDS_E_INVALID;
    double tmin = INFINITY, tmax = -INFINITY, dsum = 0.0;
    double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (uint32_t b = 0; b < nb; ++b) {
        const double* q = &hpart[kPart * (size_t)b];
        tmin = std::fmin(tmin, q[0]);
        tmax = std::fmax(tmax, q[1]);
        dsum += q[2];
        for (int k = 0; k < 3; ++k) {
            clo[k] = std::fmin(clo[k], q[3 + 2 * k]);
            chi[k] = std::fmax(chi[k], q[4 + 2 * k]);
        }
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

    // ---- sort: by t_start, or by (bin, spatial cell)
    int key_bits = 64;
    if (layout == TDS_LAYOUT_SPATIAL) {
        float lo[3], sc[3];
        for (int k = 0; k < 3; ++k) {
            const double ext = chi[k] - clo[k];
            lo[k] = (float)clo[k];
            sc[k] = (ext > 0.0 && std::isfinite(ext)) ? (float)(1024.0 / ext) : 0.f;
        }
        hipLaunchKernelGGL(k_spatial_key, dim3(nb), dim3(kBT), 0, stream, n, tmp64, tmp32, tmin,
                           bw, m, lo[0], lo[1], lo[2], sc[0], sc[1], sc[2], keys);
        TDS_HIP(hipGetLastError());
        int bin_bits = 0;
        while ((1u << bin_bits) < m) ++bin_bits;
        key_bits = 30 + bin_bits;
    }
    TDS_TRY(radix_sort_u64(keys, vals, keys2, vals2, (uint32_t)n, key_bits, stream));

    // ---- the index object
    tds_index* idx = new (std::nothrow) tds_index();
    if (!idx) return TDS_E_NOMEM;
    idx->device = dev;
    idx->n = n;
    idx->m = m;
    idx->t_min = tmin;
    idx->t_max = tmax;
    idx->bw = bw;
    idx->layout = layout;
    const uint32_t nblk = ceil_div(n, 1u << kBoxShift);
    int st = TDS_OK;
    do {
        if ((st = dmalloc(&idx->e64, n))) break;
        if ((st = dmalloc(&idx->e32, n))) break;
        if ((st = dmalloc(&idx->ev32, n))) break;
        if ((st = dmalloc(&idx->seg_id, n))) break;
        if ((st = dmalloc(&idx->traj, n))) break;
        if ((st = dmalloc(&idx->bin_first, (size_t)m + 1))) break;
        if ((st = dmalloc(&idx->min_ts, m))) break;
        if ((st = dmalloc(&idx->max_te, m))) break;
        if ((st = dmalloc(&idx->min_te, m))) break;
        if ((st = dmalloc(&idx->cmax_te, m))) break;
        if ((st = dmalloc(&idx->lo_ts, m))) break;
        if ((st = dmalloc(&idx->max_ts, m))) break;
        if (layout == TDS_LAYOUT_SPATIAL && (st = dmalloc(&idx->bbox, nblk))) break;
    } while (0);
    if (st != TDS_OK) {
        destroy_index(idx);
        return st;
    }
    idx->device_bytes = n * (sizeof(EntryF64) + sizeof(EntryF32) + sizeof(EntryV32) + 8) +
                        (size_t)m * 52 + 4 +
                        (idx->bbox ? (size_t)nblk * sizeof(BlockBox) : 0);
    hipLaunchKernelGGL(k_gather, dim3(nb), dim3(kBT), 0, stream, n, vals, tmp64, tmp32, S.traj,
                       idx->e64, idx->e32, idx->ev32, idx->seg_id, idx->traj);
    hipLaunchKernelGGL(k_bin_first, dim3(nb), dim3(kBT), 0, stream, n, idx->e64, tmin, bw, m,
                       idx->bin_first);
    hipLaunchKernelGGL(k_bin_stats, dim3(m), dim3(kBT), 0, stream, idx->e64, idx->bin_first,
                       idx->min_ts, idx->max_ts, idx->min_te, idx->max_te);
    hipLaunchKernelGGL(k_bin_scan<true>, dim3(1), dim3(1024), 0, stream, idx->max_te, idx->cmax_te,
                       m);
    hipLaunchKernelGGL(k_bin_scan<false>, dim3(1), dim3(1024), 0, stream, idx->min_ts, idx->lo_ts,
                       m);
    if (idx->bbox)
        hipLaunchKernelGGL(k_block_box, dim3(ceil_div(nblk, kBT / kWave)), dim3(kBT), 0, stream, n,
                           idx->e64, idx->bbox, nblk);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(stream) != hipSuccess) {
        destroy_index(idx);
        return TDS_E_DEVICE;
    }
    *out = idx;
    return TDS_OK;
}

}  // namespace tds
