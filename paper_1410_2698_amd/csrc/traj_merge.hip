// Trajectory-level output: segment-level result records merged into maximal
// time intervals per (q_traj, e_traj) pair (the trajectory-level answer to
// the motivating query of Sec. 1, built on the segment records of Sec. 3.1).
//
//   1. stable radix sort of the record indices by t_lo, then by the
//      trajectory pair: the records in (q_traj, e_traj, t_lo) order, equal
//      keys in input order;
//   2. k_run_heads / scan: one run per trajectory pair;
//   3. k_merge_runs<false>: one thread per run walks its records and counts
//      the merged intervals (an interval is extended while the next record
//      starts no later than the running end); scan of the counts;
//   4. k_merge_runs<true>: the same walk writes the intervals at their offsets
//      (only those below the capacity).
#include <algorithm>

#include "tds_internal.hpp"

namespace tds {

namespace {

constexpr int kMT = 256;

__device__ inline uint64_t order_key_f64(double t) {
    // order-preserving map of a double to u64 (-0 and +0 are equal)
    uint64_t u = (t == 0.0) ? 0ull : (uint64_t)__double_as_longlong(t);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

__device__ inline uint64_t pair_key(const tds_result& r) {
    return ((uint64_t)r.q_traj << 32) | r.e_traj;
}

__global__ __launch_bounds__(kMT) void k_keys_tlo(const tds_result* __restrict__ recs, uint32_t n,
                                                  uint64_t* __restrict__ keys,
                                                  uint32_t* __restrict__ vals) {
    const uint32_t i = blockIdx.x * kMT + threadIdx.x;
    if (i >= n) return;
    keys[i] = order_key_f64(recs[i].t_lo);
    vals[i] = i;
}

__global__ __launch_bounds__(kMT) void k_keys_pair(const tds_result* __restrict__ recs, uint32_t n,
                                                   const uint32_t* __restrict__ vals,
                                                   uint64_t* __restrict__ keys) {
    const uint32_t i = blockIdx.x * kMT + threadIdx.x;
    if (i >= n) return;
    keys[i] = pair_key(recs[vals[i]]);
}

// head[i] = 1 where a new trajectory pair starts in sorted order.
__global__ __launch_bounds__(kMT) void k_run_heads(const uint64_t* __restrict__ keys, uint32_t n,
                                                   uint32_t* __restrict__ head) {
    const uint32_t i = blockIdx.x * kMT + threadIdx.x;
    if (i >= n) return;
    head[i] = (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
}

// run_start[run index] = first sorted position of the run (from the
// exclusive scan of the heads and the heads themselves).
__global__ __launch_bounds__(kMT) void k_run_starts(const uint64_t* __restrict__ keys, uint32_t n,
                                                    const uint32_t* __restrict__ run_of,
                                                    uint32_t* __restrict__ run_start,
                                                    uint32_t n_runs) {
    const uint32_t i = blockIdx.x * kMT + threadIdx.x;
    if (i >= n) return;
    if (i == 0 || keys[i] != keys[i - 1]) run_start[run_of[i]] = i;
    if (i == 0) run_start[n_runs] = n;
}

// One thread per run: the merged intervals of one trajectory pair, counted
// (kWrite false: cnt[r]) or written from offset cnt[r] (kWrite true).
template <bool kWrite>
__global__ __launch_bounds__(kMT) void k_merge_runs(const tds_result* __restrict__ recs,
                                                    const uint32_t* __restrict__ order,
                                                    const uint32_t* __restrict__ run_start,
                                                    uint32_t n_runs, uint32_t* __restrict__ cnt,
                                                    tds_traj_interval* __restrict__ out,
                                                    uint64_t capacity) {
    const uint32_t r = blockIdx.x * kMT + threadIdx.x;
    if (r >= n_runs) return;
    const uint32_t b = run_start[r], e = run_start[r + 1];
    uint64_t pos = kWrite ? cnt[r] : 0u;
    uint32_t c = 0;
    const tds_result first = recs[order[b]];
    double lo = first.t_lo, hi = first.t_hi;
    for (uint32_t i = b + 1; i <= e; ++i) {
        bool close = (i == e);
        double nlo = 0.0, nhi = 0.0;
        if (!close) {
            const tds_result x = recs[order[i]];
            nlo = x.t_lo;
            nhi = x.t_hi;
            close = nlo > hi;  // a gap: the current interval is complete
        }
        if (close) {
            if (kWrite && pos < capacity) {
                tds_traj_interval o;
                o.q_traj = first.q_traj;
                o.e_traj = first.e_traj;
                o.t_lo = lo;
                o.t_hi = hi;
                out[pos] = o;
            }
            ++pos;
            ++c;
            lo = nlo;
            hi = nhi;
        } else if (nhi > hi) {
            hi = nhi;
        }
    }
    if (!kWrite) cnt[r] = c;
}

struct Bufs {
    void* p[8] = {};
    ~Bufs() {
        for (void* q : p) dfree(q);
    }
};

}  // namespace

int merge_impl(const tds_result* recs, uint64_t n, bool recs_dev, tds_traj_interval* out,
               uint64_t capacity, bool out_dev, uint64_t* n_out, hipStream_t s) {
    if (!n_out) return TDS_E_INVALID;
    *n_out = 0;
    if (n == 0) return TDS_OK;
    if (!recs || (capacity && !out) || n >= 0xFFFFFFFFull) return TDS_E_INVALID;
    const uint32_t nn = (uint32_t)n;
    const uint32_t nb = ceil_div(nn, kMT);
    Bufs B;
    const tds_result* R = recs;
    if (!recs_dev) {
        tds_result* d = nullptr;
        TDS_TRY(dmalloc(&d, n));
        B.p[0] = d;
        TDS_HIP(hipMemcpyAsync(d, recs, n * sizeof(tds_result), hipMemcpyHostToDevice, s));
        R = d;
    }
    uint64_t *k1 = nullptr, *k2 = nullptr;
    uint32_t *v1 = nullptr, *v2 = nullptr, *runs = nullptr;
    TDS_TRY(dmalloc(&k1, n));
    B.p[1] = k1;
    TDS_TRY(dmalloc(&k2, n));
    B.p[2] = k2;
    TDS_TRY(dmalloc(&v1, n));
    B.p[3] = v1;
    TDS_TRY(dmalloc(&v2, n));
    B.p[4] = v2;
    TDS_TRY(dmalloc(&runs, n));
    B.p[5] = runs;
    // (q_traj, e_traj, t_lo) order: by t_lo, then stably by the pair
    hipLaunchKernelGGL(k_keys_tlo, dim3(nb), dim3(kMT), 0, s, R, nn, k1, v1);
    TDS_HIP(hipGetLastError());
    TDS_TRY(radix_sort_u64(k1, v1, k2, v2, nn, 64, s));
    hipLaunchKernelGGL(k_keys_pair, dim3(nb), dim3(kMT), 0, s, R, nn, v1, k1);
    TDS_HIP(hipGetLastError());
    TDS_TRY(radix_sort_u64(k1, v1, k2, v2, nn, 64, s));
    // runs of equal pairs
    hipLaunchKernelGGL(k_run_heads, dim3(nb), dim3(kMT), 0, s, k1, nn, runs);
    TDS_HIP(hipGetLastError());
    uint32_t n_runs = 0;
    TDS_TRY(exclusive_scan_u32(runs, nn, &n_runs, s));
    uint32_t *run_start = nullptr, *cnt = nullptr;
    TDS_TRY(dmalloc(&run_start, (size_t)n_runs + 1));
    B.p[6] = run_start;
    TDS_TRY(dmalloc(&cnt, n_runs));
    B.p[7] = cnt;
    hipLaunchKernelGGL(k_run_starts, dim3(nb), dim3(kMT), 0, s, k1, nn, runs, run_start, n_runs);
    const uint32_t rb = ceil_div(n_runs, kMT);
    hipLaunchKernelGGL(k_merge_runs<false>, dim3(rb), dim3(kMT), 0, s, R, v1, run_start, n_runs,
                       cnt, nullptr, 0ull);
    TDS_HIP(hipGetLastError());
    uint32_t total = 0;
    TDS_TRY(exclusive_scan_u32(cnt, n_runs, &total, s));
    *n_out = total;
    const uint64_t keep = std::min<uint64_t>(total, capacity);
    if (keep) {
        tds_traj_interval* dst = out;
        tds_traj_interval* stage = nullptr;
        if (!out_dev) {
            TDS_TRY(dmalloc(&stage, keep));
            dst = stage;
        }
        hipLaunchKernelGGL(k_merge_runs<true>, dim3(rb), dim3(kMT), 0, s, R, v1, run_start, n_runs,
                           cnt, dst, keep);
        int st = (hipGetLastError() == hipSuccess) ? TDS_OK : TDS_E_DEVICE;
        if (st == TDS_OK && !out_dev &&
            hipMemcpyAsync(out, stage, keep * sizeof(tds_traj_interval), hipMemcpyDeviceToHost,
                           s) != hipSuccess)
            st = TDS_E_DEVICE;
        if (st == TDS_OK && hipStreamSynchronize(s) != hipSuccess) st = TDS_E_DEVICE;
        dfree(stage);
        TDS_TRY(st);
    }
    return total > capacity ? TDS_E_OVERFLOW : TDS_OK;
}

}  // namespace tds
