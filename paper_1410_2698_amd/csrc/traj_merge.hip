// Trajectory-level output: segment-level result records merged into maximal
// time intervals per (q_traj, e_traj) pair (the trajectory-level answer to
// the motivating query of Sec. 1, built on the segment records of Sec. 3.1).
//
//   1. stable radix sort of the record indices by t_lo, then by the
//      trajectory pair: the records in (q_traj, e_traj, t_lo) order, equal
//      keys in input order.  One reduction first finds which 8-bit digits of
//      the t_lo keys differ and how many bits the trajectory ids need, so the
//      sorts make only the passes that can change the order;
//   2. k_run_heads / scan: one run per trajectory pair;
//   3. k_merge_runs<false>: one thread per run walks its records and counts
//      the merged intervals (an interval is extended while the next record
//      starts no later than the running end); scan of the counts;
//   4. k_merge_runs<true>: the same walk writes the intervals at their offsets
//      (only those below the capacity).
#include <algorithm>
#include <mutex>

#include "tds_internal.hpp"

namespace tds {

namespace {

constexpr int kMT = 256;

__device__ inline uint64_t order_key_f64(double t) {
    // order-preserving map of a double to u64 (-0 and +0 are equal)
    uint64_t u = (t == 0.0) ? 0ull : (uint64_t)__double_as_longlong(t);
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

// red[0] = OR of the t_lo keys, red[1] = AND, red[2] = max q_traj, red[3] =
// max e_traj (k_red_init sets the identities).
__global__ void k_red_init(unsigned long long* red) {
    red[0] = 0ull;
    red[1] = ~0ull;
    red[2] = 0ull;
    red[3] = 0ull;
}

__global__ __launch_bounds__(kMT) void k_keys_tlo(const tds_result* __restrict__ recs, uint32_t n,
                                                  uint64_t* __restrict__ keys,
                                                  uint32_t* __restrict__ vals,
                                                  unsigned long long* red) {
    __shared__ unsigned long long s_or[kMT], s_and[kMT], s_q[kMT], s_e[kMT];
    const uint32_t i = blockIdx.x * kMT + threadIdx.x;
    unsigned long long ko = 0ull, ka = ~0ull, mq = 0ull, me = 0ull;
    if (i < n) {
        const tds_result r = recs[i];
        const uint64_t k = order_key_f64(r.t_lo);
        keys[i] = k;
        vals[i] = i;
        ko = ka = k;
        mq = r.q_traj;
        me = r.e_traj;
    }
    s_or[threadIdx.x] = ko;
    s_and[threadIdx.x] = ka;
    s_q[threadIdx.x] = mq;
    s_e[threadIdx.x] = me;
    __syncthreads();
    for (uint32_t off = kMT / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) {
            s_or[threadIdx.x] |= s_or[threadIdx.x + off];
            s_and[threadIdx.x] &= s_and[threadIdx.x + off];
            s_q[threadIdx.x] = max(s_q[threadIdx.x], s_q[threadIdx.x + off]);
            s_e[threadIdx.x] = max(s_e[threadIdx.x], s_e[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        atomicOr(&red[0], s_or[0]);
        atomicAnd(&red[1], s_and[0]);
        atomicMax(&red[2], s_q[0]);
        atomicMax(&red[3], s_e[0]);
    }
}

// Pair key q_traj << e_bits | e_traj (e_bits: bits of the largest e_traj).
__global__ __launch_bounds__(kMT) void k_keys_pair(const tds_result* __restrict__ recs, uint32_t n,
                                                   const uint32_t* __restrict__ vals, uint32_t e_bits,
                                                   uint64_t* __restrict__ keys) {
    const uint32_t i = blockIdx.x * kMT + threadIdx.x;
    if (i >= n) return;
    const tds_result r = recs[vals[i]];
    keys[i] = ((uint64_t)r.q_traj << e_bits) | r.e_traj;
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

// Device scratch of the merge, per device, grown on demand and kept until the
// process ends (the merge is called repeatedly on result sets of similar
// size; allocating and freeing per call cost more than the kernels).
struct MergeScratch {
    std::mutex mu;
    size_t cap = 0;  // records the buffers hold
    tds_result* recs = nullptr;
    uint64_t *k1 = nullptr, *k2 = nullptr;
    uint32_t *v1 = nullptr, *v2 = nullptr, *runs = nullptr, *run_start = nullptr, *cnt = nullptr;
    uint32_t *hist = nullptr, *part = nullptr;
    tds_traj_interval* stage = nullptr;
    unsigned long long* red = nullptr;
    unsigned long long* red_host = nullptr;  // pinned

    void release() {
        dfree(recs);
        dfree(k1);
        dfree(k2);
        dfree(v1);
        dfree(v2);
        dfree(runs);
        dfree(run_start);
        dfree(cnt);
        dfree(hist);
        dfree(part);
        dfree(stage);
        recs = nullptr;
        k1 = k2 = nullptr;
        v1 = v2 = runs = run_start = cnt = hist = part = nullptr;
        stage = nullptr;
        cap = 0;
    }

    int reserve(size_t n) {
        if (!red) {
            TDS_TRY(dmalloc(&red, 4));
            if (hipHostMalloc(reinterpret_cast<void**>(&red_host), 4 * sizeof(unsigned long long),
                              hipHostMallocDefault) != hipSuccess) {
                (void)hipGetLastError();
                red_host = nullptr;
                return TDS_E_NOMEM;
            }
        }
        if (n <= cap) return TDS_OK;
        release();
        const size_t c = std::max<size_t>(n, 1024);
        const size_t parts = std::max(scan_part_len(radix_hist_len((uint32_t)c)), scan_part_len(c));
        int st = TDS_OK;
        if (st == TDS_OK) st = dmalloc(&recs, c);
        if (st == TDS_OK) st = dmalloc(&k1, c);
        if (st == TDS_OK) st = dmalloc(&k2, c);
        if (st == TDS_OK) st = dmalloc(&v1, c);
        if (st == TDS_OK) st = dmalloc(&v2, c);
        if (st == TDS_OK) st = dmalloc(&runs, c);
        if (st == TDS_OK) st = dmalloc(&run_start, c + 1);
        if (st == TDS_OK) st = dmalloc(&cnt, c);
        if (st == TDS_OK) st = dmalloc(&hist, radix_hist_len((uint32_t)c));
        if (st == TDS_OK) st = dmalloc(&part, parts);
        if (st == TDS_OK) st = dmalloc(&stage, c);
        if (st != TDS_OK) {
            release();
            return st;
        }
        cap = c;
        return TDS_OK;
    }
};

constexpr int kMaxDevices = 64;
MergeScratch g_scratch[kMaxDevices];

// 8-bit digits in which some of the keys differ.
uint32_t varying_digits(uint64_t ored, uint64_t anded) {
    const uint64_t v = ored ^ anded;
    uint32_t m = 0;
    for (int p = 0; p < 8; ++p)
        if ((v >> (8 * p)) & 0xFFull) m |= 1u << p;
    return m;
}

uint32_t bit_width(uint64_t v) {
    uint32_t b = 0;
    while (v) {
        ++b;
        v >>= 1;
    }
    return b;
}

}  // namespace

int merge_impl(const tds_result* recs, uint64_t n, bool recs_dev, tds_traj_interval* out,
               uint64_t capacity, bool out_dev, uint64_t* n_out, hipStream_t s) {
    if (!n_out) return TDS_E_INVALID;
    *n_out = 0;
    if (n == 0) return TDS_OK;
    if (!recs || (capacity && !out) || n >= 0xFFFFFFFFull) return TDS_E_INVALID;
    int dev = 0;
    TDS_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return TDS_E_DEVICE;
    MergeScratch& M = g_scratch[dev];
    // one merge at a time per device: every call waits for its own work
    // before it returns, so the next call finds the scratch free
    std::lock_guard<std::mutex> lock(M.mu);
    TDS_TRY(M.reserve(n));
    const uint32_t nn = (uint32_t)n;
    const uint32_t nb = ceil_div(nn, kMT);
    const tds_result* R = recs;
    if (!recs_dev) {
        TDS_HIP(hipMemcpyAsync(M.recs, recs, n * sizeof(tds_result), hipMemcpyHostToDevice, s));
        R = M.recs;
    }
    // keys, and which digits and id bits the sorts need
    hipLaunchKernelGGL(k_red_init, dim3(1), dim3(1), 0, s, M.red);
    hipLaunchKernelGGL(k_keys_tlo, dim3(nb), dim3(kMT), 0, s, R, nn, M.k1, M.v1, M.red);
    TDS_HIP(hipGetLastError());
    TDS_HIP(hipMemcpyAsync(M.red_host, M.red, 4 * sizeof(unsigned long long), hipMemcpyDeviceToHost,
                           s));
    TDS_HIP(hipStreamSynchronize(s));
    const uint32_t t_digits = varying_digits(M.red_host[0], M.red_host[1]);
    const uint32_t e_bits = std::max(1u, bit_width(M.red_host[3]));
    const uint32_t pair_bits = bit_width(M.red_host[2]) + e_bits;
    const uint32_t pair_digits = (pair_bits >= 64) ? 0xFFu : ((1u << ((pair_bits + 7) / 8)) - 1u);
    // (q_traj, e_traj, t_lo) order: by t_lo, then stably by the pair
    TDS_TRY(radix_sort_u64_digits(M.k1, M.v1, M.k2, M.v2, nn, t_digits, s, M.hist, M.part));
    hipLaunchKernelGGL(k_keys_pair, dim3(nb), dim3(kMT), 0, s, R, nn, M.v1, e_bits, M.k1);
    TDS_HIP(hipGetLastError());
    TDS_TRY(radix_sort_u64_digits(M.k1, M.v1, M.k2, M.v2, nn, pair_digits, s, M.hist, M.part));
    // runs of equal pairs
    hipLaunchKernelGGL(k_run_heads, dim3(nb), dim3(kMT), 0, s, M.k1, nn, M.runs);
    TDS_HIP(hipGetLastError());
    uint32_t n_runs = 0;
    TDS_TRY(exclusive_scan_u32_with(M.runs, nn, &n_runs, s, M.part));
    hipLaunchKernelGGL(k_run_starts, dim3(nb), dim3(kMT), 0, s, M.k1, nn, M.runs, M.run_start,
                       n_runs);
    const uint32_t rb = ceil_div(n_runs, kMT);
    hipLaunchKernelGGL(k_merge_runs<false>, dim3(rb), dim3(kMT), 0, s, R, M.v1, M.run_start, n_runs,
                       M.cnt, nullptr, 0ull);
    TDS_HIP(hipGetLastError());
    uint32_t total = 0;
    TDS_TRY(exclusive_scan_u32_with(M.cnt, n_runs, &total, s, M.part));
    *n_out = total;
    const uint64_t keep = std::min<uint64_t>(total, capacity);
    if (keep) {
        // at most one interval per record, so the staging buffer fits
        tds_traj_interval* dst = out_dev ? out : M.stage;
        hipLaunchKernelGGL(k_merge_runs<true>, dim3(rb), dim3(kMT), 0, s, R, M.v1, M.run_start,
                           n_runs, M.cnt, dst, keep);
        TDS_HIP(hipGetLastError());
        if (!out_dev)
            TDS_HIP(hipMemcpyAsync(out, M.stage, keep * sizeof(tds_traj_interval),
                                   hipMemcpyDeviceToHost, s));
        TDS_HIP(hipStreamSynchronize(s));
    }
    return total > capacity ? TDS_E_OVERFLOW : TDS_OK;
}

}  // namespace tds
