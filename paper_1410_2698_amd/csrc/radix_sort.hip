// Stable LSD radix sort of (u64 key, u32 value) pairs with 8-bit digits.
//
// Used by the index build to order the entry segments by t_start (Sec. 4.2.1
// sorts D by ascending start time and renumbers it); stability keeps equal
// start times in input order, which makes the renumbering deterministic.
//
// One pass per digit, five kernels per pass:
//   rs_hist    each block counts the digits of its 2048-key tile in LDS;
//   rs_scan_*  turn the digit-major count table into exclusive offsets
//              (digit d of block b starts after every smaller digit and after
//              digit d of the blocks before b): tile sums, a scan of the tile
//              sums, then each tile scanned from its offset;
//   rs_scatter each block re-reads its tile and writes every key to its
//              offset; the rank of a key among equal digits of its tile comes
//              from wave ballots (wave-local) plus per-wave digit counts in
//              LDS, processed in tile order, so the pass is stable.
#include <algorithm>

#include "tds_internal.hpp"

namespace tds {

namespace {

constexpr int kRsThreads = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kRsThreads * kRsItems;
constexpr int kRadix = 256;
constexpr int kRsWaves = kRsThreads / kWave;

__global__ __launch_bounds__(kRsThreads) void rs_hist(const uint64_t* __restrict__ keys, uint32_t n,
                                                      int shift, uint32_t* __restrict__ hist,
                                                      uint32_t nblocks) {
    __shared__ uint32_t h[kRadix];
    const int tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const uint64_t base = (uint64_t)blockIdx.x * kRsTile;
    for (int k = 0; k < kRsItems; ++k) {
        uint64_t i = base + (uint64_t)k * kRsThreads + tid;
        if (i < n) atomicAdd(&h[(uint32_t)(keys[i] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[(uint64_t)tid * nblocks + blockIdx.x] = h[tid];
}

// Exclusive scan of `len` u32 values in place, in three coalesced steps:
//   rs_scan_part  each block sums its tile of kScanTile values;
//   rs_scan_top   one block scans the tile sums (looping over them);
//   rs_scan_down  each block scans its tile again, offset by its tile's sum.
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 4;
constexpr int kScanTile = kScanThreads * kScanPer;

// Inclusive scan of one value per thread over a block of kScanThreads
// (Hillis-Steele in LDS); returns the inclusive prefix, *total the block sum.
__device__ inline uint32_t block_scan(uint32_t x, uint32_t* lds, uint32_t* total) {
    const uint32_t tid = threadIdx.x;
    lds[tid] = x;
    __syncthreads();
    for (uint32_t off = 1; off < kScanThreads; off <<= 1) {
        const uint32_t t = (tid >= off) ? lds[tid - off] : 0u;
        __syncthreads();
        lds[tid] += t;
        __syncthreads();
    }
    const uint32_t r = lds[tid];
    *total = lds[kScanThreads - 1];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kScanThreads) void rs_scan_part(const uint32_t* __restrict__ v,
                                                             uint32_t len,
                                                             uint32_t* __restrict__ part) {
    __shared__ uint32_t lds[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (int k = 0; k < kScanPer; ++k) {
        const uint64_t i = base + (uint64_t)k * kScanThreads + threadIdx.x;
        if (i < len) s += v[i];
    }
    uint32_t total;
    block_scan(s, lds, &total);
    if (threadIdx.x == 0) part[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void rs_scan_top(uint32_t* __restrict__ part,
                                                            uint32_t nparts) {
    __shared__ uint32_t lds[kScanThreads];
    uint32_t carry = 0;
    for (uint32_t b = 0; b < nparts; b += kScanThreads) {
        const uint32_t i = b + threadIdx.x;
        const uint32_t x = (i < nparts) ? part[i] : 0u;
        uint32_t total;
        const uint32_t inc = block_scan(x, lds, &total);
        if (i < nparts) part[i] = carry + inc - x;
        carry += total;
    }
    if (threadIdx.x == 0) part[nparts] = carry;  // the grand total
}

__global__ __launch_bounds__(kScanThreads) void rs_scan_down(uint32_t* __restrict__ v, uint32_t len,
                                                             const uint32_t* __restrict__ part) {
    __shared__ uint32_t lds[kScanThreads];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    // thread t scans kScanPer consecutive values: t's values are
    // base + t * kScanPer + [0, kScanPer)
    uint32_t x[kScanPer];
    uint32_t s = 0;
    for (int k = 0; k < kScanPer; ++k) {
        const uint64_t i = base + (uint64_t)threadIdx.x * kScanPer + k;
        x[k] = (i < len) ? v[i] : 0u;
        s += x[k];
    }
    uint32_t total;
    uint32_t run = block_scan(s, lds, &total) - s + part[blockIdx.x];
    for (int k = 0; k < kScanPer; ++k) {
        const uint64_t i = base + (uint64_t)threadIdx.x * kScanPer + k;
        if (i < len) v[i] = run;
        run += x[k];
    }
}

__device__ inline uint64_t lanemask_lt() {
    const uint32_t lane = __lane_id();
    return (lane == 0) ? 0ull : (~0ull >> (64 - lane));
}

__global__ __launch_bounds__(kRsThreads) void rs_scatter(const uint64_t* __restrict__ kin,
                                                         const uint32_t* __restrict__ vin,
                                                         uint64_t* __restrict__ kout,
                                                         uint32_t* __restrict__ vout, uint32_t n,
                                                         int shift,
                                                         const uint32_t* __restrict__ offs,
                                                         uint32_t nblocks) {
    __shared__ uint32_t base[kRadix];
    __shared__ uint32_t wcnt[kRsWaves][kRadix];
    const int tid = threadIdx.x;
    const int wave = tid / kWave;
    base[tid] = offs[(uint64_t)tid * nblocks + blockIdx.x];
    for (int w = 0; w < kRsWaves; ++w) wcnt[w][tid] = 0;
    __syncthreads();
    const uint64_t tile = (uint64_t)blockIdx.x * kRsTile;
    for (int k = 0; k < kRsItems; ++k) {
        const uint64_t i = tile + (uint64_t)k * kRsThreads + tid;
        const bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0ull;
        uint32_t val = valid ? vin[i] : 0u;
        // 9-bit class: digits 0..255, 256 for lanes without a key
        const uint32_t digit = valid ? ((uint32_t)(key >> shift) & (kRadix - 1)) : (uint32_t)kRadix;
        uint64_t same = __ballot(1);
        for (int bit = 0; bit < 9; ++bit) {
            const bool set = (digit >> bit) & 1u;
            const uint64_t m = __ballot(set);
            same &= set ? m : ~m;
        }
        const uint32_t rank = __popcll(same & lanemask_lt());
        const bool leader = rank == 0;
        if (valid && leader) wcnt[wave][digit] = __popcll(same);
        __syncthreads();
        // per digit: exclusive offsets over the waves of this round
        {
            uint32_t run = 0;
            for (int w = 0; w < kRsWaves; ++w) {
                uint32_t c = wcnt[w][tid];
                wcnt[w][tid] = run;
                run += c;
            }
            // run = total of digit tid in this round; add after the scatter
            __syncthreads();
            if (valid) {
                const uint32_t pos = base[digit] + wcnt[wave][digit] + rank;
                kout[pos] = key;
                vout[pos] = val;
            }
            __syncthreads();
            base[tid] += run;
            for (int w = 0; w < kRsWaves; ++w) wcnt[w][tid] = 0;
            __syncthreads();
        }
    }
}

}  // namespace

size_t radix_hist_len(uint32_t n) { return (size_t)kRadix * ceil_div(n, kRsTile); }

size_t scan_part_len(size_t len) { return (size_t)ceil_div(len, kScanTile) + 1; }

int radix_sort_u64_digits(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                          uint32_t n, uint32_t digit_mask, hipStream_t stream, uint32_t* hist,
                          uint32_t* part) {
    if (n <= 1) return TDS_OK;
    const uint32_t nblocks = ceil_div(n, kRsTile);
    const uint64_t hlen = (uint64_t)kRadix * nblocks;
    if (hlen >= (1ull << 32)) return TDS_E_INVALID;
    const uint32_t nparts = ceil_div(hlen, kScanTile);
    uint32_t* own_hist = nullptr;
    uint32_t* own_part = nullptr;
    if (!hist) {
        TDS_TRY(dmalloc(&own_hist, hlen));
        hist = own_hist;
    }
    if (!part) {
        if (dmalloc(&own_part, (size_t)nparts + 1) != TDS_OK) {
            dfree(own_hist);
            return TDS_E_NOMEM;
        }
        part = own_part;
    }
    uint64_t* ka = keys;
    uint32_t* va = vals;
    uint64_t* kb = keys_alt;
    uint32_t* vb = vals_alt;
    int status = TDS_OK;
    for (int p = 0; p < 8; ++p) {
        if (!((digit_mask >> p) & 1u)) continue;
        const int shift = 8 * p;
        hipLaunchKernelGGL(rs_hist, dim3(nblocks), dim3(kRsThreads), 0, stream, ka, n, shift, hist,
                           nblocks);
        hipLaunchKernelGGL(rs_scan_part, dim3(nparts), dim3(kScanThreads), 0, stream, hist,
                           (uint32_t)hlen, part);
        hipLaunchKernelGGL(rs_scan_top, dim3(1), dim3(kScanThreads), 0, stream, part, nparts);
        hipLaunchKernelGGL(rs_scan_down, dim3(nparts), dim3(kScanThreads), 0, stream, hist,
                           (uint32_t)hlen, part);
        hipLaunchKernelGGL(rs_scatter, dim3(nblocks), dim3(kRsThreads), 0, stream, ka, va, kb, vb,
                           n, shift, hist, nblocks);
        if (hipGetLastError() != hipSuccess) {
            status = TDS_E_DEVICE;
            break;
        }
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (status == TDS_OK && ka != keys) {
        if (hipMemcpyAsync(keys, ka, (size_t)n * sizeof(uint64_t), hipMemcpyDeviceToDevice, stream) !=
                hipSuccess ||
            hipMemcpyAsync(vals, va, (size_t)n * sizeof(uint32_t), hipMemcpyDeviceToDevice, stream) !=
                hipSuccess)
            status = TDS_E_DEVICE;
    }
    if (own_hist || own_part) {
        // buffers of this call: wait before freeing them
        if (hipStreamSynchronize(stream) != hipSuccess) status = TDS_E_DEVICE;
        dfree(own_hist);
        dfree(own_part);
    }
    return status;
}

int radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                   uint32_t n, int key_bits, hipStream_t stream) {
    const int passes = std::min(8, (key_bits + 7) / 8);
    const uint32_t mask = (passes >= 8) ? 0xFFu : ((1u << passes) - 1u);
    int st = radix_sort_u64_digits(keys, vals, keys_alt, vals_alt, n, mask, stream, nullptr, nullptr);
    if (st == TDS_OK && hipStreamSynchronize(stream) != hipSuccess) st = TDS_E_DEVICE;
    return st;
}

int exclusive_scan_u32(uint32_t* v, uint32_t len, uint32_t* total, hipStream_t stream) {
    return exclusive_scan_u32_with(v, len, total, stream, nullptr);
}

int exclusive_scan_u32_with(uint32_t* v, uint32_t len, uint32_t* total, hipStream_t stream,
                            uint32_t* scratch) {
    if (len == 0) {
        if (total) *total = 0;
        return TDS_OK;
    }
    const uint32_t nparts = ceil_div(len, kScanTile);
    uint32_t* part = scratch;
    if (!part) TDS_TRY(dmalloc(&part, (size_t)nparts + 1));
    hipLaunchKernelGGL(rs_scan_part, dim3(nparts), dim3(kScanThreads), 0, stream, v, len, part);
    hipLaunchKernelGGL(rs_scan_top, dim3(1), dim3(kScanThreads), 0, stream, part, nparts);
    hipLaunchKernelGGL(rs_scan_down, dim3(nparts), dim3(kScanThreads), 0, stream, v, len, part);
    int st = (hipGetLastError() == hipSuccess) ? TDS_OK : TDS_E_DEVICE;
    if (st == TDS_OK && total) {
        if (hipMemcpyAsync(total, part + nparts, sizeof(uint32_t), hipMemcpyDeviceToHost, stream) !=
                hipSuccess ||
            hipStreamSynchronize(stream) != hipSuccess)
            st = TDS_E_DEVICE;
    }
    if (!total && hipStreamSynchronize(stream) != hipSuccess) st = TDS_E_DEVICE;
    if (!scratch) dfree(part);
    return st;
}

}  // namespace tds
