// tds_search_noalloc: the search of tds_search for callers that cannot
// allocate device or pinned memory.  Every buffer the search kernels need
// beyond the caller's inputs and outputs (query records, bucket tables, the
// work-item table, the control block, per-workgroup counters and the result
// stages) is carved from one file-scope device array, `scratch`, whose
// device address is looked up once per device.
#include <chrono>
#include <cmath>
#include <mutex>

#include "tds_internal.hpp"

namespace tds {

namespace {

// Limits of one call (the carved buffers are sized for them).
constexpr uint64_t kNaMaxQuery = 65536;       // query segments
constexpr uint32_t kNaGridWaves = 1024;       // distance-kernel waves (256 workgroups)
constexpr uint32_t kNaStagePerWave = 256;     // result-stage records per wave
constexpr uint64_t kNaItems = 1ull << 19;     // work-item table entries
constexpr size_t kAlign = 256;

constexpr size_t up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

// Byte offsets of the carved buffers.
struct Carve {
    size_t qfu, qreq, qkey, qslot, qsorted, qf;
    size_t b_count, b_hi, b_start, b_nch, binfo;
    size_t item_bucket, item_count, bstats;
    size_t stage, stage_meta;
    size_t desc, req, hdr, ctr, dyn;
    size_t total;
};

constexpr Carve carve() {
    Carve c{};
    size_t o = 0;
    auto take = [&o](size_t bytes) {
        const size_t at = o;
        o = up(o + bytes);
        return at;
    };
    c.qfu = take(kNaMaxQuery * sizeof(QF32));
    c.qreq = take(kNaMaxQuery * sizeof(uint32_t));
    c.qkey = take(kNaMaxQuery * sizeof(uint32_t));
    c.qslot = take(kNaMaxQuery * sizeof(uint32_t));
    c.qsorted = take(kNaMaxQuery * sizeof(uint32_t));
    c.qf = take((kNaMaxQuery + kQfPad) * sizeof(QF32));
    c.b_count = take(kMaxBuckets * sizeof(uint32_t));
    c.b_hi = take(kMaxBuckets * sizeof(uint32_t));
    c.b_start = take(kMaxBuckets * sizeof(uint32_t));
    c.b_nch = take(kMaxBuckets * sizeof(uint32_t));
    c.binfo = take(kMaxBuckets * sizeof(BucketInfo));
    c.item_bucket = take(kNaItems * sizeof(uint32_t));
    c.item_count = take(kNaItems * sizeof(uint32_t));
    c.bstats = take((kNaGridWaves / kWavesPerBlock) * sizeof(BlockStats));
    c.stage = take((size_t)kNaGridWaves * kNaStagePerWave * sizeof(tds_result));
    c.stage_meta = take((size_t)kNaGridWaves * kNaStagePerWave * sizeof(uint32_t));
    c.desc = take(sizeof(BatchDesc));
    c.req = take(sizeof(Request));
    c.hdr = take(sizeof(SearchHeader));
    c.ctr = take(sizeof(ReqCounter));
    c.dyn = take((size_t)kCtrSlots * kCtrStride * sizeof(unsigned long long));
    c.total = o;
    return c;
}

constexpr Carve kCarve = carve();
constexpr size_t kScratchBytes = 28ull << 20;  // 28 MiB per device
static_assert(kCarve.total <= kScratchBytes, "scratch layout exceeds the array");

// The search's scratch memory on every device the library runs on (held
// until the process ends).  Host code never uses this name as an address:
// the device address comes from hipGetSymbolAddress (scratch_base).
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
char* g_base[kMaxDevices] = {};

// Device address of `scratch` on device dev (current), looked up on the
// first call on that device.
int scratch_base(int dev, char** out) {
    if (dev < 0 || dev >= kMaxDevices) return TDS_E_DEVICE;
    std::lock_guard<std::mutex> g(g_mu);
    if (!g_base[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return TDS_E_DEVICE;
        }
        g_base[dev] = static_cast<char*>(p);
    }
    *out = g_base[dev];
    return TDS_OK;
}

// Writes the batch descriptor and the request (kernel arguments, so no
// host staging memory is needed).
__global__ void k_put_ctl(BatchDesc* desc, BatchDesc dv, Request* req, Request rv) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        *desc = dv;
        *req = rv;
    }
}

// A workspace whose buffers are views into the scratch array: nothing of it
// is freed when it goes out of scope.
struct ScratchWorkspace : Workspace {
    explicit ScratchWorkspace(char* base, int dev) {
        device = dev;
        q_cap = kNaMaxQuery;
        r_cap = 1;
        qfu = reinterpret_cast<QF32*>(base + kCarve.qfu);
        qreq = reinterpret_cast<uint32_t*>(base + kCarve.qreq);
        qkey = reinterpret_cast<uint32_t*>(base + kCarve.qkey);
        qslot = reinterpret_cast<uint32_t*>(base + kCarve.qslot);
        qsorted = reinterpret_cast<uint32_t*>(base + kCarve.qsorted);
        qf = reinterpret_cast<QF32*>(base + kCarve.qf);
        b_count = reinterpret_cast<uint32_t*>(base + kCarve.b_count);
        b_hi = reinterpret_cast<uint32_t*>(base + kCarve.b_hi);
        b_start = reinterpret_cast<uint32_t*>(base + kCarve.b_start);
        b_nch = reinterpret_cast<uint32_t*>(base + kCarve.b_nch);
        binfo = reinterpret_cast<BucketInfo*>(base + kCarve.binfo);
        item_bucket = reinterpret_cast<uint32_t*>(base + kCarve.item_bucket);
        item_bucket_cap = kNaItems;
        item_count = reinterpret_cast<uint32_t*>(base + kCarve.item_count);
        item_cap = kNaItems;
        bstats = reinterpret_cast<BlockStats*>(base + kCarve.bstats);
        stage = reinterpret_cast<tds_result*>(base + kCarve.stage);
        stage_meta = reinterpret_cast<uint32_t*>(base + kCarve.stage_meta);
        stage_recs = (size_t)kNaGridWaves * kNaStagePerWave;
        desc = reinterpret_cast<BatchDesc*>(base + kCarve.desc);
        req = reinterpret_cast<Request*>(base + kCarve.req);
        hdr = reinterpret_cast<SearchHeader*>(base + kCarve.hdr);
        req_ctr = reinterpret_cast<ReqCounter*>(base + kCarve.ctr);
        dyn_ctr = reinterpret_cast<unsigned long long*>(base + kCarve.dyn);
    }
    ~ScratchWorkspace() {
        // views only: leave nothing for ~Workspace to free
        qfu = qf = nullptr;
        qreq = qkey = qslot = qsorted = nullptr;
        b_count = b_hi = b_start = b_nch = nullptr;
        binfo = nullptr;
        item_bucket = item_count = nullptr;
        bstats = nullptr;
        stage = nullptr;
        stage_meta = nullptr;
        desc = nullptr;
        req = nullptr;
        hdr = nullptr;
        req_ctr = nullptr;
        dyn_ctr = nullptr;
    }
};

int search_noalloc_impl(tds_index* idx, const tds_segments* Q, double d, double t_start,
                        double t_end, tds_result* out, uint64_t capacity, uint64_t* n_out,
                        const tds_search_params* params, hipStream_t s, tds_stats* stats) {
    const auto t_begin = std::chrono::steady_clock::now();
    if (!idx || !n_out) return TDS_E_INVALID;
    *n_out = 0;
    TDS_TRY(validate_segments_args(Q));
    if (!Q->on_device || Q->n > kNaMaxQuery) return TDS_E_INVALID;
    if (!(d >= 0.0) || std::isinf(d) || !(t_start < t_end)) return TDS_E_INVALID;
    if (capacity > 0 && !out) return TDS_E_INVALID;
    PipelineConfig cfg;
    TDS_TRY(resolve_config(params, &cfg));
    cfg.grid_waves = std::min(cfg.grid_waves, kNaGridWaves);
    char* base = nullptr;
    TDS_TRY(scratch_base(idx->device, &base));
    ScratchWorkspace w(base, idx->device);

    BatchDesc D{};
    D.nq = Q->n;
    D.nreq = 1;
    D.item_cap = (uint32_t)kNaItems;
    Request R{};
    R.q_begin = 0;
    R.q_count = Q->n;
    R.d = d;
    R.t_start = t_start;
    R.t_end = t_end;
    R.out_offset = 0;
    R.out_capacity = capacity;
    hipLaunchKernelGGL(k_put_ctl, dim3(1), dim3(64), 0, s, w.desc, D, w.req, R);
    TDS_HIP(hipGetLastError());
    const double* qa[8] = {Q->xs, Q->ys, Q->zs, Q->ts, Q->xe, Q->ye, Q->ze, Q->te};
    TDS_TRY(enqueue_search(idx, &w, qa, Q->traj_id, Q->n, 1, cfg, out, s));
    SearchHeader h{};
    ReqCounter rc{};
    TDS_HIP(hipMemcpyAsync(&h, w.hdr, sizeof(h), hipMemcpyDeviceToHost, s));
    TDS_HIP(hipMemcpyAsync(&rc, w.req_ctr, sizeof(rc), hipMemcpyDeviceToHost, s));
    TDS_HIP(hipStreamSynchronize(s));
    if (h.err & 1u) return TDS_E_INVALID;
    if (h.err & 2u) return TDS_E_NOMEM;  // more work items than the scratch table holds
    *n_out = rc.count;
    tds_stats st{};
    st.query_segments = Q->n;
    st.active_segments = h.active;
    st.work_items = h.n_items;
    st.candidate_tests = h.tests;
    st.filter_tests = h.ftests;
    st.block_tests = h.btests;
    st.fp64_evals = h.evals;
    st.stage_flushes = h.flushes;
    st.results = rc.count;
    st.passes = 1;
    st.total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_begin).count();
    if (stats) *stats = st;
    return rc.count > capacity ? TDS_E_OVERFLOW : TDS_OK;
}

}  // namespace

}  // namespace tds

extern "C" int tds_search_noalloc(const tds_index* index, const tds_segments* Q, double d,
                                  double t_start, double t_end, tds_result* out,
                                  uint64_t capacity, uint64_t* n_out,
                                  const tds_search_params* params, void* stream,
                                  tds_stats* stats) {
    if (!index) return TDS_E_INVALID;
    tds::DeviceGuard g(index->device);
    if (!g.ok) return TDS_E_DEVICE;
    return tds::search_noalloc_impl(const_cast<tds_index*>(index), Q, d, t_start, t_end, out,
                                    capacity, n_out, params, (hipStream_t)stream, stats);
}
