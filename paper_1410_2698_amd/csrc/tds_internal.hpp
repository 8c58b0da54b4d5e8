// Internal types of libtds: device record layouts, the index object, the
// per-search workspace and the launch helpers shared by the HIP sources.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "tds.h"

namespace tds {

// ---------------------------------------------------------------- constants

constexpr int kWave = 64;               // CDNA wavefront width
constexpr int kBlock = 256;             // threads per block of the search kernels
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr uint32_t kXcds = 8;            // accelerator complex dies (own L2 each)
constexpr uint32_t kCtrStride = 8;       // 64-bit counters 64 bytes apart (own cache lines)
// counters of the distance kernel: one dynamic item counter per XCD part, and
// the reservation counter of direct output (the last slot)
constexpr uint32_t kCtrSlots = kXcds + 1;
constexpr uint32_t kMaxBins = 65535;
constexpr uint32_t kMaxBuckets = 65536; // query buckets of one search
constexpr uint32_t kSpanClasses = 4;    // bin-span classes per first bin
constexpr uint64_t kDefaultDevCap = 1ull << 24;
constexpr uint32_t kQfPad = 4;          // query records read past a group's end

// ---------------------------------------------------------------- records

// Canonical FP64 entry record, one per indexed segment in index order.
// 64 bytes so that one wave-uniform scalar load brings a whole record.
struct alignas(64) EntryF64 {
    double x, y, z;     // start point
    double vx, vy, vz;  // velocity (P_end - P_start) / (t_end - t_start)
    double ts, te;
};
static_assert(sizeof(EntryF64) == 64, "EntryF64 layout");

// FP32 filter record: bounding sphere of the segment (centre rounded to
// nearest, radius inflated and rounded up) and the time extent rounded
// outwards.  32 bytes: one scalar load.
struct alignas(32) EntryF32 {
    float cx, cy, cz, r;
    float ts, te;       // ts rounded down, te rounded up
    float pad0, pad1;
};
static_assert(sizeof(EntryF32) == 32, "EntryF32 layout");

// FP32 motion of an index entry for the closest-approach refinement of the
// FP32 filter: velocity and the mid time of its extent, each rounded to
// nearest (16 bytes: one vector load per lane).  The sphere centre of its
// EntryF32 record is the position at that time.
struct alignas(16) EntryV32 {
    float vx, vy, vz;
    float tm;
};
static_assert(sizeof(EntryV32) == 16, "EntryV32 layout");

// Box of one aligned block of 64 index entries (spatial layout): the union of
// their segments' boxes (seg_box32), so every position the canonical
// evaluation computes for an entry of the block lies in [lo, hi], margins
// included.  32 bytes: one scalar load.
struct Box32 {
    float lx, ly, lz;  // lower corner
    float hx, hy, hz;  // upper corner
};
struct alignas(32) BlockBox {
    Box32 b;
    float pad0, pad1;
};
static_assert(sizeof(BlockBox) == 32, "BlockBox layout");
constexpr uint32_t kBoxShift = 6;  // log2 of the entries per box (one wave)

// FP32 filter record of a query segment (32 bytes: one wave-uniform scalar
// load), written by the preparation kernel in query order and copied into
// bucket order.  The FP64 data of a query segment is not stored: where it is
// needed (recheck, plain form) it is derived again from the query arrays by
// the same operations.
struct alignas(64) QF32 {
    float cx, cy, cz, R;  // sphere of the clipped segment, R >= r + d + margins
    float a32, b32;       // clipped window rounded outwards
    uint32_t lo, hi;      // candidate range
    Box32 box;            // box of the clipped segment grown by d (seg_box32)
    float pad[2];
};
static_assert(sizeof(QF32) == 64, "QF32 layout");

// Per-bucket work description, written by the bucket scan (64 bytes: one
// scalar load in the distance kernel).
struct alignas(64) BucketInfo {
    uint32_t lo, hi;      // candidate range of the bucket
    uint32_t nch, clen;   // chunks and chunk length
    uint32_t count;       // query segments in the bucket
    uint32_t start;       // their first position in bucket order
    uint32_t item0;       // first work item of the bucket
    uint32_t pad;
    double tmin_te;       // min t_end over the candidate range (-inf: unknown)
    double tmax_ts;       // max t_start over the candidate range (+inf: unknown)
    double pad2[2];
};
static_assert(sizeof(BucketInfo) == 64, "BucketInfo layout");

// One request of a batch: a contiguous slice of the batch's query segments
// with its own distance and window, and its own slice of the result buffer.
struct Request {
    uint64_t q_begin, q_count;
    double d, t_start, t_end;
    uint64_t out_offset, out_capacity;  // slice of the result buffer
    uint64_t pad;
};

// Sizes of the current batch, in device memory so that a captured graph can
// be replayed for batches of any size up to the workspace capacities.
struct alignas(64) BatchDesc {
    uint64_t nq;        // query segments
    uint32_t nreq;      // requests
    uint32_t item_cap;  // capacity of the work-item table
    uint64_t pad[6];
};

// Device-side header of one search; zeroed before every search.
struct alignas(64) SearchHeader {
    uint32_t pad0;
    uint32_t n_items;       // total work items
    uint32_t err;           // input validation failure flag
    uint32_t active;        // active query segments
    uint64_t tests;         // candidate tests executed
    uint64_t evals;         // canonical FP64 evaluations
    uint64_t results;       // total results (all requests)
    uint32_t n_buckets;     // buckets in use
    uint32_t flushes;       // result-stage flushes at the end of a work item
    uint64_t ftests;        // pairs through the FP32 filter / FP64 predicate
    uint64_t btests;        // (query, block) bounding-box tests
};
static_assert(sizeof(SearchHeader) == 64, "SearchHeader layout");

// Per-workgroup counters of the distance kernel, folded into the header by a
// one-block kernel after the launch (no contended atomics).
struct alignas(64) BlockStats {
    uint64_t tests, evals, ftests, btests;
    uint64_t flushes;  // result-stage flushes at the end of a work item
    uint64_t pad[3];
};
constexpr uint32_t kMaxDistBlocks = 16384;  // grid limit of the distance kernel

// Per-request device counters.
struct alignas(16) ReqCounter {
    unsigned long long count;  // results of the request (keeps counting past capacity)
    unsigned long long pad;
};

// ---------------------------------------------------------------- host objects

struct Workspace {
    int device = 0;
    // query-side buffers, sized for `q_cap` query segments and `r_cap` requests
    size_t q_cap = 0, r_cap = 0, item_cap = 0, res_cap = 0;
    QF32* qfu = nullptr;            // filter records in query order
    uint32_t* qreq = nullptr;       // request of each query segment
    uint32_t* qkey = nullptr;
    uint32_t* qslot = nullptr;
    uint32_t* qsorted = nullptr;
    QF32* qf = nullptr;             // q_cap + kQfPad records
    double* qstage = nullptr;       // staging of host query arrays (8 * stage_cap doubles)
    uint32_t* qtraj_stage = nullptr;
    size_t stage_cap = 0, traj_cap = 0;
    // control block, one device allocation and its pinned host mirror, laid
    // out as [desc | req x r_cap | hdr | req_ctr x r_cap]: the batch goes to
    // the device with one copy (desc and requests) and its counters come back
    // with one (header and request counters)
    char* ctl = nullptr;
    char* ctl_host = nullptr;
    Request* req = nullptr;
    ReqCounter* req_ctr = nullptr;
    Request* req_host = nullptr;       // pinned staging of the requests (r_cap)
    ReqCounter* rc_host = nullptr;     // pinned mirror of the request counters (r_cap)
    // bucket tables (kMaxBuckets each)
    uint32_t* b_count = nullptr;    // slot counters, in parts (k_qprep)
    uint32_t* b_hi = nullptr;       // candidate range ends of the members, in parts
    uint32_t* b_start = nullptr;
    uint32_t* b_nch = nullptr;      // work items of each bucket (k_bucket_scan)
    BucketInfo* binfo = nullptr;    // kMaxBuckets
    uint32_t* item_bucket = nullptr; // bucket of every work item
    size_t item_bucket_cap = 0;
    uint32_t* item_count = nullptr; // results per work item (incremental mode)
    tds_result* res = nullptr;      // device result buffer (host-output mode)
    // result stages of the distance kernel's waves (stage_recs records and
    // their metadata, split evenly over the waves of a launch)
    tds_result* stage = nullptr;
    uint32_t* stage_meta = nullptr;
    size_t stage_recs = 0;
    unsigned long long* dyn_ctr = nullptr;  // kCtrSlots counters, kCtrStride apart
    // direct output (one-request searches): each wave's last reservation and
    // the plan of the pass that fills the holes (sized for stage_waves waves)
    uint64_t* dlast = nullptr;
    uint64_t* fill_s = nullptr;      // stage_waves + 2 source prefix sums
    uint64_t* fill_d = nullptr;      // stage_waves + 1 hole prefix sums
    uint64_t* fill_dstart = nullptr; // stage_waves hole starts
    uint64_t* fill_plan = nullptr;   // T, c0, ns, total
    uint32_t stage_waves = 0;
    SearchHeader* hdr = nullptr;
    SearchHeader* hdr_host = nullptr;  // pinned mirror
    BlockStats* bstats = nullptr;      // kMaxDistBlocks per-workgroup counters
    BatchDesc* desc = nullptr;
    BatchDesc* desc_host = nullptr;    // pinned staging of the descriptor
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    ~Workspace();
};

}  // namespace tds

struct tds_index {
    int device = 0;
    uint64_t n = 0;
    uint32_t m = 0;
    double t_min = 0, t_max = 0, bw = 0;
    tds::EntryF64* e64 = nullptr;
    tds::EntryF32* e32 = nullptr;
    tds::EntryV32* ev32 = nullptr; // FP32 velocity and mid time (refinement of the filter)
    uint32_t* seg_id = nullptr;    // index position -> input position
    uint32_t* traj = nullptr;      // index position -> trajectory id
    uint32_t* bin_first = nullptr; // m + 1
    double* min_ts = nullptr;      // m
    double* max_te = nullptr;      // m
    double* min_te = nullptr;      // m: min t_end per bin (+inf when empty)
    double* cmax_te = nullptr;     // m
    double* lo_ts = nullptr;       // m: min t_start over bins >= j (+inf when none)
    double* max_ts = nullptr;      // m: max t_start per bin (-inf when empty)
    tds::BlockBox* bbox = nullptr; // ceil(n / 64) block boxes (spatial layout)
    uint32_t layout = TDS_LAYOUT_TEMPORAL;
    uint64_t device_bytes = 0;
    std::mutex mu;
    std::vector<tds::Workspace*> pool;
    tds_stats last{};
};

// Fixed spatial grid over the entries of an index (fsg.hip).
struct tds_fsg {
    const tds_index* idx = nullptr;
    int device = 0;
    uint32_t g[3] = {1, 1, 1};
    double lo[3] = {0, 0, 0};        // grid origin
    double cw[3] = {1, 1, 1};        // cell widths (0 on a flat axis)
    uint32_t* cell_first = nullptr;  // ncells + 1
    uint32_t* list = nullptr;        // entry positions grouped by cell
    uint64_t nlist = 0;
};

namespace tds {

// Makes a device current for the duration of a call (restores the caller's).
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) {
            (void)hipGetLastError();
            ok = false;
            return;
        }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) {
            (void)hipGetLastError();
            ok = false;
        }
    }
    ~DeviceGuard() {
        if (ok && prev >= 0) (void)hipSetDevice(prev);
    }
};

// Error propagation for HIP calls inside functions returning a TDS status.
#define TDS_HIP(call)                                        \
    do {                                                     \
        hipError_t e_ = (call);                              \
        if (e_ != hipSuccess) {                              \
            (void)hipGetLastError();                         \
            return (e_ == hipErrorOutOfMemory) ? TDS_E_NOMEM \
                                               : TDS_E_DEVICE; \
        }                                                    \
    } while (0)

#define TDS_TRY(call)              \
    do {                           \
        int s_ = (call);           \
        if (s_ != TDS_OK) return s_; \
    } while (0)

template <typename T>
int dmalloc(T** p, size_t count) {
    *p = nullptr;
    if (count == 0) count = 1;
    hipError_t e = hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
    if (e != hipSuccess) {
        (void)hipGetLastError();
        *p = nullptr;
        return e == hipErrorOutOfMemory ? TDS_E_NOMEM : TDS_E_DEVICE;
    }
    return TDS_OK;
}

inline void dfree(void* p) {
    if (p) (void)hipFree(p);
}

inline uint32_t ceil_div(uint64_t a, uint64_t b) { return (uint32_t)((a + b - 1) / b); }

// FP64 -> FP32 conversions rounded to nearest, downwards and upwards (host
// and device code alike): rounded to nearest, then, where that went the
// wrong way, moved to the adjacent float by stepping its encoding (as an
// unsigned integer) by one: away from zero for a float on the side of the
// step, towards zero otherwise, and from zero to the smallest subnormal of
// the step's sign.  Infinities step to the largest finite float; NaN stays.
__host__ __device__ inline float f32_rn(double x) { return (float)x; }
__host__ __device__ inline float f32_step(float f, bool up) {
    uint32_t b = __builtin_bit_cast(uint32_t, f);
    if (f == 0.f) b = up ? 0x00000001u : 0x80000001u;
    else b = ((f > 0.f) == up) ? b + 1u : b - 1u;
    return __builtin_bit_cast(float, b);
}
__host__ __device__ inline float f32_ru(double x) {
    const float f = (float)x;
    return (double)f < x ? f32_step(f, true) : f;
}
__host__ __device__ inline float f32_rd(double x) {
    const float f = (float)x;
    return (double)f > x ? f32_step(f, false) : f;
}

// FP32 bounding sphere of the segment from a to b (FP64 end points), used by
// the FP32 candidate filter: centre rounded to nearest; radius
// (r + extra)(1 + 8u) + 2u|c| + 1e-18 rounded up, u = 2^-24.  The margin
// covers the rounding of both spheres' centres to FP32, the FP32 evaluation
// of the squared centre distance and of (R_q + r_l)^2, and the FP64 rounding
// of the canonical arithmetic, so a pair whose canonical evaluation is a
// result always passes the filter.  Beyond 1e18 the radius is +inf and the
// centre 0 (the pair always passes).
__host__ __device__ inline void sphere32(double ax, double ay, double az, double bx, double by,
                                         double bz, double extra, float& cx32, float& cy32,
                                         float& cz32, float& r32) {
    const double u = 5.9604644775390625e-08;
    const double cx = 0.5 * (ax + bx), cy = 0.5 * (ay + by), cz = 0.5 * (az + bz);
    const double hx = 0.5 * (bx - ax), hy = 0.5 * (by - ay), hz = 0.5 * (bz - az);
    const double rr = sqrt(hx * hx + hy * hy + hz * hz);
    const double cn = sqrt(cx * cx + cy * cy + cz * cz);
    const double R = (rr + extra) * (1.0 + 8.0 * u) + 2.0 * u * cn + 1e-18;
    cx32 = f32_rn(cx);
    cy32 = f32_rn(cy);
    cz32 = f32_rn(cz);
    if (R < 1e18 && cn < 1e18) {
        r32 = f32_ru(R);
    } else {
        // infinite radius, centre at the origin: every distance test against
        // it passes without forming inf - inf
        cx32 = cy32 = cz32 = 0.f;
        r32 = INFINITY;
    }
}

// The FP32 filter of a pair: the bounding spheres of the query (centre c,
// radius R = its own radius + d + margins) and of the entry come within
// reach, and the outward-rounded time extents overlap strictly.  A pair that
// fails cannot be a result of the canonical evaluation (sphere32).
__host__ __device__ inline bool sphere_pass(float cx, float cy, float cz, float R, float ecx,
                                            float ecy, float ecz, float er) {
    const float dx = ecx - cx, dy = ecy - cy, dz = ecz - cz;
    const float s = fmaf(dz, dz, fmaf(dy, dy, dx * dx));
    const float Rr = R + er;
    return s <= Rr * Rr;
}

// Box of the segment from a to b (FP64 end points, as the canonical
// evaluation computes them), grown on every side by extra + the margin
// m = 8u(|h|_1 + extra) + 2u|c|_1 + 1e-18 (u = 2^-24, c the midpoint, h half
// of b - a) and rounded outwards to FP32.  The margin is the one sphere32
// adds to a radius (with L1 norms, which bound the L2 ones).  For a pair that
// the canonical evaluation accepts there is a common time at which the two
// segments' positions lie in their unmargined boxes and are less than d plus
// both margins apart (the slack the sphere test's radii allow), so the
// query's box (extra = d) and the entry's box overlap on every axis.  Unlike
// the sphere test this one spends none of the margin on its own arithmetic
// (outward rounding, exact comparisons).  Beyond 1e18 the box is the whole
// space.
__host__ __device__ inline Box32 seg_box32(double ax, double ay, double az, double bx, double by,
                                           double bz, double extra) {
    const double u = 5.9604644775390625e-08;
    const double cn = fabs(0.5 * (ax + bx)) + fabs(0.5 * (ay + by)) + fabs(0.5 * (az + bz));
    const double hn = fabs(0.5 * (bx - ax)) + fabs(0.5 * (by - ay)) + fabs(0.5 * (bz - az));
    const double m = extra + (8.0 * u) * (hn + extra) + (2.0 * u) * cn + 1e-18;
    if (!(m < 1e18 && cn < 1e18))
        return {-INFINITY, -INFINITY, -INFINITY, INFINITY, INFINITY, INFINITY};
    // the FP64 sum's own rounding (at most 2^-53 of it) moved outwards too
    const auto lo = [m](double a, double b) {
        const double v = fmin(a, b) - m;
        return f32_rd(v - fabs(v) * 0x1p-50);
    };
    const auto hi = [m](double a, double b) {
        const double v = fmax(a, b) + m;
        return f32_ru(v + fabs(v) * 0x1p-50);
    };
    return {lo(ax, bx), lo(ay, by), lo(az, bz), hi(ax, bx), hi(ay, by), hi(az, bz)};
}

// Block culling: the query's box (seg_box32 of the clipped query segment with
// extra = d) and a block box overlap on every axis.  Whenever the canonical
// evaluation accepts a pair of the block, this passes.
__host__ __device__ inline bool box_overlap(const Box32& b, const Box32& q) {
    return (b.lx <= q.hx) & (q.lx <= b.hx) & (b.ly <= q.hy) & (q.ly <= b.hy) & (b.lz <= q.hz) &
           (q.lz <= b.hz);
}

// Stable LSD radix sort of (key, value) pairs on `stream`; keys_bits is the
// number of low key bits that may differ (passes of 8 bits).  Buffers *_alt
// are scratch of the same size; the sorted data ends up in keys/vals.
int radix_sort_u64(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                   uint32_t n, int key_bits, hipStream_t stream);

// The same sort over the 8-bit digits set in digit_mask (bit p: key bits
// 8p..8p+7), e.g. only the digits that differ between keys.  hist
// (radix_hist_len(n) entries) and part (scan_part_len(radix_hist_len(n)))
// are device scratch; when null they are allocated and freed by the call
// (which then waits for the stream).  With caller scratch the call does not
// wait: the sorted data is ready in stream order.
int radix_sort_u64_digits(uint64_t* keys, uint32_t* vals, uint64_t* keys_alt, uint32_t* vals_alt,
                          uint32_t n, uint32_t digit_mask, hipStream_t stream, uint32_t* hist,
                          uint32_t* part);
size_t radix_hist_len(uint32_t n);
size_t scan_part_len(size_t len);

// Device segment staging: copies host arrays to the device when needed.
struct SegView {
    const double* a[8];     // xs, ys, zs, ts, xe, ye, ze, te (device)
    const uint32_t* traj;   // device or nullptr
    uint64_t n;
};

int validate_segments_args(const tds_segments* S);

// Workspace set-up and growth (search.hip).
int ws_init(Workspace* w);
int ws_reserve(Workspace* w, size_t nq, size_t nreq);
// Host copy of an index for the host search (host_search.hip): the entries
// in index order and the tables that give a query's candidate range.
struct HostIndex {
    uint64_t n = 0;
    uint32_t m = 0;
    std::vector<EntryF64> e64;
    std::vector<EntryF32> e32;
    std::vector<BlockBox> bbox;  // spatial layout only
    std::vector<uint32_t> seg_id, traj, bin_first;
    std::vector<double> cmax_te, lo_ts;
};
// Copies the index tables to host memory (waits for the device).
int host_index_load(const tds_index* idx, HostIndex* h);
// The candidate pairs of Q (8 arrays of L values, xs .. te, host memory) in
// the window: over its active query segments, the lengths of their candidate
// ranges (before any spatial pruning); the sum stops growing once it exceeds
// `limit`.  Two bisections per segment: the serving loop's cost model.
uint64_t host_candidates(const HostIndex& h, const double* q, uint64_t L, double t0, double t1,
                         uint64_t limit);
// The search of Q (validated values) on the host; records in query order.
void host_search(const HostIndex& h, const double* q, const uint32_t* qtraj, uint64_t L,
                 double d, double t0, double t1, std::vector<tds_result>* out);

// Sizes the result stages for distance-kernel launches of up to grid_waves
// waves (a resolved value, see resolve_config).
int ws_reserve_stage(Workspace* w, uint32_t grid_waves);
// Copies the batch descriptor and the first nreq requests to the device, and
// the header and the first nreq request counters back (one copy each).
int ws_upload(Workspace* w, uint32_t nreq, hipStream_t s);
int ws_download(Workspace* w, uint32_t nreq, hipStream_t s);

// Batched search and the graph-replaying batcher (search.hip, batch.hip).
int batch_impl(tds_index* idx, const tds_segments* Q, const tds_request* reqs, uint32_t nreq,
               tds_result* out, uint64_t out_capacity, uint64_t* counts,
               const tds_search_params* params, hipStream_t s, tds_stats* stats);
int validate_requests(const tds_request* reqs, uint32_t nreq, uint64_t nq, uint64_t out_cap);

// Pieces of the search pipeline used by the batcher (search.hip).
struct PipelineConfig {
    int prec;
    uint32_t chunk;
    uint32_t grid_waves;
    uint32_t cpl;  // FP32 form: candidates per lane per tile
};
int resolve_config(const tds_search_params* params, PipelineConfig* cfg);
uint64_t item_table_bound(const tds_index* idx, uint64_t nq, uint32_t chunk);
// Enqueues the fixed-shape launch sequence for the batch described by the
// workspace's descriptor and requests; query arrays at qarrays[0..7] (stride
// q_grid doubles apart is not required: any device pointers), traj may be
// nullptr.
int enqueue_search(const tds_index* idx, Workspace* w, const double* const* qarrays,
                   const uint32_t* qtraj, size_t q_grid, uint32_t r_cap,
                   const PipelineConfig& cfg, tds_result* out, hipStream_t s);

// Search implementation (search.hip).
int search_impl(tds_index* idx, const tds_segments* Q, double d, double t_start,
                double t_end, tds_result* out, uint64_t capacity, uint64_t* n_out,
                const tds_search_params* params, hipStream_t stream, tds_stats* stats);
// tds_search_begin / tds_search_end: the pending search is an opaque object
// the library allocates in begin and frees in end.
int search_begin_impl(tds_index* idx, const tds_segments* Q, double d, double t_start,
                      double t_end, tds_result* out, uint64_t capacity,
                      const tds_search_params* params, hipStream_t s, void** pending);
int search_end_impl(void* pending, uint64_t* n_out, tds_stats* stats);
int self_join_impl(tds_index* idx, double d, double t_start, double t_end, tds_result* out,
                   uint64_t capacity, uint64_t* n_out, const tds_search_params* params,
                   hipStream_t s, tds_stats* stats);
// Fixed spatial grid index (fsg.hip).
int fsg_build(const tds_index* idx, uint32_t gx, uint32_t gy, uint32_t gz, hipStream_t s,
              tds_fsg** out);
void fsg_destroy(tds_fsg* f);
int fsg_search(const tds_fsg* f, const tds_segments* Q, double d, double t_start, double t_end,
               tds_result* out, uint64_t capacity, uint64_t* n_out,
               const tds_search_params* params, hipStream_t s, tds_stats* stats);

// Trajectory-level merge of result records (traj_merge.hip).
int merge_impl(const tds_result* recs, uint64_t n, bool recs_dev, tds_traj_interval* out,
               uint64_t capacity, bool out_dev, uint64_t* n_out, hipStream_t s);

// Exclusive scan of len u32 values in place on `stream`; *total (may be
// NULL) receives the sum, which costs a synchronisation (radix_sort.hip).
int exclusive_scan_u32(uint32_t* v, uint32_t len, uint32_t* total, hipStream_t stream);
// The same with caller scratch of scan_part_len(len) entries (null: allocated).
int exclusive_scan_u32_with(uint32_t* v, uint32_t len, uint32_t* total, hipStream_t stream,
                            uint32_t* scratch);

int schedule_impl(tds_index* idx, const tds_segments* Q, double t_start, double t_end,
                  uint32_t* lo, uint32_t* hi, hipStream_t stream);
// Index build implementation (index_build.hip).
int build_impl(const tds_segments* D, const tds_build_params* p, hipStream_t stream,
               tds_index** out);
void destroy_index(tds_index* idx);

}  // namespace tds
