// Batched search with a captured launch sequence (tds_batcher) and the
// serving loop built on it (tds_server).
//
// A Batcher owns one workspace shaped for fixed capacities (query segments,
// requests, result records), pinned host staging, and one hipGraph holding
// the whole fixed-shape launch sequence of a search (clear, query
// preparation, bucketing, ordering, item table, persistent distance kernel).
// Sizes travel in device memory, so the graph is captured on the first batch
// and replayed for every later one.  Copies in and out stay outside the
// graph.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unordered_map>

#include "batch.hpp"

namespace tds {

// Host threads of the serving loop's host route (tds_server_params.cpu_route_tests),
// and the requests that may wait for them: beyond that a request the cost
// model sends to the host goes to the GPU batches instead, so that a burst
// is absorbed by the GPU rather than queued behind the host threads.
constexpr uint32_t kHostRouteThreads = 4;
constexpr uint32_t kHostRouteQueue = 2 * kHostRouteThreads;

namespace {

// Copies the counted records of each request of a batch (at most its
// capacity) from the device result buffer to the same positions of the pinned
// host buffer, which the kernel writes directly: a batch's reservations are
// sized before its counts are known, so one copy of the reserved ranges moves
// mostly unused records.  Workgroup b takes requests b, b + grid, ...; a
// record is two 16-byte stores.
__global__ __launch_bounds__(256) void k_copy_counted(const Request* __restrict__ req,
                                                      const ReqCounter* __restrict__ rc,
                                                      uint32_t nreq,
                                                      const tds_result* __restrict__ src,
                                                      tds_result* __restrict__ dst) {
    for (uint32_t r = blockIdx.x; r < nreq; r += gridDim.x) {
        const Request R = req[r];
        const uint64_t n = min((uint64_t)rc[r].count, R.out_capacity);
        const uint4* s = reinterpret_cast<const uint4*>(src + R.out_offset);
        uint4* d = reinterpret_cast<uint4*>(dst + R.out_offset);
        for (uint64_t i = threadIdx.x; i < 2 * n; i += blockDim.x) d[i] = s[i];
    }
}

// Host-staged query segments to the device: each thread moves segment i's
// eight values and trajectory id from the mapped host arrays (array k of
// either side at k * max_q).  A kernel rather than copy calls, so that
// queueing a batch makes no copy request of the runtime's (their first uses
// under load blocked the host for several ms).
__global__ __launch_bounds__(256) void k_stage_in(const double* __restrict__ hq,
                                                  const uint32_t* __restrict__ htraj,
                                                  double* __restrict__ dq,
                                                  uint32_t* __restrict__ dtraj, uint64_t nq,
                                                  uint64_t max_q) {
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < nq;
         i += (uint64_t)gridDim.x * 256) {
#pragma unroll
        for (int k = 0; k < 8; ++k) dq[k * max_q + i] = hq[k * max_q + i];
        dtraj[i] = htraj[i];
    }
}

}  // namespace


Batcher::~Batcher() {
    if (exec_) (void)hipGraphExecDestroy(exec_);
    if (graph_) (void)hipGraphDestroy(graph_);
    delete w_;
    dfree(dq_);
    dfree(dtraj_);
    dfree(dres_);
    if (hq_) (void)hipHostFree(hq_);
    if (htraj_) (void)hipHostFree(htraj_);
    if (hres_) (void)hipHostFree(hres_);
    if (done_) (void)hipEventDestroy(done_);
    if (own_stream_ && stream_) (void)hipStreamDestroy(stream_);
}

int Batcher::init(tds_index* idx, uint64_t max_q, uint32_t max_r, uint64_t res_cap,
                  const tds_search_params* params, hipStream_t stream) {
    if (!idx || max_q == 0 || max_r == 0 || res_cap == 0 || max_q >= 0xFFFFFFFFull)
        return TDS_E_INVALID;
    TDS_TRY(resolve_config(params, &cfg_));
    idx_ = idx;
    max_q_ = max_q;
    max_r_ = max_r;
    res_cap_ = res_cap;
    if (stream) {
        stream_ = stream;
    } else {
        TDS_HIP(hipStreamCreateWithFlags(&stream_, hipStreamNonBlocking));
        own_stream_ = true;
    }
    TDS_HIP(hipEventCreateWithFlags(&done_, hipEventDisableTiming));
    w_ = new (std::nothrow) Workspace();
    if (!w_) return TDS_E_NOMEM;
    w_->device = idx->device;
    TDS_TRY(ws_init(w_));
    TDS_TRY(ws_reserve(w_, max_q, max_r));
    TDS_TRY(ws_reserve_stage(w_, cfg_.grid_waves));
    item_cap_ = std::min<uint64_t>(item_table_bound(idx, max_q, cfg_.chunk), 1ull << 28);
    TDS_TRY(dmalloc(&w_->item_bucket, std::max<uint64_t>(item_cap_, 1)));
    w_->item_bucket_cap = std::max<uint64_t>(item_cap_, 1);
    TDS_TRY(dmalloc(&w_->item_count, std::max<uint64_t>(item_cap_, 1)));
    w_->item_cap = std::max<uint64_t>(item_cap_, 1);
    TDS_TRY(dmalloc(&dq_, 8 * max_q));
    TDS_TRY(dmalloc(&dtraj_, max_q));
    TDS_TRY(dmalloc(&dres_, res_cap));
    TDS_HIP(hipHostMalloc((void**)&hq_, 8 * max_q * sizeof(double), hipHostMallocMapped));
    TDS_HIP(hipHostMalloc((void**)&htraj_, max_q * sizeof(uint32_t), hipHostMallocMapped));
    TDS_HIP(hipHostGetDevicePointer((void**)&hq_dev_, hq_, 0));
    TDS_HIP(hipHostGetDevicePointer((void**)&htraj_dev_, htraj_, 0));
    hreq_ = w_->req_host;  // the workspace's pinned control block (max_r requests)
    hrc_ = w_->rc_host;
    TDS_HIP(hipHostMalloc((void**)&hres_, res_cap * sizeof(tds_result), hipHostMallocMapped));
    TDS_HIP(hipHostGetDevicePointer((void**)&hres_dev_, hres_, 0));
    return TDS_OK;
}

int Batcher::stage(const tds_segments* Q) {
    TDS_TRY(validate_segments_args(Q));
    if (Q->n > max_q_) return TDS_E_INVALID;
    const double* src[8] = {Q->xs, Q->ys, Q->zs, Q->ts, Q->xe, Q->ye, Q->ze, Q->te};
    if (Q->on_device) {
        for (int k = 0; k < 8; ++k)
            TDS_HIP(hipMemcpyAsync(dq_ + k * max_q_, src[k], Q->n * sizeof(double),
                                   hipMemcpyDeviceToDevice, stream_));
        if (Q->traj_id)
            TDS_HIP(hipMemcpyAsync(dtraj_, Q->traj_id, Q->n * sizeof(uint32_t),
                                   hipMemcpyDeviceToDevice, stream_));
        else
            TDS_HIP(hipMemsetAsync(dtraj_, 0, Q->n * sizeof(uint32_t), stream_));
        staged_on_device_ = true;
    } else {
        for (int k = 0; k < 8; ++k) std::memcpy(hq_ + k * max_q_, src[k], Q->n * sizeof(double));
        if (Q->traj_id) std::memcpy(htraj_, Q->traj_id, Q->n * sizeof(uint32_t));
        else std::memset(htraj_, 0, Q->n * sizeof(uint32_t));
        staged_on_device_ = false;
    }
    return TDS_OK;
}

int Batcher::launch(uint64_t nq, const tds_request* reqs, uint32_t nreq) {
    if (nq == 0 || nq > max_q_ || nreq == 0 || nreq > max_r_) return TDS_E_INVALID;
    TDS_TRY(validate_requests(reqs, nreq, nq, res_cap_));
    nq_ = nq;
    nreq_ = nreq;
    used_ = 0;
    for (uint32_t r = 0; r < nreq; ++r) {
        Request& R = hreq_[r];
        R.q_begin = reqs[r].q_begin;
        R.q_count = reqs[r].q_count;
        R.d = reqs[r].d;
        R.t_start = reqs[r].t_start;
        R.t_end = reqs[r].t_end;
        R.out_offset = reqs[r].out_offset;
        R.out_capacity = reqs[r].out_capacity;
        R.pad = 0;
        used_ = std::max<uint64_t>(used_, reqs[r].out_offset + reqs[r].out_capacity);
    }
    t0_ = std::chrono::steady_clock::now();
    if (!staged_on_device_) {
        const uint32_t blocks = (uint32_t)std::min<uint64_t>((nq + 255) / 256, 1024);
        hipLaunchKernelGGL(k_stage_in, dim3(blocks), dim3(256), 0, stream_, hq_dev_, htraj_dev_,
                           dq_, dtraj_, nq, max_q_);
        TDS_HIP(hipGetLastError());
    }
    BatchDesc* D = w_->desc_host;
    D->nq = nq;
    D->nreq = nreq;
    D->item_cap = (uint32_t)std::min<uint64_t>(item_cap_, 0xFFFFFFFFull);
    TDS_TRY(ws_upload(w_, nreq, stream_));
    if (!exec_) {
        const double* qa[8];
        for (int k = 0; k < 8; ++k) qa[k] = dq_ + k * max_q_;
        TDS_HIP(hipStreamBeginCapture(stream_, hipStreamCaptureModeThreadLocal));
        const int st = enqueue_search(idx_, w_, qa, dtraj_, max_q_, max_r_, cfg_, dres_, stream_);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(stream_, &g);
        if (st != TDS_OK || e != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            (void)hipGetLastError();
            return st != TDS_OK ? st : TDS_E_DEVICE;
        }
        graph_ = g;
        TDS_HIP(hipGraphInstantiate(&exec_, graph_, nullptr, nullptr, 0));
    }
    TDS_HIP(hipGraphLaunch(exec_, stream_));
    ++replays_;
    TDS_TRY(ws_download(w_, nreq, stream_));
    if (copy_all_ && used_) {
        hipLaunchKernelGGL(k_copy_counted, dim3(std::min<uint32_t>(nreq, 1024u)), dim3(256), 0,
                           stream_, w_->req, w_->req_ctr, nreq, dres_, hres_dev_);
        TDS_HIP(hipGetLastError());
    }
    TDS_HIP(hipEventRecord(done_, stream_));
    return TDS_OK;
}

bool Batcher::ready() const { return hipEventQuery(done_) == hipSuccess; }

int Batcher::finish(uint64_t* counts, tds_stats* stats, bool* table_overflow) {
    TDS_HIP(hipEventSynchronize(done_));
    const SearchHeader h = *w_->hdr_host;
    *table_overflow = (h.err & 2u) != 0;
    if (h.err & 1u) return TDS_E_INVALID;
    int status = TDS_OK;
    uint64_t total = 0;
    for (uint32_t r = 0; r < nreq_; ++r) {
        counts[r] = hrc_[r].count;
        total += hrc_[r].count;
        if (hrc_[r].count > hreq_[r].out_capacity) status = TDS_E_OVERFLOW;
    }
    if (stats) {
        tds_stats st{};
        st.query_segments = nq_;
        st.active_segments = h.active;
        st.work_items = h.n_items;
        st.candidate_tests = h.tests;
        st.filter_tests = h.ftests;
        st.block_tests = h.btests;
        st.fp64_evals = h.evals;
        st.stage_flushes = h.flushes;
        st.results = total;
        st.passes = 1;
        st.total_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() -
                                                                t0_)
                          .count();
        *stats = st;
    }
    return status;
}

int Batcher::copy_out(tds_result* out, const uint64_t* counts) {
    for (uint32_t r = 0; r < nreq_; ++r) {
        const uint64_t k = std::min<uint64_t>(counts[r], hreq_[r].out_capacity);
        if (!k) continue;
        if (copy_all_) {
            std::memcpy(out + hreq_[r].out_offset, hres_ + hreq_[r].out_offset,
                        k * sizeof(tds_result));
        } else {
            TDS_HIP(hipMemcpyAsync(out + hreq_[r].out_offset, dres_ + hreq_[r].out_offset,
                                   k * sizeof(tds_result), hipMemcpyDeviceToHost, stream_));
        }
    }
    if (!copy_all_) TDS_HIP(hipStreamSynchronize(stream_));
    return TDS_OK;
}

int Batcher::run(const tds_segments* Q, const tds_request* reqs, uint32_t nreq, tds_result* out,
                 uint64_t* counts, tds_stats* stats) {
    if (!out || !counts) return TDS_E_INVALID;
    TDS_TRY(stage(Q));
    TDS_TRY(launch(Q->n, reqs, nreq));
    bool overflowed = false;
    const int st = finish(counts, stats, &overflowed);
    if (overflowed) {
        // the fixed item table was too small for this batch: run it through
        // the exactly sized path instead
        tds_search_params P;
        tds_search_params_default(&P);
        P.precision = cfg_.prec;
        P.chunk = cfg_.chunk;
        P.grid_waves = cfg_.grid_waves;
        return batch_impl(idx_, Q, reqs, nreq, out, res_cap_, counts, &P, stream_, stats);
    }
    if (st != TDS_OK && st != TDS_E_OVERFLOW) return st;
    TDS_TRY(copy_out(out, counts));
    return st;
}

// ------------------------------------------------------------ serving loop

struct ServerTicket {
    uint64_t id = 0;
    uint64_t L = 0;             // query segments
    std::vector<double> q;      // 8 arrays of L doubles (xs .. te)
    std::vector<uint32_t> traj; // L ids, or empty (ids 0)
    double d = 0, t0 = 0, t1 = 0;
    uint64_t reserve = 0;
    std::chrono::steady_clock::time_point submit, done;
    std::vector<tds_result> results;
    uint64_t count = 0;
    int status = TDS_OK;
    bool finished = false;
    bool solo = false;          // next batch: this request alone (item table overflowed)
    bool cpu = false;           // routed to the host search
};

struct ServerSlot {
    Batcher b;
    std::vector<ServerTicket*> batch;
    std::vector<tds_request> reqs;
    std::vector<uint64_t> counts;
    bool busy = false;
};

}  // namespace tds

struct tds_server {
    tds_index* idx = nullptr;
    int device = 0;
    tds_server_params P{};
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::deque<tds::ServerTicket*> pending;
    std::unordered_map<uint64_t, tds::ServerTicket*> tickets;
    std::vector<std::unique_ptr<tds::ServerSlot>> slots;
    std::thread worker;
    // host route: requests with few candidate pairs run on host threads
    std::unique_ptr<tds::HostIndex> host;
    std::deque<tds::ServerTicket*> cpu_pending;
    std::condition_variable cv_cpu;
    std::vector<std::thread> cpu_workers;
    bool stop = false;
    uint64_t next_id = 1;
    tds_server_stats stats{};
    void run();
    void cpu_run();
    int run_exact(tds::ServerTicket* t);
};

// Host-route worker: searches queued small requests on the host copy of the
// index, one at a time, until the server stops and its queue is empty.
void tds_server::cpu_run() {
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        cv_cpu.wait(lk, [&] { return stop || !cpu_pending.empty(); });
        if (cpu_pending.empty()) break;  // stopping
        tds::ServerTicket* t = cpu_pending.front();
        cpu_pending.pop_front();
        lk.unlock();
        std::vector<tds_result> r;
        tds::host_search(*host, t->q.data(), t->traj.empty() ? nullptr : t->traj.data(), t->L,
                         t->d, t->t0, t->t1, &r);
        lk.lock();
        t->count = r.size();
        t->results = std::move(r);
        t->status = TDS_OK;
        t->finished = true;
        t->done = std::chrono::steady_clock::now();
        ++stats.completed;
        ++stats.cpu_routed;
        cv_done.notify_all();
    }
}

// One request through tds_search's path (work-item table sized exactly),
// results into the ticket; called by the worker without the lock.
int tds_server::run_exact(tds::ServerTicket* t) {
    tds_segments Q{};
    const uint64_t L = t->L;
    Q.xs = t->q.data();
    Q.ys = t->q.data() + L;
    Q.zs = t->q.data() + 2 * L;
    Q.ts = t->q.data() + 3 * L;
    Q.xe = t->q.data() + 4 * L;
    Q.ye = t->q.data() + 5 * L;
    Q.ze = t->q.data() + 6 * L;
    Q.te = t->q.data() + 7 * L;
    Q.traj_id = t->traj.empty() ? nullptr : t->traj.data();
    Q.n = L;
    Q.on_device = 0;
    tds_search_params sp = P.search;
    sp.out_on_device = 0;
    uint64_t cap = std::max<uint64_t>(t->reserve, 1);
    for (int attempt = 0; attempt < 2; ++attempt) {
        t->results.resize(cap);
        uint64_t n = 0;
        const int st = tds::search_impl(idx, &Q, t->d, t->t0, t->t1, t->results.data(), cap, &n,
                                        &sp, nullptr, nullptr);
        if (st == TDS_OK) {
            t->results.resize(n);
            t->count = n;
            return TDS_OK;
        }
        if (st != TDS_E_OVERFLOW) return st;
        cap = n;
    }
    return TDS_E_DEVICE;
}

namespace tds {

namespace {

void finish_ticket(tds_server* S, ServerTicket* t, int status) {
    t->status = status;
    t->finished = true;
    t->done = std::chrono::steady_clock::now();
    if (status == TDS_OK) ++S->stats.completed;
    else ++S->stats.failed;
}

// One empty batch on a slot before the server takes requests: its graph is
// captured and instantiated and its stream gets a hardware queue then, not
// while requests wait (a second slot is first needed only under load, and
// that first use stalled the requests queued behind it for several ms).
// The batch is one segment on [0, 1] searched in the window [2, 3]: its
// clipped extent is empty, so it has no candidates and no results; its
// one-record output slice makes the launch include the copy of the counted
// records, as a serving batch's does.
int warm_slot(Batcher& b) {
    for (int k = 0; k < 8; ++k) b.host_array(k)[0] = (k == 7) ? 1.0 : 0.0;  // ts = 0, te = 1
    b.host_traj()[0] = 0u;
    b.mark_host_staged();
    tds_request r{};
    r.q_begin = 0;
    r.q_count = 1;
    r.d = 0.0;
    r.t_start = 2.0;
    r.t_end = 3.0;
    r.out_offset = 0;
    r.out_capacity = 1;
    TDS_TRY(b.launch(1, &r, 1));
    uint64_t count = 0;
    bool table_overflow = false;
    return b.finish(&count, nullptr, &table_overflow);
}

}  // namespace

}  // namespace tds

// Worker: completes finished batches, forms and launches new ones on free
// slots, and sleeps only when there is nothing to do.
void tds_server::run() {
    using namespace tds;
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    std::vector<ServerTicket*> requeue, exact;
    for (;;) {
        bool progressed = false;
        // completions
        for (auto& sp : slots) {
            ServerSlot& sl = *sp;
            if (!sl.busy || !sl.b.ready()) continue;
            lk.unlock();
            bool table_overflow = false;
            const int st = sl.b.finish(sl.counts.data(), nullptr, &table_overflow);
            lk.lock();
            const tds_result* hr = sl.b.host_results();
            for (size_t i = 0; i < sl.batch.size(); ++i) {
                ServerTicket* t = sl.batch[i];
                const uint64_t c = sl.counts[i];
                if (table_overflow || (st != TDS_OK && st != TDS_E_OVERFLOW)) {
                    if (table_overflow && t->solo) {
                        exact.push_back(t);  // alone and still too large
                    } else if (table_overflow) {
                        // retried alone; alone and still too large, it runs
                        // through the exactly sized path
                        t->solo = true;
                        requeue.push_back(t);
                        ++stats.requeued;
                    } else {
                        finish_ticket(this, t, st);
                    }
                } else if (c <= sl.reqs[i].out_capacity) {
                    const tds_result* src = hr + sl.reqs[i].out_offset;
                    t->results.assign(src, src + c);
                    t->count = c;
                    finish_ticket(this, t, TDS_OK);
                } else {
                    t->reserve = c;  // exact size now known
                    requeue.push_back(t);
                    ++stats.requeued;
                }
            }
            // back to the front of the queue, in their order
            for (auto it = requeue.rbegin(); it != requeue.rend(); ++it) pending.push_front(*it);
            requeue.clear();
            // a request whose work items alone exceed the batcher's fixed item
            // table runs through the exactly sized search path
            for (ServerTicket* t : exact) {
                lk.unlock();
                const int est = run_exact(t);
                lk.lock();
                finish_ticket(this, t, est);
            }
            exact.clear();
            sl.batch.clear();
            sl.busy = false;
            progressed = true;
            cv_done.notify_all();
        }
        // launches
        for (auto& sp : slots) {
            ServerSlot& sl = *sp;
            if (sl.busy || pending.empty()) continue;
            sl.batch.clear();
            sl.reqs.clear();
            uint64_t segs = 0, res = 0;
            while (!pending.empty()) {
                ServerTicket* t = pending.front();
                if (t->reserve > sl.b.res_cap()) {
                    pending.pop_front();
                    finish_ticket(this, t, TDS_E_NOMEM);
                    cv_done.notify_all();
                    continue;
                }
                if (t->solo && !sl.batch.empty()) break;  // it goes alone
                if (sl.batch.size() == sl.b.max_r() || segs + t->L > sl.b.max_q() ||
                    res + t->reserve > sl.b.res_cap())
                    break;
                pending.pop_front();
                tds_request rq;
                rq.q_begin = segs;
                rq.q_count = t->L;
                rq.d = t->d;
                rq.t_start = t->t0;
                rq.t_end = t->t1;
                rq.out_offset = res;
                rq.out_capacity = t->reserve;
                sl.batch.push_back(t);
                sl.reqs.push_back(rq);
                segs += t->L;
                res += t->reserve;
                if (t->solo) break;
            }
            if (sl.batch.empty()) continue;
            stats.max_batch_requests_seen =
                std::max<uint64_t>(stats.max_batch_requests_seen, sl.batch.size());
            lk.unlock();
            uint64_t off = 0;
            for (ServerTicket* t : sl.batch) {
                for (int k = 0; k < 8; ++k)
                    std::memcpy(sl.b.host_array(k) + off, t->q.data() + (size_t)k * t->L,
                                t->L * sizeof(double));
                if (t->traj.empty()) std::memset(sl.b.host_traj() + off, 0, t->L * sizeof(uint32_t));
                else std::memcpy(sl.b.host_traj() + off, t->traj.data(), t->L * sizeof(uint32_t));
                off += t->L;
            }
            sl.b.mark_host_staged();
            sl.counts.assign(sl.batch.size(), 0);
            const int st = sl.b.launch(segs, sl.reqs.data(), (uint32_t)sl.reqs.size());
            lk.lock();
            if (st != TDS_OK) {
                for (ServerTicket* t : sl.batch) finish_ticket(this, t, st);
                sl.batch.clear();
                cv_done.notify_all();
            } else {
                sl.busy = true;
                ++stats.batches;
            }
            progressed = true;
        }
        bool any_busy = false;
        for (auto& sp : slots) any_busy = any_busy || sp->busy;
        if (stop && pending.empty() && !any_busy) break;
        if (!progressed) {
            if (any_busy) {
                lk.unlock();
                std::this_thread::sleep_for(std::chrono::microseconds(10));
                lk.lock();
            } else {
                cv_work.wait(lk, [&] { return stop || !pending.empty(); });
            }
        }
    }
}

extern "C" {

int tds_search_batch(const tds_index* index, const tds_segments* Q, const tds_request* reqs,
                     uint32_t nreq, tds_result* out, uint64_t out_capacity, uint64_t* counts,
                     const tds_search_params* params, void* stream, tds_stats* stats) {
    if (!index) return TDS_E_INVALID;
    tds::DeviceGuard g(index->device);
    if (!g.ok) return TDS_E_DEVICE;
    return tds::batch_impl(const_cast<tds_index*>(index), Q, reqs, nreq, out, out_capacity, counts,
                           params, (hipStream_t)stream, stats);
}

int tds_batcher_create(const tds_index* index, uint64_t max_segments, uint32_t max_requests,
                       uint64_t result_capacity, const tds_search_params* params, void* stream,
                       tds_batcher** out) {
    if (!out || !index) return TDS_E_INVALID;
    *out = nullptr;
    tds::DeviceGuard g(index->device);
    if (!g.ok) return TDS_E_DEVICE;
    tds_batcher* b = new (std::nothrow) tds_batcher();
    if (!b) return TDS_E_NOMEM;
    const int st = b->impl.init(const_cast<tds_index*>(index), max_segments, max_requests,
                                result_capacity, params, (hipStream_t)stream);
    if (st != TDS_OK) {
        delete b;
        return st;
    }
    b->device = index->device;
    *out = b;
    return TDS_OK;
}

int tds_batcher_run(tds_batcher* b, const tds_segments* Q, const tds_request* reqs, uint32_t nreq,
                    tds_result* out, uint64_t* counts, tds_stats* stats) {
    if (!b) return TDS_E_INVALID;
    tds::DeviceGuard g(b->device);
    if (!g.ok) return TDS_E_DEVICE;
    return b->impl.run(Q, reqs, nreq, out, counts, stats);
}

uint64_t tds_batcher_replays(const tds_batcher* b) { return b ? b->impl.replays() : 0; }

int tds_batcher_destroy(tds_batcher* b) {
    if (!b) return TDS_OK;
    tds::DeviceGuard g(b->device);
    delete b;
    return TDS_OK;
}

}  // extern "C"

extern "C" {

int tds_server_create(const tds_index* index, const tds_server_params* params, tds_server** out) {
    if (!index || !out) return TDS_E_INVALID;
    *out = nullptr;
    tds::DeviceGuard g(index->device);
    if (!g.ok) return TDS_E_DEVICE;
    tds_server_params P{};
    if (params) P = *params;
    else tds_search_params_default(&P.search);
    if (!P.max_batch_segments) P.max_batch_segments = 262144;
    if (!P.max_batch_requests) P.max_batch_requests = 4096;
    if (!P.slots) P.slots = 2;
    if (!P.result_capacity) P.result_capacity = 1ull << 21;
    if (!P.default_reserve) P.default_reserve = 1024;
    if (!P.max_pending) P.max_pending = 1u << 20;
    if (P.slots > 8) return TDS_E_INVALID;
    P.search.out_on_device = 0;
    tds_server* S = new (std::nothrow) tds_server();
    if (!S) return TDS_E_NOMEM;
    S->idx = const_cast<tds_index*>(index);
    S->device = index->device;
    S->P = P;
    for (uint32_t i = 0; i < P.slots; ++i) {
        auto sl = std::make_unique<tds::ServerSlot>();
        const int st = sl->b.init(S->idx, P.max_batch_segments, P.max_batch_requests,
                                  P.result_capacity, &P.search, nullptr);
        if (st != TDS_OK) {
            delete S;
            return st;
        }
        sl->b.set_copy_all(true);
        const int wst = tds::warm_slot(sl->b);
        if (wst != TDS_OK) {
            delete S;
            return wst;
        }
        S->slots.push_back(std::move(sl));
    }
    if (P.cpu_route_tests) {
        S->host = std::make_unique<tds::HostIndex>();
        const int st = tds::host_index_load(S->idx, S->host.get());
        if (st != TDS_OK) {
            delete S;
            return st;
        }
        for (uint32_t i = 0; i < tds::kHostRouteThreads; ++i)
            S->cpu_workers.emplace_back([S] { S->cpu_run(); });
    }
    S->worker = std::thread([S] { S->run(); });
    *out = S;
    return TDS_OK;
}

int tds_server_submit(tds_server* S, const tds_segments* Q, double d, double t_start,
                      double t_end, uint64_t reserve, int blocking, uint64_t* ticket) {
    if (!S || !ticket) return TDS_E_INVALID;
    if (tds::validate_segments_args(Q) != TDS_OK || Q->on_device) return TDS_E_INVALID;
    if (Q->n > S->P.max_batch_segments) return TDS_E_INVALID;
    if (!(d >= 0.0) || std::isinf(d) || !(t_start < t_end)) return TDS_E_INVALID;
    auto* t = new (std::nothrow) tds::ServerTicket();
    if (!t) return TDS_E_NOMEM;
    t->L = Q->n;
    t->q.resize(8 * Q->n);
    const double* src[8] = {Q->xs, Q->ys, Q->zs, Q->ts, Q->xe, Q->ye, Q->ze, Q->te};
    for (int k = 0; k < 8; ++k) std::memcpy(t->q.data() + (size_t)k * Q->n, src[k], Q->n * sizeof(double));
    // the values are checked here, where they were copied: a bad segment would
    // otherwise fail the whole batch it joins, other clients' requests included
    for (size_t i = 0; i < 8 * (size_t)Q->n; ++i) {
        if (!std::isfinite(t->q[i])) {
            delete t;
            return TDS_E_INVALID;
        }
    }
    for (uint64_t i = 0; i < Q->n; ++i) {
        if (!(t->q[7 * Q->n + i] > t->q[3 * Q->n + i])) {  // te > ts
            delete t;
            return TDS_E_INVALID;
        }
    }
    if (Q->traj_id) t->traj.assign(Q->traj_id, Q->traj_id + Q->n);
    t->d = d;
    t->t0 = t_start;
    t->t1 = t_end;
    t->reserve = reserve ? reserve : S->P.default_reserve;
    // host route: a request with few candidate pairs (the cost model: the
    // pairs of its candidate ranges, which the host search prunes with the
    // block boxes) is searched on the host
    if (S->host)
        t->cpu = tds::host_candidates(*S->host, t->q.data(), t->L, t_start, t_end,
                                      S->P.cpu_route_tests) <= S->P.cpu_route_tests;
    std::unique_lock<std::mutex> lk(S->mu);
    auto queued = [&] { return S->pending.size() + S->cpu_pending.size(); };
    if (queued() >= S->P.max_pending) {
        if (!blocking) {
            delete t;
            return TDS_E_BUSY;
        }
        S->cv_done.wait(lk, [&] { return queued() < S->P.max_pending; });
    }
    t->id = S->next_id++;
    t->submit = std::chrono::steady_clock::now();
    S->tickets[t->id] = t;
    ++S->stats.submitted;
    *ticket = t->id;
    if (t->cpu && S->cpu_pending.size() >= tds::kHostRouteQueue) t->cpu = false;  // host busy
    if (t->cpu) {
        S->cpu_pending.push_back(t);
        S->cv_cpu.notify_one();
    } else {
        S->pending.push_back(t);
        S->cv_work.notify_one();
    }
    return TDS_OK;
}

int tds_server_poll(tds_server* S, uint64_t ticket, int* done) {
    if (!S || !done) return TDS_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return TDS_E_INVALID;
    *done = it->second->finished ? 1 : 0;
    return TDS_OK;
}

int tds_server_wait(tds_server* S, uint64_t ticket, tds_result* out, uint64_t capacity,
                    uint64_t* n_out, double* latency_ms) {
    if (!S) return TDS_E_INVALID;
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->tickets.find(ticket);
    if (it == S->tickets.end()) return TDS_E_INVALID;
    tds::ServerTicket* t = it->second;
    S->cv_done.wait(lk, [&] { return t->finished; });
    if (n_out) *n_out = t->count;
    if (latency_ms)
        *latency_ms = std::chrono::duration<double, std::milli>(t->done - t->submit).count();
    int st = t->status;
    if (st == TDS_OK) {
        if (t->count > capacity || (t->count && !out)) return TDS_E_OVERFLOW;
        if (t->count) std::memcpy(out, t->results.data(), t->count * sizeof(tds_result));
    }
    S->tickets.erase(it);
    delete t;
    return st;
}

int tds_server_stats_get(tds_server* S, tds_server_stats* stats) {
    if (!S || !stats) return TDS_E_INVALID;
    std::lock_guard<std::mutex> lk(S->mu);
    *stats = S->stats;
    return TDS_OK;
}

int tds_server_destroy(tds_server* S) {
    if (!S) return TDS_OK;
    {
        std::lock_guard<std::mutex> lk(S->mu);
        S->stop = true;
    }
    S->cv_work.notify_all();
    S->cv_cpu.notify_all();
    if (S->worker.joinable()) S->worker.join();
    for (auto& th : S->cpu_workers)
        if (th.joinable()) th.join();
    tds::DeviceGuard g(S->device);
    for (auto& kv : S->tickets) delete kv.second;
    S->tickets.clear();
    S->slots.clear();
    delete S;
    return TDS_OK;
}

}  // extern "C"
