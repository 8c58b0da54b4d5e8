// Batcher: fixed-capacity batched search replayed from a captured hipGraph
// (implementation in batch.hip).
#pragma once

#include <chrono>

#include "tds_internal.hpp"

namespace tds {

class Batcher {
public:
    ~Batcher();
    int init(tds_index* idx, uint64_t max_q, uint32_t max_r, uint64_t res_cap,
             const tds_search_params* params, hipStream_t stream);
    // Copies the query segments into the staging buffers (host arrays into
    // pinned memory, device arrays into the device buffers).
    int stage(const tds_segments* Q);
    // Pinned staging of host query arrays, for callers that fill it directly:
    // array k (xs, ys, zs, ts, xe, ye, ze, te) holds max_q() doubles.
    double* host_array(int k) { return hq_ + (size_t)k * max_q_; }
    uint32_t* host_traj() { return htraj_; }
    void mark_host_staged() { staged_on_device_ = false; }
    // Enqueues one batch: copies in, graph replay, copies out; returns
    // without waiting.
    int launch(uint64_t nq, const tds_request* reqs, uint32_t nreq);
    bool ready() const;
    // Waits for the batch and reads the per-request totals.
    int finish(uint64_t* counts, tds_stats* stats, bool* table_overflow);
    // Copies each request's records into out (after finish).
    int copy_out(tds_result* out, const uint64_t* counts);
    // Records of the batch in pinned memory, at their requests' offsets
    // (after finish, copy_all mode: the counted records of each request).
    const tds_result* host_results() const { return hres_; }
    int run(const tds_segments* Q, const tds_request* reqs, uint32_t nreq, tds_result* out,
            uint64_t* counts, tds_stats* stats);
    void set_copy_all(bool v) { copy_all_ = v; }
    uint64_t replays() const { return replays_; }
    uint64_t max_q() const { return max_q_; }
    uint32_t max_r() const { return max_r_; }
    uint64_t res_cap() const { return res_cap_; }
    hipStream_t stream() const { return stream_; }
    const PipelineConfig& config() const { return cfg_; }

private:
    tds_index* idx_ = nullptr;
    Workspace* w_ = nullptr;
    hipStream_t stream_ = nullptr;
    bool own_stream_ = false;
    hipEvent_t done_ = nullptr;
    PipelineConfig cfg_{};
    uint64_t max_q_ = 0, res_cap_ = 0, item_cap_ = 0, nq_ = 0, used_ = 0, replays_ = 0;
    uint32_t max_r_ = 0, nreq_ = 0;
    double* dq_ = nullptr;
    uint32_t* dtraj_ = nullptr;
    tds_result* dres_ = nullptr;
    double* hq_ = nullptr;        // mapped pinned host memory: staged query arrays
    uint32_t* htraj_ = nullptr;
    double* hq_dev_ = nullptr;    // hq_ and htraj_ as the device sees them
    uint32_t* htraj_dev_ = nullptr;
    Request* hreq_ = nullptr;     // in the workspace's pinned control block
    ReqCounter* hrc_ = nullptr;   // (owned by the workspace)
    tds_result* hres_ = nullptr;
    tds_result* hres_dev_ = nullptr;  // hres_ as the device sees it
    bool staged_on_device_ = false;
    bool copy_all_ = false;
    hipGraph_t graph_ = nullptr;
    hipGraphExec_t exec_ = nullptr;
    std::chrono::steady_clock::time_point t0_;
};

}  // namespace tds

struct tds_batcher {
    tds::Batcher impl;
    int device = 0;
};
