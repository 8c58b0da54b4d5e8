// C ABI of libtds (declared in include/tds.h): argument checks, device
// selection and dispatch to the implementation files.
#include <cmath>

#include "tds_internal.hpp"

using tds::DeviceGuard;

extern "C" {

uint32_t tds_abi_version(void) { return TDS_ABI_VERSION; }

const char* tds_status_str(int status) {
    switch (status) {
        case TDS_OK: return "TDS_OK";
        case TDS_E_INVALID: return "TDS_E_INVALID: invalid argument or input value";
        case TDS_E_OVERFLOW: return "TDS_E_OVERFLOW: more results than the output capacity";
        case TDS_E_NOMEM: return "TDS_E_NOMEM: allocation failed";
        case TDS_E_DEVICE: return "TDS_E_DEVICE: a HIP call failed";
        case TDS_E_BUSY: return "TDS_E_BUSY: admission refused";
        default: return "unknown tds status";
    }
}

void tds_search_params_default(tds_search_params* p) {
    if (!p) return;
    std::memset(p, 0, sizeof(*p));
    p->precision = TDS_PREC_FP32_RECHECK;
}

int tds_build_index(const tds_segments* D, const tds_build_params* params, void* stream,
                    tds_index** out) {
    if (!out) return TDS_E_INVALID;
    *out = nullptr;
    int st = tds::validate_segments_args(D);
    if (st != TDS_OK) return st;
    return tds::build_impl(D, params, (hipStream_t)stream, out);
}

int tds_index_destroy(tds_index* index) {
    if (!index) return TDS_OK;
    tds::destroy_index(index);
    return TDS_OK;
}

int tds_index_info_get(const tds_index* index, tds_index_info* info) {
    if (!index || !info) return TDS_E_INVALID;
    info->n = index->n;
    info->num_bins = index->m;
    info->device = (uint32_t)index->device;
    info->t_min = index->t_min;
    info->t_max = index->t_max;
    info->bin_width = index->bw;
    info->device_bytes = index->device_bytes;
    info->layout = index->layout;
    info->reserved = 0;
    return TDS_OK;
}

int tds_index_export(const tds_index* index, uint32_t* order, uint32_t* bin_first, double* min_ts,
                     double* max_te, double* cmax_te) {
    if (!index) return TDS_E_INVALID;
    DeviceGuard g(index->device);
    if (!g.ok) return TDS_E_DEVICE;
    const size_t n = index->n, m = index->m;
    if (order && hipMemcpy(order, index->seg_id, n * sizeof(uint32_t), hipMemcpyDeviceToHost))
        return TDS_E_DEVICE;
    if (bin_first &&
        hipMemcpy(bin_first, index->bin_first, (m + 1) * sizeof(uint32_t), hipMemcpyDeviceToHost))
        return TDS_E_DEVICE;
    if (min_ts && hipMemcpy(min_ts, index->min_ts, m * sizeof(double), hipMemcpyDeviceToHost))
        return TDS_E_DEVICE;
    if (max_te && hipMemcpy(max_te, index->max_te, m * sizeof(double), hipMemcpyDeviceToHost))
        return TDS_E_DEVICE;
    if (cmax_te && hipMemcpy(cmax_te, index->cmax_te, m * sizeof(double), hipMemcpyDeviceToHost))
        return TDS_E_DEVICE;
    return TDS_OK;
}

int tds_schedule(const tds_index* index, const tds_segments* Q, double t_start, double t_end,
                 uint32_t* lo, uint32_t* hi, void* stream) {
    if (!index) return TDS_E_INVALID;
    DeviceGuard g(index->device);
    if (!g.ok) return TDS_E_DEVICE;
    return tds::schedule_impl(const_cast<tds_index*>(index), Q, t_start, t_end, lo, hi,
                              (hipStream_t)stream);
}

struct tds_pending {
    int device;
    void* impl;  // tds::PendingSearch
};

int tds_search_begin(const tds_index* index, const tds_segments* Q, double d, double t_start,
                     double t_end, tds_result* out, uint64_t capacity,
                     const tds_search_params* params, void* stream, tds_pending** pending) {
    if (!pending) return TDS_E_INVALID;
    *pending = nullptr;
    if (!index || !Q || Q->n == 0) return TDS_E_INVALID;
    tds_pending* p = new (std::nothrow) tds_pending();
    if (!p) return TDS_E_NOMEM;
    p->device = index->device;
    DeviceGuard g(index->device);
    if (!g.ok) {
        delete p;
        return TDS_E_DEVICE;
    }
    const int st = tds::search_begin_impl(const_cast<tds_index*>(index), Q, d, t_start, t_end,
                                          out, capacity, params, (hipStream_t)stream, &p->impl);
    if (st != TDS_OK) {
        delete p;
        return st;
    }
    *pending = p;
    return TDS_OK;
}

int tds_search_end(tds_pending* pending, uint64_t* n_out, tds_stats* stats) {
    if (!pending) return TDS_E_INVALID;
    if (n_out) *n_out = 0;
    DeviceGuard g(pending->device);
    const int st = g.ok ? tds::search_end_impl(pending->impl, n_out, stats) : TDS_E_DEVICE;
    delete pending;
    return st;
}

int tds_search(const tds_index* index, const tds_segments* Q, double d, double t_start,
               double t_end, tds_result* out, uint64_t capacity, uint64_t* n_out,
               const tds_search_params* params, void* stream, tds_stats* stats) {
    if (!index || !n_out || !Q) return TDS_E_INVALID;
    *n_out = 0;
    if (Q->n == 0) {
        if (!(d >= 0.0) || std::isinf(d) || !(t_start < t_end)) return TDS_E_INVALID;
        if (stats) *stats = tds_stats{};
        return TDS_OK;
    }
    DeviceGuard g(index->device);
    if (!g.ok) return TDS_E_DEVICE;
    return tds::search_impl(const_cast<tds_index*>(index), Q, d, t_start, t_end, out, capacity,
                            n_out, params, (hipStream_t)stream, stats);
}

int tds_self_join(const tds_index* index, double d, double t_start, double t_end,
                  tds_result* out, uint64_t capacity, uint64_t* n_out,
                  const tds_search_params* params, void* stream, tds_stats* stats) {
    if (!index || !n_out) return TDS_E_INVALID;
    *n_out = 0;
    DeviceGuard g(index->device);
    if (!g.ok) return TDS_E_DEVICE;
    return tds::self_join_impl(const_cast<tds_index*>(index), d, t_start, t_end, out, capacity,
                               n_out, params, (hipStream_t)stream, stats);
}

int tds_fsg_build(const tds_index* index, uint32_t gx, uint32_t gy, uint32_t gz, void* stream,
                  tds_fsg** out) {
    if (!index || !out) return TDS_E_INVALID;
    *out = nullptr;
    DeviceGuard g(index->device);
    if (!g.ok) return TDS_E_DEVICE;
    return tds::fsg_build(index, gx, gy, gz, (hipStream_t)stream, out);
}

int tds_fsg_destroy(tds_fsg* grid) {
    tds::fsg_destroy(grid);
    return TDS_OK;
}

int tds_fsg_search(const tds_fsg* grid, const tds_segments* Q, double d, double t_start,
                   double t_end, tds_result* out, uint64_t capacity, uint64_t* n_out,
                   const tds_search_params* params, void* stream, tds_stats* stats) {
    if (!grid || !n_out || !Q) return TDS_E_INVALID;
    *n_out = 0;
    if (Q->n == 0) {
        if (!(d >= 0.0) || std::isinf(d) || !(t_start < t_end)) return TDS_E_INVALID;
        if (stats) *stats = tds_stats{};
        return TDS_OK;
    }
    DeviceGuard g(grid->device);
    if (!g.ok) return TDS_E_DEVICE;
    return tds::fsg_search(grid, Q, d, t_start, t_end, out, capacity, n_out, params,
                           (hipStream_t)stream, stats);
}

int tds_merge_trajectories(const tds_result* recs, uint64_t n, int recs_on_device,
                           tds_traj_interval* out, uint64_t capacity, int out_on_device,
                           uint64_t* n_out, void* stream) {
    if (!n_out) return TDS_E_INVALID;
    *n_out = 0;
    return tds::merge_impl(recs, n, recs_on_device != 0, out, capacity, out_on_device != 0, n_out,
                           (hipStream_t)stream);
}

int tds_last_stats(const tds_index* index, tds_stats* stats) {
    if (!index || !stats) return TDS_E_INVALID;
    tds_index* ix = const_cast<tds_index*>(index);
    std::lock_guard<std::mutex> lk(ix->mu);
    *stats = ix->last;
    return TDS_OK;
}

}  // extern "C"
