/*
 * tds.h - C ABI of the trajectory distance-threshold search library (libtds.so)
 * for AMD Instinct MI355X (gfx950).
 *
 * Problem (Gowanlock & Casanova, arXiv:1410.2698, Sec. 3.1): a database D of
 * 4-D entry line segments (x, y, z, t start point; end point; segment id;
 * trajectory id) is indexed once and kept resident in GPU memory (Sec. 3.1,
 * in-memory database); a set Q of query segments is then searched against it:
 * for every query segment q and every entry segment l that overlap in time,
 * the library reports the time interval during which the two linearly moving
 * points are within Euclidean distance d (Sec. 4.1) of each other, as a
 * record (q, l, [t_lo, t_hi]) (the result set of Sec. 3.1).
 *
 * Semantics fixed by this library where the paper is silent:
 *   - time overlap is strict after clipping to the search window
 *     [t_start, t_end] (the search interval of Sec. 1): pairs that only touch
 *     at one instant are not results;
 *   - "within d" is inclusive; a tangent pair gives t_lo == t_hi;
 *   - one record per (query segment, entry segment) pair; intervals are not
 *     merged across consecutive segments; each record carries both
 *     trajectory ids;
 *   - membership and endpoints follow one fixed FP64 evaluation order (no
 *     fused multiply-add), so the result set is reproducible bit for bit.
 *
 * Conventions for every entry point:
 *   - return value: a TDS_* status code; TDS_OK is 0;
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream);
 *     work is ordered on it; calls that return counts wait for it;
 *   - pointers flagged as device memory must be allocated on the device that
 *     was current when the index was built;
 *   - no entry point keeps a caller pointer after it returns.
 */
#ifndef TDS_H
#define TDS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define TDS_ABI_VERSION 4u

/* Status codes. */
enum {
    TDS_OK = 0,
    TDS_E_INVALID = 1,  /* bad argument or input value (NaN, t_end <= t_start, ...) */
    TDS_E_OVERFLOW = 2, /* more results than the output capacity; *n_out holds the total */
    TDS_E_NOMEM = 3,    /* device or host allocation failed */
    TDS_E_DEVICE = 4,   /* a HIP call failed */
    TDS_E_BUSY = 5      /* admission refused (serving, non-blocking submit) */
};

/* Arithmetic of the candidate filter inside the distance kernel. */
enum {
    /* Library default (currently TDS_PREC_FP32_RECHECK). */
    TDS_PREC_DEFAULT = 0,
    /* Plain form: every candidate pair is evaluated with the canonical FP64
       predicate. */
    TDS_PREC_FP64 = 1,
    /* FP32 bulk test with a rigorous error margin around d (a pair is dropped
       only when it provably has no result); the surviving pairs are decided,
       and their endpoints computed, by the canonical FP64 evaluation.  Result
       set and endpoints are identical to TDS_PREC_FP64. */
    TDS_PREC_FP32_RECHECK = 2
};

/*
 * A set of segments in structure-of-arrays form.  Segment k runs from
 * (xs[k], ys[k], zs[k]) at time ts[k] to (xe[k], ye[k], ze[k]) at time te[k]
 * (Sec. 3.1).  The segment id is the array position k.  traj_id may be NULL
 * (every id 0).  All arrays hold n elements and live in host memory
 * (on_device = 0) or device memory (on_device = 1).  Borrowed for the call.
 * Requirements: every value finite, te[k] > ts[k], n < 2^32.
 */
typedef struct tds_segments {
    const double* xs;
    const double* ys;
    const double* zs;
    const double* ts;
    const double* xe;
    const double* ye;
    const double* ze;
    const double* te;
    const uint32_t* traj_id;
    uint64_t n;
    int32_t on_device;
    int32_t reserved;
} tds_segments;

/* Order of the entries inside each temporal bin. */
enum {
    /* Library default (currently TDS_LAYOUT_SPATIAL). */
    TDS_LAYOUT_DEFAULT = 0,
    /* Temporal index of Sec. 4.2.1 only: entries sorted by t_start. */
    TDS_LAYOUT_TEMPORAL = 1,
    /* Spatial subdivision of every temporal bin (the idea of the
       spatiotemporal index, Sec. 4.3): inside a bin, entries are ordered by
       the Hilbert index of their bounding-sphere centre's cell on a 1024^3
       grid over the data's extent, and every aligned block of 64 entries
       carries a bounding box, against which the FP32 form tests each query
       before it tests the block's entries.  Bins, candidate ranges and results are
       the same as with TDS_LAYOUT_TEMPORAL. */
    TDS_LAYOUT_SPATIAL = 2
};

/* Place of the FP32 form's closest-approach refinement: a pair that passes
   the bounding-sphere test is dropped when FP32 lower bounds on the smallest
   distance of the two moving points exceed d by more than the rounding of
   the FP32 data and arithmetic; the rest are decided in FP64. */
enum {
    TDS_REFINE_DEFAULT = 0, /* currently TDS_REFINE_QUEUED */
    /* A stage of the pair queue, 64 pairs at a time (least register pressure
       in the filter; best where few pairs pass the sphere test). */
    TDS_REFINE_QUEUED = 1,
    /* In the filter's walk over the queries of a block, from the candidate's
       data in registers (best where most pairs pass the sphere test). */
    TDS_REFINE_INLINE = 2
};

/* Dealing of the distance kernel's work items to its waves.  Items are split
   into one contiguous part per XCD (so a candidate range stays under one
   L2) and every wave first takes one item of its part. */
enum {
    TDS_DEAL_DEFAULT = 0, /* currently TDS_DEAL_DYNAMIC */
    /* The rest from per-part counters, a wave whose part is used up taking
       from the others (balances searches whose item costs vary widely). */
    TDS_DEAL_DYNAMIC = 1,
    /* The rest round-robin over the part's waves, no counters (cheapest when
       items cost about the same). */
    TDS_DEAL_STATIC = 2
};

/* How the results of a one-request search (tds_search, tds_self_join, a
   one-request tds_search_batch) reach the output buffer.  Batches of several
   requests, the batcher and the server always stage.  Both modes give the
   same records; positions within a request are in no fixed order. */
enum {
    TDS_OUTPUT_DEFAULT = 0, /* currently TDS_OUTPUT_DIRECT */
    /* Each wave reserves a chunk of output positions at a time (one
       device-scope atomic per chunk) and writes its results straight to it;
       a short pass after the distance kernel moves the results found past the
       final count into the chunks' unused tails.  Positions of the buffer
       between the count and the capacity may be written as well. */
    TDS_OUTPUT_DIRECT = 1,
    /* Each wave stages its results in device memory and, at the end of each
       work item (or when the stage is full), reserves exactly their number
       per request and copies them out. */
    TDS_OUTPUT_STAGED = 2
};

/* Index parameters; a NULL pointer or 0 fields select defaults. */
typedef struct tds_build_params {
    /* Number m of temporal bins (Sec. 4.2.1).  0 = auto: the full temporal
       extent divided by the mean segment duration, rounded, clamped to
       [1, 65535]. */
    uint32_t num_bins;
    uint32_t layout; /* TDS_LAYOUT_* */
    uint32_t reserved[6];
} tds_build_params;

/* One result record (32 bytes): the interaction of query segment q_seg with
   entry segment e_seg is within d during [t_lo, t_hi] (Sec. 3.1). */
typedef struct tds_result {
    uint32_t q_seg;  /* query segment id (position in the request's Q) */
    uint32_t e_seg;  /* entry segment id (position in the D given to build) */
    uint32_t q_traj; /* trajectory id of the query segment */
    uint32_t e_traj; /* trajectory id of the entry segment */
    double t_lo;
    double t_hi;
} tds_result;

/* Search parameters; a NULL pointer or 0 fields select defaults. */
typedef struct tds_search_params {
    int32_t precision;     /* TDS_PREC_* */
    int32_t out_on_device; /* 1: `out` is device memory, else host memory */
    uint32_t chunk;        /* candidates per work item; 0 = auto */
    uint32_t grid_waves;   /* waves of the persistent distance kernel; 0 = auto */
    /* Host output only: size, in records, of the device result buffer
       (the paper's fixed result buffer, Sec. 5.2).  When the results exceed
       it, the search is re-run in increments that each fit (Sec. 3.2).
       0 = min(capacity, 2^24). */
    uint64_t device_capacity;
    /* FP32 form: candidates each lane holds per tile of the distance kernel
       (the tile is 64 x this); 2 or 4, 0 = 4. */
    uint32_t tile;
    /* FP32 form: where the closest-approach refinement of the filter runs
       (TDS_REFINE_*).  Both places drop the same pairs. */
    uint32_t refine;
    /* How the distance kernel's work items reach its waves (TDS_DEAL_*). */
    uint32_t deal;
    /* How a one-request search's results reach the output (TDS_OUTPUT_*). */
    uint32_t output;
    uint64_t reserved[2];
} tds_search_params;

/* Counters of the last search (tests and benchmarks). */
typedef struct tds_stats {
    uint64_t query_segments;  /* query segments given */
    uint64_t active_segments; /* with a non-empty window and candidate range */
    uint64_t work_items;      /* (query group, candidate chunk) items */
    uint64_t candidate_tests; /* (query, entry) pairs in the candidate ranges */
    uint64_t fp64_evals;      /* pairs evaluated by the canonical FP64 code */
    uint64_t results;         /* result records found (may exceed the capacity) */
    uint32_t passes;          /* distance-kernel launches (> 1: incremental) */
    uint32_t stage_flushes;   /* first pass, staged output: work items whose results
                                 were reserved and written at the item's end (one
                                 device-scope atomic per request in the item); direct
                                 output: chunk reservations */
    double kernel_ms;         /* distance kernel(s), measured with HIP events */
    double total_ms;          /* whole call, host wall clock */
    uint64_t filter_tests;    /* pairs put through the FP32 filter (FP32 form) or the
                                 FP64 predicate (plain form) */
    uint64_t block_tests;     /* (query, 64-entry block) bounding-box tests */
} tds_stats;

/* Index description. */
typedef struct tds_index_info {
    uint64_t n;         /* entry segments */
    uint32_t num_bins;  /* m */
    uint32_t device;    /* HIP device ordinal */
    double t_min;       /* min t_start over D */
    double t_max;       /* max t_end over D */
    double bin_width;   /* (t_max - t_min) / m */
    uint64_t device_bytes;
    uint32_t layout;    /* TDS_LAYOUT_TEMPORAL or TDS_LAYOUT_SPATIAL */
    uint32_t reserved;
} tds_index_info;

typedef struct tds_index tds_index;

/* ABI version (TDS_ABI_VERSION of the built library).  Never fails. */
uint32_t tds_abi_version(void);

/* Static string naming a status code.  Never fails. */
const char* tds_status_str(int status);

/*
 * Build the temporal index of D on the current HIP device (Sec. 4.2.1): assign
 * the entries to m bins of equal width over [t_min, t_max] by t_start, store
 * them bin after bin (inside a bin by t_start, ties in input order, or, with
 * the spatial layout, by spatial cell, ties in input order), and record per
 * bin its first entry and the data extents used to compute candidate ranges.
 * Errors also: TDS_E_INVALID for an unknown layout.  The entries are
 * copied; the index owns all its device memory until tds_index_destroy.
 * Waits for `stream` before returning.
 * Errors: TDS_E_INVALID (NULL pointers, n == 0, n >= 2^32 - 1, a non-finite
 * value or te <= ts in D), TDS_E_NOMEM, TDS_E_DEVICE.
 */
int tds_build_index(const tds_segments* D, const tds_build_params* params,
                    void* stream, tds_index** out);

/* Free the index and its device memory.  NULL is accepted.  The caller must
   ensure no search on it is still running. */
int tds_index_destroy(tds_index* index);

/* Describe the index.  Errors: TDS_E_INVALID (NULL pointers). */
int tds_index_info_get(const tds_index* index, tds_index_info* info);

/*
 * Copy index tables to host memory (for inspection and tests); any output
 * may be NULL.  order[n]: input position of the i-th entry in index order.
 * bin_first[m + 1]: sorted position of the first entry of bin j
 * (bin_first[m] = n; bin j holds [bin_first[j], bin_first[j+1])).
 * min_ts[m], max_te[m]: data extents of bin j (+inf / -inf when empty).
 * cmax_te[m]: running maximum of max_te over bins 0..j.
 * Errors: TDS_E_INVALID, TDS_E_DEVICE.
 */
int tds_index_export(const tds_index* index, uint32_t* order, uint32_t* bin_first,
                     double* min_ts, double* max_te, double* cmax_te);

/*
 * Candidate range (the schedule S of Sec. 4.2.2) of each query segment: the
 * contiguous span E_k = [lo[k], hi[k]) of sorted entry positions from the
 * first entry of the first bin whose running max t_end exceeds a_q to the last
 * entry of the last non-empty bin whose smallest t_start is below b_q, where
 * [a_q, b_q] is the query segment clipped to [t_start, t_end].  Every entry that strictly overlaps the clipped query in
 * time lies in the span.  Empty windows or spans give lo = hi = 0.  lo and hi
 * are host arrays of Q->n elements.  Waits for `stream`.
 * Errors: TDS_E_INVALID (bad pointers or Q values, t_start >= t_end or NaN),
 * TDS_E_NOMEM, TDS_E_DEVICE.
 */
int tds_schedule(const tds_index* index, const tds_segments* Q, double t_start,
                 double t_end, uint32_t* lo, uint32_t* hi, void* stream);

/*
 * Distance threshold search of Q against the index (Sec. 3.1, Sec. 4.2.2).
 * Records go to `out` (host or device memory per params->out_on_device) in
 * unspecified order; *n_out is always set to the total number of results.
 * d finite and >= 0; t_start < t_end (either may be infinite).  Waits for `stream`.
 *   TDS_OK          all *n_out records are in out[0 .. *n_out).
 *   TDS_E_OVERFLOW  *n_out > capacity: out holds an unspecified subset of at
 *                   most `capacity` records; call again with a larger buffer.
 * Host output larger than params->device_capacity is produced in several
 * distance-kernel passes, each writing a slice that fits the device buffer.
 * stats may be NULL.
 * Errors: TDS_E_INVALID (bad pointers, d < 0 or NaN, t_start >= t_end, a
 * non-finite value or te <= ts in Q), TDS_E_NOMEM, TDS_E_DEVICE.
 */
int tds_search(const tds_index* index, const tds_segments* Q, double d,
               double t_start, double t_end, tds_result* out, uint64_t capacity,
               uint64_t* n_out, const tds_search_params* params, void* stream,
               tds_stats* stats);

/*
 * tds_search in two halves, for callers that overlap the search with other
 * work on the host: tds_search_begin orders the whole search on `stream`
 * (query preparation, bucket table, distance kernel, and for direct output
 * the fill pass) and returns without waiting for the device; tds_search_end
 * waits for it and reports as tds_search does.  The output is device memory
 * (params->out_on_device must be 1) and Q may be in host memory (copied to
 * the device before begin returns) or device memory (it must stay valid and
 * unchanged until end).  No incremental passes: on TDS_E_OVERFLOW `out` holds
 * an unspecified subset of `capacity` records and *n_out the total.  The
 * pending search holds a workspace of the index until end; every begin must
 * be matched by exactly one end (which frees *pending, also on errors), and
 * the index must outlive it.  Searches begun on different streams run
 * concurrently.  The rare search whose work items outgrow the table sized
 * from their bound runs a second time inside end.
 * Errors (begin): as tds_search, plus TDS_E_INVALID for host output; then
 * *pending is NULL and nothing is left running.  Errors (end): TDS_E_INVALID
 * (a NULL handle or invalid Q values found on the device), TDS_E_DEVICE.
 */
typedef struct tds_pending tds_pending;
int tds_search_begin(const tds_index* index, const tds_segments* Q, double d, double t_start,
                     double t_end, tds_result* out, uint64_t capacity,
                     const tds_search_params* params, void* stream, tds_pending** pending);
int tds_search_end(tds_pending* pending, uint64_t* n_out, tds_stats* stats);

/*
 * tds_search for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * search, records and status codes as tds_search with device output, but
 * every buffer beyond the caller's inputs and outputs comes from one
 * statically sized device array of 28 MiB per device (held by the library
 * until the process ends; its address is looked up on the first call on a
 * device).  The call allocates no device, host or pinned memory.
 * Requirements beyond tds_search's: Q in device memory (Q->on_device = 1) with
 * at most 65,536 segments; `out` is device memory (params->out_on_device is
 * ignored); at most 1,024 distance-kernel waves (params->grid_waves is capped)
 * and at most 524,288 work items (a larger search returns TDS_E_NOMEM: split
 * Q or use tds_search).  No incremental passes: on TDS_E_OVERFLOW `out` holds
 * an unspecified subset of `capacity` records.  stats->kernel_ms is 0 (no
 * timing events).  Every call on a device shares that device's array and
 * clears what it needs at its start: calls that overlap on one device (other
 * streams or threads) race and must be serialised by the caller.  Waits for
 * `stream`.
 * Errors: TDS_E_INVALID (as tds_search, plus host-memory Q or more than 65,536
 * query segments), TDS_E_NOMEM (work items beyond the table), TDS_E_DEVICE.
 */
int tds_search_noalloc(const tds_index* index, const tds_segments* Q, double d,
                       double t_start, double t_end, tds_result* out, uint64_t capacity,
                       uint64_t* n_out, const tds_search_params* params, void* stream,
                       tds_stats* stats);

/*
 * Self-join of the indexed database (the "every trajectory against every
 * other" search that motivates the paper, Sec. 1): every pair of entry
 * segments of different trajectories that is within d during the window,
 * each unordered pair once, as a record whose q_seg is the lower of the two
 * segment ids (q_traj its trajectory).  Records, intervals, output and
 * overflow behaviour as for tds_search with Q = the indexed segments; the
 * query data is read from the index itself.  Each pair is tested once, from
 * the entry stored first in the index.  Waits for `stream`.
 * Errors: TDS_E_INVALID (bad pointers, d < 0 or NaN, t_start >= t_end),
 * TDS_E_NOMEM, TDS_E_DEVICE.
 */
int tds_self_join(const tds_index* index, double d, double t_start, double t_end,
                  tds_result* out, uint64_t capacity, uint64_t* n_out,
                  const tds_search_params* params, void* stream, tds_stats* stats);

/* One trajectory-level result: trajectories q_traj and e_traj are within d
   throughout [t_lo, t_hi] (24 bytes). */
typedef struct tds_traj_interval {
    uint32_t q_traj;
    uint32_t e_traj;
    double t_lo;
    double t_hi;
} tds_traj_interval;

/*
 * Trajectory-level output: merges segment-level records into maximal time
 * intervals per (q_traj, e_traj).  Two intervals of the same trajectory pair
 * are merged when they overlap or touch (the next one starts no later than
 * the current one ends), so consecutive segment pairs whose intervals meet at
 * the shared timestep become one interval; endpoints are taken unchanged from
 * the records.  Output sorted by (q_traj, e_traj, t_lo).  recs (n records,
 * device memory if recs_on_device, else host) is only read; out holds
 * `capacity` intervals (device memory if out_on_device).  *n_out is always set
 * to the total; when it exceeds capacity, out holds the first `capacity`
 * intervals in that order and the call returns TDS_E_OVERFLOW.  Runs on the
 * current HIP device and waits for `stream`.  The library keeps the merge's
 * device scratch per device (grown to the largest n merged, about 60 bytes
 * per record, held until the process ends); calls on one device run one at a
 * time.
 * Errors: TDS_E_INVALID (NULL pointers, n >= 2^32 - 1), TDS_E_NOMEM,
 * TDS_E_DEVICE.
 */
int tds_merge_trajectories(const tds_result* recs, uint64_t n, int recs_on_device,
                           tds_traj_interval* out, uint64_t capacity, int out_on_device,
                           uint64_t* n_out, void* stream);

/*
 * Fixed spatial grid (FSG) index over the entries of an existing index: the
 * spatial method of Sec. 4.1 (Alg. 1, GPUSpatial).  The entries' spatial
 * extent is divided into gx x gy x gz equal cells (0 selects 50, the size the
 * paper found best); every entry is listed in each cell its bounding box
 * (grown by a relative 1e-9 so that rounding cannot drop a result) overlaps,
 * so ids repeat across cells.  A search visits the cells overlapped by each
 * query segment's box grown by d, compares the listed entries with the
 * canonical FP64 evaluation, and reports a pair found in several cells once:
 * from the lowest cell that both boxes overlap.  The grid keeps a reference
 * to `index` (not owned; destroy the grid first).  Requirements:
 * gx, gy, gz <= 1024, gx * gy * gz <= 2^24.  Waits for `stream`.
 * Errors: TDS_E_INVALID (bad pointers or sizes), TDS_E_NOMEM (more than
 * 2^32 - 1 listings), TDS_E_DEVICE.
 */
typedef struct tds_fsg tds_fsg;
int tds_fsg_build(const tds_index* index, uint32_t gx, uint32_t gy, uint32_t gz, void* stream,
                  tds_fsg** out);

/* Free the grid.  NULL is accepted. */
int tds_fsg_destroy(tds_fsg* grid);

/*
 * Distance threshold search through the grid: the records, the meaning of
 * out / capacity / *n_out, host or device output (params->out_on_device) and
 * TDS_E_OVERFLOW are those of tds_search, without incremental passes (when
 * the results exceed `capacity`, out holds an unspecified subset).  The
 * comparison is always the canonical FP64 one (params->precision is ignored).
 * stats: query_segments, candidate_tests (listings compared, repeats
 * included), results, kernel_ms, total_ms.  Waits for `stream`.
 * Errors: as tds_search.
 */
int tds_fsg_search(const tds_fsg* grid, const tds_segments* Q, double d, double t_start,
                   double t_end, tds_result* out, uint64_t capacity, uint64_t* n_out,
                   const tds_search_params* params, void* stream, tds_stats* stats);

/*
 * One request of a batch: a slice of the batch's query segments searched with
 * its own distance and window, writing into its own slice of the output.
 * Requests of a batch must tile the query segments in order: the first
 * starts at 0 and each starts where the previous one ends.  q_seg in the
 * records of a request counts from its q_begin.
 */
typedef struct tds_request {
    uint64_t q_begin, q_count;
    double d, t_start, t_end;          /* as for tds_search */
    uint64_t out_offset, out_capacity; /* output slice, in records */
} tds_request;

/*
 * Batched search: all requests in one pass of the search kernels (their query
 * segments share work items; each record goes to its request's slice).
 * counts[r] (host, nreq entries) is set to the total results of request r;
 * a request whose total exceeds its out_capacity keeps an unspecified subset
 * and makes the call return TDS_E_OVERFLOW (the other requests are complete).
 * `out` holds out_capacity records in host or device memory
 * (params->out_on_device).  Waits for `stream`.
 * Errors: TDS_E_INVALID (requests that do not tile Q, slices outside out,
 * bad d or window, bad Q values), TDS_E_NOMEM, TDS_E_DEVICE.
 */
int tds_search_batch(const tds_index* index, const tds_segments* Q, const tds_request* reqs,
                     uint32_t nreq, tds_result* out, uint64_t out_capacity, uint64_t* counts,
                     const tds_search_params* params, void* stream, tds_stats* stats);

/*
 * Batcher: a reusable batched search with fixed capacities whose launch
 * sequence is captured once in a hipGraph and replayed for every batch
 * (sizes are read from device memory).  It owns its device buffers and
 * pinned staging; `stream` (kept, not owned; NULL = a stream of its own) is
 * where it works.  One batch at a time per batcher.
 */
typedef struct tds_batcher tds_batcher;

/* Errors: TDS_E_INVALID (zero capacities, bad params), TDS_E_NOMEM, TDS_E_DEVICE. */
int tds_batcher_create(const tds_index* index, uint64_t max_segments, uint32_t max_requests,
                       uint64_t result_capacity, const tds_search_params* params, void* stream,
                       tds_batcher** out);

/*
 * Run one batch (Q in host or device memory, at most max_segments; at most
 * max_requests requests; output slices within result_capacity).  `out` is
 * host memory of result_capacity records; counts as for tds_search_batch.
 * Returns after the results are in `out`.  Same status codes as
 * tds_search_batch.
 */
int tds_batcher_run(tds_batcher* b, const tds_segments* Q, const tds_request* reqs, uint32_t nreq,
                    tds_result* out, uint64_t* counts, tds_stats* stats);

/* Number of graph replays so far (0 until the first batch). */
uint64_t tds_batcher_replays(const tds_batcher* b);

int tds_batcher_destroy(tds_batcher* b);

/*
 * Serving loop over a resident index (the in-memory database of Sec. 3.1,
 * queried many times).  Requests (one query trajectory each, host memory,
 * with its own d and window) are admitted in arrival order into batches by
 * free batch slots, query-segment capacity and result-memory reservations;
 * batches run on `slots` streams at once (continuous batching: requests that
 * arrive while batches run join the next batch to start).  A request whose
 * results exceed its reservation is re-queued with the exact size, so every
 * request completes with all its records.  Each request's records are the
 * same as from tds_search on its own.
 */
typedef struct tds_server tds_server;

typedef struct tds_server_params {
    uint64_t max_batch_segments; /* query segments per batch (0 = 262144) */
    uint32_t max_batch_requests; /* requests per batch (0 = 4096) */
    uint32_t slots;              /* batches in flight (0 = 2) */
    uint64_t result_capacity;    /* result records per batch (0 = 2^21) */
    uint64_t default_reserve;    /* records reserved per request until known (0 = 1024) */
    uint32_t max_pending;        /* queued requests before submit refuses (0 = 1 << 20) */
    /* Host route (hybrid CPU + GPU serving, 0 = off): a request whose
       candidate ranges hold at most this many (query, entry) pairs is
       searched on 4 host threads over a host copy of the index, with the
       GPU's filter (block boxes of the spatial layout, spheres) and canonical
       evaluation (the same records as on the GPU, bit for bit), as long as at
       most 8 such requests wait for those threads; the rest go to GPU batches
       (so a burst is absorbed by the GPU).  The host copy takes about 105
       bytes per entry of host memory. */
    uint32_t cpu_route_tests;
    tds_search_params search;    /* precision, chunk, grid (output fields ignored) */
} tds_server_params;

typedef struct tds_server_stats {
    uint64_t submitted, completed, batches, requeued, failed;
    uint64_t max_batch_requests_seen;
    uint64_t cpu_routed; /* requests completed by the host route */
} tds_server_stats;

/* Creation runs one empty batch on every slot (its graph is captured and its
 * stream set up before the first request needs it) and returns when they are
 * done.  Errors: TDS_E_INVALID, TDS_E_NOMEM, TDS_E_DEVICE.  params may be
 * NULL. */
int tds_server_create(const tds_index* index, const tds_server_params* params, tds_server** out);

/*
 * Queue one request (Q in host memory, copied; at most max_batch_segments
 * segments).  reserve = result records to reserve (0 = default).  When the
 * queue is full: blocking != 0 waits, else TDS_E_BUSY.  *ticket identifies
 * the request for tds_server_wait / tds_server_poll.
 * Errors: TDS_E_INVALID (bad Q, d or window), TDS_E_BUSY.
 */
int tds_server_submit(tds_server* srv, const tds_segments* Q, double d, double t_start,
                      double t_end, uint64_t reserve, int blocking, uint64_t* ticket);

/* *done = 1 once the request has completed (or failed). */
int tds_server_poll(tds_server* srv, uint64_t ticket, int* done);

/*
 * Wait for a request and copy its records (host memory).  *n_out = number of
 * records, *latency_ms = time from submit to completion (either may be NULL).
 * TDS_E_OVERFLOW: more than `capacity` records; nothing copied, the request
 * stays available for another call.  On any other return the ticket is
 * released.  Errors: TDS_E_INVALID (unknown ticket), or the request's failure.
 */
int tds_server_wait(tds_server* srv, uint64_t ticket, tds_result* out, uint64_t capacity,
                    uint64_t* n_out, double* latency_ms);

int tds_server_stats_get(tds_server* srv, tds_server_stats* stats);

/* Finishes queued requests, stops the worker and frees everything. */
int tds_server_destroy(tds_server* srv);

/* Fill *p with the defaults (TDS_PREC_FP32_RECHECK, host output, auto sizes). */
void tds_search_params_default(tds_search_params* p);

/* Counters of the last tds_search on this index (any thread).  Errors:
   TDS_E_INVALID. */
int tds_last_stats(const tds_index* index, tds_stats* stats);

#ifdef __cplusplus
}
#endif

#endif /* TDS_H */
