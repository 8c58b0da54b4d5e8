"""Benchmark of the distance threshold search on one MI355X.

Headline workload (one "step" = one pass of the whole search path over one
batch): the random-uniform 1M database (2,500 trajectories x 401 timesteps =
1,000,000 segments, start U[0,1000]^3, per-step velocity U[-5,5]^3), the full
query set of 500 query trajectories (200,000 query segments) over [0, 400],
searched at d = 1, 5 and 25 (three requests over the same query segments,
run as one batch per step), FP32 bulk filter with FP64 recheck, spatial index
layout, index and queries resident in HBM, results written to a device
buffer.  Launch parameters (bin count, chunk, grid) are the library defaults
(chosen by sweeps on this workload); --tune runs the autotuner on the full
workload before the timed region instead.

value = strictly time-overlapping (query, entry) segment pairs resolved per
second (index independent: every such pair is decided exactly).

Also reported: candidate tests per kernel-second, queries/s (one query = one
query trajectory at one d), the roofline of the distance kernel, the
self-join of the 1M entries at d = 25 with its trajectory-level merge, the
served form (open-loop replay of the request stream: Poisson arrivals at 5,000/s of
query trajectories of 5-400 segments with random windows and d in [1, 25],
through the serving loop) and the plain form (FP64 canonical test of every
candidate, one request per call, host memory in and out) on the same stream,
each with p50/p99 latency, and the oracle timed on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-serve]
                       [--no-self-join] [--tune] [--unbatched]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "segment-pair tests/s + queries/s at exact results; p50/p99 latency vs plain GPU"

# MI355X published FP32 vector peak: 256 CUs x 2.4 GHz x 256 FLOP/clk/CU
# = 157.3 TFLOP/s.
PEAK_FP32_TFLOPS = 256 * 256 * 2.4e9 / 1e12
PEAK_HBM_BPS = 8.0e12  # MI355X HBM3E, bytes/s
# FP operations of one FP32 filter test: 3 sub, 1 mul, 2 FMA (2 flops each),
# 1 add, 1 mul, 3 compares (1 each) = 13.
FLOPS_PER_TEST_FP32 = 13
# FP operations of one (query, 64-entry block) bounding-box test: per axis 2
# sub + 2 max, then 1 mul, 2 FMA (2 each), 1 add, 1 mul, 1 compare = 20.
FLOPS_PER_BLOCK_TEST = 20
KERNEL = "k_distance<FP32_RECHECK>"


def overlap_pairs(D, Q, t0, t1):
    """Number of strictly time-overlapping (query, entry) pairs within the
    window: N(ts < b_q) - N(te <= a_q) per query segment."""
    ts = np.sort(D.ts)
    te = np.sort(D.te)
    aq = np.maximum(Q.ts, t0)
    bq = np.minimum(Q.te, t1)
    ok = aq < bq
    n = np.searchsorted(ts, bq[ok], side="left") - np.searchsorted(te, aq[ok], side="right")
    return int(n.sum())


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def pct(x, q):
    return round(float(np.percentile(np.asarray(x), q)), 4)


KERNEL_SOURCES = ("search.hip", "canon.hpp", "tds_internal.hpp")
TRAFFIC_JSON = os.path.join(ROOT, "profiles", "k_distance_fp32_uniform1m_traffic.json")
VALU_JSON = os.path.join(ROOT, "profiles", "k_distance_fp32_uniform1m_valu.json")
# wave64 VALU instructions the chip can issue per second: 256 CUs x 4 SIMDs,
# one wave64 FP32 instruction per SIMD every 4 cycles (16 lanes), 2.4 GHz
PEAK_VALU_WAVE_INSTS = 256 * 4 * 2.4e9 / 4


def kernel_source_hash():
    """Hash of the sources the distance kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1410_2698_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_profile():
    """HBM bytes per launch of the distance kernel from the committed counter
    summary, if it was taken on the current kernel sources (else None)."""
    try:
        with open(TRAFFIC_JSON) as f:
            rec = json.load(f)
        h = kernel_source_hash()
    except (OSError, ValueError):
        return None
    return rec.get("bytes_per_launch") if rec.get("kernel_sources_sha256_16") == h else None


def valu_from_profile():
    """VALU and SALU instructions per launch of the distance kernel from the
    committed counter summary, if taken on the current kernel sources."""
    try:
        with open(VALU_JSON) as f:
            rec = json.load(f)
        h = kernel_source_hash()
    except (OSError, ValueError):
        return None
    return rec if rec.get("kernel_sources_sha256_16") == h else None


def summarize_valu(csv_path, command):
    """Counter CSV of one rocprofv3 --pmc run (SQ_INSTS_VALU SQ_INSTS_SALU
    SQ_WAVES) -> the distance kernel's instruction counts per launch."""
    import csv
    with open(csv_path) as f:
        rows = [r for r in csv.DictReader(f) if "k_distance<2>" in r["Kernel_Name"]]
    per = {}
    for r in rows:
        per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if not per:
        raise SystemExit(f"{csv_path}: no distance-kernel rows")
    rec = {"kernel": "k_distance<FP32_RECHECK>", "workload": "uniform1m, d in {1,5,25}",
           "launches": len(next(iter(per.values())))}
    for name, vals in per.items():
        rec[name.lower() + "_per_launch"] = sum(vals) / len(vals)
    rec["kernel_sources_sha256_16"] = kernel_source_hash()
    rec["command"] = command
    with open(VALU_JSON, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def summarize_traffic(fetch_csv, write_csv, command):
    """Counter CSVs of two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE,
    each with --calib-copy-mb 256) -> the traffic summary: the distance
    kernel's average per launch, scaled by what the same counter reads for the
    256 MiB calibration copy."""
    import csv

    def per_kernel(path, counter):
        with open(path) as f:
            rows = [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]
        dist = [float(r["Counter_Value"]) for r in rows if "k_distance<2>" in r["Kernel_Name"]]
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        if not dist or not copies:
            raise SystemExit(f"{path}: no {counter} rows for the distance kernel or the copy")
        return dist, max(copies)

    fd, fcopy = per_kernel(fetch_csv, "FETCH_SIZE")
    wd, wcopy = per_kernel(write_csv, "WRITE_SIZE")
    ref_kib = 256 * 1024
    ffac, wfac = ref_kib / fcopy, ref_kib / wcopy
    fetch_b = sum(fd) / len(fd) * 1024 * ffac
    write_b = sum(wd) / len(wd) * 1024 * wfac
    rec = {"kernel": "k_distance<FP32_RECHECK>", "workload": "uniform1m, d in {1,5,25}",
           "launches": len(fd), "fetch_kib_raw_avg": sum(fd) / len(fd),
           "write_kib_raw_avg": sum(wd) / len(wd),
           "copy_calibration": {"bytes": 256 << 20, "fetch_kib": fcopy, "write_kib": wcopy,
                                "fetch_factor": ffac, "write_factor": wfac},
           "bytes_per_launch": round(fetch_b + write_b),
           "kernel_sources_sha256_16": kernel_source_hash(), "command": command}
    with open(TRAFFIC_JSON, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def self_join_leg(tds, idx, D, d, reps=3):
    """The all-against-all form over the resident index: the self-join of the
    1M entries at distance d (device output), then the trajectory-level merge
    of its records (device to device)."""
    import torch
    st, n, _ = idx.self_join_raw(d, out_ptr=0, capacity=0, out_on_device=True)
    cap = n + 1
    rec = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
    out = torch.empty(cap * 24, dtype=torch.uint8, device="cuda")
    ts, tm, kern = [], [], []
    m = 0
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st, n2, s = idx.self_join_raw(d, out_ptr=rec.data_ptr(), capacity=cap, out_on_device=True)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st2, m = tds.merge_trajectories_raw(rec.data_ptr(), n2, True, out.data_ptr(), cap, True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if st != tds.TDS_OK or st2 != tds.TDS_OK or n2 != n:
            raise RuntimeError("self-join failed")
        if r:
            ts.append(t1 - t0)
            tm.append(t2 - t1)
            kern.append(s["kernel_ms"])
    # trajectories are time-monotone, so within its own trajectory a segment
    # overlaps only itself: the pairs resolved are the cross-trajectory ones
    pairs = (overlap_pairs(D, D, -np.inf, np.inf) - len(D)) // 2
    t_sj = float(np.median(ts))
    return {"d": d, "pairs_resolved": pairs, "pairs_per_s": round(pairs / t_sj, 1),
            "ms": round(1e3 * t_sj, 4), "kernel_ms": round(float(np.median(kern)), 4),
            "records": n, "merge_ms": round(1e3 * float(np.median(tm)), 4),
            "trajectory_intervals": m}


def fsg_leg(tds, idx, Qt, counts, ds, t0, t1, grids=(20, 50, 100), reps=3):
    """The fixed spatial grid (Alg. 1) over the same resident entries and
    queries: build time, and per d the search time and the listings compared,
    next to the index search's counts (the records must agree in number)."""
    import torch
    rows = []
    cap = max(counts.values()) + 1
    out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
    for g in grids:
        torch.cuda.synchronize()
        tb = time.perf_counter()
        grid = tds.FSG(idx, g, g, g)
        torch.cuda.synchronize()
        build_ms = 1e3 * (time.perf_counter() - tb)
        for d in ds:
            ts, kern, tested = [], [], 0
            for r in range(reps + 1):
                torch.cuda.synchronize()
                ta = time.perf_counter()
                st, n, s = grid.search_raw(Qt, d, t0, t1, out_ptr=out.data_ptr(), capacity=cap,
                                           out_on_device=True)
                torch.cuda.synchronize()
                if st != tds.TDS_OK or n != counts[d]:
                    raise RuntimeError(f"grid search failed: status {st}, {n} vs {counts[d]}")
                if r:
                    ts.append(time.perf_counter() - ta)
                    kern.append(s["kernel_ms"])
                    tested = s["candidate_tests"]
            rows.append({"cells_per_axis": g, "d": d, "build_ms": round(build_ms, 3),
                         "ms": round(1e3 * float(np.median(ts)), 4),
                         "kernel_ms": round(float(np.median(kern)), 4),
                         "listings_compared": int(tested), "records": int(n)})
        grid.close()
    return {"fsg": rows}


def open_loop(tds, idx, reqs):
    """Submits reqs at their arrival times from a thread while the main thread
    collects them; returns (latencies in ms, records, elapsed s, server stats)."""
    srv = tds.Server(idx, max_batch_segments=1 << 17, max_batch_requests=2048, slots=2,
                     result_capacity=1 << 21, default_reserve=512)
    for r in reqs[:200]:  # warm-up, not timed
        srv.wait(srv.submit(r.Q, r.d, r.t_start, r.t_end))
    reqs = reqs[200:]
    base = reqs[0].arrival
    tickets = [None] * len(reqs)
    t_start = time.perf_counter()

    def submitter():
        for i, r in enumerate(reqs):
            dt = (r.arrival - base) - (time.perf_counter() - t_start)
            if dt > 0:
                time.sleep(dt)
            tickets[i] = srv.submit(r.Q, r.d, r.t_start, r.t_end)

    th = threading.Thread(target=submitter)
    th.start()
    lat, n_rec = [], 0
    for i in range(len(reqs)):
        while tickets[i] is None:
            time.sleep(0.0002)
        recs, ms = srv.wait(tickets[i])
        lat.append(ms)
        n_rec += recs.size
    th.join()
    elapsed = time.perf_counter() - t_start
    st = srv.stats()
    srv.close()
    return lat, n_rec, elapsed, st


def serve_leg(tds, idx, seconds, rate, sweep=(10000.0, 20000.0, 40000.0)):
    """The request stream through tds_server: an open-loop run at `rate` for
    `seconds`, the plain FP64 form (one request per call) on its first 5,000
    requests, and shorter open-loop runs at higher offered rates."""
    import trajgen
    n_req = int(seconds * rate)
    reqs = trajgen.request_stream(n_req + 200, rate=rate)
    lat, n_rec, elapsed, st = open_loop(tds, idx, reqs)
    served = {"offered_rate": rate, "requests": len(lat),
              "requests_per_s": round(len(lat) / elapsed, 1),
              "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99), "records": n_rec,
              "batches": st["batches"], "requeued": st["requeued"],
              "max_batch_requests": st["max_batch_requests_seen"]}
    plain = []
    for r in reqs[200:5200]:
        t0 = time.perf_counter()
        idx.search(r.Q, r.d, r.t_start, r.t_end, precision="fp64", capacity=4096)
        plain.append(1e3 * (time.perf_counter() - t0))
    rows = []
    for rt in sweep:
        sreqs = trajgen.request_stream(5200, rate=rt)
        slat, _, sel, sst = open_loop(tds, idx, sreqs)
        rows.append({"offered_rate": rt, "requests_per_s": round(len(slat) / sel, 1),
                     "p50_ms": pct(slat, 50), "p99_ms": pct(slat, 99),
                     "batches": sst["batches"]})
    return {
        "served_fp32": served,
        "served_rate_sweep": rows,
        "plain_fp64": {"requests": len(plain),
                       "requests_per_s": round(len(plain) / (sum(plain) * 1e-3), 1),
                       "p50_ms": pct(plain, 50), "p99_ms": pct(plain, 99),
                       "note": "one request per call, back to back (service time, no queueing)"},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-self-join", action="store_true")
    ap.add_argument("--no-fsg", action="store_true", help="skip the fixed spatial grid leg")
    ap.add_argument("--summarize-traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic summary from two counter CSVs and exit (no GPU)")
    ap.add_argument("--summarize-valu", metavar="CSV",
                    help="write the VALU instruction summary from a counter CSV and exit (no GPU)")
    ap.add_argument("--tune", action="store_true", help="autotune before timing")
    ap.add_argument("--unbatched", action="store_true",
                    help="also time the step as three separate searches (context)")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the open-loop serving run at 5,000 requests/s")
    ap.add_argument("--cpu-traj", type=int, default=500, help="query trajectories in the oracle sample")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--grid-waves", type=int, default=0)
    ap.add_argument("--num-bins", type=int, default=0)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.summarize_valu:
        summarize_valu(args.summarize_valu,
                       "rocprofv3 --pmc SQ_INSTS_VALU SQ_INSTS_SALU SQ_WAVES --output-format csv "
                       "-d gpurun_out/pmc -o p -- python3 bench.py --steps 3 --warmup 1 "
                       "--no-cpu --no-serve --no-self-join --no-fsg")
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic,
                          "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv "
                          "-d gpurun_out/pmc -o p -- python3 bench.py --steps 3 --warmup 1 "
                          "--no-cpu --no-serve --no-self-join --no-fsg --calib-copy-mb 256")
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1410_2698_amd as tds
    import trajgen
    from paper_1410_2698_amd import autotune

    torch.cuda.set_device(0)
    if args.calib_copy_mb:
        n = args.calib_copy_mb << 20
        src = torch.ones(n, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    w = trajgen.uniform1m()
    ds = w.ds
    t0, t1 = w.window
    tuned = {"num_bins": args.num_bins, "chunk": args.chunk, "grid_waves": args.grid_waves}
    if args.tune and not (args.chunk or args.grid_waves or args.num_bins):
        best = autotune.tune(w.D, w.Q, ds, w.window, cache=None)
        tuned = {k: best[k] for k in ("num_bins", "chunk", "grid_waves")}
    idx = tds.Index(w.D, num_bins=tuned["num_bins"])
    Qt = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in w.Q.arrays().items()
          if k != "traj"}
    Qt["traj"] = torch.from_numpy(w.Q.traj.astype(np.int32)).cuda()
    pairs = overlap_pairs(w.D, w.Q, t0, t1)

    # one batch per step: the query segments once per d, one request each;
    # a first batch with no output space counts the results
    nq = len(w.Q)
    Qb = {k: torch.cat([v] * len(ds)) for k, v in Qt.items()}
    _, want, _ = idx.search_batch_raw(Qb, [(i * nq, nq, d, t0, t1, 0, 0) for i, d in enumerate(ds)],
                                      out_ptr=0, out_capacity=0, out_on_device=True,
                                      chunk=tuned["chunk"], grid_waves=tuned["grid_waves"])
    counts = dict(zip(ds, want))
    cap = max(want) + 1
    out = torch.empty(len(ds) * cap * 32, dtype=torch.uint8, device="cuda")
    reqs = [(i * nq, nq, d, t0, t1, i * cap, cap) for i, d in enumerate(ds)]

    kern_ms, tests, evals, launches, ftests, btests = 0.0, 0, 0, 0, 0, 0

    def step(record):
        nonlocal kern_ms, tests, evals, launches, ftests, btests
        st, got, s = idx.search_batch_raw(Qb, reqs, out_ptr=out.data_ptr(),
                                          out_capacity=len(ds) * cap, out_on_device=True,
                                          chunk=tuned["chunk"], grid_waves=tuned["grid_waves"])
        if st != tds.TDS_OK or got != want:
            raise RuntimeError(f"search failed: status {st}, {got} vs {want}")
        if record:
            kern_ms += s["kernel_ms"]
            tests += s["candidate_tests"]
            evals += s["fp64_evals"]
            launches += s["passes"]
            ftests += s["filter_tests"]
            btests += s["block_tests"]

    def step_unbatched():
        for d in ds:
            st, n, _ = idx.search_raw(Qt, d, t0, t1, out_ptr=out.data_ptr(), capacity=cap,
                                      out_on_device=True, chunk=tuned["chunk"],
                                      grid_waves=tuned["grid_waves"])
            if st != tds.TDS_OK or n != counts[d]:
                raise RuntimeError(f"search failed: status {st}, {n} vs {counts[d]}")

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - tb
    ms_per_step = 1e3 * elapsed / args.steps
    ms_unbatched = None
    if args.unbatched:
        # context: the same step as three separate searches (not the headline)
        step_unbatched()
        torch.cuda.synchronize()
        tu = time.perf_counter()
        for _ in range(3):
            step_unbatched()
        torch.cuda.synchronize()
        ms_unbatched = round(1e3 * (time.perf_counter() - tu) / 3, 4)
    n_queries = len(w.query_traj_slices()) * len(ds)
    value = args.steps * pairs * len(ds) / elapsed

    avg_ms = kern_ms / max(launches, 1)
    tests_per_launch = tests / max(launches, 1)
    # algorithmic work of one launch: the FP32 filter tests and block tests it
    # performs (pairs removed by the block boxes are not counted)
    flops = (FLOPS_PER_TEST_FP32 * ftests + FLOPS_PER_BLOCK_TEST * btests) / max(launches, 1)
    achieved = flops / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_FP32_TFLOPS, 1),
                "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_TFLOPS, 4),
                "traffic": traffic_from_profile(), "kernel": KERNEL,
                "avg_launch_ms": round(avg_ms, 4), "flops_per_launch": int(flops),
                "flops_per_filter_test": FLOPS_PER_TEST_FP32,
                "flops_per_block_test": FLOPS_PER_BLOCK_TEST}
    # the other two views of the same launch: the candidate stream the method
    # reads per pair (32-B FP32 records, as if each pair fetched its own), and
    # the HBM bytes the counters saw
    traffic = roofline["traffic"]
    roofline["views"] = {
        "candidate_stream_tb_s": round(tests_per_launch * 32 / (avg_ms * 1e-3) / 1e12, 2),
        "candidate_stream_frac_of_hbm": round(tests_per_launch * 32 / (avg_ms * 1e-3) / PEAK_HBM_BPS, 3),
        "dram_tb_s": round(traffic / (avg_ms * 1e-3) / 1e12, 3) if traffic else None,
        "dram_frac_of_hbm": round(traffic / (avg_ms * 1e-3) / PEAK_HBM_BPS, 4) if traffic else None,
        "alu_frac": roofline["frac"]}
    valu = valu_from_profile()
    if valu and valu.get("sq_insts_valu_per_launch"):
        # VALU issue utilisation: wave64 VALU instructions per launch (counter
        # run of the same command) over the launch time, against the issue peak
        vi = valu["sq_insts_valu_per_launch"]
        roofline["views"]["valu_wave_insts_per_launch"] = int(vi)
        roofline["views"]["valu_issue_frac"] = round(vi / (avg_ms * 1e-3) / PEAK_VALU_WAVE_INSTS, 3)
        if valu.get("sq_insts_salu_per_launch"):
            roofline["views"]["salu_wave_insts_per_launch"] = int(valu["sq_insts_salu_per_launch"])

    extra = {"queries_per_s": round(n_queries * args.steps / elapsed, 1),
             "candidate_tests_per_kernel_s": round(tests / (kern_ms * 1e-3), 1) if kern_ms else None,
             "candidate_pairs_per_launch": int(tests_per_launch),
             "fp64_recheck_fraction": round(evals / max(tests, 1), 8),
             "filter_tests_per_launch": int(ftests / max(launches, 1)),
             "block_tests_per_launch": int(btests / max(launches, 1)),
             "layout": {1: "temporal", 2: "spatial"}.get(idx.info()["layout"]),
             "fp32_endpoint_error": 0.0,
             "results_per_d": {str(d): counts[d] for d in ds},
             "overlap_pairs_per_search": pairs, "tuned": tuned,
             "batch_latency_ms": round(ms_per_step, 4),
             "ms_per_step_as_three_searches": ms_unbatched}

    if not args.no_serve:
        extra.update(serve_leg(tds, idx, args.serve_seconds, 5000.0))
    if not args.no_self_join:
        extra["self_join"] = self_join_leg(tds, idx, w.D, 25.0)
    if not args.no_fsg:
        extra.update(fsg_leg(tds, idx, Qt, counts, ds, t0, t1))

    cpu = None
    if not args.no_cpu:
        import oracle
        sl = w.query_traj_slices()
        k = max(1, min(args.cpu_traj, len(sl)))
        sub = w.Q.take(np.arange(sl[0][0], sl[k - 1][1]))
        cores = os.cpu_count() or 1
        tc = time.perf_counter()
        oracle.search(sub, w.D, 5.0, t0, t1, threads=cores)
        dt = time.perf_counter() - tc
        cpu = {"value": round(overlap_pairs(w.D, sub, t0, t1) / dt, 1), "unit": "pair tests/s",
               "cores": cores, "kind": "oracle",
               "sample": f"{k} of 500 query trajectories ({len(sub)} query segments) x 1,000,000 "
                         f"entries at d=5, brute force over all pairs; {dt:.2f} s"}
        # the same on one core, over a twentieth of the query trajectories
        k1 = max(1, k // 20)
        sub1 = w.Q.take(np.arange(sl[0][0], sl[k1 - 1][1]))
        tc = time.perf_counter()
        oracle.search(sub1, w.D, 5.0, t0, t1, threads=1)
        dt1 = time.perf_counter() - tc
        cpu["single_core"] = {"value": round(overlap_pairs(w.D, sub1, t0, t1) / dt1, 1),
                              "sample": f"{k1} query trajectories ({len(sub1)} query segments); "
                                        f"{dt1:.2f} s"}
        cpu["cpu_model"] = cpu_model()

    rec = {"metric": METRIC, "value": round(value, 1), "unit": "pair tests/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": "uniform1m: 2,500 trajectories x 401 timesteps (1,000,000 "
                                  "segments), 500 query trajectories (200,000 segments) over "
                                  "[0,400], d in {1,5,25} as three requests of one batch, "
                                  "FP32 filter + FP64 recheck, spatial layout",
                      "n_entries": len(w.D), "n_query_segments": len(w.Q), "d": ds,
                      "num_bins": idx.info()["num_bins"]},
           "roofline": roofline, "cpu_baseline": cpu, **extra}
    print(json.dumps(rec), flush=True)
    idx.close()


if __name__ == "__main__":
    main()
