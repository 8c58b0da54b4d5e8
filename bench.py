"""Benchmark of the distance threshold search on one MI355X.

Workload (one "step" = one pass of the whole search path over one batch):
the random-uniform 1M database (2,500 trajectories x 401 timesteps =
1,000,000 segments, start U[0,1000]^3, per-step velocity U[-5,5]^3), the full
query set of 500 query trajectories (200,000 query segments) over [0, 400],
searched at d = 1, 5 and 25 (three searches per step), FP32 bulk filter with
FP64 recheck, index and queries resident in HBM, results written to a device
buffer.

value = strictly time-overlapping (query, entry) segment pairs resolved per
second (index independent: every such pair is decided exactly), over the
timed steps.  Also reported: candidate tests per kernel-second, queries/s
(one query = one query trajectory at one d), the plain form (FP64 canonical
test of every candidate, one query trajectory per call, host memory in and
out) with its p50/p99 latency, the roofline of the distance kernel, and the
oracle timed on the host on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--no-plain]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "segment-pair tests/s + queries/s at exact results; p50/p99 latency vs plain GPU"

# MI355X: 256 CUs, 4 SIMD16 per CU (wave64 over 4 cycles), 2.4 GHz.  Packed
# FP32 is not used, so one FP32 FMA per lane per cycle:
# 256 * 64 lanes * 2 flops * 2.4e9 = 78.6 TFLOP/s.
PEAK_FP32_NONPACKED_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12
# FP operations of one FP32 filter test: 3 sub, 1 mul, 2 FMA (2 flops each),
# 1 add, 1 mul, 3 compares (1 each) = 13.
FLOPS_PER_TEST_FP32 = 13


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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--cpu-traj", type=int, default=8, help="query trajectories in the oracle sample")
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--grid-waves", type=int, default=0)
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1410_2698_amd as tds
    import trajgen

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
    idx = tds.Index(w.D)
    Qt = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in w.Q.arrays().items()
          if k != "traj"}
    Qt["traj"] = torch.from_numpy(w.Q.traj.astype(np.int32)).cuda()
    pairs = overlap_pairs(w.D, w.Q, t0, t1)

    # size the device result buffer from one untimed search per d
    counts = {}
    for d in ds:
        _, n, _ = idx.search_raw(Qt, d, t0, t1, out_ptr=0, capacity=0, out_on_device=True)
        counts[d] = n
    cap = max(counts.values()) + 1
    out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")

    kern_ms = 0.0
    tests = 0
    launches = 0

    def step(record):
        nonlocal kern_ms, tests, launches
        for d in ds:
            st, n, s = idx.search_raw(Qt, d, t0, t1, out_ptr=out.data_ptr(), capacity=cap,
                                      out_on_device=True, chunk=args.chunk,
                                      grid_waves=args.grid_waves)
            if st != tds.TDS_OK or n != counts[d]:
                raise RuntimeError(f"search failed: status {st}, {n} vs {counts[d]}")
            if record:
                kern_ms += s["kernel_ms"]
                tests += s["candidate_tests"]
                launches += s["passes"]

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    tb = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - tb
    ms_per_step = 1e3 * elapsed / args.steps
    n_queries = len(w.query_traj_slices()) * len(ds)
    value = args.steps * pairs * len(ds) / elapsed

    avg_ms = kern_ms / max(launches, 1)
    tests_per_launch = tests / max(launches, 1)
    achieved = FLOPS_PER_TEST_FP32 * tests_per_launch / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "achieved": round(achieved, 3),
                "peak": round(PEAK_FP32_NONPACKED_TFLOPS, 1), "unit": "TFLOP/s",
                "frac": round(achieved / PEAK_FP32_NONPACKED_TFLOPS, 4), "traffic": None,
                "kernel": "k_distance<FP32_RECHECK>", "avg_launch_ms": round(avg_ms, 4),
                "tests_per_launch": int(tests_per_launch)}

    extra = {"queries_per_s": round(n_queries * args.steps / elapsed, 1),
             "candidate_tests_per_kernel_s": round(tests / (kern_ms * 1e-3), 1) if kern_ms else None,
             "results_per_d": {str(d): counts[d] for d in ds},
             "overlap_pairs_per_search": pairs}

    # plain form: FP64 test of every candidate, one query trajectory per call,
    # queries from host memory and results back to host memory
    if not args.no_plain:
        lat = []
        sl = w.query_traj_slices()
        d = 5.0
        for i, (b, e) in enumerate(sl):
            sub = w.Q.take(np.arange(b, e))
            tq = time.perf_counter()
            idx.search(sub, d, t0, t1, precision="fp64", capacity=4096)
            lat.append(time.perf_counter() - tq)
        lat = np.array(lat) * 1e3
        extra["plain_fp64"] = {"queries_per_s": round(len(lat) / (lat.sum() * 1e-3), 1),
                               "p50_ms": round(float(np.percentile(lat, 50)), 4),
                               "p99_ms": round(float(np.percentile(lat, 99)), 4), "d": d}
        extra["batched_fp32"] = {"queries_per_s": extra["queries_per_s"],
                                 "batch_latency_ms": round(ms_per_step / len(ds), 4)}

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
                         f"entries at d=5, brute force; {dt:.2f} s"}

    rec = {"metric": METRIC, "value": round(value, 1), "unit": "pair tests/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": "uniform1m: 2,500 trajectories x 401 timesteps (1,000,000 "
                                  "segments), 500 query trajectories (200,000 segments) over "
                                  "[0,400], d in {1,5,25}, FP32 filter + FP64 recheck",
                      "n_entries": len(w.D), "n_query_segments": len(w.Q), "d": ds,
                      "num_bins": idx.info()["num_bins"]},
           "roofline": roofline, "cpu_baseline": cpu, **extra}
    print(json.dumps(rec), flush=True)
    idx.close()


if __name__ == "__main__":
    main()
