"""Benchmark of the distance threshold search on one MI355X.

Headline workload (one "step" = one pass of the whole search path over one
batch of queries): the galaxy-merger-shaped database (2 x 100,000 particles in
two Plummer spheres on an approaching orbit, 20 snapshots = 3,800,000 entry
segments) searched with 2,000 query particles (38,000 query segments) at
d = 0.5 kpc over the full time span, FP32 bulk filter with FP64 recheck,
spatial index layout, index and queries resident in HBM, results
(1.7e8 records) written to a device buffer sized by a counting call.

value = strictly time-overlapping (query, entry) segment pairs resolved per
second (index independent: every such pair is decided exactly; 7.6e9 per
search).  Also reported for the headline: queries/s (one query = one query
trajectory), the filter tests and FP64 evaluations the kernel performed per
second, the roofline of the distance kernel (HBM and ALU views), the FP32
endpoint error (records of the FP32-filter form against the plain FP64 form)
and the oracle timed on the host on a sample of the same workload.

The other workloads run as legs of their own (each with its step time,
roofline, endpoint error and oracle sample): uniform1m (1M entries, 200,000
query segments at d = 1, 5, 25 as three requests of one batch), dense (1M
entries in [0,50]^3, 100,000 query segments, d = 2) and tiny (98,000 entries,
4,900 query segments, d = 5); the served form on the request stream over the
uniform1m index (Poisson arrivals of query trajectories of 5-400 segments with
random windows and d in [1, 25]) with an open-loop rate sweep to saturation,
and the plain FP64 form (one request per call) on the same stream; the
self-join of the uniform1m entries and the fixed spatial grid.

Each search leg first runs the autotuner on its workload (bin count, chunk,
grid, tile, wavefront mapping; untimed) and times the configuration it picks.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--legs a,b,...]
                       [--no-cpu] [--no-tune] [--no-fp64-form]
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
UNIT = "time-overlapping segment pairs resolved/s"

# MI355X published peaks: FP32 vector 256 CUs x 2.4 GHz x 256 FLOP/clk/CU =
# 157.3 TFLOP/s, FP64 vector 78.6 TFLOP/s, HBM3E 8 TB/s.
PEAK_FP32 = 256 * 256 * 2.4e9
PEAK_FP64 = 78.6e12
PEAK_HBM_BPS = 8.0e12
# wave64 VALU instructions the chip can issue per second: 256 CUs x 4 SIMDs,
# one wave64 instruction per SIMD every 4 cycles (16 lanes), 2.4 GHz
PEAK_VALU_WAVE_INSTS = 256 * 4 * 2.4e9 / 4

# Algorithmic work of the distance kernel, per unit (counted by the kernel):
# FP32 filter test: 3 sub, 1 mul, 2 FMA (2 flops each), 1 add, 1 mul,
#   3 compares = 13;
# (query, 64-entry block) box test: 2 compares per axis = 6;
# canonical FP64 membership of one pair: extent 2 min/max + 1 compare + 1 sub,
#   4 time offsets, 6 position differences of 5, 3 relative velocities, d^2,
#   C0 and C1 (6 each), A and B (5 each), the vertex clause (3 mul, 1 sub,
#   6 compares) = 74;
# interval of a result: discriminant 3, sqrt 1, max 1, root numerator 2,
#   2 divisions + 1 compare, both ends clamped (5 each), order check 1 = 21.
FLOPS_FILTER = 13
FLOPS_BOX = 6
FLOPS_EVAL64 = 74
FLOPS_RESULT64 = 21
# Bytes the kernel must move, per unit: a result record written (32 B); per
# entry of the searched candidate ranges, its FP32 filter record (32 B), FP64
# record (64 B) and ids (8 B), each read once; per query segment its end
# points (64 B).
BYTES_RESULT = 32
BYTES_ENTRY = 32 + 64 + 8
BYTES_QUERY = 64
KERNEL = "k_distance<FP32_RECHECK>"
KERNEL_SOURCES = ("search.hip", "canon.hpp", "tds_internal.hpp")


def prof_path(workload, kind):
    return os.path.join(ROOT, "profiles", f"k_distance_fp32_{workload}_{kind}.json")


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


def kernel_source_hash():
    """Hash of the sources the distance kernel is compiled from."""
    import hashlib
    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1410_2698_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_profile(workload, kind):
    """A committed counter summary of the distance kernel on `workload`, if
    it was taken on the current kernel sources (else None)."""
    try:
        with open(prof_path(workload, kind)) as f:
            rec = json.load(f)
        h = kernel_source_hash()
    except (OSError, ValueError):
        return None
    return rec if rec.get("kernel_sources_sha256_16") == h else None


# Launch parameters the profiles are taken with (the autotuner's choice for
# the workload on MI355X; the bench's own tuning picks them again).
PROFILE_PARAMS = {
    "galaxy": "num_bins=19,chunk=2048,grid_waves=4096,tile=2,refine=inline,deal=dynamic,"
              "output=direct,precision=fp32",
    "uniform1m": "num_bins=400,chunk=8192,grid_waves=4096,tile=2,refine=queued,deal=static,"
                 "output=staged,precision=fp32"}


def start_space(autotune, workload):
    """The autotuner's search space with the launch parameters measured best
    for `workload` (PROFILE_PARAMS) as its starting point, where there are
    such: its coordinate descent keeps the start unless a neighbour times
    faster, so a noisy early comparison cannot walk it off to a worse corner
    of the space (the bin count stays a factor of the automatic one)."""
    if workload not in PROFILE_PARAMS:
        return None
    start = dict(kv.split("=") for kv in PROFILE_PARAMS[workload].split(","))
    space = {}
    for knob, values in autotune.SPACE.items():
        if knob not in start:
            continue
        v0 = type(values[0])(start[knob])
        space[knob] = (v0,) + tuple(v for v in values if v != v0)
    return space


def profile_command(workload, counters):
    return (f"rocprofv3 --pmc {counters} --output-format csv -d gpurun_out/pmc -o p -- "
            f"python3 bench.py --legs {workload} --steps 2 --warmup 1 --no-cpu --no-fp64-form "
            f"--calib-copy-mb 256 --fixed {PROFILE_PARAMS[workload]}")


def summarize_valu(workload, csv_path):
    """Counter CSV of one rocprofv3 --pmc run (SQ_INSTS_VALU SQ_INSTS_SALU
    SQ_WAVES ...) -> the distance kernel's counts per launch."""
    import csv
    with open(csv_path) as f:
        rows = [r for r in csv.DictReader(f) if "k_distance<2," in r["Kernel_Name"]]
    per = {}
    for r in rows:
        per.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    if not per:
        raise SystemExit(f"{csv_path}: no distance-kernel rows")
    rec = {"kernel": KERNEL, "workload": workload, "launches": len(next(iter(per.values())))}
    for name, vals in per.items():
        rec[name.lower() + "_per_launch"] = sum(vals) / len(vals)
    rec["kernel_sources_sha256_16"] = kernel_source_hash()
    rec["command"] = profile_command(workload, " ".join(sorted(per)))
    with open(prof_path(workload, "valu"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def summarize_traffic(workload, fetch_csv, write_csv):
    """Counter CSVs of two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE,
    each with --calib-copy-mb 256) -> the traffic summary: the distance
    kernel's average per launch, scaled by what the same counter reads for the
    256 MiB calibration copy."""
    import csv

    def per_kernel(path, counter):
        with open(path) as f:
            rows = [r for r in csv.DictReader(f) if r["Counter_Name"] == counter]
        dist = [float(r["Counter_Value"]) for r in rows if "k_distance<2," in r["Kernel_Name"]]
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
    rec = {"kernel": KERNEL, "workload": workload,
           "launches": len(fd), "fetch_kib_raw_avg": sum(fd) / len(fd),
           "write_kib_raw_avg": sum(wd) / len(wd),
           "copy_calibration": {"bytes": 256 << 20, "fetch_kib": fcopy, "write_kib": wcopy,
                                "fetch_factor": ffac, "write_factor": wfac},
           "fetch_bytes_per_launch": round(fetch_b), "write_bytes_per_launch": round(write_b),
           "bytes_per_launch": round(fetch_b + write_b),
           "kernel_sources_sha256_16": kernel_source_hash(),
           "command": profile_command(workload, "FETCH_SIZE") + " (then WRITE_SIZE)"}
    with open(prof_path(workload, "traffic"), "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


def roofline(workload, st, launches, n_entries_ranged, nq):
    """Roofline of the distance kernel from the counters it keeps (summed over
    `launches` launches in `st`): the HBM view (algorithmic bytes per launch
    over the launch's time) and the ALU view (FP32 filter and box arithmetic
    at the FP32 peak, FP64 evaluations at the FP64 peak); `bound` is the view
    closer to its roof."""
    L = max(launches, 1)
    avg_s = st["kernel_ms"] / L * 1e-3
    res = st["results"] / L
    byts = BYTES_RESULT * res + BYTES_ENTRY * n_entries_ranged + BYTES_QUERY * nq
    f32 = (FLOPS_FILTER * st["filter_tests"] + FLOPS_BOX * st["block_tests"]) / L
    f64 = (FLOPS_EVAL64 * st["fp64_evals"] + FLOPS_RESULT64 * st["results"]) / L
    alu_time = f32 / PEAK_FP32 + f64 / PEAK_FP64  # at both peaks
    alu_peak = (f32 + f64) / alu_time if alu_time else PEAK_FP32
    hbm = {"achieved": byts / avg_s, "peak": PEAK_HBM_BPS}
    alu = {"achieved": (f32 + f64) / avg_s, "peak": alu_peak}
    hbm_frac = hbm["achieved"] / hbm["peak"]
    alu_frac = alu["achieved"] / alu["peak"]
    traffic = load_profile(workload, "traffic")
    valu = load_profile(workload, "valu")
    views = {"hbm_tb_s": round(hbm["achieved"] / 1e12, 4), "hbm_frac": round(hbm_frac, 4),
             "alu_tflop_s": round(alu["achieved"] / 1e12, 3),
             "alu_peak_tflop_s": round(alu_peak / 1e12, 2), "alu_frac": round(alu_frac, 4),
             "algorithmic_bytes_per_launch": int(byts),
             "fp32_flops_per_launch": int(f32), "fp64_flops_per_launch": int(f64),
             "filter_tests_per_s": round(st["filter_tests"] / L / avg_s, 1),
             # the bandwidth a kernel streaming one 32-B FP32 record per executed
             # filter test would need (the per-query access model); not bounded
             # by HBM here, records are reused from registers by 64 queries
             "filter_test_stream_tb_s": round(32 * st["filter_tests"] / L / avg_s / 1e12, 3),
             "fp64_evals_per_s": round(st["fp64_evals"] / L / avg_s, 1)}
    if traffic:
        views["dram_tb_s"] = round(traffic["bytes_per_launch"] / avg_s / 1e12, 4)
        views["dram_frac_of_hbm"] = round(traffic["bytes_per_launch"] / avg_s / PEAK_HBM_BPS, 4)
    if valu and valu.get("sq_insts_valu_per_launch"):
        vi = valu["sq_insts_valu_per_launch"]
        views["valu_wave_insts_per_launch"] = int(vi)
        views["valu_issue_frac"] = round(vi / avg_s / PEAK_VALU_WAVE_INSTS, 3)
    if hbm_frac >= alu_frac:
        r = {"bound": "hbm", "achieved": round(hbm["achieved"] / 1e9, 2), "peak": 8000.0,
             "unit": "GB/s", "frac": round(hbm_frac, 4)}
    else:
        r = {"bound": "alu", "achieved": round(alu["achieved"] / 1e12, 3),
             "peak": round(alu_peak / 1e12, 2), "unit": "TFLOP/s", "frac": round(alu_frac, 4)}
    r["traffic"] = traffic["bytes_per_launch"] if traffic else None
    r["kernel"] = KERNEL
    r["avg_launch_ms"] = round(avg_s * 1e3, 4)
    r["views"] = views
    return r


def ranged_entries(idx_info, D, Q, t0, t1):
    """Entries in the union of the query segments' temporal candidate ranges
    (bins overlapping the clipped query extents): each is read at least once."""
    edges = np.linspace(idx_info["t_min"], idx_info["t_max"], idx_info["num_bins"] + 1)
    a = np.maximum(Q.ts, t0)
    b = np.minimum(Q.te, t1)
    ok = a < b
    if not ok.any():
        return 0
    lo = max(float(a[ok].min()), float(edges[0]))
    hi = float(b[ok].max())
    return int(np.count_nonzero((D.te > lo) & (D.ts < hi)))


def device_segments(S):
    """The segment arrays of S as contiguous CUDA tensors (float64, int32 traj)."""
    import torch
    out = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda()
           for k, v in S.arrays().items() if k != "traj"}
    out["traj"] = torch.from_numpy(np.ascontiguousarray(S.traj).astype(np.int32)).cuda()
    return out


def sorted_records(buf, n):
    """The n records in a CUDA byte tensor as an (n, 4) int64 tensor ordered
    by (q_seg, e_seg)."""
    import torch
    rec = buf[: n * 32].view(torch.int64).view(n, 4)
    ids = rec[:, 0]
    key = ((ids & 0xFFFFFFFF) << 32) | ((ids >> 32) & 0xFFFFFFFF)
    _, perm = torch.sort(key)
    return rec[perm]


def endpoint_error(buf32, buf64, n):
    """FP32-filter form against the plain FP64 form (both on the device):
    identical (q_seg, e_seg, trajectory) sets required; max and p99 of the
    endpoint differences."""
    import torch
    a = sorted_records(buf32, n)
    b = sorted_records(buf64, n)
    if not torch.equal(a[:, :2], b[:, :2]):
        raise RuntimeError("FP32 and FP64 forms give different record sets")
    da = torch.cat([(a[:, 2].view(torch.float64) - b[:, 2].view(torch.float64)).abs(),
                    (a[:, 3].view(torch.float64) - b[:, 3].view(torch.float64)).abs()])
    p99 = 0.0
    if n:
        # p99 over a uniform sample of at most 2^24 differences
        pick = torch.randint(0, da.numel(), (min(da.numel(), 1 << 24),), device=da.device,
                             generator=torch.Generator(device=da.device).manual_seed(1))
        p99 = float(torch.quantile(da[pick], 0.99).item())
    out = {"records_compared": int(n), "max_abs": float(da.max().item()) if n else 0.0,
           "p99_abs": p99, "bit_identical": bool(torch.equal(a, b))}
    del a, b, da
    return out


def oracle_sample(w, d, n_traj, cores):
    """The oracle (plain FP64 brute force) on the first n_traj query
    trajectories at distance d, on `cores` threads: time-overlapping pairs
    resolved per second."""
    import oracle
    sl = w.query_traj_slices()
    k = max(1, min(n_traj, len(sl)))
    sub = w.Q.take(np.arange(sl[0][0], sl[k - 1][1]))
    t0, t1 = w.window
    tc = time.perf_counter()
    oracle.search(sub, w.D, d, t0, t1, threads=cores)
    dt = time.perf_counter() - tc
    return {"value": round(overlap_pairs(w.D, sub, t0, t1) / dt, 1), "unit": UNIT,
            "cores": cores, "kind": "oracle",
            "sample": f"{k} of {len(sl)} query trajectories ({len(sub)} query segments) x "
                      f"{len(w.D):,} entries at d={d}, brute force over all pairs; {dt:.2f} s"}


class SearchLeg:
    """One workload on the resident index: the search of all its query
    segments at every d of the workload (one request per d, one batch), into
    device memory sized by a counting call."""

    def __init__(self, tds, w, tuned=None, precision=None):
        import torch
        self.tds, self.w = tds, w
        self.tuned = dict({"num_bins": 0, "chunk": 0, "grid_waves": 0, "tile": 0,
                           "refine": "default", "deal": "default", "output": "default",
                           "precision": "fp32"}, **(tuned or {}))
        torch.cuda.synchronize()
        tb = time.perf_counter()
        self.idx = tds.Index(w.D, num_bins=self.tuned["num_bins"])
        torch.cuda.synchronize()
        # index build, host arrays in (upload included): reported apart from
        # the search, as the paper's response time excludes it
        self.build_ms = 1e3 * (time.perf_counter() - tb)
        Qt = device_segments(w.Q)
        nq = len(w.Q)
        self.Qb = {k: torch.cat([v] * len(w.ds)) if len(w.ds) > 1 else v for k, v in Qt.items()}
        t0, t1 = w.window
        self.count_reqs = [(i * nq, nq, d, t0, t1, 0, 0) for i, d in enumerate(w.ds)]
        self.precision = precision or self.tuned["precision"]
        _, want, _ = self.run(self.count_reqs, 0, 0)
        self.counts = want
        self.cap = max(want) + 1
        self.out = torch.empty(len(w.ds) * self.cap * 32, dtype=torch.uint8, device="cuda")
        self.reqs = [(i * nq, nq, d, t0, t1, i * self.cap, self.cap) for i, d in enumerate(w.ds)]

    def run(self, reqs, out_ptr, cap, precision=None):
        return self.idx.search_batch_raw(self.Qb, reqs, out_ptr=out_ptr, out_capacity=cap,
                                         out_on_device=True,
                                         precision=precision or self.precision,
                                         chunk=self.tuned["chunk"],
                                         grid_waves=self.tuned["grid_waves"],
                                         tile=self.tuned["tile"], refine=self.tuned["refine"],
                                         deal=self.tuned["deal"], output=self.tuned["output"])

    def step(self):
        st, got, s = self.run(self.reqs, self.out.data_ptr(), len(self.w.ds) * self.cap)
        if st != self.tds.TDS_OK or got != self.counts:
            raise RuntimeError(f"search failed: status {st}, {got} vs {self.counts}")
        return s

    def timed(self, steps, warmup):
        import torch
        for _ in range(warmup):
            self.step()
        acc = None
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for _ in range(steps):
            s = self.step()
            if acc is None:
                acc = dict(s)
            else:
                for k in ("kernel_ms", "candidate_tests", "fp64_evals", "results", "filter_tests",
                          "block_tests", "passes", "stage_flushes"):
                    acc[k] += s[k]
        torch.cuda.synchronize()
        return time.perf_counter() - tb, acc

    def fp64_form(self):
        """The plain FP64 form of the same batch (one launch), its time, and
        the FP32 endpoint error against it, request by request."""
        import torch
        out64 = torch.empty_like(self.out)
        torch.cuda.synchronize()
        t = time.perf_counter()
        st, got, s = self.run(self.reqs, out64.data_ptr(), len(self.w.ds) * self.cap, "fp64")
        torch.cuda.synchronize()
        t = time.perf_counter() - t
        if st != self.tds.TDS_OK or got != self.counts:
            raise RuntimeError(f"FP64 search failed: status {st}, {got} vs {self.counts}")
        errs = {}
        for i, d in enumerate(self.w.ds):
            a = self.out[i * self.cap * 32:]
            b = out64[i * self.cap * 32:]
            errs[str(d)] = endpoint_error(a, b, self.counts[i])
        del out64
        return {"ms": round(1e3 * t, 3), "kernel_ms": round(s["kernel_ms"], 3)}, errs

    def report(self, steps, warmup, cpu_traj, cores, with_cpu=True, with_fp64=True):
        w = self.w
        elapsed, acc = self.timed(steps, warmup)
        t0, t1 = w.window
        pairs = overlap_pairs(w.D, w.Q, t0, t1) * len(w.ds)
        info = self.idx.info()
        n_ranged = ranged_entries(info, w.D, w.Q, t0, t1)
        fp64, errs = self.fp64_form() if with_fp64 else (None, {})
        out = {
            "workload": w.name, "n_entries": len(w.D), "n_query_segments": len(w.Q),
            "d": w.ds, "num_bins": info["num_bins"],
            "ms_per_step": round(1e3 * elapsed / steps, 4),
            "value": round(steps * pairs / elapsed, 1), "unit": UNIT,
            "queries_per_s": round(len(w.query_traj_slices()) * len(w.ds) * steps / elapsed, 1),
            "overlap_pairs_per_step": pairs,
            "results_per_d": {str(d): c for d, c in zip(w.ds, self.counts)},
            "kernel_ms": round(acc["kernel_ms"] / steps, 4),
            "filter_tests_per_step": acc["filter_tests"] // steps,
            "block_tests_per_step": acc["block_tests"] // steps,
            "fp64_evals_per_step": acc["fp64_evals"] // steps,
            "fp64_recheck_fraction": round(acc["fp64_evals"] / max(acc["candidate_tests"], 1), 8),
            "stage_flushes_per_step": acc["stage_flushes"] // steps,
            "index_build_ms": round(self.build_ms, 2),
            "roofline": roofline(w.name, acc, acc["passes"], n_ranged, len(w.Q) * len(w.ds)),
            "fp64_form": fp64,
            "fp32_endpoint_error": {"max_abs": max(e["max_abs"] for e in errs.values()),
                                    "p99_abs": max(e["p99_abs"] for e in errs.values()),
                                    "per_d": errs} if errs else None,
            "tuned": self.tuned,
        }
        if with_cpu:
            out["cpu_baseline"] = oracle_sample(w, w.ds[len(w.ds) // 2], cpu_traj, cores)
        return out

    def close(self):
        self.idx.close()


def self_join_leg(tds, idx, D, d, reps=3):
    """The all-against-all form over the resident index: the self-join of the
    entries at distance d (device output), then the trajectory-level merge of
    its records (device to device)."""
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
    return rows


def open_loop(tds, idx, reqs, route=0):
    """Submits reqs at their arrival times from a thread while the main thread
    collects them.  Returns (latency from submission in ms, latency from the
    scheduled arrival in ms, records, elapsed s, server stats): when the
    submitting thread falls behind the arrivals, the second shows it."""
    srv = tds.Server(idx, max_batch_segments=1 << 17, max_batch_requests=2048, slots=2,
                     result_capacity=1 << 21, default_reserve=512, cpu_route_tests=route)
    # warm-up, not timed: the requests one at a time, then all at once (full
    # batches on both slots)
    for r in reqs[:100]:
        srv.wait(srv.submit(r.Q, r.d, r.t_start, r.t_end))
    for t in [srv.submit(r.Q, r.d, r.t_start, r.t_end) for r in reqs[100:200]]:
        srv.wait(t)
    reqs = reqs[200:]
    handles = [tds.prepare_segments(r.Q) for r in reqs]  # marshalled before the run
    base = reqs[0].arrival
    tickets = [None] * len(reqs)
    late = [0.0] * len(reqs)
    t_start = time.perf_counter()

    def submitter():
        for i, r in enumerate(reqs):
            due = r.arrival - base
            dt = due - (time.perf_counter() - t_start)
            if dt > 0:
                time.sleep(dt)
            late[i] = max(0.0, time.perf_counter() - t_start - due)
            tickets[i] = srv.submit(handles[i], r.d, r.t_start, r.t_end)

    th = threading.Thread(target=submitter)
    th.start()
    lat, lat_arr, n_rec = [], [], 0
    for i in range(len(reqs)):
        while tickets[i] is None:
            time.sleep(0.0002)
        recs, ms = srv.wait(tickets[i])
        lat.append(ms)
        lat_arr.append(ms + 1e3 * late[i])
        n_rec += recs.size
    th.join()
    elapsed = time.perf_counter() - t_start
    st = srv.stats()
    srv.close()
    return lat, lat_arr, n_rec, elapsed, st


def flood(tds, idx, reqs, route=0):
    """Every request submitted at once (marshalled beforehand): the server's
    throughput when it always has work queued, and the latencies then."""
    srv = tds.Server(idx, max_batch_segments=1 << 17, max_batch_requests=2048, slots=2,
                     result_capacity=1 << 21, default_reserve=512, max_pending=len(reqs) + 1,
                     cpu_route_tests=route)
    for r in reqs[:200]:
        srv.wait(srv.submit(r.Q, r.d, r.t_start, r.t_end))
    reqs = reqs[200:]
    handles = [tds.prepare_segments(r.Q) for r in reqs]
    t0 = time.perf_counter()
    tickets = [srv.submit(h, r.d, r.t_start, r.t_end) for h, r in zip(handles, reqs)]
    t_sub = time.perf_counter() - t0
    lat = [srv.wait(t)[1] for t in tickets]
    elapsed = time.perf_counter() - t0
    st = srv.stats()
    srv.close()
    out = {"requests": len(reqs), "requests_per_s": round(len(reqs) / elapsed, 1),
           "submit_s": round(t_sub, 4), "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
           "batches": st["batches"], "max_batch_requests": st["max_batch_requests_seen"]}
    if route:
        out["cpu_route_tests"] = route
        out["cpu_routed"] = st["cpu_routed"]
    return out


def serve_leg(tds, idx, seconds, rate, sweep=(10000.0, 20000.0, 40000.0, 80000.0, 160000.0,
                                              320000.0)):
    """The request stream through tds_server: an open-loop run at `rate` for
    `seconds`, the plain FP64 form (one request per call) on its first 5,000
    requests, open-loop runs at rising offered rates until the achieved rate
    falls below the offered one, and a flood of 20,000 requests submitted at
    once (the server's saturation throughput)."""
    import trajgen
    n_req = int(seconds * rate)
    reqs = trajgen.request_stream(n_req + 200, rate=rate)
    lat, lat_arr, n_rec, elapsed, st = open_loop(tds, idx, reqs)
    served = {"offered_rate": rate, "requests": len(lat),
              "requests_per_s": round(len(lat) / elapsed, 1),
              "p50_ms": pct(lat, 50), "p99_ms": pct(lat, 99),
              "p50_from_arrival_ms": pct(lat_arr, 50), "p99_from_arrival_ms": pct(lat_arr, 99),
              "records": n_rec, "batches": st["batches"], "requeued": st["requeued"],
              "max_batch_requests": st["max_batch_requests_seen"]}
    plain = []
    for r in reqs[200:5200]:
        t0 = time.perf_counter()
        idx.search(r.Q, r.d, r.t_start, r.t_end, precision="fp64", capacity=4096)
        plain.append(1e3 * (time.perf_counter() - t0))
    rows = []
    for rt in sweep:
        sreqs = trajgen.request_stream(10200, rate=rt)
        slat, sarr, _, sel, sst = open_loop(tds, idx, sreqs)
        rows.append({"offered_rate": rt, "requests_per_s": round(len(slat) / sel, 1),
                     "p50_ms": pct(slat, 50), "p99_ms": pct(slat, 99),
                     "p50_from_arrival_ms": pct(sarr, 50), "p99_from_arrival_ms": pct(sarr, 99),
                     "batches": sst["batches"]})
        if len(slat) / sel < 0.9 * rt:
            break
    fl = flood(tds, idx, trajgen.request_stream(20200, rate=1e9, seed=91))
    # hybrid: requests with at most HOST_ROUTE_TESTS candidate pairs searched
    # on host threads, the same stream
    rlat, rarr, rrec, rel, rst = open_loop(tds, idx, reqs, route=HOST_ROUTE_TESTS)
    routed = {"offered_rate": rate, "requests": len(rlat), "cpu_route_tests": HOST_ROUTE_TESTS,
              "cpu_routed": rst["cpu_routed"], "requests_per_s": round(len(rlat) / rel, 1),
              "p50_ms": pct(rlat, 50), "p99_ms": pct(rlat, 99),
              "p50_from_arrival_ms": pct(rarr, 50), "p99_from_arrival_ms": pct(rarr, 99),
              "records": rrec, "batches": rst["batches"]}
    if rrec != n_rec:
        raise RuntimeError(f"routed serving found {rrec} records, GPU-only {n_rec}")
    rfl = flood(tds, idx, trajgen.request_stream(20200, rate=1e9, seed=91),
                route=HOST_ROUTE_TESTS)
    return {
        "served_fp32": served,
        "served_hybrid": routed,
        "served_rate_sweep": rows,
        "served_flood": fl,
        "served_hybrid_flood": rfl,
        "saturation_requests_per_s": max([r["requests_per_s"] for r in rows] +
                                         [fl["requests_per_s"]]),
        "plain_fp64": {"requests": len(plain),
                       "requests_per_s": round(len(plain) / (sum(plain) * 1e-3), 1),
                       "p50_ms": pct(plain, 50), "p99_ms": pct(plain, 99),
                       "note": "one request per call, back to back (service time, no queueing)"},
    }


# Host route threshold of the hybrid serving run: requests whose candidate
# ranges hold at most this many pairs run on the host (on the uniform1m index
# a clipped query segment has about 2,500-5,000 candidates, of which the
# block boxes leave a few hundred: up to about 100 active segments).
HOST_ROUTE_TESTS = 500000

LEGS = ("galaxy", "uniform1m", "dense", "tiny", "serve", "self_join", "fsg")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--legs", default=",".join(LEGS),
                    help="comma-separated legs to run (the headline is the first of "
                         "galaxy, uniform1m, dense, tiny that runs)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64-form", action="store_true",
                    help="skip the plain FP64 form and the endpoint-error comparison")
    ap.add_argument("--summarize-traffic", nargs=3, metavar=("WORKLOAD", "FETCH_CSV", "WRITE_CSV"),
                    help="write the traffic summary from two counter CSVs and exit (no GPU)")
    ap.add_argument("--summarize-valu", nargs=2, metavar=("WORKLOAD", "CSV"),
                    help="write the instruction-counter summary from a counter CSV and exit")
    ap.add_argument("--no-tune", action="store_true",
                    help="library defaults instead of the autotuner's choice for each search leg")
    ap.add_argument("--fixed", default="",
                    help="launch parameters for every search leg instead of tuning, e.g. "
                         "num_bins=38,chunk=1024,grid_waves=8192,tile=4,precision=fp32")
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="length of the open-loop serving run at 5,000 requests/s")
    ap.add_argument("--calib-copy-mb", type=int, default=0,
                    help="run one device copy of this many MiB first (counter calibration)")
    args = ap.parse_args()
    if args.summarize_valu:
        summarize_valu(*args.summarize_valu)
        return
    if args.summarize_traffic:
        summarize_traffic(*args.summarize_traffic)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(sharding is described in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    legs = [x for x in args.legs.split(",") if x]
    for x in legs:
        if x not in LEGS:
            raise SystemExit(f"unknown leg {x}; legs are {','.join(LEGS)}")

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
    cores = os.cpu_count() or 1
    with_cpu = not args.no_cpu
    # oracle samples: about 10-15 s for the headline, a few s for the others
    cpu_traj = {"galaxy": 200, "uniform1m": 100, "dense": 100, "tiny": 100}
    results = {}
    uni = None
    for name in ("galaxy", "uniform1m", "dense", "tiny"):
        if name not in legs and not (name == "uniform1m" and
                                     any(x in legs for x in ("serve", "self_join", "fsg"))):
            continue
        w = getattr(trajgen, name)()
        tuned = None
        if args.fixed:
            tuned = {"num_bins": 0, "chunk": 0, "grid_waves": 0, "tile": 0, "refine": "default",
                     "deal": "default", "output": "default", "precision": "fp32"}
            for kv in args.fixed.split(","):
                k, v = kv.split("=")
                tuned[k] = v if k in ("precision", "refine", "deal", "output") else int(v)
        elif not args.no_tune and name in legs:
            tb = time.perf_counter()
            best = autotune.tune(w.D, w.Q, w.ds, w.window, cache=None,
                                 space=start_space(autotune, name))
            tuned = {k: best[k] for k in ("num_bins", "chunk", "grid_waves", "tile", "refine",
                                          "deal", "output", "precision")}
            tuned["trials"] = best["trials"]
            tuned["tuning_s"] = round(time.perf_counter() - tb, 2)
        leg = SearchLeg(tds, w, tuned)
        if name in legs:
            first = not results
            results[name] = leg.report(args.steps if first else max(3, args.steps // 2),
                                       args.warmup if first else 1, cpu_traj[name], cores,
                                       with_cpu, not args.no_fp64_form)
            print(f"# {name}: {json.dumps(results[name])}", file=sys.stderr, flush=True)
        if name == "uniform1m":
            uni = (w, leg)
        else:
            leg.close()
            del leg
        torch.cuda.empty_cache()
    extra = {}
    if uni is not None:
        w, leg = uni
        if "serve" in legs:
            extra.update(serve_leg(tds, leg.idx, args.serve_seconds, 5000.0))
        if "self_join" in legs:
            extra["self_join"] = self_join_leg(tds, leg.idx, w.D, 25.0)
        if "fsg" in legs:
            extra["fsg"] = fsg_leg(tds, leg.idx, device_segments(w.Q),
                                   dict(zip(w.ds, leg.counts)), w.ds, *w.window)
        leg.close()
    if not results:
        print(json.dumps({"metric": METRIC, "legs": extra}), flush=True)
        return
    head_name = next(iter(results))
    head = results[head_name]
    descr = {
        "galaxy": "galaxy: 2 x 100,000 Plummer particles on an approaching orbit, 20 snapshots "
                  "(3,800,000 entry segments); 2,000 query particles (38,000 segments), "
                  "d = 0.5 kpc over the full span; FP32 filter + FP64 recheck, spatial layout",
        "uniform1m": "uniform1m: 2,500 trajectories x 401 timesteps (1,000,000 segments), "
                     "500 query trajectories (200,000 segments) over [0,400], d in {1,5,25} as "
                     "three requests of one batch; FP32 filter + FP64 recheck, spatial layout",
        "dense": "dense: 10,000 trajectories x 101 timesteps in [0,50]^3 (1,000,000 segments), "
                 "1,000 query trajectories (100,000 segments), d = 2; FP32 filter + FP64 recheck",
        "tiny": "tiny: 2,000 trajectories x 50 timesteps (98,000 segments), 100 query "
                "trajectories (4,900 segments), d = 5; FP32 filter + FP64 recheck",
    }[head_name]
    rec = {"metric": METRIC, "value": head["value"], "unit": UNIT, "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": head["ms_per_step"],
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32+f64",
           "data": "synthetic",
           "config": {"workload": descr, "n_entries": head["n_entries"],
                      "n_query_segments": head["n_query_segments"], "d": head["d"],
                      "num_bins": head["num_bins"]},
           "roofline": head["roofline"], "cpu_baseline": head.get("cpu_baseline"),
           "queries_per_s": head["queries_per_s"],
           "results_per_step": sum(head["results_per_d"].values()),
           "fp32_endpoint_error": head["fp32_endpoint_error"],
           "headline": head}
    if rec["cpu_baseline"]:
        rec["cpu_baseline"]["cpu_model"] = cpu_model()
    rec["configs"] = {k: v for k, v in results.items() if k != head_name}
    rec.update(extra)
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
