"""The library's kernels run on the CPU: the HIP sources of the index build,
the search (query preparation, bucket scan, distance kernel, FP64 recheck,
result append), the fixed spatial grid, the merge and the radix sort are
compiled as host code with clang++ and AddressSanitizer against a small
emulation of the HIP runtime (tests/emu/hip: the threads of a block as host
threads, wave intrinsics through a per-wave barrier, device memory from
malloc).  Every memory access the kernels make is then bounds-checked, and
their results are compared with the oracle's.  This checks the kernels'
indexing and the host code around them on a machine without a GPU; the GPU
parity tests check the same entry points on the device.

The emulated runs spend most of their time waiting in barriers, not
computing, so all of them are started together (a module fixture) and each
test checks its own run's output."""
import concurrent.futures as cf
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import trajgen

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1410_2698_amd", "csrc")
RESULT_DTYPE = np.dtype([("q_seg", "<u4"), ("e_seg", "<u4"), ("q_traj", "<u4"), ("e_traj", "<u4"),
                         ("t_lo", "<f8"), ("t_hi", "<f8")])
TEMPORAL, SPATIAL = 1, 2  # index layouts (C ABI values)
FP64, FP32 = 1, 2         # search precisions (C ABI values)
QUEUED, INLINE = 1, 2     # places of the FP32 refinement (C ABI values)
DIRECT, STAGED = 1, 2     # output modes (C ABI values)


def columns(S):
    return np.stack([np.asarray(getattr(S, k), np.float64)
                     for k in ("xs", "ys", "zs", "ts", "xe", "ye", "ze", "te")]
                    + [np.asarray(S.traj, np.float64)])


def _merge_random():
    rng = np.random.default_rng(4)
    n = 3000  # two radix-sort tiles
    recs = np.zeros(n, RESULT_DTYPE)
    recs["q_seg"] = np.arange(n)
    recs["q_traj"] = rng.integers(0, 40, n)
    recs["e_traj"] = rng.integers(0, 40, n) * 70001  # ids of 22 bits: 4 pair digits
    lo = rng.integers(-800, 800, n) / 8.0
    recs["t_lo"] = lo
    recs["t_hi"] = lo + rng.integers(0, 24, n) / 8.0
    return recs


def _merge_degenerate():
    # one t_lo for every record (no t_lo digit differs: no pass of that
    # sort) and the largest ids (all eight pair digits)
    n = 600
    recs = np.zeros(n, RESULT_DTYPE)
    recs["q_traj"] = np.where(np.arange(n) % 3 == 0, 0xFFFFFFFF, 7)
    recs["e_traj"] = np.where(np.arange(n) % 2 == 0, 0xFFFFFFFF, 0)
    recs["t_lo"] = 2.5
    recs["t_hi"] = 2.5 + (np.arange(n) % 5)
    return recs


FILL_CASES = {
    "fill_exact": (1, 64, 64, 6, 1.0, 0, 0),            # capacity = count
    "fill_more": (2, 64, 128, 6, 1.0, 5000, 0),         # room to spare: holes below count
    "fill_less_one": (3, 37, 64, 3, 1.0, -1, 0),        # one short, an odd wave count
    "fill_half": (4, 200, 64, 8, 0.5, 0, 0),            # overflow
    "fill_aligned": (5, 200, 256, 10, 0.6, 0, 1),       # capacity a multiple of the chunk
    "fill_big_chunk": (6, 48, 2048, 40, 0.9, 0, 0),     # the largest chunk
    "fill_zero_cap": (7, 16, 64, 4, 0.0, 0, 0),         # nothing kept
    "fill_empty": (8, 16, 64, 0, 1.0, 0, 0),            # no results, no reservation
    "fill_max_waves": (9, 16384, 64, 2, 1.0, 0, 0),     # the most waves of a direct launch
}


def _cvt_inputs():
    """Doubles for the directed FP64 -> FP32 conversions: random magnitudes
    over the whole double range, floats exactly, their neighbours and
    midpoints, zeros, subnormals, the float range's ends, infinities."""
    rng = np.random.default_rng(12)
    x = [rng.standard_normal(20000) * 10.0 ** rng.uniform(-330, 300, 20000)]
    f = rng.standard_normal(5000).astype(np.float32).astype(np.float64)
    x += [f, np.nextafter(f, np.inf), np.nextafter(f, -np.inf),
          (f + np.nextafter(f.astype(np.float32), np.float32(np.inf)).astype(np.float64)) / 2]
    fl = np.finfo(np.float32)
    x.append(np.array([0.0, -0.0, 1e-50, -1e-50, 1e-45, -1e-45, 1.4e-45, float(fl.tiny),
                       -float(fl.tiny), float(fl.max), -float(fl.max), float(fl.max) * 1.0000001,
                       -float(fl.max) * 1.0000001, 1e300, -1e300, np.inf, -np.inf]))
    return np.concatenate(x)


def _jobs():
    """Every emulated run: name -> (kind, inputs, arguments after the inputs).
    Kinds "search" and "fsg" take D and Q, "selfjoin" D, "merge" records."""
    tiny = trajgen.tiny(scale=0.05)  # 100 trajectories (4,900 entries), 5 query trajectories
    tiny04 = trajgen.tiny(scale=0.04)
    J = {}
    for g in [(1, 1, 1), (7, 3, 5), (50, 50, 50)]:
        J["fsg_%dx%dx%d" % g] = ("fsg", (tiny.D, tiny.Q), [*g, 8.0, 0.0, 49.0])
    for layout, prec, d in [(SPATIAL, FP32, 8.0), (SPATIAL, FP64, 30.0), (TEMPORAL, FP32, 30.0)]:
        J[f"search_{layout}_{prec}_{d:g}"] = ("search", (tiny.D, tiny.Q),
                                              [layout, prec, d, 0.0, 49.0, 100000])
    # the database against itself at a distance larger than the data's
    # extent: every time-overlapping pair is a result (each query segment
    # meets the co-temporal segment of each of the 100 trajectories), so a
    # work item of 64 query segments has 6,400 results and fills its wave's
    # 2,048-record stage several times before it ends; the items outnumber
    # the emulated waves, so the dynamic item counters are used as well
    for prec in (FP32, FP64):
        J[f"flush_{prec}"] = ("search", (tiny.D, tiny.D),
                              [SPATIAL, prec, 250.0, 0.0, 49.0, 600000, 0, 0, 0, STAGED])
    # direct output of the same search: chunk reservations kept across
    # items, and a buffer whose capacity is the exact count (positions past
    # it go to the scratch buffer and come back in the fill) or less than it
    for cap in (490000, 489999, 1000):
        J[f"direct_{cap}"] = ("search", (tiny.D, tiny.D),
                              [SPATIAL, FP32, 250.0, 0.0, 49.0, cap, 0, 0, 0, DIRECT])
    # the closest-approach refinement inline in the filter walk, at both
    # tiles, on a sparse and a dense search (at d = 250 every time-overlapping
    # pair passes every test)
    for d, tile in [(8.0, 2), (30.0, 4), (250.0, 2)]:
        J[f"inline_{d:g}_{tile}"] = ("search", (tiny.D, tiny.Q),
                                     [SPATIAL, FP32, d, 0.0, 49.0, 100000, 0, INLINE, tile])
    # more query buckets than the parted slot counters take (2,000 bins:
    # 8,000 buckets, one counter part); merged keys (over 16,384 bins) take
    # minutes here and are covered by the GPU tests
    J["many_bins"] = ("search", (tiny.D, tiny.Q), [SPATIAL, FP32, 8.0, 0.0, 49.0, 100000, 2000])
    # a result buffer smaller than the result set: the total is reported
    J["overflow"] = ("search", (tiny.D, tiny.Q), [SPATIAL, FP32, 30.0, 0.0, 49.0, 100])
    J["selfjoin"] = ("selfjoin", (tiny04.D,), [SPATIAL, FP32, 4.0, 0.0, 49.0, 200000])
    # pairs built to pass at d (1 + eps) around coordinates of 1e6, eps down
    # to 0 (decided by the canonical evaluation's rounding): every filter in
    # front of it must keep every pair the oracle accepts
    gD, gQ = trajgen.grazing(660, 77, 0.5, 1e6)
    for refine, tile in [(QUEUED, 4), (INLINE, 2)]:
        J[f"graze_{refine}"] = ("search", (gD, gQ),
                                [SPATIAL, FP32, 0.5, -1e9, 1e9, 100000, 0, refine, tile])
    J["hostsearch_graze"] = ("hostsearch", (gD, gQ), [0.5, -1e9, 1e9])
    # the serving loop's host route over a host copy of the index
    J["hostsearch"] = ("hostsearch", (tiny.D, tiny.Q), [30.0, 3.5, 40.25])
    J["hostsearch_all"] = ("hostsearch", (tiny.D, tiny.Q), [250.0, 3.5, 40.25])
    # the direct output's fill pass alone on synthetic reservation patterns
    # (seed, waves, chunk, runs per wave at most, capacity = floor(count *
    # frac) + add, rounded down to a multiple of the chunk if align)
    for name, args in FILL_CASES.items():
        J[name] = ("fill", None, list(args))
    # the FP32 filter against the canonical evaluation on two million grazing
    # pairs at random scales
    J["filtercheck"] = ("filtercheck", None, [5, 2000000])
    J["cvt"] = ("cvt", _cvt_inputs(), [])
    J["merge_random"] = ("merge", _merge_random(), [3000])
    J["merge_degenerate"] = ("merge", _merge_degenerate(), [600])
    J["merge_degenerate_cap3"] = ("merge", _merge_degenerate(), [3])
    return J, {"tiny": tiny, "tiny04": tiny04, "graze": (gD, gQ)}


def _build_harness(out):
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    cxx = os.path.join(rocm, "llvm", "bin", "clang++")
    if not os.path.exists(cxx):
        cxx = shutil.which("clang++")
    if cxx is None:
        pytest.skip("clang++ not available")
    # host-only build (no GPU code); the canonical evaluation is compiled
    # without contraction, as for the GPU; search.hip is included by the
    # harness itself
    cmd = [cxx, "-std=c++20", "-O1", "-g", "-fsanitize=address", "-fno-omit-frame-pointer",
           "-ffp-contract=off", "-Wno-unknown-attributes", "-Wno-ignored-attributes",
           "-I", os.path.join(ROOT, "tests", "emu"), "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           "-x", "c++", os.path.join(CSRC, "fsg.hip"), os.path.join(CSRC, "radix_sort.hip"),
           os.path.join(CSRC, "traj_merge.hip"), os.path.join(CSRC, "index_build.hip"),
           os.path.join(CSRC, "host_search.hip"), "-x", "none",
           os.path.join(ROOT, "tests", "emu", "harness.cpp"), "-o", out, "-lpthread"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("emulation build failed:\n" + r.stderr[-4000:])


def _run_job(harness, d, kind, inputs, args):
    os.makedirs(d, exist_ok=True)
    out = os.path.join(d, "out.bin")
    if kind == "merge":
        inputs.astype(RESULT_DTYPE).tofile(os.path.join(d, "recs.bin"))
        argv = [harness, "merge", os.path.join(d, "recs.bin"), *args, out]
    elif kind == "fill":
        out = os.path.join(d, "fill")
        argv = [harness, "fill", *args, out]
    elif kind == "filtercheck":
        argv = [harness, "filtercheck", *args]
    elif kind == "cvt":
        inputs.astype(np.float64).tofile(os.path.join(d, "x.bin"))
        argv = [harness, "cvt", os.path.join(d, "x.bin"), out]
    else:
        files = []
        for i, S in enumerate(inputs):
            f = os.path.join(d, f"in{i}.bin")
            columns(S).tofile(f)
            files.append(f)
        if kind == "hostsearch":  # harness hostsearch D Q d t0 t1 <out>
            argv = [harness, kind, *files, *args, out]
        else:  # harness <kind> <inputs> <six numbers> <out> [bins]
            argv = [harness, kind, *files, *args[:6], out, *args[6:]]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    r = subprocess.run([str(a) for a in argv], capture_output=True, text=True, env=env,
                       timeout=900)
    return r, out


@pytest.fixture(scope="module")
def emu(tmp_path_factory):
    base = tmp_path_factory.mktemp("emu")
    harness = str(base / "harness")
    _build_harness(harness)
    jobs, data = _jobs()
    order = sorted(jobs, key=lambda n: (not n.startswith("flush"), n))  # heaviest first
    with cf.ThreadPoolExecutor(4) as ex:
        futs = {n: ex.submit(_run_job, harness, str(base / n), *jobs[n]) for n in order}
        res = {n: f.result() for n, f in futs.items()}
    return res, data


def result(emu, name):
    """(integers the harness printed, path of its output file) of one run."""
    r, out = emu[0][name]
    assert r.returncode == 0, f"emulated kernels failed:\n{r.stdout[-2000:]}\n{r.stderr[-6000:]}"
    return tuple(int(v) for v in r.stdout.split()), out


def same_records(got, want):
    key = lambda r: np.lexsort((r["e_seg"], r["q_seg"]))
    got, want = got[key(got)], want[key(want)]
    assert got.size == want.size
    for f in ("q_seg", "e_seg", "q_traj", "e_traj"):
        assert np.array_equal(got[f], want[f]), f
    for f in ("t_lo", "t_hi"):
        assert np.all(np.abs(got[f] - want[f]) <= 1e-9 * np.maximum(1.0, np.abs(want[f]))), f


@pytest.mark.parametrize("grid", ["1x1x1", "7x3x5", "50x50x50"])
def test_grid_search_emulated(emu, grid):
    (st, n), out = result(emu, f"fsg_{grid}")
    w = emu[1]["tiny"]
    assert st == 0
    want = oracle.search(w.Q, w.D, 8.0, 0.0, 49.0)
    assert want.size > 0 and n == want.size
    same_records(np.fromfile(out, dtype=RESULT_DTYPE), want)


@pytest.mark.parametrize("layout,prec,d", [(SPATIAL, FP32, 8.0), (SPATIAL, FP64, 30.0),
                                           (TEMPORAL, FP32, 30.0)])
def test_search_emulated(emu, layout, prec, d):
    # the whole search path on the CPU: index build, query preparation,
    # buckets, work items, distance kernel, FP64 recheck and append
    (st, n, ftests, _), out = result(emu, f"search_{layout}_{prec}_{d:g}")
    w = emu[1]["tiny"]
    assert st == 0
    want = oracle.search(w.Q, w.D, d, 0.0, 49.0)
    assert want.size > 0 and n == want.size and ftests > 0
    same_records(np.fromfile(out, dtype=RESULT_DTYPE), want)


@pytest.mark.parametrize("prec", [FP32, FP64])
def test_search_emulated_stage_flushes(emu, prec):
    (st, n, _, flushes), out = result(emu, f"flush_{prec}")
    w = emu[1]["tiny"]
    assert st == 0
    want = oracle.search(w.D, w.D, 250.0, 0.0, 49.0)
    assert want.size == len(w.D) * 100 and n == want.size
    assert flushes > 0
    same_records(np.fromfile(out, dtype=RESULT_DTYPE), want)


@pytest.mark.parametrize("d,tile", [(8.0, 2), (30.0, 4), (250.0, 2)])
def test_search_emulated_inline_refinement(emu, d, tile):
    (st, n, ftests, _), out = result(emu, f"inline_{d:g}_{tile}")
    w = emu[1]["tiny"]
    assert st == 0
    want = oracle.search(w.Q, w.D, d, 0.0, 49.0)
    assert want.size > 0 and n == want.size and ftests > 0
    if d == 250.0:
        assert want.size == len(w.Q) * 100
    same_records(np.fromfile(out, dtype=RESULT_DTYPE), want)


@pytest.mark.parametrize("cap", [490000, 489999, 1000])
def test_search_emulated_direct_output(emu, cap):
    # 490,000 results: at the exact capacity the output is dense and equals
    # the oracle's set; below it the call overflows and the buffer holds
    # `cap` distinct results (the holes below the capacity were filled)
    (st, n, _, reservations), out = result(emu, f"direct_{cap}")
    w = emu[1]["tiny"]
    want = oracle.search(w.D, w.D, 250.0, 0.0, 49.0)
    assert want.size == 490000 and n == want.size and reservations > 0
    got = np.fromfile(out, dtype=RESULT_DTYPE)
    if cap >= n:
        assert st == 0
        same_records(got, want)
    else:
        assert st == 2  # TDS_E_OVERFLOW
        assert got.size == cap
        keys = lambda r: set(zip(r["q_seg"].tolist(), r["e_seg"].tolist()))
        k = keys(got)
        assert len(k) == cap and k <= keys(want)


def test_search_emulated_many_bins(emu):
    (st, n, _, _), out = result(emu, "many_bins")
    w = emu[1]["tiny"]
    assert st == 0
    want = oracle.search(w.Q, w.D, 8.0, 0.0, 49.0)
    assert want.size > 0 and n == want.size
    same_records(np.fromfile(out, dtype=RESULT_DTYPE), want)


def test_search_emulated_overflow(emu):
    (st, n, _, _), _ = result(emu, "overflow")
    w = emu[1]["tiny"]
    want = oracle.search(w.Q, w.D, 30.0, 0.0, 49.0)
    assert st == 2 and n == want.size  # TDS_E_OVERFLOW


def test_self_join_emulated(emu):
    (st, n, _, _), out = result(emu, "selfjoin")
    w = emu[1]["tiny04"]
    assert st == 0
    want = oracle.self_join(w.D, 4.0, 0.0, 49.0)
    assert want.size > 0 and n == want.size
    same_records(np.fromfile(out, dtype=RESULT_DTYPE), want)


@pytest.mark.parametrize("job,d", [("hostsearch", 30.0), ("hostsearch_all", 250.0)])
def test_host_search_emulated(emu, job, d):
    """The host search of the serving loop's host route (host copy of the
    index, same candidate ranges, FP32 filter and canonical FP64 evaluation)
    against the oracle, in a window that clips segments at both ends.  At
    d = 30 the block boxes prune candidates; at d = 250 every time-overlapping
    pair is a result and nothing is pruned."""
    (st, n, cand), out = result(emu, job)
    w = emu[1]["tiny"]
    assert st == 0
    want = oracle.search(w.Q, w.D, d, 3.5, 40.25)
    assert want.size > 100 and n == want.size
    # the routing cost model: the candidate pairs of the clipped segments'
    # ranges, at least one per trajectory and clipped segment, whatever d
    assert cand >= 5 * 36 * 100 and cand >= n
    assert cand == result(emu, "hostsearch_all")[0][2]
    got = np.fromfile(out, dtype=RESULT_DTYPE)
    same_records(got, want)
    # the evaluation is the kernels' canonical one: endpoints bit for bit
    key = lambda r: np.lexsort((r["e_seg"], r["q_seg"]))
    assert got[key(got)].tobytes() == want[key(want)].tobytes()


@pytest.mark.parametrize("name", list(FILL_CASES))
def test_fill_pass_emulated(emu, name):
    """The direct output's fill pass on a synthetic reservation pattern: the
    first T = min(count, capacity) positions must end dense, the results the
    distance kernel placed below T must stay where they are, and the holes
    must be filled by the first results past T in position order (those the
    pass takes), each once."""
    (st, count, cap, T, holes, R), prefix = result(emu, name)
    assert st == 0 and T == min(count, cap)
    allr = np.fromfile(prefix + ".all", dtype=RESULT_DTYPE)
    before = np.fromfile(prefix + ".before", dtype=RESULT_DTYPE)
    after = np.fromfile(prefix + ".after", dtype=RESULT_DTYPE)
    assert allr.size == count and before.size == T and after.size == T
    assert np.array_equal(allr["q_seg"], np.arange(count))
    hole = before["q_seg"] == 0xFFFFFFFF
    assert int(hole.sum()) == holes and R >= count + holes
    assert not np.any(after["q_seg"] == 0xFFFFFFFF)
    # every record is one of the results, as it was placed, and appears once
    assert np.array_equal(after["e_seg"], allr["e_seg"][after["q_seg"]])
    assert np.unique(after["q_seg"]).size == T
    assert np.array_equal(after[~hole], before[~hole])
    pos = allr["e_seg"].astype(np.int64)
    past = np.sort(pos[pos >= T])[:holes]
    moved = np.sort(after["e_seg"][hole].astype(np.int64))
    assert np.array_equal(moved, past)
    assert np.all(allr["e_traj"][after["q_seg"][hole]] == 1)  # kept in output or scratch
    if count <= cap:
        assert np.array_equal(np.sort(after["q_seg"]), np.arange(count))
    if name == "fill_empty":
        assert count == 0 and R == 0
    if name == "fill_zero_cap":
        assert T == 0 and count > 0
    if name == "fill_exact":
        assert count == cap and holes > 0


@pytest.mark.parametrize("job", ["graze_1", "graze_2", "hostsearch_graze"])
def test_grazing_pairs_emulated(emu, job):
    """Grazing pairs (see trajgen.grazing) through the FP32 kernel form with
    the refinement queued and inline, and through the host route: the same
    records as the oracle, whose evaluation decides the closest pairs by its
    FP64 rounding."""
    (st, n, *_), out = result(emu, job)
    gD, gQ = emu[1]["graze"]
    assert st == 0
    want = oracle.search(gQ, gD, 0.5, -1e9, 1e9)
    assert want.size > 200 and n == want.size
    same_records(np.fromfile(out, dtype=RESULT_DTYPE), want)


def test_directed_conversions(emu):
    """f32_rd / f32_ru (the outward roundings of the filter's spheres, time
    extents and boxes) against their definition: the largest float not above
    x and the smallest float not below it, from numpy's float32 rounding to
    nearest and one step with nextafter where it went the wrong way."""
    (st, n), out = result(emu, "cvt")
    x = _cvt_inputs()
    assert st == 0 and n == x.size
    got = np.fromfile(out, dtype=np.float32).reshape(-1, 2)
    with np.errstate(over="ignore"):  # FLT_MAX steps to infinity, as it should
        f = x.astype(np.float32)
        up = np.where(f.astype(np.float64) < x, np.nextafter(f, np.float32(np.inf)), f)
        dn = np.where(f.astype(np.float64) > x, np.nextafter(f, np.float32(-np.inf)), f)
    assert np.array_equal(got[:, 0].view(np.uint32), dn.view(np.uint32))
    assert np.array_equal(got[:, 1].view(np.uint32), up.view(np.uint32))


def test_filter_keeps_every_accepted_pair(emu):
    """Two million pairs built to pass at d (1 + eps), eps down to 0, with
    lengths, coordinate magnitudes and d spread over twelve decades: every
    pair the canonical FP64 evaluation accepts passes the FP32 sphere test,
    the outward-rounded time test and the segment-box test, each built from
    the end points as the kernels build it.  Boxes without the margins and
    the outward rounding would drop some accepted pairs: the pairs are close
    enough to the boundary for the margins to matter."""
    (st, accepted, misses, naive), _ = result(emu, "filtercheck")
    assert st == 0
    assert accepted > 500000
    assert misses == 0
    assert naive > 0


def same_intervals(got, want):
    assert got.size == want.size
    for f in ("q_traj", "e_traj", "t_lo", "t_hi"):
        assert np.array_equal(got[f], want[f]), f


def test_merge_emulated_random(emu):
    (st, m), out = result(emu, "merge_random")
    assert st == 0
    same_intervals(np.fromfile(out, dtype=oracle.TRAJ_DTYPE),
                   oracle.merge_trajectories(_merge_random()))


def test_merge_emulated_degenerate_keys(emu):
    recs = _merge_degenerate()
    want = oracle.merge_trajectories(recs)
    assert want.size == 4
    (st, m), out = result(emu, "merge_degenerate")
    assert st == 0
    same_intervals(np.fromfile(out, dtype=oracle.TRAJ_DTYPE), want)
    # capacity below the total: the first intervals in order, the total reported
    (st, m), out = result(emu, "merge_degenerate_cap3")
    assert st == 2 and m == 4  # TDS_E_OVERFLOW
    same_intervals(np.fromfile(out, dtype=oracle.TRAJ_DTYPE), want[:3])
