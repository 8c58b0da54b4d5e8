"""GPU parity: the HIP library against the FP64 CPU oracle, through the C ABI.

Result sets must be identical (same (q_seg, e_seg) pairs, ids, no
duplicates); interval endpoints must agree within 1e-9 relative (the GPU
evaluates the same FP64 operation sequence, so they are expected to be
bit-identical and the tests also report how many are).
"""
import math

import numpy as np
import pytest

import oracle
import trajgen

torch = pytest.importorskip("torch")
import paper_1410_2698_amd as tds  # noqa: E402

pytestmark = pytest.mark.gpu

REL = 1e-9


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    tds.load()


def compare(got, want, label=""):
    got = tds.sort_records(got)
    want = oracle.sort_results(want)
    kg = got["q_seg"].astype(np.uint64) << np.uint64(32) | got["e_seg"]
    assert np.unique(kg).size == kg.size, f"{label}: duplicate records"
    assert got.size == want.size, f"{label}: {got.size} records, oracle {want.size}"
    for f in ("q_seg", "e_seg", "q_traj", "e_traj"):
        assert np.array_equal(got[f], want[f]), f"{label}: field {f} differs"
    for f in ("t_lo", "t_hi"):
        err = np.abs(got[f] - want[f])
        tol = REL * np.maximum(1.0, np.abs(want[f]))
        assert np.all(err <= tol), f"{label}: {f} max err {err.max()}"
    return int(np.sum((got["t_lo"] == want["t_lo"]) & (got["t_hi"] == want["t_hi"])))


def build(D, m=0, layout="default"):
    return tds.Index(D, num_bins=m, layout=layout)


def check_tables(ex, ob, n, layout):
    """Bin tables equal the oracle's; the order equals the oracle's t_start
    order (temporal layout) or holds the same entries bin by bin (spatial
    layout, where only the order inside a bin differs)."""
    assert np.array_equal(ex["bin_first"][:-1].astype(np.int64), ob["first"])
    assert ex["bin_first"][-1] == n
    assert np.array_equal(ex["min_ts"], ob["min_ts"])
    assert np.array_equal(ex["max_te"], ob["max_te"])
    assert np.array_equal(ex["cmax_te"], ob["cmax_te"])
    order = ex["order"].astype(np.int64)
    if layout == "temporal":
        assert np.array_equal(order, ob["order"])
    else:
        assert np.array_equal(np.sort(order), np.arange(n))
        f = ex["bin_first"].astype(np.int64)
        for j in range(len(f) - 1):
            assert np.array_equal(np.sort(order[f[j]:f[j + 1]]), np.sort(ob["order"][f[j]:f[j + 1]]))


# ---------------------------------------------------------------- index build

@pytest.mark.parametrize("layout", ["temporal", "spatial"])
@pytest.mark.parametrize("m", [0, 1, 7, 49])
def test_index_tables_match_oracle(m, layout):
    w = trajgen.tiny(scale=0.05)
    idx = build(w.D, m, layout)
    inf = idx.info()
    mm = inf["num_bins"]
    assert inf["layout"] == tds.LAYOUTS[layout]
    if m == 0:
        assert mm == 49  # span 49 / mean duration 1
    ob = oracle.bins(w.D.ts, w.D.te, mm)
    check_tables(idx.export(), ob, len(w.D), layout)
    idx.close()


@pytest.mark.parametrize("layout", ["temporal", "spatial"])
def test_index_tables_large(layout):
    """98,000 entries: the radix sort's count table spans several scan tiles."""
    w = trajgen.tiny()
    idx = build(w.D, 0, layout)
    ob = oracle.bins(w.D.ts, w.D.te, idx.info()["num_bins"])
    check_tables(idx.export(), ob, len(w.D), layout)
    idx.close()


def test_default_layout_is_spatial():
    w = trajgen.tiny(scale=0.01)
    idx = build(w.D)
    assert idx.info()["layout"] == tds.LAYOUTS["spatial"]
    idx.close()


def test_index_tables_irregular_times():
    rng = np.random.default_rng(3)
    n = 5000
    ts = np.round(rng.uniform(-20, 80, n), 2)
    ts[::7] = 0.0
    ts[1::11] = -0.0  # equal start times keep input order
    te = ts + rng.uniform(0.01, 9, n)
    D = trajgen.Segments(xs=rng.normal(size=n), ys=rng.normal(size=n), zs=rng.normal(size=n), ts=ts,
                         xe=rng.normal(size=n), ye=rng.normal(size=n), ze=rng.normal(size=n), te=te,
                         traj=np.arange(n, dtype=np.uint32))
    for m in (1, 13, 1000):
        for layout in ("temporal", "spatial"):
            idx = build(D, m, layout)
            check_tables(idx.export(), oracle.bins(ts, te, m), n, layout)
            idx.close()


def test_paper_example_index_on_gpu():
    """The worked example of the temporal index (15 segments, 4 bins)."""
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", "example_index.txt")
    segs = [l.split() for l in open(path) if l.startswith("segment")]
    bins = [l.split() for l in open(path) if l.startswith("bin")]
    ts = np.array([float(s[2]) for s in segs])
    te = np.array([float(s[3]) for s in segs])
    z = np.zeros_like(ts)
    D = trajgen.Segments(xs=z, ys=z, zs=z, ts=ts, xe=z, ye=z, ze=z, te=te,
                         traj=np.zeros(15, np.uint32))
    idx = build(D, 4)
    ex = idx.export()
    assert list(ex["order"]) == list(range(15))
    for b in bins:
        j, first, last = int(b[1]), int(b[4]), int(b[5])
        assert ex["bin_first"][j] == first and ex["bin_first"][j + 1] - 1 == last
    idx.close()


# ---------------------------------------------------------------- schedule

@pytest.mark.parametrize("window", [(-math.inf, math.inf), (3.5, 40.25), (10.0, 10.5)])
def test_schedule_matches_oracle(window):
    w = trajgen.tiny(scale=0.05)
    idx = build(w.D, 0)
    m = idx.info()["num_bins"]
    rng = np.random.default_rng(11)
    nq = 3000
    qts = rng.uniform(-3, 52, nq)
    qte = qts + rng.uniform(0.001, 4, nq)
    qts[:49] = np.arange(49.0)
    qte[:49] = qts[:49] + 1.0
    z = np.zeros(nq)
    Q = trajgen.Segments(xs=z, ys=z, zs=z, ts=qts, xe=z, ye=z, ze=z, te=qte,
                         traj=np.zeros(nq, np.uint32))
    lo, hi = idx.schedule(Q, *window)
    olo, ohi = oracle.schedule(w.D.ts, w.D.te, m, qts, qte, *window)
    assert np.array_equal(lo.astype(np.int64), olo)
    assert np.array_equal(hi.astype(np.int64), ohi)
    idx.close()


# ---------------------------------------------------------------- search parity

@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_tiny_config_full(prec):
    """2,000 trajectories x 50 steps (98,000 segments), 100 query trajectories,
    d = 5 on [0, 49]."""
    w = trajgen.tiny()
    idx = build(w.D)
    want = oracle.search(w.Q, w.D, 5.0, 0.0, 49.0)
    got = idx.search(w.Q, 5.0, 0.0, 49.0, precision=prec)
    same = compare(got, want, f"tiny/{prec}")
    print(f"tiny/{prec}: {got.size} records, {same} bit-identical endpoints, stats {idx.last_stats}")
    assert len(want) > 1000
    idx.close()


@pytest.mark.parametrize("cfg,scale,d", [
    ("uniform1m", 0.02, 150.0),
    ("uniform1m", 0.02, 60.0),
    ("dense", 0.02, 2.0),
    ("galaxy", 0.01, 0.5),
])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_reduced_configs(cfg, scale, d, prec):
    kw = {"n_pts": 61} if cfg in ("uniform1m", "dense") else {}
    w = trajgen.CONFIGS[cfg](scale, **kw)
    idx = build(w.D)
    want = oracle.search(w.Q, w.D, d, *w.window)
    got = idx.search(w.Q, d, *w.window, precision=prec)
    compare(got, want, f"{cfg}/{prec}")
    print(f"{cfg} d={d} {prec}: {got.size} records, stats {idx.last_stats}")
    idx.close()


@pytest.mark.parametrize("cfg,scale,d", [
    ("uniform1m", 0.02, 25.0),
    ("dense", 0.02, 2.0),
    ("galaxy", 0.01, 0.5),
])
def test_spatial_and_temporal_layouts_same_results(cfg, scale, d):
    """Subdividing the bins in space changes which pairs are tested, never the
    result: both layouts give the oracle's set with identical bytes."""
    kw = {"n_pts": 61} if cfg in ("uniform1m", "dense") else {}
    w = trajgen.CONFIGS[cfg](scale, **kw)
    want = oracle.search(w.Q, w.D, d, *w.window)
    got, stats = {}, {}
    for layout in ("temporal", "spatial"):
        idx = build(w.D, 0, layout)
        for prec in ("fp32", "fp64"):
            r = idx.search(w.Q, d, *w.window, precision=prec)
            compare(r, want, f"{cfg}/{layout}/{prec}")
            got[layout, prec] = tds.sort_records(r).tobytes()
            stats[layout, prec] = dict(idx.last_stats)
        idx.close()
    assert len(set(got.values())) == 1
    t, s = stats["temporal", "fp32"], stats["spatial", "fp32"]
    assert t["candidate_tests"] == s["candidate_tests"]
    assert t["block_tests"] == 0 and s["block_tests"] > 0
    assert t["filter_tests"] <= t["candidate_tests"]
    assert s["filter_tests"] <= t["filter_tests"]
    print(f"{cfg}: candidate {s['candidate_tests']}, filter temporal {t['filter_tests']}, "
          f"spatial {s['filter_tests']} after {s['block_tests']} block tests")


def test_spatial_layout_culls_pairs():
    """With hundreds of entries per bin, the block boxes remove most pairs
    before the filter; the result stays the oracle's."""
    w = trajgen.uniform1m(0.2, n_pts=61)  # 500 trajectories: 500 entries per bin
    sl = w.query_traj_slices()
    Q = w.Q.take(np.arange(sl[0][0], sl[19][1]))
    want = oracle.search(Q, w.D, 5.0, *w.window)
    stats = {}
    for layout in ("temporal", "spatial"):
        idx = build(w.D, 0, layout)
        compare(idx.search(Q, 5.0, *w.window), want, layout)
        stats[layout] = dict(idx.last_stats)
        idx.close()
    t, s = stats["temporal"], stats["spatial"]
    print(f"filter tests: temporal {t['filter_tests']}, spatial {s['filter_tests']}")
    assert s["filter_tests"] < 0.7 * t["filter_tests"]


def test_huge_coordinates():
    """Positions near the top of the double range: FP32 spheres become
    infinite and must pass every pair on to the FP64 code."""
    rng = np.random.default_rng(8)
    rows = []
    for k in range(300):
        big = 10.0 ** float(rng.choice([20, 100, 300, 307]))
        p = rng.choice([-1.0, 1.0], 3) * big
        q = p + rng.normal(size=3) * float(rng.choice([0.0, 1.0, big * 1e-3]))
        t = float(rng.integers(0, 20))
        rows.append([*p, t, *q, t + 1.0])
    rows += [[0, 0, 0, 0, 1, 1, 1, 5], [1e308, 0, 0, 2, -1e308, 0, 0, 3]]
    D = _seg(rows)
    Q = _seg(rows[::3])
    for layout in ("temporal", "spatial"):
        idx = build(D, 0, layout)
        for d in (0.0, 1.0, 1e300):
            want = oracle.search(Q, D, d, -math.inf, math.inf)
            for prec in ("fp32", "fp64"):
                compare(idx.search(Q, d, precision=prec), want, f"huge {layout} d={d} {prec}")
        idx.close()


@pytest.mark.parametrize("offset", [0.0, 1e3, 1e6])
def test_grazing_pairs(offset):
    """Pairs built to pass at d (1 + eps), eps from 1e-5 down to 0, around
    coordinates of magnitude `offset`: the closest ones are decided by the
    FP64 rounding of the canonical evaluation, so every filter in front of it
    (block boxes, spheres and time extents, the closest-approach refinement,
    in every kernel form) must keep every pair the oracle accepts."""
    D, Q = trajgen.grazing(2000, 77, 0.5, offset)
    want = oracle.search(Q, D, 0.5, -math.inf, math.inf)
    assert want.size > 600  # about half of the closest pairs and all at eps < 0
    for layout in ("spatial", "temporal"):
        idx = build(D, 0, layout)
        for kw in ({"precision": "fp32", "refine": "queued", "tile": 4},
                   {"precision": "fp32", "refine": "inline", "tile": 2},
                   {"precision": "fp32", "refine": "inline", "tile": 4, "output": "staged"},
                   {"precision": "fp64"}):
            compare(idx.search(Q, 0.5, **kw), want, f"grazing {offset} {layout} {kw}")
        idx.close()


def test_fp32_and_fp64_forms_bit_identical():
    w = trajgen.dense(0.03, n_pts=41)
    idx = build(w.D)
    a = tds.sort_records(idx.search(w.Q, 3.0, *w.window, precision="fp32"))
    s32 = dict(idx.last_stats)
    b = tds.sort_records(idx.search(w.Q, 3.0, *w.window, precision="fp64"))
    assert a.size > 100
    assert a.tobytes() == b.tobytes()
    assert s32["fp64_evals"] < s32["candidate_tests"]
    idx.close()


def test_random_windows_and_ragged_queries():
    w = trajgen.uniform1m(0.01, n_pts=81)
    idx = build(w.D)
    rng = np.random.default_rng(21)
    # ragged query trajectories: random sub-ranges of each query trajectory
    keep = []
    for b, e in w.query_traj_slices():
        s0 = int(rng.integers(b, e))
        keep.extend(range(s0, int(rng.integers(s0 + 1, e + 1))))
    Q = w.Q.take(np.array(keep))
    for t0, t1, d in [(-math.inf, math.inf, 30.0), (12.3, 55.7, 40.0), (0.5, 0.75, 80.0),
                      (79.9, 1e9, 50.0), (-5.0, 0.0, 50.0)]:
        want = oracle.search(Q, w.D, d, t0, t1)
        got = idx.search(Q, d, t0, t1)
        compare(got, want, f"window {t0},{t1}")
    idx.close()


def test_swap_symmetry_on_gpu():
    """Searching D against Q gives the swapped records with identical intervals."""
    w = trajgen.dense(0.01, n_pts=31)
    i1 = build(w.D)
    r1 = tds.sort_records(i1.search(w.Q, 4.0, *w.window))
    i2 = build(w.Q)
    r2 = i2.search(w.D, 4.0, *w.window)
    sw = r2.copy()
    sw["q_seg"], sw["e_seg"] = r2["e_seg"], r2["q_seg"]
    sw["q_traj"], sw["e_traj"] = r2["e_traj"], r2["q_traj"]
    assert r1.size > 50
    assert tds.sort_records(sw).tobytes() == r1.tobytes()
    i1.close()
    i2.close()


# ---------------------------------------------------------------- capacity

def test_overflow_reports_total_and_incremental_passes_match():
    w = trajgen.dense(0.02, n_pts=31)
    idx = build(w.D)
    want = oracle.search(w.Q, w.D, 6.0, *w.window)
    n = len(want)
    assert n > 500
    buf = np.empty(10, tds.RESULT_DTYPE)
    st, total, _ = idx.search_raw(w.Q, 6.0, *w.window, out_ptr=buf.ctypes.data, capacity=10,
                                  out_on_device=False)
    assert st == tds.TDS_E_OVERFLOW and total == n
    for dev_cap in (1, 7, 1000, n - 1, n):
        got = idx.search(w.Q, 6.0, *w.window, capacity=n, device_capacity=dev_cap)
        compare(got, want, f"device_capacity={dev_cap}")
        if dev_cap < n:
            assert idx.last_stats["passes"] > 1
    idx.close()


def test_device_output_buffer():
    w = trajgen.dense(0.02, n_pts=31)
    idx = build(w.D)
    want = oracle.search(w.Q, w.D, 6.0, *w.window)
    cap = len(want) + 100
    out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
    st, total, _ = idx.search_raw(w.Q, 6.0, *w.window, out_ptr=out.data_ptr(), capacity=cap,
                                  out_on_device=True)
    assert st == tds.TDS_OK and total == len(want)
    torch.cuda.synchronize()
    got = np.frombuffer(out[: total * 32].cpu().numpy().tobytes(), dtype=tds.RESULT_DTYPE)
    compare(got, want, "device out")
    small = torch.empty(5 * 32, dtype=torch.uint8, device="cuda")
    st, total2, _ = idx.search_raw(w.Q, 6.0, *w.window, out_ptr=small.data_ptr(), capacity=5,
                                   out_on_device=True)
    assert st == tds.TDS_E_OVERFLOW and total2 == len(want)
    idx.close()


def test_device_resident_inputs():
    w = trajgen.tiny(0.05)
    Dt = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in w.D.arrays().items()
          if k != "traj"}
    Dt["traj"] = torch.from_numpy(w.D.traj.astype(np.int32)).cuda()
    Qt = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in w.Q.arrays().items()
          if k != "traj"}
    Qt["traj"] = torch.from_numpy(w.Q.traj.astype(np.int32)).cuda()
    idx = build(Dt)
    want = oracle.search(w.Q, w.D, 10.0, *w.window)
    compare(idx.search(Qt, 10.0, *w.window), want, "device inputs")
    idx.close()


# ---------------------------------------------------------------- launch shapes

def test_results_independent_of_bins_chunks_and_grid():
    w = trajgen.dense(0.01, n_pts=41)
    want = oracle.search(w.Q, w.D, 3.0, *w.window)
    for m in (1, 10, 0, 400):
        idx = build(w.D, m)
        for chunk, gw in ((64, 1), (333, 5), (5000, 0), (0, 3)):
            for prec in ("fp32", "fp64"):
                compare(idx.search(w.Q, 3.0, *w.window, chunk=chunk, grid_waves=gw, precision=prec),
                        want, f"m={m} chunk={chunk} grid={gw} {prec}")
        idx.close()


def test_bucket_counter_forms():
    """Bin counts whose query buckets use the parted slot counters (400 bins),
    one counter part (2,000 bins: 8,000 buckets) and keys merged by a shift
    (20,000 and 65,535 bins: more bin-span codes than bucket-table entries),
    in single searches and in a batch of two requests."""
    w = trajgen.dense(0.01, n_pts=41)
    ds = (1.5, 3.0)
    want = {d: oracle.search(w.Q, w.D, d, *w.window) for d in ds}
    for m in (400, 2000, 20000, 65535):
        idx = build(w.D, m)
        assert idx.info()["num_bins"] == m
        for d in ds:
            compare(idx.search(w.Q, d, *w.window), want[d], f"m={m} d={d}")
        out = idx.search_batch([(w.Q, d, *w.window) for d in ds])
        for d, got in zip(ds, out):
            compare(got, want[d], f"batch m={m} d={d}")
        idx.close()


# ---------------------------------------------------------------- edge cases

def _seg(rows, traj=None):
    a = np.array(rows, dtype=np.float64).reshape(-1, 8)
    n = a.shape[0]
    return trajgen.Segments(xs=a[:, 0], ys=a[:, 1], zs=a[:, 2], ts=a[:, 3], xe=a[:, 4], ye=a[:, 5],
                            ze=a[:, 6], te=a[:, 7],
                            traj=np.arange(n, dtype=np.uint32) if traj is None else traj)


def test_closed_form_cases_on_gpu():
    D = _seg([[0, 3, 4, 0, 10, 3, 4, 10],      # co-moving at distance 5
              [10, 3, 0, 0, -10, 3, 0, 10],    # head-on, closest 3 at t = 5
              [0, 0, 0, 0, 0, 0, 0, 2],        # stationary at the origin
              [0, 0, 0, 10, 0, 0, 0, 11]])     # touches q's end only
    Q = _seg([[0, 0, 0, 0, 10, 0, 0, 10], [-1, 5, 0, 0, 1, 5, 0, 2]])
    idx = build(D, 2)
    for d, t0, t1 in [(5.0, -math.inf, math.inf), (4.999, -math.inf, math.inf), (0.0, 0.0, 10.0),
                      (5.0, 4.5, 5.5), (3.0, 0.0, 10.0)]:
        for prec in ("fp32", "fp64"):
            compare(idx.search(Q, d, t0, t1, precision=prec), oracle.search(Q, D, d, t0, t1),
                    f"closed d={d} {prec}")
    got = tds.sort_records(idx.search(Q, 5.0))
    pairs = {(int(r["q_seg"]), int(r["e_seg"])): (r["t_lo"], r["t_hi"]) for r in got}
    assert pairs[(0, 0)] == (0.0, 10.0)
    assert pairs[(1, 2)] == (1.0, 1.0)   # tangent at d
    assert (0, 3) not in pairs           # touch-only
    idx.close()


def test_zero_distance_identical_trajectories():
    w = trajgen.tiny(0.01)
    idx = build(w.D)
    got = idx.search(w.D, 0.0, *w.window)
    want = oracle.search(w.D, w.D, 0.0, *w.window)
    compare(got, want, "d=0 self")
    assert np.all(got["q_seg"] == got["e_seg"]) and got.size == len(w.D)
    idx.close()


def test_invalid_inputs_raise():
    w = trajgen.tiny(0.01)
    idx = build(w.D)
    Q = w.Q.take(np.arange(5))
    for d, t0, t1 in [(-1.0, 0, 1), (math.nan, 0, 1), (1.0, 5.0, 5.0), (1.0, 6.0, 5.0),
                      (math.inf, 0, 1)]:
        with pytest.raises(tds.TdsError) as e:
            idx.search(Q, d, t0, t1)
        assert e.value.status == tds._lib.TDS_E_INVALID
    bad = w.Q.take(np.arange(5))
    bad.xs = bad.xs.copy()
    bad.xs[2] = np.nan
    with pytest.raises(tds.TdsError):
        idx.search(bad, 1.0)
    bad2 = w.Q.take(np.arange(5))
    bad2.te = bad2.ts.copy()
    with pytest.raises(tds.TdsError):
        idx.search(bad2, 1.0)
    with pytest.raises(tds.TdsError):
        tds.Index(bad2)
    # queries outside the database's time span, and an empty query set
    far = w.Q.take(np.arange(5))
    far.ts = far.ts + 1000.0
    far.te = far.te + 1000.0
    assert idx.search(far, 50.0).size == 0
    assert idx.search(w.Q.take(np.arange(0)), 1.0).size == 0
    idx.close()


def test_single_entry_database():
    D = _seg([[0, 0, 0, 0, 1, 1, 1, 1]])
    Q = _seg([[0, 0, 0.5, 0, 1, 1, 0.5, 1], [5, 5, 5, 0.5, 5, 5, 5, 2]])
    idx = build(D)
    compare(idx.search(Q, 0.6), oracle.search(Q, D, 0.6), "single entry")
    idx.close()


# ---------------------------------------------------------------- full sizes

@pytest.mark.parametrize("cfg,ds,n_traj", [("uniform1m", (1.0, 5.0, 25.0), 3), ("dense", (2.0,), 3)])
def test_full_size_sampled(cfg, ds, n_traj):
    """Full-size database; the oracle checks a sample of query trajectories
    (the search runs on the whole query set, as in the benchmark)."""
    w = trajgen.CONFIGS[cfg]()
    idx = build(w.D)
    sl = w.query_traj_slices()
    pick = np.linspace(0, len(sl) - 1, n_traj).astype(int)
    qsel = np.concatenate([np.arange(*sl[i]) for i in pick])
    for d in ds:
        got = idx.search(w.Q, d, *w.window)
        mask = np.isin(got["q_seg"], qsel)
        sub = w.Q.take(qsel)
        want = oracle.search(sub, w.D, d, *w.window)
        want["q_seg"] = qsel[want["q_seg"]]
        compare(got[mask], want, f"{cfg} d={d}")
        print(f"{cfg} d={d}: {got.size} records total, stats {idx.last_stats}")
    idx.close()


def test_galaxy_full_database_sampled_queries():
    """The merger-shaped database at full size (2 x 100,000 Plummer particles,
    20 snapshots: 3.8M segments); a sample of the query particles against the
    oracle, both forms."""
    w = trajgen.galaxy()
    assert len(w.D) == 3_800_000
    idx = build(w.D)
    sl = w.query_traj_slices()
    pick = np.linspace(0, len(sl) - 1, 6).astype(int)
    qsel = np.concatenate([np.arange(*sl[i]) for i in pick])
    sub = w.Q.take(qsel)
    want = oracle.search(sub, w.D, 0.5, *w.window)
    assert len(want) > 1000
    for prec in ("fp32", "fp64"):
        got = idx.search(sub, 0.5, *w.window, precision=prec)
        compare(got, want, f"galaxy {prec}")
    print(f"galaxy sample: {len(want)} records, stats {idx.last_stats}")
    idx.close()
