"""GPU parity of the self-join and of the trajectory-level merge, through the
C ABI, against the oracle.  Self-join records must be the oracle's (same
pairs, ids, orientation; endpoints within 1e-9 relative); merged intervals
must equal the oracle's merge of the same records exactly (the merge copies
endpoints, it computes none)."""
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


def compare(got, want, label):
    got = tds.sort_records(got)
    want = oracle.sort_results(want)
    assert got.size == want.size, f"{label}: {got.size} records, oracle {want.size}"
    for f in ("q_seg", "e_seg", "q_traj", "e_traj"):
        assert np.array_equal(got[f], want[f]), f"{label}: field {f} differs"
    for f in ("t_lo", "t_hi"):
        err = np.abs(got[f] - want[f])
        assert np.all(err <= REL * np.maximum(1.0, np.abs(want[f]))), f"{label}: {f}"


def same_intervals(got, want, label):
    assert got.dtype == tds.TRAJ_DTYPE
    assert got.size == want.size, f"{label}: {got.size} intervals, oracle {want.size}"
    for f in ("q_traj", "e_traj", "t_lo", "t_hi"):
        assert np.array_equal(got[f], want[f]), f"{label}: field {f} differs"


@pytest.mark.parametrize("layout", ["temporal", "spatial"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_self_join_matches_oracle(layout, prec):
    w = trajgen.tiny(scale=0.2)  # 400 trajectories, 19,600 segments
    want = oracle.self_join(w.D, 4.0, 0.0, 49.0)
    assert want.size > 1000
    idx = tds.Index(w.D, layout=layout)
    got = idx.self_join(4.0, 0.0, 49.0, precision=prec)
    compare(got, want, f"self-join {layout}/{prec}")
    s = idx.last_stats
    if prec == "fp32":
        # each pair is tested from one side only: with the temporal layout the
        # filter sees about half of the pairs it sees when D is searched
        # against itself; with the spatial one, the pairs left after the block
        # boxes cluster around each query's own position, so fewer go
        idx.search(w.D, 4.0, 0.0, 49.0, precision=prec)
        bound = 0.6 if layout == "temporal" else 0.85
        assert s["filter_tests"] < bound * idx.last_stats["filter_tests"]
    idx.close()


def test_self_join_windows_dense_and_incremental():
    w = trajgen.dense(0.02, n_pts=41)
    idx = tds.Index(w.D)
    for t0, t1, d in [(-math.inf, math.inf, 1.5), (10.25, 20.5, 2.0)]:
        want = oracle.self_join(w.D, d, t0, t1)
        compare(idx.self_join(d, t0, t1), want, f"dense {t0},{t1}")
        # a device buffer far smaller than the result: incremental passes
        got = idx.self_join(d, t0, t1, device_capacity=max(1, want.size // 7))
        compare(got, want, "incremental")
        assert idx.last_stats["passes"] > 1
    idx.close()


def test_self_join_single_trajectory_has_no_pairs():
    rng = np.random.default_rng(2)
    n = 50
    t = np.arange(n + 1, dtype=np.float64)
    p = np.cumsum(rng.normal(size=(n + 1, 3)), axis=0)
    D = trajgen.Segments(xs=p[:-1, 0], ys=p[:-1, 1], zs=p[:-1, 2], ts=t[:-1], xe=p[1:, 0],
                         ye=p[1:, 1], ze=p[1:, 2], te=t[1:], traj=np.zeros(n, np.uint32))
    idx = tds.Index(D)
    assert idx.self_join(100.0).size == 0
    idx.close()


def test_merge_matches_oracle_on_self_join_records():
    w = trajgen.tiny(scale=0.2)
    idx = tds.Index(w.D)
    recs = idx.self_join(4.0, 0.0, 49.0)
    idx.close()
    want = oracle.merge_trajectories(recs)
    got = tds.merge_trajectories(recs)
    same_intervals(got, want, "self-join records")
    assert got.size < recs.size  # consecutive segment pairs merged


def test_merge_matches_oracle_on_random_records():
    rng = np.random.default_rng(9)
    n = 200_000  # several radix-sort scan tiles
    recs = np.zeros(n, tds.RESULT_DTYPE)
    recs["q_seg"] = np.arange(n)
    recs["e_seg"] = rng.integers(0, 1 << 31, n)
    recs["q_traj"] = rng.integers(0, 300, n)
    recs["e_traj"] = rng.integers(0, 300, n) * 4099  # large ids
    lo = rng.integers(0, 4000, n) / 8.0
    recs["t_lo"] = lo
    recs["t_hi"] = lo + rng.integers(0, 16, n) / 8.0
    recs["t_lo"][::11] = -recs["t_lo"][::11]  # negative times
    recs["t_hi"][::11] = recs["t_lo"][::11] + 0.5
    got = tds.merge_trajectories(recs)
    same_intervals(got, oracle.merge_trajectories(recs), "random")


def test_merge_edge_cases_and_overflow():
    empty = np.zeros(0, tds.RESULT_DTYPE)
    assert tds.merge_trajectories(empty).size == 0
    one = np.zeros(1, tds.RESULT_DTYPE)
    one[0] = (3, 4, 5, 6, 1.5, 2.5)
    same_intervals(tds.merge_trajectories(one), oracle.merge_trajectories(one), "one")
    rows = np.zeros(6, tds.RESULT_DTYPE)
    rows["q_traj"] = [7, 7, 7, 1, 1, 7]
    rows["e_traj"] = [2, 2, 2, 9, 9, 2]
    rows["t_lo"] = [0.0, 1.0, 3.0, 0.0, 0.0, 1.0]
    rows["t_hi"] = [1.0, 2.0, 3.0, 4.0, 1.0, 1.5]
    want = oracle.merge_trajectories(rows)  # (1,9,[0,4]), (7,2,[0,2]), (7,2,[3,3])
    assert want.size == 3
    same_intervals(tds.merge_trajectories(rows), want, "small")
    # capacity 2: overflow, the first two intervals in order, the total reported
    out = np.zeros(2, tds.TRAJ_DTYPE)
    st, n = tds.merge_trajectories_raw(rows.ctypes.data, rows.size, False, out.ctypes.data, 2, False)
    assert st == tds.TDS_E_OVERFLOW and n == 3
    same_intervals(out, want[:2], "overflow prefix")


def test_merge_device_buffers():
    w = trajgen.tiny(scale=0.1)
    idx = tds.Index(w.D)
    cap = 1 << 16
    rec_dev = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
    st, n, _ = idx.self_join_raw(5.0, out_ptr=rec_dev.data_ptr(), capacity=cap, out_on_device=True)
    assert st == tds.TDS_OK and 0 < n < cap
    out_dev = torch.empty(n * 24, dtype=torch.uint8, device="cuda")
    st, m = tds.merge_trajectories_raw(rec_dev.data_ptr(), n, True, out_dev.data_ptr(), n, True)
    assert st == tds.TDS_OK and 0 < m <= n
    got = np.frombuffer(out_dev.cpu().numpy().tobytes()[: m * 24], dtype=tds.TRAJ_DTYPE)
    recs = np.frombuffer(rec_dev.cpu().numpy().tobytes()[: n * 32], dtype=tds.RESULT_DTYPE)
    same_intervals(got, oracle.merge_trajectories(recs), "device")
    idx.close()
