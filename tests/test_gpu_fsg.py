"""GPU parity of the fixed spatial grid search (Alg. 1) against the oracle,
through the C ABI: the same records as the brute-force search (the grid
only chooses candidates; duplicates across cells must not appear)."""
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
    kg = got["q_seg"].astype(np.uint64) << np.uint64(32) | got["e_seg"]
    assert np.unique(kg).size == kg.size, f"{label}: duplicate records"
    assert got.size == want.size, f"{label}: {got.size} records, oracle {want.size}"
    for f in ("q_seg", "e_seg", "q_traj", "e_traj"):
        assert np.array_equal(got[f], want[f]), f"{label}: field {f} differs"
    for f in ("t_lo", "t_hi"):
        err = np.abs(got[f] - want[f])
        assert np.all(err <= REL * np.maximum(1.0, np.abs(want[f]))), f"{label}: {f}"


@pytest.mark.parametrize("grid", [(1, 1, 1), (7, 3, 5), (50, 50, 50)])
def test_fsg_tiny(grid):
    w = trajgen.tiny(scale=0.2)
    idx = tds.Index(w.D)
    g = tds.FSG(idx, *grid)
    want = oracle.search(w.Q, w.D, 5.0, 0.0, 49.0)
    got = g.search(w.Q, 5.0, 0.0, 49.0)
    compare(got, want, f"grid {grid}")
    # the same records as the temporal index search, bit for bit
    assert tds.sort_records(got).tobytes() == tds.sort_records(idx.search(w.Q, 5.0, 0.0, 49.0)).tobytes()
    g.close()
    idx.close()


@pytest.mark.parametrize("cfg,scale,d", [("uniform1m", 0.02, 40.0), ("dense", 0.02, 2.0),
                                         ("galaxy", 0.01, 0.5)])
def test_fsg_reduced_configs(cfg, scale, d):
    kw = {"n_pts": 61} if cfg in ("uniform1m", "dense") else {}
    w = trajgen.CONFIGS[cfg](scale, **kw)
    idx = tds.Index(w.D)
    g = tds.FSG(idx, 20, 20, 20)
    compare(g.search(w.Q, d, *w.window), oracle.search(w.Q, w.D, d, *w.window), cfg)
    g.close()
    idx.close()


def test_fsg_windows_overflow_and_device_output():
    w = trajgen.dense(0.02, n_pts=41)
    idx = tds.Index(w.D)
    g = tds.FSG(idx)
    for t0, t1, d in [(12.5, 17.25, 3.0), (-math.inf, 3.0, 1.0), (30.0, math.inf, 2.5)]:
        compare(g.search(w.Q, d, t0, t1), oracle.search(w.Q, w.D, d, t0, t1), f"window {t0},{t1}")
    want = oracle.search(w.Q, w.D, 3.0, *w.window)
    buf = np.empty(5, tds.RESULT_DTYPE)
    st, n, _ = g.search_raw(w.Q, 3.0, *w.window, out_ptr=buf.ctypes.data, capacity=5,
                            out_on_device=False)
    assert st == tds.TDS_E_OVERFLOW and n == want.size
    dev = torch.empty((n + 1) * 32, dtype=torch.uint8, device="cuda")
    st, n2, s = g.search_raw(w.Q, 3.0, *w.window, out_ptr=dev.data_ptr(), capacity=n + 1,
                             out_on_device=True)
    assert st == tds.TDS_OK and n2 == n and s["candidate_tests"] > 0
    got = np.frombuffer(dev.cpu().numpy().tobytes()[: n * 32], dtype=tds.RESULT_DTYPE)
    compare(got, want, "device output")
    g.close()
    idx.close()


def test_fsg_largest_grid():
    # 256^3 = 2^24 cells, the largest grid accepted: mostly empty cells
    w = trajgen.tiny(scale=0.05)
    idx = tds.Index(w.D)
    g = tds.FSG(idx, 256, 256, 256)
    compare(g.search(w.Q, 3.0, 0.0, 49.0), oracle.search(w.Q, w.D, 3.0, 0.0, 49.0), "256^3")
    g.close()
    with pytest.raises(tds.TdsError):
        tds.FSG(idx, 256, 256, 257)
    idx.close()


def test_fsg_invalid_arguments():
    w = trajgen.tiny(scale=0.01)
    idx = tds.Index(w.D)
    with pytest.raises(tds.TdsError):
        tds.FSG(idx, 2000, 1, 1)
    with pytest.raises(tds.TdsError):
        tds.FSG(idx, 1024, 1024, 1024)
    g = tds.FSG(idx, 4, 4, 4)
    with pytest.raises(tds.TdsError):
        g.search(w.Q, -1.0)
    bad = w.Q.take(np.arange(3))
    bad.te[1] = bad.ts[1]
    with pytest.raises(tds.TdsError):
        g.search(bad, 1.0)
    g.close()
    idx.close()
