"""tds_search_noalloc (the search for callers that cannot allocate: every
buffer beyond the inputs and outputs comes from one static device array)
against tds_search with device output, the entry point it is a variant of:
the same records, bit for bit, on calls in a row that reuse the array with
smaller inputs, and the oracle's records (Sec. 3.1 result set)."""
import numpy as np
import pytest

import oracle
import trajgen
from parity import DeviceRecords, compare, device_segments

torch = pytest.importorskip("torch")
import paper_1410_2698_amd as tds  # noqa: E402

pytestmark = pytest.mark.gpu


def both(idx, Qt, d, window):
    """Records of tds_search and of tds_search_noalloc (device output), each
    ordered on the device; the no-alloc call's stats."""
    st, n, _ = idx.search_raw(Qt, d, *window, out_ptr=0, capacity=0, out_on_device=True)
    assert st in (tds.TDS_OK, tds.TDS_E_OVERFLOW)
    a = torch.empty(max(n, 1) * 32, dtype=torch.uint8, device="cuda")
    st, n1, _ = idx.search_raw(Qt, d, *window, out_ptr=a.data_ptr(), capacity=n, out_on_device=True)
    assert st == tds.TDS_OK and n1 == n
    b = torch.full((max(n, 1) * 32,), 0xAB, dtype=torch.uint8, device="cuda")
    st, n2, stats = idx.search_noalloc_raw(Qt, d, *window, out_ptr=b.data_ptr(), capacity=n)
    assert st == tds.TDS_OK and n2 == n, (st, n2, n)
    return DeviceRecords(a, n), DeviceRecords(b, n), stats


def sub_segments(Qt, k):
    return {key: v[:k].contiguous() for key, v in Qt.items()}


def test_noalloc_matches_search_on_calls_in_a_row():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    # galaxy-shaped (dense cores: work items fill the 256-record stages
    # many times over), then two smaller calls on another index
    g = trajgen.galaxy(scale=0.05)  # 10,000 particles, 190,000 entries; 50 query particles
    gidx = tds.Index(g.D)
    Qg = device_segments(g.Q)
    a, b, st = both(gidx, Qg, 0.5, g.window)
    assert a.n > 50000 and b.unique and a.equal(b)
    assert st["results"] == a.n and st["stage_flushes"] > 0
    want = oracle.sort_results(oracle.search(g.Q, g.D, 0.5, *g.window))
    compare(b.q_range(0, len(g.Q)), want, "noalloc galaxy")
    gidx.close()

    u = trajgen.uniform1m(scale=0.1)  # 250 trajectories (100,000 entries); 50 queries
    uidx = tds.Index(u.D)
    Qu = device_segments(u.Q)
    assert len(u.Q) == 20000
    a, b, _ = both(uidx, Qu, 25.0, u.window)
    assert a.n > 100 and b.unique and a.equal(b)
    # the second call: fewer query segments, a narrower window, FP64 form
    Qs = sub_segments(Qu, 4000)
    st, n, _ = uidx.search_raw(Qs, 40.0, 50.0, 300.0, out_ptr=0, capacity=0, out_on_device=True,
                               precision="fp64")
    ref = torch.empty(max(n, 1) * 32, dtype=torch.uint8, device="cuda")
    uidx.search_raw(Qs, 40.0, 50.0, 300.0, out_ptr=ref.data_ptr(), capacity=n,
                    out_on_device=True, precision="fp64")
    got = torch.full((max(n, 1) * 32,), 0xCD, dtype=torch.uint8, device="cuda")
    st2, n2, _ = uidx.search_noalloc_raw(Qs, 40.0, 50.0, 300.0, out_ptr=got.data_ptr(),
                                         capacity=n, precision="fp64")
    assert st2 == tds.TDS_OK and n2 == n and n > 10
    ra, rb = DeviceRecords(ref, n), DeviceRecords(got, n)
    assert rb.unique and ra.equal(rb)
    want = oracle.sort_results(oracle.search(u.Q.take(np.arange(4000)), u.D, 40.0, 50.0, 300.0))
    compare(rb.q_range(0, 4000), want, "noalloc uniform second call")
    uidx.close()


def test_noalloc_limits_and_overflow():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    u = trajgen.uniform1m(scale=0.05, n_pts=81)
    idx = tds.Index(u.D)
    Qt = device_segments(u.Q)
    # overflow: the total is reported, at most `capacity` records written
    st, n, _ = idx.search_raw(Qt, 60.0, *u.window, out_ptr=0, capacity=0, out_on_device=True)
    assert n > 20
    buf = torch.empty(n * 32, dtype=torch.uint8, device="cuda")
    st, n2, _ = idx.search_noalloc_raw(Qt, 60.0, *u.window, out_ptr=buf.data_ptr(), capacity=10)
    assert st == tds.TDS_E_OVERFLOW and n2 == n
    # more query segments than the scratch array is laid out for
    big = {k: torch.cat([v] * (65536 // len(u.Q) + 1)) for k, v in Qt.items()}
    st, _, _ = idx.search_noalloc_raw(big, 5.0, *u.window, out_ptr=buf.data_ptr(), capacity=n)
    assert st == tds.TDS_E_INVALID
    # host-memory queries are refused (a device copy would need memory)
    st, _, _ = idx.search_noalloc_raw(u.Q, 5.0, *u.window, out_ptr=buf.data_ptr(), capacity=n)
    assert st == tds.TDS_E_INVALID
    # still usable afterwards
    a, b, _ = both(idx, Qt, 60.0, u.window)
    assert a.equal(b)
    idx.close()
