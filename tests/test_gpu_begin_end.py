"""tds_search_begin / tds_search_end: the search ordered on a stream by one
call and collected by another gives the records of tds_search (Sec. 3.1
result set, checked against the oracle), also with two searches in flight on
two streams and ended in the other order, and reports an overflow with the
total."""
import numpy as np
import pytest

import oracle
import trajgen
from parity import compare, device_segments

torch = pytest.importorskip("torch")
import paper_1410_2698_amd as tds  # noqa: E402

pytestmark = pytest.mark.gpu


def records(buf, n):
    return np.frombuffer(buf[: n * 32].cpu().numpy().tobytes(), dtype=tds.RESULT_DTYPE)


def test_begin_end_matches_oracle_and_search():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = trajgen.tiny()
    idx = tds.Index(w.D)
    d = 5.0
    want = oracle.sort_results(oracle.search(w.Q, w.D, d, *w.window))
    assert want.size > 1000
    out = torch.empty((want.size + 10) * 32, dtype=torch.uint8, device="cuda")
    p = idx.search_begin(w.Q, d, *w.window, out_ptr=out.data_ptr(), capacity=want.size + 10)
    st, n, s = p.end()
    assert st == tds.TDS_OK and n == want.size and s["results"] == n
    compare(tds.sort_records(records(out, n)), want, "begin/end")
    with pytest.raises(RuntimeError):
        p.end()
    # device-resident queries, staged output, the same records bit for bit
    Qt = device_segments(w.Q)
    out2 = torch.empty((want.size + 10) * 32, dtype=torch.uint8, device="cuda")
    p = idx.search_begin(Qt, d, *w.window, out_ptr=out2.data_ptr(), capacity=want.size + 10,
                         output="staged")
    st, n2, _ = p.end()
    assert st == tds.TDS_OK and n2 == n
    assert tds.sort_records(records(out2, n)).tobytes() == \
        tds.sort_records(records(out, n)).tobytes()
    idx.close()


def test_two_searches_in_flight_on_two_streams():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = trajgen.dense(0.05, n_pts=81)
    idx = tds.Index(w.D)
    Qt = device_segments(w.Q)
    ref = {}
    for d in (4.0, 8.0):
        r = idx.search(w.Q, d, *w.window)
        ref[d] = tds.sort_records(r).tobytes()
        assert r.size > 1000
    bufs, pend = {}, {}
    streams = {4.0: torch.cuda.Stream(), 8.0: torch.cuda.Stream()}
    for d, s in streams.items():
        n = len(ref[d]) // 32
        bufs[d] = torch.empty((n + 64) * 32, dtype=torch.uint8, device="cuda")
        with torch.cuda.stream(s):
            pend[d] = idx.search_begin(Qt, d, *w.window, out_ptr=bufs[d].data_ptr(),
                                       capacity=n + 64)
    for d in (8.0, 4.0):  # ended in the other order
        st, n, _ = pend[d].end()
        assert st == tds.TDS_OK and n == len(ref[d]) // 32
        assert tds.sort_records(records(bufs[d], n)).tobytes() == ref[d], d
    idx.close()


def test_begin_end_overflow_reports_the_total():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = trajgen.tiny()
    idx = tds.Index(w.D)
    want = oracle.search(w.Q, w.D, 5.0, *w.window)
    cap = want.size // 2
    out = torch.empty(cap * 32, dtype=torch.uint8, device="cuda")
    st, n, _ = idx.search_begin(w.Q, 5.0, *w.window, out_ptr=out.data_ptr(),
                                capacity=cap).end()
    assert st == tds.TDS_E_OVERFLOW and n == want.size
    got = records(out, cap)
    keys = set(zip(got["q_seg"].tolist(), got["e_seg"].tolist()))
    assert len(keys) == cap
    assert keys <= set(zip(want["q_seg"].tolist(), want["e_seg"].tolist()))
    idx.close()
