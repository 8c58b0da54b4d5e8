"""Parity at the full sizes of the four database configurations and of the
request stream, in the launch configuration the benchmark times (index and
queries resident in device memory, device output sized by a counting call).

Every record of the GPU is compared with the FP64 oracle (the brute force of
Sec. 3.1): identical result sets and trajectory ids, no duplicates, interval
endpoints within 1e-9 relative.  The galaxy-merger-shaped search (1.7e8
records) is ordered on the device and compared a slice of query particles at
a time, so that the host never holds the whole set twice.
"""
import concurrent.futures as cf
import os

import numpy as np
import pytest

import oracle
import trajgen
from parity import DeviceRecords, compare, device_segments

torch = pytest.importorskip("torch")
import paper_1410_2698_amd as tds  # noqa: E402

pytestmark = pytest.mark.gpu

THREADS = min(16, os.cpu_count() or 1)


def full_search(idx, Qt, d, window, **kw):
    """One search of the whole query set into device memory, as the benchmark
    runs it: a counting call without output space, then the search with a
    buffer of exactly the counted size."""
    st, n, _ = idx.search_raw(Qt, d, *window, out_ptr=0, capacity=0, out_on_device=True, **kw)
    assert st in (tds.TDS_OK, tds.TDS_E_OVERFLOW)
    buf = torch.empty(max(n, 1) * 32, dtype=torch.uint8, device="cuda")
    st, n2, stats = idx.search_raw(Qt, d, *window, out_ptr=buf.data_ptr(), capacity=n,
                                   out_on_device=True, **kw)
    assert st == tds.TDS_OK and n2 == n, (st, n2, n)
    return buf, n, stats


def oracle_slices(w, d, slices):
    """Oracle records of the query trajectories in `slices` (list of (begin,
    end) segment ranges), q_seg counted in the whole query set."""
    qsel = np.concatenate([np.arange(a, b) for a, b in slices])
    want = oracle.search(w.Q.take(qsel), w.D, d, *w.window, threads=THREADS)
    want["q_seg"] = qsel[want["q_seg"]]
    return oracle.sort_results(want)


# ---------------------------------------------------------------- uniform1m

@pytest.fixture(scope="module")
def uniform():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = trajgen.uniform1m()
    idx = tds.Index(w.D)
    yield w, idx
    idx.close()


@pytest.fixture(scope="module")
def uniform_batch(uniform):
    """The benchmark's step: the 200,000 query segments once per d as three
    requests of one batch, device output."""
    w, idx = uniform
    ds = w.ds
    nq = len(w.Q)
    Qt = device_segments(w.Q)
    Qb = {k: torch.cat([v] * len(ds)) for k, v in Qt.items()}
    t0, t1 = w.window
    st, counts, _ = idx.search_batch_raw(Qb, [(i * nq, nq, d, t0, t1, 0, 0) for i, d in enumerate(ds)],
                                         out_ptr=0, out_capacity=0, out_on_device=True)
    cap = max(counts) + 1
    out = torch.empty(len(ds) * cap * 32, dtype=torch.uint8, device="cuda")
    reqs = [(i * nq, nq, d, t0, t1, i * cap, cap) for i, d in enumerate(ds)]
    st, got, stats = idx.search_batch_raw(Qb, reqs, out_ptr=out.data_ptr(),
                                          out_capacity=len(ds) * cap, out_on_device=True)
    assert st == tds.TDS_OK and got == counts
    per_d = {}
    for i, d in enumerate(ds):
        part = out[i * cap * 32:(i * cap + counts[i]) * 32]
        per_d[d] = DeviceRecords(part, counts[i])
    return per_d


@pytest.mark.parametrize("d", [1.0, 5.0, 25.0])
def test_uniform1m_all_queries(uniform, uniform_batch, d):
    """All 500 query trajectories (200,000 segments) against the 1M entries,
    at each d of the batch."""
    w, _ = uniform
    rec = uniform_batch[d]
    assert rec.unique
    got = rec.q_range(0, len(w.Q))
    want = oracle_slices(w, d, [(0, len(w.Q))])
    assert want.size >= {1.0: 1, 5.0: 100, 25.0: 10000}[d]
    same = compare(got, want, f"uniform1m d={d}")
    print(f"uniform1m d={d}: {got.size} records, {same} bit-identical endpoints")


# ---------------------------------------------------------------- dense

def test_dense_all_queries():
    """All 1,000 query trajectories (100,000 segments) against the 1M entries
    confined to [0,50]^3, d = 2."""
    w = trajgen.dense()
    idx = tds.Index(w.D)
    buf, n, stats = full_search(idx, device_segments(w.Q), 2.0, w.window)
    rec = DeviceRecords(buf, n)
    del buf
    assert rec.unique
    got = rec.q_range(0, len(w.Q))
    want = oracle_slices(w, 2.0, [(0, len(w.Q))])
    assert want.size > 100000
    same = compare(got, want, "dense d=2")
    print(f"dense: {got.size} records, {same} bit-identical endpoints, stats {stats}")
    idx.close()


# ---------------------------------------------------------------- galaxy

GALAXY_CHUNKS = 10  # slices of 200 query particles


@pytest.fixture(scope="module")
def galaxy():
    """The whole galaxy search (38,000 query segments against 3.8M entries)
    in both forms, ordered on the device."""
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = trajgen.galaxy()
    idx = tds.Index(w.D)
    Qt = device_segments(w.Q)
    buf, n, stats = full_search(idx, Qt, 0.5, w.window)
    rec32 = DeviceRecords(buf, n)
    del buf
    buf, n64, stats64 = full_search(idx, Qt, 0.5, w.window, precision="fp64")
    rec64 = DeviceRecords(buf, n64)
    del buf
    print(f"galaxy: {n} records; FP32 form {stats}; FP64 form {stats64}")
    yield w, rec32, rec64, stats
    idx.close()


def test_galaxy_forms_bit_identical(galaxy):
    """The FP32-filter form and the plain FP64 form give bit-identical record
    sets over the whole search (the FP32 endpoint error is zero)."""
    w, rec32, rec64, stats = galaxy
    assert rec32.n > 10_000_000 and rec32.unique
    assert rec32.n == stats["results"]
    assert rec32.equal(rec64)


@pytest.mark.parametrize("chunk", range(GALAXY_CHUNKS))
def test_galaxy_all_queries(galaxy, chunk):
    """Query particles [200 c, 200 c + 200) of the 2,000: every record of
    the full search against the oracle's."""
    w, rec32, _, _ = galaxy
    sl = w.query_traj_slices()
    per = len(sl) // GALAXY_CHUNKS
    part = sl[chunk * per:(chunk + 1) * per] if chunk < GALAXY_CHUNKS - 1 else sl[chunk * per:]
    q0, q1 = part[0][0], part[-1][1]
    got = rec32.q_range(q0, q1)
    want = oracle_slices(w, 0.5, part)
    assert want.size > 100000
    same = compare(got, want, f"galaxy chunk {chunk}")
    print(f"galaxy chunk {chunk}: {got.size} records, {same} bit-identical endpoints")


# ---------------------------------------------------------------- request stream

N_STREAM = 2000


def test_stream_served_on_full_index(uniform):
    """2,000 requests of the request stream (query trajectories of 5-400
    segments, random windows, d in [1, 25]) through the serving loop on the
    full uniform1m index, submitted back to back so that batches mix many
    requests; every request's records against the oracle's for that request
    alone."""
    w, idx = uniform
    reqs = trajgen.request_stream(N_STREAM)
    srv = tds.Server(idx, max_batch_segments=1 << 17, max_batch_requests=2048, slots=2,
                     result_capacity=1 << 21, default_reserve=64)
    tickets = [srv.submit(r.Q, r.d, r.t_start, r.t_end) for r in reqs]
    got = [srv.wait(t)[0] for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == N_STREAM and st["failed"] == 0
    assert st["max_batch_requests_seen"] > 1

    def want(r):
        return oracle.sort_results(oracle.search(r.Q, w.D, r.d, r.t_start, r.t_end, threads=1))

    total = 0
    with cf.ThreadPoolExecutor(THREADS) as ex:
        for i, (g, wnt) in enumerate(zip(got, ex.map(want, reqs))):
            compare(tds.sort_records(g), wnt, f"request {i}")
            total += wnt.size
    assert total > 2000  # about 2.5 records per request
    print(f"stream: {N_STREAM} requests, {total} records, {st}")
