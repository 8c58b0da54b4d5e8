"""GPU tests of the batched forms: tds_search_batch, the graph-replaying
batcher and the serving loop.  Every request's records must equal the
oracle's for that request (same set, endpoints within 1e-9 relative) and be
bit-identical to the same request searched on its own."""
import numpy as np
import pytest

import oracle
import trajgen

torch = pytest.importorskip("torch")
import paper_1410_2698_amd as tds  # noqa: E402

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = trajgen.uniform1m(0.05, n_pts=81)
    idx = tds.Index(w.D)
    stream = trajgen.request_stream(48, n_pts=81, seed=77)
    # distances scaled up for the thinner database (125 trajectories)
    reqs = [(r.Q, r.d * 6.0, r.t_start, r.t_end) for r in stream]
    yield w, idx, reqs
    idx.close()


def key_sorted(r):
    return tds.sort_records(r).tobytes()


def check_oracle(got, Q, D, d, t0, t1):
    want = oracle.sort_results(oracle.search(Q, D, d, t0, t1))
    got = tds.sort_records(got)
    assert got.size == want.size
    for f in ("q_seg", "e_seg", "q_traj", "e_traj"):
        assert np.array_equal(got[f], want[f])
    for f in ("t_lo", "t_hi"):
        assert np.all(np.abs(got[f] - want[f]) <= 1e-9 * np.maximum(1.0, np.abs(want[f])))
    return want.size


def test_batch_matches_oracle_and_alone(setup):
    w, idx, reqs = setup
    out = idx.search_batch(reqs)
    assert len(out) == len(reqs)
    total = 0
    for (Q, d, t0, t1), got in zip(reqs, out):
        total += check_oracle(got, Q, w.D, d, t0, t1)
        alone = idx.search(Q, d, t0, t1)
        assert key_sorted(alone) == key_sorted(got)
    assert total > 100
    # the FP64 form gives the same records
    out64 = idx.search_batch(reqs, precision="fp64")
    for a, b in zip(out, out64):
        assert key_sorted(a) == key_sorted(b)


def test_device_resident_batch_of_distances(setup):
    """The bench's step form: the same query segments once per d as requests
    of one batch, inputs and outputs in device memory; a first call without
    output space only counts."""
    w, idx, _ = setup
    Qt = {k: torch.from_numpy(np.ascontiguousarray(v)).cuda() for k, v in w.Q.arrays().items()
          if k != "traj"}
    Qt["traj"] = torch.from_numpy(w.Q.traj.astype(np.int32)).cuda()
    ds = (6.0, 30.0, 150.0)
    nq = len(w.Q)
    Qb = {k: torch.cat([v] * len(ds)) for k, v in Qt.items()}
    st, counts, _ = idx.search_batch_raw(
        Qb, [(i * nq, nq, d, 0.0, 80.0, 0, 0) for i, d in enumerate(ds)], out_ptr=0,
        out_capacity=0, out_on_device=True)
    assert st == tds.TDS_E_OVERFLOW and counts[2] > counts[0]
    cap = max(counts) + 3
    out = torch.empty(len(ds) * cap * 32, dtype=torch.uint8, device="cuda")
    reqs = [(i * nq, nq, d, 0.0, 80.0, i * cap, cap) for i, d in enumerate(ds)]
    st, got, stats = idx.search_batch_raw(Qb, reqs, out_ptr=out.data_ptr(),
                                          out_capacity=len(ds) * cap, out_on_device=True)
    assert st == tds.TDS_OK and got == counts and stats["passes"] == 1
    recs = np.frombuffer(out.cpu().numpy().tobytes(), dtype=tds.RESULT_DTYPE)
    for i, d in enumerate(ds):
        part = recs[i * cap: i * cap + counts[i]].copy()
        check_oracle(part, w.Q, w.D, d, 0.0, 80.0)
        assert key_sorted(part) == key_sorted(idx.search(w.Q, d, 0.0, 80.0))


def test_batch_overflow_is_per_request(setup):
    w, idx, reqs = setup
    b = tds.Batcher(idx, max_segments=20000, max_requests=64, result_capacity=64 * 2)
    recs, counts, status = b.run(reqs, slice_capacity=2)
    want = [len(oracle.search(Q, w.D, d, t0, t1)) for (Q, d, t0, t1) in reqs]
    assert counts == want
    assert (status == tds.TDS_E_OVERFLOW) == any(c > 2 for c in want)
    for c, r in zip(counts, recs):
        assert r.size == min(c, 2)
    b.close()


def test_batcher_graph_replays_match_eager(setup):
    w, idx, reqs = setup
    b = tds.Batcher(idx, max_segments=20000, max_requests=64, result_capacity=64 * 4096)
    subsets = [reqs[:5], reqs[5:30], reqs[30:31], reqs[10:48], reqs[:48]]
    for i, sub in enumerate(subsets):
        eager = idx.search_batch(sub)
        # unrelated eager work and a synchronisation between replays
        x = torch.randn(1 << 16, device="cuda")
        float(x.sum())
        torch.cuda.synchronize()
        got, counts, status = b.run(sub, slice_capacity=4096)
        assert status == tds.TDS_OK
        assert b.replays == i + 1
        for e, g in zip(eager, got):
            assert key_sorted(e) == key_sorted(g)
        # every replay against the oracle, request by request
        for (Q, d, t0, t1), g in zip(sub, got):
            check_oracle(g, Q, w.D, d, t0, t1)
    # fp64 batcher
    b64 = tds.Batcher(idx, max_segments=20000, max_requests=64, result_capacity=64 * 4096,
                      precision="fp64")
    got, _, _ = b64.run(reqs[:20], slice_capacity=4096)
    for e, g in zip(idx.search_batch(reqs[:20]), got):
        assert key_sorted(e) == key_sorted(g)
    b.close()
    b64.close()


def test_server_alone_vs_mix(setup):
    w, idx, reqs = setup
    srv = tds.Server(idx, max_batch_segments=20000, max_batch_requests=16, slots=2,
                     result_capacity=1 << 16, default_reserve=4)
    alone = []
    for Q, d, t0, t1 in reqs:
        t = srv.submit(Q, d, t0, t1)
        recs, lat = srv.wait(t)
        assert lat > 0
        alone.append(recs)
    tickets = [srv.submit(Q, d, t0, t1) for Q, d, t0, t1 in reqs]
    mixed = [srv.wait(t)[0] for t in tickets]
    st = srv.stats()
    srv.close()
    for (Q, d, t0, t1), a, m in zip(reqs, alone, mixed):
        assert key_sorted(a) == key_sorted(m)
    for i in range(0, len(reqs), 7):
        Q, d, t0, t1 = reqs[i]
        check_oracle(mixed[i], Q, w.D, d, t0, t1)
    assert st["completed"] == 2 * len(reqs) and st["failed"] == 0
    assert st["requeued"] > 0             # small reservations forced exact re-runs
    assert st["max_batch_requests_seen"] > 1  # requests shared batches
    assert st["batches"] < 2 * len(reqs) + st["requeued"]


def test_server_rejects_a_bad_request_alone(setup):
    """A request with a non-finite value or an empty segment is refused at
    submission; the valid requests around it complete with the records they
    get alone (a bad request never fails a batch it would have joined)."""
    w, idx, reqs = setup
    srv = tds.Server(idx, max_batch_segments=20000, max_batch_requests=16, slots=2,
                     result_capacity=1 << 16, default_reserve=64)
    tickets = []
    refused = 0
    for i, (Q, d, t0, t1) in enumerate(reqs[:24]):
        tickets.append(srv.submit(Q, d, t0, t1))
        if i % 6 == 2:
            arrs = {k: np.array(v, copy=True) for k, v in Q.arrays().items()}
            bad = [dict(arrs), dict(arrs)]
            bad[0]["ys"] = arrs["ys"].copy()
            bad[0]["ys"][len(Q) // 2] = np.nan
            bad[1]["te"] = arrs["te"].copy()
            bad[1]["te"][0] = arrs["ts"][0]  # te == ts
            for b in bad:
                with pytest.raises(tds.TdsError) as e:
                    srv.submit(b, d, t0, t1)
                assert e.value.status == tds.TDS_E_INVALID
                refused += 1
    got = [srv.wait(t)[0] for t in tickets]
    st = srv.stats()
    srv.close()
    assert refused == 8
    assert st["completed"] == 24 and st["failed"] == 0 and st["submitted"] == 24
    for (Q, d, t0, t1), g in zip(reqs[:24], got):
        check_oracle(g, Q, w.D, d, t0, t1)
        assert key_sorted(g) == key_sorted(idx.search(Q, d, t0, t1))


def test_repeated_batch_on_the_same_buffers(setup):
    """tds_search_batch called again and again on the same query and output
    buffers (the bench's step), with the requests' contents and the query
    values changing between calls: every call's records must equal direct
    searches of what the buffers hold at that call (nothing is carried over
    from one call to the next)."""
    w, idx, _ = setup
    host = {k: np.ascontiguousarray(v) for k, v in w.Q.arrays().items() if k != "traj"}
    Qt = {k: torch.from_numpy(v).cuda() for k, v in host.items()}
    Qt["traj"] = torch.from_numpy(w.Q.traj.astype(np.int32)).cuda()
    nq = len(w.Q)
    Qb = {k: torch.cat([v] * 3) for k, v in Qt.items()}
    _, counts, _ = idx.search_batch_raw(
        Qb, [(i * nq, nq, 150.0, 0.0, 80.0, 0, 0) for i in range(3)], out_ptr=0, out_capacity=0,
        out_on_device=True)
    cap = 4 * max(counts) + 16
    out = torch.empty(3 * cap * 32, dtype=torch.uint8, device="cuda")
    # the direct searches first, so that the batch calls follow each other
    sequence = [((6.0, 30.0, 150.0), 0.0)] * 3 + [((12.0, 60.0, 150.0), 0.0)] * 2 + \
               [((6.0, 30.0, 150.0), 0.0)] + [((6.0, 30.0, 150.0), 0.5)] * 2
    direct = {}
    for ds, shift in sequence:
        for d in ds:
            if (d, shift) not in direct:
                Q = dict(host, traj=w.Q.traj.astype(np.uint32))
                Q["xs"] = host["xs"] + shift
                Q["xe"] = host["xe"] + shift
                direct[(d, shift)] = key_sorted(idx.search(Q, d, 0.0, 80.0))
    shifted = False
    for ds, shift in sequence:
        if shift and not shifted:
            # new query values in the same device buffers
            for k in ("xs", "xe"):
                Qb[k].add_(shift)
            shifted = True
        reqs = [(i * nq, nq, d, 0.0, 80.0, i * cap, cap) for i, d in enumerate(ds)]
        # unrelated eager work and a synchronisation between the calls
        x = torch.randn(1 << 16, device="cuda")
        float(x.sum())
        torch.cuda.synchronize()
        st, got, stats = idx.search_batch_raw(Qb, reqs, out_ptr=out.data_ptr(),
                                              out_capacity=3 * cap, out_on_device=True)
        assert st == tds.TDS_OK and stats["kernel_ms"] > 0
        recs = np.frombuffer(out.cpu().numpy().tobytes(), dtype=tds.RESULT_DTYPE)
        for i, d in enumerate(ds):
            assert got[i] <= cap
            assert key_sorted(recs[i * cap: i * cap + got[i]].copy()) == direct[(d, shift)]


def test_server_host_route_matches_gpu_and_oracle(setup):
    """Hybrid serving: requests whose candidate ranges hold few pairs are
    searched on host threads over a host copy of the index, the rest in GPU
    batches; every request's records are the oracle's and bit-identical to
    tds_search on its own, whichever side ran it."""
    w, idx, reqs = setup
    # the candidate pairs of each request decide its route: a threshold at
    # their median sends about half of the requests to each side
    lens = []
    for Q, d, t0, t1 in reqs:
        a = np.maximum(Q.ts, t0)
        b = np.minimum(Q.te, t1)
        lens.append(int(np.sum(b > a)))
    srv = tds.Server(idx, max_batch_segments=20000, max_batch_requests=16, slots=2,
                     result_capacity=1 << 16, default_reserve=64,
                     cpu_route_tests=int(np.median(lens)) * 125)
    tickets = [srv.submit(Q, d, t0, t1) for Q, d, t0, t1 in reqs]
    got = [srv.wait(t)[0] for t in tickets]
    st = srv.stats()
    srv.close()
    assert st["completed"] == len(reqs) and st["failed"] == 0
    assert 0 < st["cpu_routed"] < len(reqs), st
    for (Q, d, t0, t1), g in zip(reqs, got):
        check_oracle(g, Q, w.D, d, t0, t1)
        assert key_sorted(g) == key_sorted(idx.search(Q, d, t0, t1))
