"""The autotuner (bin count, chunk, grid, tile, wavefront mapping chosen by
timing batched searches) on a reduced uniform workload: the configuration it
picks gives the oracle's records (Sec. 3.1 result set), and a second call
with the same workload and search space is served from its cache."""
import numpy as np
import pytest

import oracle
import trajgen
from parity import compare, device_segments

torch = pytest.importorskip("torch")
import paper_1410_2698_amd as tds  # noqa: E402
from paper_1410_2698_amd import autotune  # noqa: E402

pytestmark = pytest.mark.gpu

KEYS = ("num_bins", "chunk", "grid_waves", "tile", "refine", "deal", "output", "precision")


def records_of(buf, n):
    """The first n records of a CUDA byte tensor as an (n, 4) int64 NumPy
    array (q_seg | e_seg << 32, trajectories, t_lo bits, t_hi bits)."""
    a = buf[: n * 32].cpu().numpy().view(np.int64).reshape(n, 4)
    ids = a[:, 0]
    return np.stack([ids & 0xFFFFFFFF, (ids >> 32) & 0xFFFFFFFF, a[:, 2], a[:, 3]], axis=1)


def test_autotune_choice_is_exact_and_cached(tmp_path):
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = trajgen.uniform1m(0.05, n_pts=81)  # 10,000 entries, 2,000 query segments
    ds = [30.0, 90.0]
    space = {"bins_factor": (1.0, 2.0), "chunk": (4096, 1024), "grid_waves": (4096, 1024),
             "tile": (4, 2), "refine": ("queued", "inline"), "deal": ("dynamic", "static"),
             "output": ("direct", "staged"), "precision": ("fp32", "fp64")}
    cache = str(tmp_path / "tune.json")
    best = autotune.tune(w.D, w.Q, ds, w.window, space=space, reps=1, cache=cache)
    assert not best["cached"]
    assert best["trials"] >= 6  # the starting point and one move per knob at least
    assert best["tile"] in (2, 4) and best["precision"] in ("fp32", "fp64")
    idx = tds.Index(w.D, num_bins=best["num_bins"])
    total = 0
    for d in ds:
        got = idx.search(w.Q, d, *w.window, precision=best["precision"], chunk=best["chunk"],
                         grid_waves=best["grid_waves"], tile=best["tile"], refine=best["refine"],
                         deal=best["deal"])
        want = oracle.sort_results(oracle.search(w.Q, w.D, d, *w.window))
        compare(tds.sort_records(got), want, f"tuned d={d}")
        total += want.size
    idx.close()
    assert total > 100
    again = autotune.tune(w.D, w.Q, ds, w.window, space=space, reps=1, cache=cache)
    assert again["cached"]
    assert {k: again[k] for k in KEYS} == {k: best[k] for k in KEYS}


def test_every_tile_and_mapping_gives_the_same_records():
    """The knobs the autotuner moves do not change the records: both tiles
    and both places of the refinement in the FP32 form, both output modes,
    and the FP64 form, bit for bit."""
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = trajgen.dense(0.02, n_pts=41)
    idx = tds.Index(w.D)
    ref = tds.sort_records(idx.search(w.Q, 4.0, *w.window, precision="fp64", output="staged"))
    assert ref.size > 100
    for tile in (2, 4):
        for refine in ("queued", "inline"):
            for chunk, deal, output in ((256, "dynamic", "direct"), (256, "static", "staged"),
                                        (1024, "dynamic", "staged"), (4096, "static", "direct")):
                got = tds.sort_records(idx.search(w.Q, 4.0, *w.window, tile=tile, chunk=chunk,
                                                  refine=refine, deal=deal, output=output,
                                                  grid_waves=256))
                assert got.tobytes() == ref.tobytes(), (tile, refine, chunk, deal, output)
    got = tds.sort_records(idx.search(w.Q, 4.0, *w.window, precision="fp64", output="direct"))
    assert got.tobytes() == ref.tobytes()
    with pytest.raises(tds.TdsError):
        idx.search(w.Q, 4.0, *w.window, tile=3)
    idx.close()


@pytest.mark.parametrize("grid_waves", [256, 4096, 8192, 20480])
def test_direct_output_capacities_on_the_device(grid_waves):
    """Direct output into a device buffer: at the exact count the records
    are the staged search's; one short of it (and far short) the call
    overflows and the buffer holds that many distinct results; with room to
    spare the first `count` records are the results.  Many waves end with
    partly used chunks, so the fill has work at every grid; a grid of more
    waves than the fill plan takes (16,384) stages instead, unasked."""
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = trajgen.dense(0.05, n_pts=81)
    idx = tds.Index(w.D)
    Qt = device_segments(w.Q)
    d = 12.0
    st, n, _ = idx.search_raw(Qt, d, *w.window, out_ptr=0, capacity=0, out_on_device=True,
                              output="staged")
    assert st == tds.TDS_E_OVERFLOW and n > 10000
    ref = torch.empty(n * 32, dtype=torch.uint8, device="cuda")
    st, n2, _ = idx.search_raw(Qt, d, *w.window, out_ptr=ref.data_ptr(), capacity=n,
                               out_on_device=True, output="staged")
    assert st == tds.TDS_OK and n2 == n
    want = set(map(tuple, records_of(ref, n)[:, :2].tolist()))
    assert len(want) == n
    for cap in (n + 1000, n, n - 1, n // 3):
        buf = torch.full(((n + 1000) * 32,), 0xAB, dtype=torch.uint8, device="cuda")
        st, m, s = idx.search_raw(Qt, d, *w.window, out_ptr=buf.data_ptr(), capacity=cap,
                                  out_on_device=True, output="direct", grid_waves=grid_waves)
        assert m == n and s["stage_flushes"] > 0, (cap, m, n)
        k = min(cap, n)
        got = records_of(buf, k)
        keys = set(map(tuple, got[:, :2].tolist()))
        assert len(keys) == k and keys <= want, (cap, grid_waves)
        if cap >= n:
            assert st == tds.TDS_OK
            assert tds.sort_records(np.frombuffer(buf[: n * 32].cpu().numpy().tobytes(),
                                                  dtype=tds.RESULT_DTYPE)).tobytes() == \
                tds.sort_records(np.frombuffer(ref.cpu().numpy().tobytes(),
                                               dtype=tds.RESULT_DTYPE)).tobytes()
        else:
            assert st == tds.TDS_E_OVERFLOW
    idx.close()
