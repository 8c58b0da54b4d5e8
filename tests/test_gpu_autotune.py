"""The autotuner (bin count, chunk, grid, tile, wavefront mapping chosen by
timing batched searches) on a reduced uniform workload: the configuration it
picks gives the oracle's records (Sec. 3.1 result set), and a second call
with the same workload and search space is served from its cache."""
import numpy as np
import pytest

import oracle
import trajgen
from parity import compare

torch = pytest.importorskip("torch")
import paper_1410_2698_amd as tds  # noqa: E402
from paper_1410_2698_amd import autotune  # noqa: E402

pytestmark = pytest.mark.gpu

KEYS = ("num_bins", "chunk", "grid_waves", "tile", "refine", "deal", "precision")


def test_autotune_choice_is_exact_and_cached(tmp_path):
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = trajgen.uniform1m(0.05, n_pts=81)  # 10,000 entries, 2,000 query segments
    ds = [30.0, 90.0]
    space = {"bins_factor": (1.0, 2.0), "chunk": (4096, 1024), "grid_waves": (4096, 1024),
             "tile": (4, 2), "refine": ("queued", "inline"), "deal": ("dynamic", "static"),
             "precision": ("fp32", "fp64")}
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
    and both places of the refinement in the FP32 form and the FP64 form,
    bit for bit."""
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    w = trajgen.dense(0.02, n_pts=41)
    idx = tds.Index(w.D)
    ref = tds.sort_records(idx.search(w.Q, 4.0, *w.window, precision="fp64"))
    assert ref.size > 100
    for tile in (2, 4):
        for refine in ("queued", "inline"):
            for chunk, deal in ((256, "dynamic"), (256, "static"), (1024, "dynamic"),
                                (4096, "static")):
                got = tds.sort_records(idx.search(w.Q, 4.0, *w.window, tile=tile, chunk=chunk,
                                                  refine=refine, deal=deal, grid_waves=256))
                assert got.tobytes() == ref.tobytes(), (tile, refine, chunk, deal)
    with pytest.raises(tds.TdsError):
        idx.search(w.Q, 4.0, *w.window, tile=3)
    idx.close()
