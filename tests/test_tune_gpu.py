"""The autotuner on the GPU: it times the shapes that hold each length range
of a catalog and then the frequency tile, installs the fastest, caches the
choices, and the search keeps its oracle parity under the tuned settings."""
import json

import numpy as np
import pytest

import oracle
import paper_2111_07396_amd as ssg
from paper_2111_07396_amd import synth, tune

pytestmark = pytest.mark.gpu


def test_tuner_installs_valid_shapes_and_keeps_parity(tmp_path):
    import torch
    cat = synth.make_catalog(12, 40, (40, 300), 1000.0, (0.2, 10.0), 0.05)
    grid = (0.1, 10.0, 1500)
    ctx = ssg.Context(0)
    cache = str(tmp_path / "tune.json")
    chosen, tile = tune.tune(ctx, cat.offsets, cat.t, cat.y, cat.e, grid, sample_objects=16,
                             sample_freqs=256, cache_path=cache)
    assert tile is not None and tile[0] in tune.TILES and tile[1] > 0
    lens = np.diff(cat.offsets)
    assert chosen
    for (lo, hi), (nw, ppl, rate) in chosen.items():
        assert (nw, ppl) in ssg.shapes() and 64 * nw * ppl >= hi and rate > 0
        assert ((lens > lo) & (lens <= hi)).any()
    with open(cache) as f:
        assert len(json.load(f)) == len(chosen) + 1  # the ranges and the tile
    # a second tuner call reuses the cache
    again, tile2 = tune.tune(ctx, cat.offsets, cat.t, cat.y, cat.e, grid, cache_path=cache)
    assert {k: v[:2] for k, v in again.items()} == {k: v[:2] for k, v in chosen.items()}
    assert tile2[0] == tile[0]
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    bi, bp, bw, st = ctx.ss_best_period(oracle.SS, dc, grid)
    torch.cuda.synchronize()
    po, so = oracle.periodogram(oracle.SS, cat.offsets, cat.t, cat.y, cat.e, *grid)
    bi, bw = bi.cpu().numpy(), bw.cpu().numpy()
    for o in range(cat.n_obj):
        ko = oracle.best(po[o])
        assert abs(bw[o] - po[o, ko]) <= 1e-4 * (1 - po[o, ko]) + 1e-12
        if bi[o] != ko:
            assert po[o, ko] - po[o, bi[o]] <= 1e-4 * (1 - po[o, ko])
    ctx.close()
