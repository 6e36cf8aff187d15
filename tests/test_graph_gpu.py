"""A best-period call captured into a HIP graph and replayed on new data.

The library plans on the device (shape classes and work queues are built by
the prep kernel, counters are cleared by a kernel), so a call with a grown
workspace contains no host synchronisation and no allocation and can be
captured.  Every replay is checked against an eager call on the same data,
with eager work and synchronisations between the replays."""
import numpy as np
import pytest

import paper_2111_07396_amd as ssg
from paper_2111_07396_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("method", [ssg.SS_METHOD_SS, ssg.SS_METHOD_SSSP])
def test_captured_call_replays_match_eager(method):
    import torch
    base, _ = synth.catalog_uneven(seed=61, n_obj=48)
    grid = (0.1, 10.0, 600)
    ctx = ssg.Context(0)
    dc = ssg.DeviceCatalog.from_numpy(base.offsets, base.t, base.y, base.e)
    n = dc.n_obj
    out = (torch.empty(n, dtype=torch.int64, device="cuda"),
           torch.empty(n, dtype=torch.float64, device="cuda"),
           torch.empty(n, dtype=torch.float64, device="cuda"),
           torch.empty(n, dtype=torch.int32, device="cuda"))
    ctx.ss_best_period(method, dc, grid, out=out)  # grows the workspace
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.ss_best_period(method, dc, grid, out=out)
    torch.cuda.synchronize()
    for rep in range(3):
        # same object lengths, new light curves
        nxt = synth.make_catalog(700 + rep, n, (50, 400), 1000.0, (0.2, 10.0), 0.05)
        lens = np.diff(base.offsets)
        t = np.concatenate([np.sort(np.random.default_rng(rep).uniform(0, 1000, L)) for L in lens])
        y = np.resize(nxt.y, t.size)
        dc.t.copy_(torch.from_numpy(t))
        dc.y.copy_(torch.from_numpy(y))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [o.clone() for o in out]
        ref = ctx.ss_best_period(method, dc, grid)
        torch.cuda.synchronize()
        for a, b in zip(got, ref):
            assert torch.equal(a.cpu(), b.cpu()), f"replay {rep}"
    ctx.close()
