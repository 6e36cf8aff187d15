"""GPU parity of the compensated-FP32 path (SS_FP32C) against the FP64 oracle.

Tolerance, derived from the arithmetic: window sums are float pairs (about
2^-44 relative after the prefix differences), every per-point fit is FP32
(unit roundoff 2^-24 over some ten operations), so a smooth carries relative
error ~1e-6 and chi^2 ~1e-5: every frequency stays within 1e-4 of the oracle
unless an FP32 rounding flips one of the method's hard decisions (the
per-point span argmin, V > vsmlsq, an exact phase tie).  Such flips are rare
and move chi^2 by at most ~1e-2 relative.  The test therefore asks for
1e-4 at >= 99.9 % of frequencies, 1e-2 everywhere, and the oracle's best
index unless the oracle's top two powers are within 1e-3 (1 - P)."""
import numpy as np
import pytest

import oracle
import paper_2111_07396_amd as ssg
from paper_2111_07396_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP])
def test_fp32c_against_fp64_oracle(method):
    import torch
    cat, grid = synth.catalog_uneven()
    sub = cat.subset(np.arange(6))
    grid = (grid[0], grid[1], 4000)
    ctx = ssg.Context(0)
    dc = ssg.DeviceCatalog.from_numpy(sub.offsets, sub.t, sub.y, sub.e)
    fn = ctx.ss_periodogram if method == oracle.SS else ctx.sssp_periodogram
    pg, st = fn(dc, grid, ssg.Params(precision=ssg.SS_FP32C))
    torch.cuda.synchronize()
    assert pg.dtype == torch.float32
    pg = pg.cpu().numpy().astype(np.float64)
    po, so = oracle.periodogram(method, sub.offsets, sub.t, sub.y, sub.e, *grid)
    assert np.array_equal(st.cpu().numpy(), so)
    rel = np.abs(pg - po) / np.maximum(1.0 - po, 1e-12)
    # P is stored as float: its own rounding (~6e-8 |P|) sits inside 1e-4.
    assert np.mean(rel > 1e-4) <= 1e-3, np.sort(rel.ravel())[-10:]
    assert rel.max() <= 1e-2
    for o in range(sub.n_obj):
        ko, kg = oracle.best(po[o]), oracle.best(pg[o])
        if ko != kg:
            top = np.sort(po[o])[::-1]
            assert top[0] - top[1] < 1e-3 * (1 - top[0]), (o, ko, kg)
    ctx.close()
