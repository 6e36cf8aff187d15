"""Debug mode (SS_FLAG_CHECK_INVARIANTS): the checked call gives the same
results as the plain one, counts every trial, finds no out-of-order sorted
key and no window with W <= 0 on valid catalogs (ties, short, long and
uneven light curves); the self-test bit makes every ordered pair count and
the call report SS_ERR_INVARIANT; the flags are refused where unsupported."""
import numpy as np
import pytest

import paper_2111_07396_amd as ssg
from paper_2111_07396_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = ssg.Context(0)
    yield c
    c.close()


def _catalog():
    # uneven lengths (several size classes, up to the uncached long groups),
    # plus one light curve with repeated times (exact phase ties)
    cats = [synth.make_catalog(71 + i, 1, n, 900.0, (0.3, 5.0), 0.05)
            for i, n in enumerate([12, 70, 200, 333, 700, 1500])]
    rng = np.random.default_rng(5)
    t = np.sort(np.repeat(rng.uniform(0, 800, 90), 2))
    y = 15 + 0.2 * np.sin(2 * np.pi * t / 2.3) + rng.normal(0, 0.05, t.size)
    e = rng.uniform(0.02, 0.06, t.size)
    ts = [c.t for c in cats] + [t]
    ys = [c.y for c in cats] + [y]
    es = [c.e for c in cats] + [e]
    offs = np.concatenate([[0], np.cumsum([a.size for a in ts])]).astype(np.int64)
    return offs, np.concatenate(ts), np.concatenate(ys), np.concatenate(es)


@pytest.mark.parametrize("method", [ssg.SS_METHOD_SS, ssg.SS_METHOD_SSSP])
def test_checked_call_equals_plain_and_counts(ctx, method):
    import torch
    offs, t, y, e = _catalog()
    grid = (0.1, 8.0, 57)
    dc = ssg.DeviceCatalog.from_numpy(offs, t, y, e)
    pg0, st0 = ctx.method_periodogram(method, dc, grid, ssg.Params())
    prm = ssg.Params(flags=ssg.SS_FLAG_CHECK_INVARIANTS)
    pg1, st1 = ctx.method_periodogram(method, dc, grid, prm)
    torch.cuda.synchronize()
    assert torch.equal(st0, st1)
    assert np.array_equal(pg0.cpu().numpy().view(np.int64), pg1.cpu().numpy().view(np.int64))
    ok = int((st1.cpu().numpy() == 0).sum())
    assert ok == offs.size - 1
    assert ctx.check_counts() == (ok * grid[2], 0, 0)
    # the best-period call with the flag
    b0 = ctx.ss_best_period(method, dc, grid, ssg.Params())
    b1 = ctx.ss_best_period(method, dc, grid, prm)
    torch.cuda.synchronize()
    assert torch.equal(b0[0], b1[0])
    assert ctx.check_counts() == (ok * grid[2], 0, 0)


def test_selftest_is_reported(ctx):
    import torch
    offs, t, y, e = _catalog()
    grid = (0.1, 8.0, 19)
    dc = ssg.DeviceCatalog.from_numpy(offs, t, y, e)
    prm = ssg.Params(flags=ssg.SS_FLAG_CHECK_INVARIANTS | ssg.SS_FLAG_CHECK_SELFTEST)
    with pytest.raises(ssg.SSError) as ei:
        ctx.method_periodogram(ssg.SS_METHOD_SSSP, dc, grid, prm)
        torch.cuda.synchronize()
    assert ei.value.code == ssg.SS_ERR_INVARIANT
    n = np.diff(offs)
    # every adjacent pair of a correct sort increases: all are reported
    assert ctx.check_counts() == (n.size * grid[2], int((n - 1).sum()) * grid[2], 0)


def test_flags_refused_where_unsupported(ctx):
    offs, t, y, e = _catalog()
    grid = (0.1, 8.0, 19)
    dc = ssg.DeviceCatalog.from_numpy(offs, t, y, e)
    for flags in (4, ssg.SS_FLAG_CHECK_SELFTEST):
        with pytest.raises(ssg.SSError) as ei:
            ctx.method_periodogram(ssg.SS_METHOD_SS, dc, grid, ssg.Params(flags=flags))
        assert ei.value.code == ssg.SS_ERR_INVALID_ARG
    with pytest.raises(ssg.SSError) as ei:
        ctx.ss_best_period_noalloc(ssg.SS_METHOD_SS, dc, grid,
                                   ssg.Params(flags=ssg.SS_FLAG_CHECK_INVARIANTS))
    assert ei.value.code == ssg.SS_ERR_INVALID_ARG
