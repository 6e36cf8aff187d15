"""Shared time sampling: objects observed at the same times fold and sort
once per trial frequency and batch.  Checked against the ordinary catalog
path on the same objects (which must give the same numbers bit for bit:
the same fold, sort and smoother arithmetic) and against the oracle run
object by object."""
import numpy as np
import pytest

import oracle
import paper_2111_07396_amd as ssg
from paper_2111_07396_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def ctx():
    c = ssg.Context(0)
    yield c
    c.close()


def _shared_set(n_obj, n, seed):
    """n_obj curves: the magnitudes of the uneven-catalog generator (each
    object its own period, shape, phase and noise) paired with one shared set
    of times, and error bars scattered over a factor 4."""
    rng = np.random.default_rng(seed)
    t = np.sort(rng.uniform(0, 1000.0, n))
    cat = synth.make_catalog(seed, n_obj, n, 1000.0, (0.2, 10.0), 0.05)
    y = cat.y.reshape(n_obj, n).copy()
    e = cat.e.reshape(n_obj, n) * rng.uniform(0.5, 2.0, (n_obj, n))
    return t, y, e


def _ordinary(ctx, method, t, y, e, grid, params=None):
    import torch
    n_obj, n = y.shape
    offs = np.arange(n_obj + 1, dtype=np.int64) * n
    dc = ssg.DeviceCatalog.from_numpy(offs, np.tile(t, n_obj), y.ravel(), e.ravel())
    pg, st = ctx.method_periodogram(method, dc, grid, params)
    best = ctx.ss_best_period(method, dc, grid, params)
    torch.cuda.synchronize()
    return pg.cpu().numpy(), st.cpu().numpy(), [b.cpu().numpy() for b in best]


@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP, oracle.SSSP2])
@pytest.mark.parametrize("n", [60, 200, 333])
def test_shared_equals_ordinary_and_oracle(ctx, method, n):
    import torch
    n_obj = 37  # batches of 8 and a ragged last batch
    t, y, e = _shared_set(n_obj, n, 100 + n)
    y[5] = 15.0                  # constant magnitudes: CONST_MAG (exact: the
    e[5] = 0.125                 # weighted mean of 15 with equal dyadic weights)
    e[11, 3] = -1.0              # bad error bar: BAD_ERR
    grid = (0.1, 8.0, 157)
    sc = ssg.SharedCatalog.from_numpy(t, y, e)
    pg, st = ctx.shared_periodogram(method, sc, grid)
    bi, bp, bw, st2 = ctx.shared_best_period(method, sc, grid)
    torch.cuda.synchronize()
    pg, st = pg.cpu().numpy(), st.cpu().numpy()
    po, so, best = _ordinary(ctx, method, t, y, e, grid)
    assert list(st) == list(so) and st[5] == ssg.OBJ_CONST_MAG and st[11] == ssg.OBJ_BAD_ERR
    np.testing.assert_array_equal(pg, po)
    np.testing.assert_array_equal(bi.cpu().numpy(), best[0])
    np.testing.assert_array_equal(bw.cpu().numpy(), best[2])
    assert np.array_equal(st2.cpu().numpy(), st)
    # the oracle, object by object (a few objects)
    for o in (0, 17, 36):
        offs = np.array([0, n], dtype=np.int64)
        ora, _ = oracle.periodogram(method, offs, t, y[o], e[o], *grid)
        ok = np.isfinite(ora[0])
        d = np.abs(pg[o][ok] - ora[0][ok])
        assert np.all(d <= TOL * np.maximum(1 - ora[0][ok], 1e-12) + 1e-12), o


def test_shared_edge_cases(ctx):
    import torch
    grid = (0.2, 3.0, 29)
    for n, want in ((4, ssg.OBJ_TOO_FEW), (5000, ssg.OBJ_TOO_LONG)):
        t, y, e = _shared_set(3, n, 7)
        sc = ssg.SharedCatalog.from_numpy(t, y, e)
        pg, st = ctx.shared_periodogram(oracle.SS, sc, grid)
        bi, _, _, _ = ctx.shared_best_period(oracle.SS, sc, grid)
        torch.cuda.synchronize()
        assert (st.cpu().numpy() == want).all()
        assert np.isnan(pg.cpu().numpy()).all()
        assert (bi.cpu().numpy() == -1).all()
    # a non-finite time: every object NONFINITE
    t, y, e = _shared_set(9, 50, 8)
    t[7] = np.nan
    pg, st = ctx.shared_periodogram(oracle.SSSP, ssg.SharedCatalog.from_numpy(t, y, e), grid)
    torch.cuda.synchronize()
    assert (st.cpu().numpy() == ssg.OBJ_NONFINITE).all()
    # a single object, and exact phase ties (dyadic times at power-of-two
    # frequencies), equal to the ordinary path
    rng = np.random.default_rng(9)
    t = np.sort(rng.choice(4096, 150, replace=False)) / 16.0
    y = 15 + 0.2 * np.sin(2 * np.pi * t / 3.0)[None, :] + rng.normal(0, 0.05, (3, t.size))
    e = rng.uniform(0.03, 0.08, (3, t.size))
    for f in (0.25, 1.0):
        g = (f, 2 * f, 1)
        for method in (oracle.SS, oracle.SSSP):
            pg, _ = ctx.shared_periodogram(method, ssg.SharedCatalog.from_numpy(t, y, e), g)
            torch.cuda.synchronize()
            po, _, _ = _ordinary(ctx, method, t, y, e, g)
            np.testing.assert_array_equal(pg.cpu().numpy(), po)
