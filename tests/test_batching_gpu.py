"""Batching: the Eq. 1 memory planner (Sec. 4.1) splits a periodogram into
object batches that fit beta times the device memory; forced small budgets
give many batches whose rows are bit for bit the one-call periodogram.
A catalog with several length classes gives the same results with its class
launches forked onto concurrent streams and run one after another, equal to
the oracle."""
import numpy as np
import pytest

import oracle
import paper_2111_07396_amd as ssg
from paper_2111_07396_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = ssg.Context(0)
    yield c
    c.close()


def test_planner_numbers(ctx):
    grid = (0.05, 20.0, 50_000)
    # 1e6 objects x 50,000 frequencies in FP32 (200 GB of output) against a
    # 64 GiB budget: Eq. 1 with beta = 0.75
    per, nb = ctx.plan_batches(1_000_000, 250_000_000, grid, ssg.SS_FP32C, True, 0.75,
                               64 << 30)
    row = 50_000 * 4 + 12 * ((50_000 + 15) // 16) + 16 + 4 * len(ssg.shapes()) + 4
    assert per == int((0.75 * (64 << 30) - 32 * 250_000_000) // row)
    assert nb == -(-1_000_000 // per) and nb > 1
    # the device's free memory when mem_bytes = 0; a budget below one object
    per0, nb0 = ctx.plan_batches(10_000, 2_000_000, grid)
    assert per0 >= 1 and nb0 >= 1
    with pytest.raises(ssg.SSError) as ei:
        ctx.plan_batches(10, 2000, grid, mem_bytes=100_000)
    assert ei.value.code == ssg.SS_ERR_OOM


@pytest.mark.parametrize("precision", [ssg.SS_FP64, ssg.SS_FP32C])
def test_forced_small_budget_is_bitwise_identical(ctx, precision):
    import torch
    cat, _ = synth.catalog_uneven(seed=91, n_obj=101)
    cat.e[cat.offsets[7]] = 0.0  # a bad object inside a batch
    grid = (0.1, 10.0, 777)
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    prm = ssg.Params(precision=precision)
    ref, st = ctx.method_periodogram(ssg.SS_METHOD_SS, dc, grid, prm)
    torch.cuda.synchronize()
    esz = 8 if precision == ssg.SS_FP64 else 4
    budget = int((32 * cat.offsets[-1] + 9 * (777 * esz + 12 * 49 + 80)) / 0.75)
    got, st2, nb = ctx.periodogram_batched(ssg.SS_METHOD_SS, dc, grid, prm, mem_bytes=budget)
    assert nb >= 10
    np.testing.assert_array_equal(got, ref.cpu().numpy())
    np.testing.assert_array_equal(st2, st.cpu().numpy())
    assert st2[7] == ssg.OBJ_BAD_ERR and np.isnan(got[7]).all()


def test_concurrent_classes_match_oracle(ctx):
    import torch
    # five length classes in one call (forked class launches), timing on
    lens = [40, 100, 180, 240, 350, 500, 60, 130, 250]
    cats = [synth.make_catalog(4000 + i, 1, n, 900.0, (0.3, 5.0), 0.05, shapes=(i % 3,))
            for i, n in enumerate(lens)]
    offs = np.concatenate([[0], np.cumsum([c.offsets[-1] for c in cats])]).astype(np.int64)
    t = np.concatenate([c.t for c in cats])
    y = np.concatenate([c.y for c in cats])
    e = np.concatenate([c.e for c in cats])
    grid = (0.2, 5.0, 211)
    dc = ssg.DeviceCatalog.from_numpy(offs, t, y, e)
    ctx.set_timing(True)
    try:
        for method in (oracle.SS, oracle.SSSP):
            ctx.set_concurrency(True)
            pg, st = ctx.method_periodogram(method, dc, grid)
            ms, n_launch = ctx.trial_kernel_ms()
            torch.cuda.synchronize()
            assert n_launch == 1 and ms > 0  # one span, fork to join
            ctx.set_concurrency(False)
            pg_serial, _ = ctx.method_periodogram(method, dc, grid)
            torch.cuda.synchronize()
            assert ctx.trial_kernel_ms()[1] > 1  # one span per class launch
            np.testing.assert_array_equal(pg.cpu().numpy(), pg_serial.cpu().numpy())
            po, so = oracle.periodogram(method, offs, t, y, e, *grid)
            pg = pg.cpu().numpy()
            d = np.abs(pg - po)
            assert np.all(d <= 1e-4 * np.maximum(1 - po, 1e-12) + 1e-12)
    finally:
        ctx.set_timing(False)
        ctx.set_concurrency(False)
