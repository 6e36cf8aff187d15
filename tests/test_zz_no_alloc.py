"""The allocation-free entry point (ss_best_period_noalloc) through the C ABI:
its outputs equal ss_best_period's bit for bit, on two calls in a row (the
second on a smaller catalog, which reuses the same fixed region), for both
methods; a catalog larger than the region is refused before any work."""
import numpy as np
import pytest

import paper_2111_07396_amd as ssg
from paper_2111_07396_amd import synth

pytestmark = pytest.mark.gpu


def test_noalloc_equals_best_period_on_two_calls():
    import torch
    ctx = ssg.Context(0)
    try:
        grid = (0.1, 10.0, 3001)
        for seed, n_obj in ((81, 300), (82, 57)):  # the second call is smaller
            cat, _ = synth.catalog_uneven(seed=seed, n_obj=n_obj)
            cat.e[cat.offsets[3]] = 0.0  # one bad object
            dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
            for method in (ssg.SS_METHOD_SS, ssg.SS_METHOD_SSSP):
                ref = ctx.ss_best_period(method, dc, grid)
                got = ctx.ss_best_period_noalloc(method, dc, grid)
                torch.cuda.synchronize()
                for a, b in zip(got, ref):  # bit patterns (NaN rows included)
                    ia = a.cpu().view(torch.int64 if a.element_size() == 8 else torch.int32)
                    ib = b.cpu().view(torch.int64 if b.element_size() == 8 else torch.int32)
                    assert torch.equal(ia, ib), (seed, method)
                assert int(got[3][3]) == ssg.OBJ_BAD_ERR and int(got[0][3]) == -1
    finally:
        ctx.close()


def test_noalloc_refuses_a_catalog_larger_than_its_region():
    import torch
    ctx = ssg.Context(0)
    try:
        # 2.2e6 points need 32 bytes each: more than the 64 MiB region
        n_obj, n = 11_000, 200
        rng = np.random.default_rng(5)
        offs = np.arange(n_obj + 1, dtype=np.int64) * n
        t = np.tile(np.sort(rng.uniform(0, 1000, n)), n_obj)
        y = 15 + rng.normal(0, 0.1, n_obj * n)
        e = np.full(n_obj * n, 0.1)
        dc = ssg.DeviceCatalog.from_numpy(offs, t, y, e)
        with pytest.raises(ssg.SSError) as ei:
            ctx.ss_best_period_noalloc(ssg.SS_METHOD_SS, dc, (0.1, 10.0, 100))
        assert ei.value.code == ssg.SS_ERR_UNSUPPORTED
        assert b"allocation-free" in ssg.load_library().ss_last_error()
        torch.cuda.synchronize()
    finally:
        ctx.close()
