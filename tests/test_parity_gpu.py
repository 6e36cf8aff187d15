"""GPU parity: the HIP path against the FP64 CPU oracle on the same seeded
inputs, through the C ABI.  Tolerance (FP64 path): at every frequency
|chi2_gpu - chi2_oracle| <= 1e-4 * chi2_oracle, i.e.
|P_gpu - P_oracle| <= 1e-4 * (1 - P_oracle); the best index must be equal
unless the oracle's two largest P differ by less than that tolerance."""
import numpy as np
import pytest

import oracle
import paper_2111_07396_amd as ssg
from paper_2111_07396_amd import synth

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def ctx():
    import torch
    c = ssg.Context(0)
    yield c
    c.close()


def _gpu_pgram(ctx, method, offs, t, y, e, grid, params=None):
    import torch
    cat = ssg.DeviceCatalog.from_numpy(offs, t, y, e)
    pg, st = ctx.method_periodogram(method, cat, grid, params)
    torch.cuda.synchronize()
    return pg.cpu().numpy().astype(np.float64), st.cpu().numpy()


def _assert_pgram_close(pg, po, tol=TOL, what=""):
    ok = np.isfinite(po)
    assert np.array_equal(ok, np.isfinite(pg)), what
    d = np.abs(pg[ok] - po[ok])
    lim = tol * np.maximum(1.0 - po[ok], 1e-12) + 1e-12
    bad = d > lim
    assert not bad.any(), f"{what}: {bad.sum()} of {bad.size} over tol, worst {np.max(d / lim)}"


def _assert_best_equal(pg, po, tol=TOL):
    for o in range(po.shape[0]):
        if not np.isfinite(po[o]).any():
            continue
        ko, kg = oracle.best(po[o]), oracle.best(pg[o])
        if ko == kg:
            continue
        top = np.sort(po[o][np.isfinite(po[o])])[::-1]
        assert top[0] - top[1] < tol * (1 - top[0]), (o, ko, kg)


@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP])
def test_single_small_full_grid(ctx, method):
    cat, grid = synth.single_small()
    po, so = oracle.periodogram(method, cat.offsets, cat.t, cat.y, cat.e, *grid)
    pg, sg = _gpu_pgram(ctx, method, cat.offsets, cat.t, cat.y, cat.e, grid)
    assert np.array_equal(so, sg)
    _assert_pgram_close(pg, po, what="single object N=100")
    _assert_best_equal(pg, po)


LENGTHS = [5, 6, 17, 63, 64, 65, 100, 128, 129, 191, 192, 193, 255, 256, 257, 300, 383, 384,
           385, 450, 511, 512]


@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP])
def test_every_size_class_and_ragged_tile(ctx, method):
    rng = np.random.default_rng(123)
    cats = [synth.make_catalog(1000 + i, 1, n, 500.0, (0.3, 5.0), 0.05, shapes=(i % 3,))
            for i, n in enumerate(LENGTHS)]
    offs = np.concatenate([[0], np.cumsum([c.offsets[-1] for c in cats])]).astype(np.int64)
    t = np.concatenate([c.t for c in cats])
    y = np.concatenate([c.y for c in cats])
    e = np.concatenate([c.e for c in cats]) * rng.uniform(0.5, 2.0, offs[-1])
    grid = (0.2, 3.3, 173)  # not a multiple of any tile
    po, so = oracle.periodogram(method, offs, t, y, e, *grid)
    pg, sg = _gpu_pgram(ctx, method, offs, t, y, e, grid)
    assert np.array_equal(so, sg)
    _assert_pgram_close(pg, po, what="size classes")
    _assert_best_equal(pg, po)


@pytest.mark.parametrize("alpha", [0.0, 4.5, 9.0, 10.0])
def test_alpha_and_fixed_span(ctx, alpha):
    cat, grid = synth.catalog_uneven(seed=21, n_obj=6)
    grid = (0.1, 10.0, 300)
    prm = ssg.Params(alpha=alpha)
    po, _ = oracle.periodogram(oracle.SS, cat.offsets, cat.t, cat.y, cat.e, *grid, alpha=alpha)
    pg, _ = _gpu_pgram(ctx, oracle.SS, cat.offsets, cat.t, cat.y, cat.e, grid, prm)
    _assert_pgram_close(pg, po, what=f"alpha={alpha}")
    for method in (oracle.SS, oracle.SSSP):
        po, _ = oracle.periodogram(method, cat.offsets, cat.t, cat.y, cat.e, *grid,
                                   fixed_span=0.3)
        pg, _ = _gpu_pgram(ctx, method, cat.offsets, cat.t, cat.y, cat.e, grid,
                           ssg.Params(fixed_span=0.3))
        _assert_pgram_close(pg, po, what=f"fixed span method={method}")


def test_sinusoid_closed_form_on_gpu(ctx):
    # t_j = j/64 d, f = 1 c/d: exact phases j/64; P has a closed form
    from tests.test_oracle_pins import _ss_closed_form, _sinusoid_object
    t, y, e = _sinusoid_object()
    offs = np.array([0, t.size], dtype=np.int64)
    pg, _ = _gpu_pgram(ctx, oracle.SS, offs, t, y, e, (1.0, 2.0, 4))
    assert abs(pg[0, 0] - _ss_closed_form(9.0)) < 1e-12


def test_statuses_and_nan_rows(ctx):
    import torch
    rng = np.random.default_rng(5)
    lens = [0, 3, 40, 40, 40, 40, 80]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    t = rng.uniform(0, 100, offs[-1])
    y = 15 + rng.normal(0, 0.1, offs[-1])
    e = np.full(offs[-1], 0.1)
    t[offs[2] + 5] = np.nan          # object 2: non-finite t
    e[offs[3] + 7] = 0.0             # object 3: bad error
    y[offs[4]:offs[5]] = 12.5        # object 4: constant
    y[offs[5] + 1] = np.inf          # object 5: non-finite y
    grid = (0.5, 2.0, 50)
    for method in (oracle.SS, oracle.SSSP):
        po, so = oracle.periodogram(method, offs, t, y, e, *grid)
        pg, sg = _gpu_pgram(ctx, method, offs, t, y, e, grid)
        assert list(sg) == [1, 1, 3, 2, 4, 3, 0]
        assert np.array_equal(so, sg)
        assert np.isnan(pg[:6]).all()
        _assert_pgram_close(pg[6:], po[6:])
        cat = ssg.DeviceCatalog.from_numpy(offs, t, y, e)
        bi, bp, bw, st = ctx.ss_best_period(method, cat, grid)
        bi = bi.cpu().numpy()
        assert list(bi[:6]) == [-1] * 6
        assert np.isnan(bp.cpu().numpy()[:6]).all()
        assert bi[6] == oracle.best(po[6])


def test_phase_ties(ctx):
    # Dyadic times folded at power-of-two frequencies: both the oracle's
    # (tt mod p)/p and the kernel's frac(tt f) are exact there, so the many
    # equal phases are exact ties on both sides (tie averaging, windows with
    # zero spread).  At other frequencies such ties are only ties up to the
    # fold's rounding, and either order is a correct answer.
    rng = np.random.default_rng(8)
    t = np.sort(rng.choice(4096, 150, replace=False)) / 16.0
    y = 15 + 0.2 * np.sin(2 * np.pi * t / 3.0) + rng.normal(0, 0.05, t.size)
    e = rng.uniform(0.03, 0.08, t.size)
    offs = np.array([0, t.size], dtype=np.int64)
    for f in (0.125, 0.25, 0.5, 1.0, 2.0, 4.0):
        grid = (f, 2 * f, 1)
        for method in (oracle.SS, oracle.SSSP):
            po, _ = oracle.periodogram(method, offs, t, y, e, *grid)
            pg, _ = _gpu_pgram(ctx, method, offs, t, y, e, grid)
            _assert_pgram_close(pg, po, what=f"ties f={f} method={method}")


@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP])
def test_best_period_matches_periodogram(ctx, method):
    import torch
    cat, _ = synth.catalog_uneven(seed=33, n_obj=40)
    grid = (0.1, 10.0, 700)
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    fn = ctx.ss_periodogram if method == oracle.SS else ctx.sssp_periodogram
    pg, st = fn(dc, grid)
    bi, bp, bw, st2 = ctx.ss_best_period(method, dc, grid)
    torch.cuda.synchronize()
    pg = pg.cpu().numpy()
    bi = bi.cpu().numpy()
    for o in range(cat.n_obj):
        k = oracle.best(pg[o])
        assert bi[o] == k
        assert bw.cpu().numpy()[o] == pg[o, k]
        f = oracle.freq(grid[0], grid[1], grid[2], k)
        assert bp.cpu().numpy()[o] == 1.0 / f


@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP])
def test_every_shape_gives_the_oracle_result(ctx, method):
    # the same light curves forced through every trial-group shape that holds
    # them: identical to the oracle within tolerance, and to each other
    import torch
    lens = [150, 200, 250]
    cats = [synth.make_catalog(300 + i, 1, n, 800.0, (0.3, 5.0), 0.05, shapes=(i % 3,))
            for i, n in enumerate(lens)]
    offs = np.concatenate([[0], np.cumsum([c.offsets[-1] for c in cats])]).astype(np.int64)
    t = np.concatenate([c.t for c in cats])
    y = np.concatenate([c.y for c in cats])
    e = np.concatenate([c.e for c in cats])
    grid = (0.2, 4.0, 37)
    po, _ = oracle.periodogram(method, offs, t, y, e, *grid)
    ref = None
    try:
        for nw, ppl in ssg.shapes():
            if 64 * nw * ppl < 250:
                continue
            ctx.set_shape(0, 0, 0)
            ctx.set_shape(250, nw, ppl)
            pg, st = _gpu_pgram(ctx, method, offs, t, y, e, grid)
            if (st == ssg.OBJ_TOO_LONG).all():  # shape does not fit the LDS at span 0.5
                continue
            _assert_pgram_close(pg, po, what=f"shape {nw}x{ppl}")
            if ref is None:
                ref = pg
            np.testing.assert_allclose(pg, ref, rtol=0, atol=1e-11)
    finally:
        ctx.set_shape(0, 0, 0)


@pytest.mark.parametrize("precision", [ssg.SS_FP64, ssg.SS_FP32C])
@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP, oracle.SSSP2])
def test_every_kernel_gives_the_oracle_result(ctx, method, precision):
    # every compiled kernel (shape x method x precision), each on a light curve
    # that fills most of its group: every kernel has its own register budget,
    # so each one is checked on its own
    tol = TOL if precision == ssg.SS_FP64 else 1e-2
    grid = (0.2, 4.0, 23)
    try:
        for i, (nw, ppl) in enumerate(ssg.shapes()):
            n = min(700, max(5, int(0.85 * 64 * nw * ppl)))
            cat = synth.make_catalog(900 + i, 1, n, 800.0, (0.3, 5.0), 0.05, shapes=(i % 3,))
            ctx.set_shape(0, 0, 0)
            ctx.set_shape(n, nw, ppl)
            po, _ = oracle.periodogram(method, cat.offsets, cat.t, cat.y, cat.e, *grid)
            pg, st = _gpu_pgram(ctx, method, cat.offsets, cat.t, cat.y, cat.e, grid,
                                ssg.Params(precision=precision))
            if (st == ssg.OBJ_TOO_LONG).all():  # shape does not fit the LDS at span 0.5
                continue
            _assert_pgram_close(pg, po, tol=tol, what=f"kernel {nw}x{ppl} n={n}")
    finally:
        ctx.set_shape(0, 0, 0)


@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP])
def test_long_light_curves(ctx, method):
    # multi-wave trial groups: lengths across the 512/1024/2048/3072 shapes,
    # including the dense 3,000-point eclipsing binary
    cats = [synth.make_catalog(500 + i, 1, n, 3000.0, (0.2, 10.0), 0.02, shapes=(2,))
            for i, n in enumerate([600, 1024, 1025, 2049, 3000])]
    offs = np.concatenate([[0], np.cumsum([c.offsets[-1] for c in cats])]).astype(np.int64)
    t = np.concatenate([c.t for c in cats])
    y = np.concatenate([c.y for c in cats])
    e = np.concatenate([c.e for c in cats])
    grid = (0.01, 20.0, 23)
    po, so = oracle.periodogram(method, offs, t, y, e, *grid)
    pg, sg = _gpu_pgram(ctx, method, offs, t, y, e, grid)
    assert np.array_equal(so, sg)
    _assert_pgram_close(pg, po, what="long light curves")
    pg32, _ = _gpu_pgram(ctx, method, offs, t, y, e, grid, ssg.Params(precision=ssg.SS_FP32C))
    rel = np.abs(pg32 - po) / np.maximum(1 - po, 1e-12)
    # the compensated-FP32 bar: 1e-4 at >= 99.9 % of trials, 1e-2 everywhere
    print(f"FP32c long curves: max {rel.max():.2e}, over 1e-4 {np.mean(rel > 1e-4):.2e}")
    assert np.mean(rel > 1e-4) <= 1e-3 and rel.max() <= 1e-2, (rel.max(), np.mean(rel > 1e-4))


def test_tile_size_does_not_change_results(ctx):
    cat, _ = synth.catalog_uneven(seed=44, n_obj=5)
    grid = (0.1, 10.0, 211)
    pg0, _ = _gpu_pgram(ctx, oracle.SS, cat.offsets, cat.t, cat.y, cat.e, grid)
    try:
        for tile in (1, 7, 64, 500):
            ctx.set_tile(tile)
            pg, _ = _gpu_pgram(ctx, oracle.SS, cat.offsets, cat.t, cat.y, cat.e, grid)
            np.testing.assert_array_equal(pg, pg0)
    finally:
        ctx.set_tile(0)


def test_size_limits(ctx):
    # the longest curve the default spans fit in LDS (3,072 points on 16x3
    # groups) against the oracle on a few frequencies; one point more, and a
    # curve above SS_MAX_POINTS, are reported too long with NaN rows
    import torch
    lens = [3072, 3073, 5000]
    cats = [synth.make_catalog(700 + i, 1, n, 3000.0, (0.2, 10.0), 0.02, shapes=(2,))
            for i, n in enumerate(lens)]
    offs = np.concatenate([[0], np.cumsum([c.offsets[-1] for c in cats])]).astype(np.int64)
    t = np.concatenate([c.t for c in cats])
    y = np.concatenate([c.y for c in cats])
    e = np.concatenate([c.e for c in cats])
    grid = (0.05, 5.0, 7)
    for method in (oracle.SS, oracle.SSSP):
        pg, st = _gpu_pgram(ctx, method, offs, t, y, e, grid)
        assert list(st) == [0, ssg.OBJ_TOO_LONG, ssg.OBJ_TOO_LONG]
        assert np.isnan(pg[1:]).all()
        po, so = oracle.periodogram(method, offs[:2], t[:3072], y[:3072], e[:3072], *grid)
        _assert_pgram_close(pg[:1], po, what=f"n=3072 method={method}")
        dc = ssg.DeviceCatalog.from_numpy(offs, t, y, e)
        bi, bp, bw, st2 = ctx.ss_best_period(method, dc, grid)
        torch.cuda.synchronize()
        assert list(bi.cpu().numpy()[1:]) == [-1, -1]


@pytest.mark.parametrize("precision", [ssg.SS_FP64, ssg.SS_FP32C])
@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP, oracle.SSSP2])
def test_ties_and_uneven_weights_on_every_shape(ctx, method, precision):
    # tie averaging on every group shape, forced for the light curve (exact
    # phase ties from dyadic times at power-of-two frequencies), and eight
    # points whose weights span four decades on every shape (almost all of a
    # group's slots are padding)
    rng = np.random.default_rng(77)
    tie_t = np.sort(rng.choice(2048, 60, replace=False)) / 16.0
    tie_y = 15 + 0.2 * np.sin(2 * np.pi * tie_t / 3.0) + rng.normal(0, 0.05, tie_t.size)
    tie_e = rng.uniform(0.03, 0.08, tie_t.size)
    fb_t = np.array([0.0, 0.31, 0.77, 1.2, 2.9, 3.3, 5.05, 7.4])
    fb_y = np.array([15.0, 15.4, 14.8, 15.2, 15.1, 14.7, 15.3, 15.0])
    fb_e = np.array([0.001, 0.2, 0.3, 0.002, 0.25, 0.1, 0.003, 0.3])
    cases = [("ties", tie_t, tie_y, tie_e, [(f, 2 * f, 1) for f in (0.25, 1.0, 4.0)]),
             ("uneven weights", fb_t, fb_y, fb_e, [(0.05, 3.0, 41)])]
    try:
        for name, t, y, e, grids in cases:
            offs = np.array([0, t.size], dtype=np.int64)
            for nw, ppl in ssg.shapes():
                ctx.set_shape(0, 0, 0)
                ctx.set_shape(t.size, nw, ppl)
                for grid in grids:
                    po, so = oracle.periodogram(method, offs, t, y, e, *grid)
                    pg, sg = _gpu_pgram(ctx, method, offs, t, y, e, grid,
                                        ssg.Params(precision=precision))
                    if (sg == ssg.OBJ_TOO_LONG).all():
                        continue
                    assert np.array_equal(so, sg)
                    _assert_pgram_close(pg, po, tol=TOL if precision == ssg.SS_FP64 else 1e-2,
                                        what=f"{name} {nw}x{ppl} grid={grid}")
    finally:
        ctx.set_shape(0, 0, 0)


OTHER_SPANS = [(0.02, 0.1, 0.3), (0.1, 0.3, 0.6), (0.05, 0.2, 1.0)]


@pytest.mark.parametrize("spans", OTHER_SPANS)
@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP, oracle.SSSP2])
def test_other_spans(ctx, method, spans):
    # span parameters other than the defaults change the half-widths, the
    # periodic extension and the LDS layout; lengths across several shapes
    lens = [23, 70, 150, 200, 333, 600]
    cats = [synth.make_catalog(1500 + i, 1, n, 900.0, (0.3, 5.0), 0.05, shapes=(i % 3,))
            for i, n in enumerate(lens)]
    offs = np.concatenate([[0], np.cumsum([c.offsets[-1] for c in cats])]).astype(np.int64)
    t = np.concatenate([c.t for c in cats])
    y = np.concatenate([c.y for c in cats])
    e = np.concatenate([c.e for c in cats]) * np.random.default_rng(4).uniform(0.5, 2.0, offs[-1])
    grid = (0.1, 6.0, 97)
    prm = ssg.Params(span_min=spans[0], span_mid=spans[1], span_max=spans[2])
    po, so = oracle.periodogram(method, offs, t, y, e, *grid, spans=spans)
    pg, sg = _gpu_pgram(ctx, method, offs, t, y, e, grid, prm)
    assert np.array_equal(so, sg)
    _assert_pgram_close(pg, po, what=f"spans={spans} method={method}")
    _assert_best_equal(pg, po)


@pytest.mark.parametrize("alpha", [2.5, 7.3])
@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP2])
def test_fractional_alpha(ctx, method, alpha):
    # non-integer 10 - alpha: the bass power goes through exp2/log2
    cat, _ = synth.catalog_uneven(seed=23, n_obj=16)
    grid = (0.1, 10.0, 301)
    po, _ = oracle.periodogram(method, cat.offsets, cat.t, cat.y, cat.e, *grid, alpha=alpha)
    pg, _ = _gpu_pgram(ctx, method, cat.offsets, cat.t, cat.y, cat.e, grid,
                       ssg.Params(alpha=alpha))
    _assert_pgram_close(pg, po, what=f"alpha={alpha} method={method}")
    _assert_best_equal(pg, po)


@pytest.mark.parametrize("spans", OTHER_SPANS)
def test_sinusoid_closed_form_other_spans_on_gpu(ctx, spans):
    from tests.test_oracle_pins import _sinusoid_object, _gains, _mix_gain
    t, y, e = _sinusoid_object()
    offs = np.array([0, t.size], dtype=np.int64)
    m, D = _gains(spans)
    c = [(1 - D[k]) / (1 - 1.0 / m[k]) for k in range(3)]
    prm = ssg.Params(span_min=spans[0], span_mid=spans[1], span_max=spans[2], alpha=9.0)
    pg, _ = _gpu_pgram(ctx, oracle.SS, offs, t, y, e, (1.0, 2.0, 4), prm)
    assert abs(pg[0, 0] - (1 - (1 - D[0] * _mix_gain(spans, c, D, 9.0)) ** 2)) < 1e-12
    pg, _ = _gpu_pgram(ctx, oracle.SSSP2, offs, t, y, e, (1.0, 2.0, 4), prm)
    assert abs(pg[0, 0] - (1 - (1 - _mix_gain(spans, c, D, 9.0)) ** 2)) < 1e-12


@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP, oracle.SSSP2])
def test_every_kernel_at_other_spans(ctx, method):
    # every compiled FP64 kernel at a non-default span triple, on several
    # objects that fill most of its group (several work items per group)
    spans = (0.1, 0.3, 0.6)
    prm = ssg.Params(span_min=spans[0], span_mid=spans[1], span_max=spans[2])
    grid = (0.2, 4.0, 41)
    try:
        for i, (nw, ppl) in enumerate(ssg.shapes()):
            n = min(700, max(5, int(0.85 * 64 * nw * ppl)))
            cat = synth.make_catalog(2900 + i, 3, n, 800.0, (0.3, 5.0), 0.05)
            ctx.set_shape(0, 0, 0)
            ctx.set_shape(n, nw, ppl)
            po, _ = oracle.periodogram(method, cat.offsets, cat.t, cat.y, cat.e, *grid,
                                       spans=spans)
            pg, st = _gpu_pgram(ctx, method, cat.offsets, cat.t, cat.y, cat.e, grid, prm)
            if (st == ssg.OBJ_TOO_LONG).all():
                continue
            _assert_pgram_close(pg, po, what=f"kernel {nw}x{ppl} n={n} spans={spans}")
    finally:
        ctx.set_shape(0, 0, 0)


def _stress_catalog(seed, n, n_obj=8):
    """Objects of n points that stress the rare paths: repeated times (each
    time observed two or three times: exact phase ties at every frequency,
    whatever the fold's rounding, so tie averaging on both sides), a few
    points with errors 200x smaller than the rest (leverage w h up to
    1 - 2e-5: CV residuals divided by a nearly vanishing 1 - w h), clumped
    times (half the points within 0.02 d), and plain ones."""
    rng = np.random.default_rng(seed)
    ts, ys, es = [], [], []
    for o in range(n_obj):
        kind = o % 4
        if kind == 0:
            t = np.sort(np.repeat(rng.uniform(0, 800, n), rng.integers(2, 4, n))[:n])
        elif kind == 2:
            t = np.sort(np.concatenate([rng.uniform(0, 800, n - n // 2),
                                        rng.uniform(100, 100.02, n // 2)]))
        else:
            t = np.sort(rng.uniform(0, 800, n))
        y = 15 + 0.3 * np.sin(2 * np.pi * t / rng.uniform(0.3, 5.0)) + rng.normal(0, 0.05, n)
        e = rng.uniform(0.02, 0.08, n)
        if kind == 1:
            e[rng.choice(n, max(2, n // 20), replace=False)] *= 0.005
        ts.append(t)
        ys.append(y)
        es.append(e)
    offs = np.concatenate([[0], np.cumsum([t.size for t in ts])]).astype(np.int64)
    return offs, np.concatenate(ts), np.concatenate(ys), np.concatenate(es)


@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP, oracle.SSSP2])
def test_every_kernel_many_items_ties_and_heavy_points(ctx, method):
    # every compiled FP64 kernel on eight objects that fill most of its group,
    # one frequency per work item (tile 1) and more items than the persistent
    # grid has workgroups, so every workgroup takes several items in a row;
    # a quarter of the objects have exact phase ties at every frequency, a
    # quarter has points of leverage close to 1.  (Ties from dyadic times at
    # frequencies whose period is not a binary fraction would not do: the
    # kernel's phase, the fraction of the exact product tt f, is exact there,
    # while the oracle's (tt mod p)/p is off by an ulp, so only one side sees
    # the tie.)
    try:
        ctx.set_tile(1)
        for i, (nw, ppl) in enumerate(ssg.shapes()):
            n = min(700, max(5, int(0.85 * 64 * nw * ppl)))
            nf = 400 if n <= 256 else 160
            grid = (0.25, 0.25 + nf / 16.0, nf)
            offs, t, y, e = _stress_catalog(3100 + i, n)
            assert (np.diff(t[offs[0]:offs[1]]) == 0).sum() >= n // 3
            ctx.set_shape(0, 0, 0)
            ctx.set_shape(n, nw, ppl)
            po, so = oracle.periodogram(method, offs, t, y, e, *grid)
            pg, sg = _gpu_pgram(ctx, method, offs, t, y, e, grid)
            if (sg == ssg.OBJ_TOO_LONG).all():
                continue
            assert np.array_equal(so, sg)
            _assert_pgram_close(pg, po, what=f"kernel {nw}x{ppl} n={n} method={method}")
    finally:
        ctx.set_shape(0, 0, 0)
        ctx.set_tile(0)
