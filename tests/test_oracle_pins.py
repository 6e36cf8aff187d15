"""Pins of the CPU oracle against things other than itself: brute-force fits,
closed forms, textbook special cases, invariants and numbers the paper prints.
CPU only."""
import json
import os

import numpy as np
import pytest

import oracle
from tests import bruteforce as bf

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
SPANS = (0.05, 0.2, 0.5)


# ----------------------------------------------------------------- smoother

@pytest.mark.parametrize("periodic", [True, False])
@pytest.mark.parametrize("span", [0.05, 0.2, 0.5, 1.0])
def test_smooth_matches_bruteforce(periodic, span):
    rng = np.random.default_rng(11 + int(span * 100) + periodic)
    for n in (5, 6, 9, 17, 40):
        x = np.sort(rng.uniform(0, 1, n))
        v = rng.normal(0, 1, n)
        w = rng.uniform(0.2, 3.0, n)
        s, r, lev = oracle.smooth(x, v, w, span, periodic=periodic, cv=True, vsmlsq=0.0)
        s2, r2, lev2 = bf.smooth(x, v, w, span, periodic=periodic, cv=True, vsmlsq=0.0)
        np.testing.assert_allclose(s, s2, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(r, r2, rtol=1e-9, atol=1e-12)
        np.testing.assert_allclose(lev, lev2, rtol=1e-10, atol=1e-12)


def test_smooth_ties_match_bruteforce():
    rng = np.random.default_rng(5)
    n = 30
    x = np.sort(np.round(rng.uniform(0, 1, n), 1))  # many exact ties
    v = rng.normal(0, 1, n)
    w = rng.uniform(0.5, 2.0, n)
    for periodic in (True, False):
        for span in SPANS:
            # a window of all-equal x has V ~ 0: vsmlsq > 0 decides it, as in
            # the driver
            s, r, _ = oracle.smooth(x, v, w, span, periodic=periodic, cv=True, vsmlsq=1e-8)
            s2, r2, _ = bf.smooth(x, v, w, span, periodic=periodic, cv=True, vsmlsq=1e-8)
            np.testing.assert_allclose(s, s2, rtol=1e-10, atol=1e-12)
            np.testing.assert_allclose(r, r2, rtol=1e-9, atol=1e-12)
            # every run of equal x carries one value
            for u in np.unique(x):
                assert np.ptp(s[x == u]) < 1e-12


def test_smooth_vsmlsq_drops_slope():
    rng = np.random.default_rng(3)
    n = 21
    x = np.sort(rng.uniform(0, 1, n))
    v = rng.normal(0, 1, n)
    w = np.ones(n)
    s, _, lev = oracle.smooth(x, v, w, 0.2, periodic=True, cv=True, vsmlsq=1e9)
    s2, _, lev2 = bf.smooth(x, v, w, 0.2, periodic=True, cv=True, vsmlsq=1e9)
    np.testing.assert_allclose(s, s2, rtol=1e-12)
    np.testing.assert_allclose(lev, 1.0 / 5.0 * np.ones(n) * (5.0 / (2 * bf.halfwidth(n, 0.2) + 1)),
                               rtol=1e-12)


@pytest.mark.parametrize("span", [0.05, 0.2, 0.5, 1.0])
def test_smooth_reproduces_exact_line(span):
    # non-periodic: a line is its own local linear fit, CV residuals vanish
    rng = np.random.default_rng(7)
    n = 33
    x = np.sort(rng.uniform(-2, 3, n))
    w = rng.uniform(0.1, 5.0, n)
    v = 1.7 - 0.6 * x
    s, r, _ = oracle.smooth(x, v, w, span, periodic=False, cv=True)
    np.testing.assert_allclose(s, v, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r, 0.0, atol=1e-11)


def test_smooth_full_window_is_global_regression():
    # non-periodic, span 1, odd n: the clamped window holds every point, so the
    # smooth is the global weighted least-squares line (numpy.polyfit)
    rng = np.random.default_rng(9)
    n = 25
    x = np.sort(rng.uniform(0, 1, n))
    v = rng.normal(0, 1, n)
    w = rng.uniform(0.5, 2.0, n)
    s, _, _ = oracle.smooth(x, v, w, 1.0, periodic=False, cv=False)
    c = np.polyfit(x, v, 1, w=np.sqrt(w))
    np.testing.assert_allclose(s, np.polyval(c, x), rtol=1e-11, atol=1e-12)


@pytest.mark.parametrize("n", [16, 64, 100])
@pytest.mark.parametrize("span", SPANS)
def test_smooth_sinusoid_closed_form(n, span):
    # equally spaced phases, equal weights: every window is centred on its
    # point, so the smooth is the m-point moving average: s = D_m * y, and the
    # leave-one-out residual is |y| (1 - D_m)/(1 - 1/m)
    A, th = 0.7, 0.3
    x = np.arange(n) / n
    y = A * np.sin(2 * np.pi * x + th)
    w = np.full(n, 2.5)
    m = 2 * oracle.halfwidth(n, span) + 1
    D = bf.dirichlet_gain(m, n)
    s, r, lev = oracle.smooth(x, y, w, span, periodic=True, cv=True)
    np.testing.assert_allclose(s, D * y, rtol=0, atol=1e-13)
    np.testing.assert_allclose(r, np.abs(y) * (1 - D) / (1 - 1.0 / m), rtol=1e-10, atol=1e-13)
    np.testing.assert_allclose(w * lev, 1.0 / m, rtol=1e-12)


def test_halfwidth_values():
    assert [oracle.halfwidth(64, s) for s in SPANS] == [2, 6, 16]
    assert [oracle.halfwidth(200, s) for s in SPANS] == [5, 20, 50]
    assert oracle.halfwidth(5, 0.5) == 2
    assert oracle.halfwidth(7, 1.0) == 3  # clamped to (n-1)/2


# ----------------------------------------------------------------- trial closed forms

def _sinusoid_object(n=64, A=0.4, th=0.3, base=15.0, err=0.05):
    # t_j = j / 64 d: at f = 1 c/d every phase j/64 is exact, so fold and sort
    # are exact and the closed forms above apply end to end
    t = np.arange(n) / 64.0
    y = base + A * np.sin(2 * np.pi * t + th)
    e = np.full(n, err)
    return t, y, e


def test_trial_fixed_span_closed_form():
    t, y, e = _sinusoid_object()
    st, tt, w, ybar, chi0 = oracle.prep(t, y, e)
    assert st == 0
    for span in SPANS:
        m = 2 * oracle.halfwidth(64, span) + 1
        D = bf.dirichlet_gain(m, 64)
        p = oracle.trial(oracle.SS, tt, y, w, chi0, 1.0, fixed_span=span)
        assert abs(p - (1 - (1 - D) ** 2)) < 1e-12
        p2 = oracle.trial(oracle.SSSP, tt, y, w, chi0, 1.0, fixed_span=span)
        assert abs(p2 - p) < 1e-12


def _ss_closed_form(alpha, n=64):
    m = [2 * oracle.halfwidth(n, s) + 1 for s in SPANS]
    D = [bf.dirichlet_gain(mm, n) for mm in m]
    c = [(1 - D[k]) / (1 - 1.0 / m[k]) for k in range(3)]
    k = int(np.argmin(c))
    span = SPANS[k]
    if 0 < alpha <= 10 and c[k] < c[2]:
        span += (SPANS[2] - span) * max(c[k] / c[2], 1e-7) ** (10 - alpha)
    span = min(max(span, SPANS[0]), SPANS[2])
    f = span - SPANS[1]
    if f < 0:
        f /= SPANS[0] - SPANS[1]
        B = (1 - f) * D[1] + f * D[0]
    else:
        f /= SPANS[2] - SPANS[1]
        B = (1 - f) * D[1] + f * D[2]
    return 1 - (1 - D[0] * B) ** 2


@pytest.mark.parametrize("alpha", [0.0, 3.5, 9.0, 10.0])
def test_trial_supersmoother_closed_form(alpha):
    # the whole driver on a sinusoid: CV residuals are c_k|y|, so the span
    # choice, the bass enhancement and the blend are all constant over the
    # points and the final curve is a known multiple of y
    t, y, e = _sinusoid_object()
    st, tt, w, ybar, chi0 = oracle.prep(t, y, e)
    p = oracle.trial(oracle.SS, tt, y, w, chi0, 1.0, alpha=alpha)
    assert abs(p - _ss_closed_form(alpha)) < 1e-12


def test_trial_sssp_closed_form():
    t, y, e = _sinusoid_object()
    st, tt, w, ybar, chi0 = oracle.prep(t, y, e)
    m = [2 * oracle.halfwidth(64, s) + 1 for s in SPANS]
    D = [bf.dirichlet_gain(mm, 64) for mm in m]
    gcv = [(1 - D[k]) ** 2 / (1 - 1.0 / m[k]) ** 2 for k in range(3)]
    k = int(np.argmin(gcv))
    p = oracle.trial(oracle.SSSP, tt, y, w, chi0, 1.0)
    assert abs(p - (1 - (1 - D[k]) ** 2)) < 1e-12
    # RSS_k and TR_k individually
    ph = oracle.fold(tt, 1.0)
    perm = oracle.argsort(ph)
    chi2, rss, tr, kb = oracle.sssp(ph[perm], y[perm], w[perm])
    assert kb == k
    np.testing.assert_allclose(tr, [64.0 / mm for mm in m], rtol=1e-12)
    np.testing.assert_allclose(rss, [chi0 * (1 - d) ** 2 for d in D], rtol=1e-10)


def _blend_gain(alpha, n=64):
    # span choice from the per-point residual ratios c_k (the same for every
    # point of the sinusoid), bass, clip, blend: the blend is B times y
    m = [2 * oracle.halfwidth(n, s) + 1 for s in SPANS]
    D = [bf.dirichlet_gain(mm, n) for mm in m]
    c = [(1 - D[k]) / (1 - 1.0 / m[k]) for k in range(3)]
    k = int(np.argmin(c))
    span = SPANS[k]
    if 0 < alpha <= 10 and c[k] < c[2]:
        span += (SPANS[2] - span) * max(c[k] / c[2], 1e-7) ** (10 - alpha)
    span = min(max(span, SPANS[0]), SPANS[2])
    f = span - SPANS[1]
    if f < 0:
        f /= SPANS[0] - SPANS[1]
        return (1 - f) * D[1] + f * D[0]
    f /= SPANS[2] - SPANS[1]
    return (1 - f) * D[1] + f * D[2]


@pytest.mark.parametrize("alpha", [0.0, 3.5, 9.0, 10.0])
def test_trial_sssp2_closed_form(alpha):
    # second single-pass reading on the sinusoid: TR_k = n/m_k, so the
    # un-smoothed residual |y - D_k y| / (1 - 1/m_k) is c_k |y| at every point;
    # the choice, bass and blend are constant and the fit is B y (no final smooth)
    t, y, e = _sinusoid_object()
    st, tt, w, ybar, chi0 = oracle.prep(t, y, e)
    p = oracle.trial(oracle.SSSP2, tt, y, w, chi0, 1.0, alpha=alpha)
    assert abs(p - (1 - (1 - _blend_gain(alpha)) ** 2)) < 1e-12
    # the Listing 1 driver is the same blend followed by the tweeter smooth
    m0 = 2 * oracle.halfwidth(64, SPANS[0]) + 1
    assert abs(_ss_closed_form(alpha) - (1 - (1 - bf.dirichlet_gain(m0, 64)
                                              * _blend_gain(alpha)) ** 2)) < 1e-12


def test_trial_sssp2_fixed_span_is_the_smooth():
    t, y, e = _sinusoid_object()
    st, tt, w, ybar, chi0 = oracle.prep(t, y, e)
    for span in SPANS:
        p = oracle.trial(oracle.SSSP2, tt, y, w, chi0, 1.0, fixed_span=span)
        assert abs(p - oracle.trial(oracle.SS, tt, y, w, chi0, 1.0, fixed_span=span)) < 1e-12


def test_supsmu_nonperiodic_line_is_fixed_point():
    rng = np.random.default_rng(2)
    n = 50
    x = np.sort(rng.uniform(0, 1, n))
    w = rng.uniform(0.5, 2, n)
    y = 3.0 + 2.0 * x
    smo = oracle.supsmu(x, y, w, periodic=False)
    np.testing.assert_allclose(smo, y, atol=1e-12)


def test_supsmu_degenerate_phases_give_weighted_mean():
    n = 12
    x = np.full(n, 0.25)
    y = np.arange(n, dtype=float)
    w = np.linspace(1, 2, n)
    smo = oracle.supsmu(x, y, w)
    np.testing.assert_allclose(smo, np.sum(w * y) / np.sum(w), rtol=1e-14)


def test_supsmu_vsmlsq_uses_listing_quartile_indices():
    # Listing 1 sets scale from sorted abscissae q-1 and 3q-1 (q = n/4).  Here
    # the cyclic window of point 0 ({6, 7, 0, 1, 2}, V = 4.88e-7) sits between
    # the threshold those indices give (3.6e-7) and the one the next indices
    # would give (1.0e-6), so a wrong index changes the fitted curve.
    x = np.array([0.0, 2e-4, 4e-4, 0.3, 0.45, 0.6, 1 - 5e-4, 1 - 2e-4])
    y = np.array([0.0, 1.0, -1.0, 2.0, 0.5, 0.3, -0.2, 0.1])
    w = np.ones(8)
    q = 8 // 4
    vs = 1e-6 * (x[3 * q - 1] - x[q - 1]) ** 2
    smo = oracle.supsmu(x, y, w, fixed_span=0.2)
    ref, _, _ = bf.smooth(x, y, w, 0.2, periodic=True, cv=True, vsmlsq=vs)
    np.testing.assert_allclose(smo, ref, rtol=1e-10, atol=1e-12)
    wrong = 1e-6 * (x[3 * q] - x[q]) ** 2
    ref_wrong, _, _ = bf.smooth(x, y, w, 0.2, periodic=True, cv=True, vsmlsq=wrong)
    assert np.max(np.abs(ref_wrong - ref)) > 1e-3


# ----------------------------------------------------------------- invariants

def _small_catalog(seed=4, n_obj=3):
    rng = np.random.default_rng(seed)
    lens = rng.integers(30, 70, n_obj)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    t = np.concatenate([np.sort(rng.choice(64 * 200, L, replace=False)) / 64.0 for L in lens])
    y = 15 + np.concatenate([0.2 * np.sin(2 * np.pi * rng.uniform(0, 1) + t[a:b] / 1.7)
                             for a, b in zip(offs[:-1], offs[1:])])
    y = y + rng.normal(0, 0.05, y.size)
    e = rng.uniform(0.03, 0.08, y.size)
    return offs, t, y, e


@pytest.mark.parametrize("method", [oracle.SS, oracle.SSSP, oracle.SSSP2])
def test_periodogram_invariances(method):
    offs, t, y, e = _small_catalog()
    grid = (0.2, 3.0, 40)
    p0, st = oracle.periodogram(method, offs, t, y, e, *grid)
    assert np.all(st == 0)
    assert np.all(p0 <= 1.0)
    checks = {
        "t+1024": (t + 1024.0, y, e),
        "y+3": (t, y + 3.0, e),
        "2y": (t, 2.0 * y, e),
        "-y": (t, -y, e),
        "2e": (t, y, 2.0 * e),
    }
    for name, (t2, y2, e2) in checks.items():
        p, _ = oracle.periodogram(method, offs, t2, y2, e2, *grid)
        tol = 1e-12 if name == "t+1024" else 1e-9
        np.testing.assert_allclose(p, p0, rtol=0, atol=tol, err_msg=name)
    # permuting the points of each object: same result.  Times drawn from a
    # continuous distribution, so no two phases tie at any trial frequency.
    rng = np.random.default_rng(1)
    t = t + rng.uniform(0, 1.0 / 64, t.size)
    p0, _ = oracle.periodogram(method, offs, t, y, e, *grid)
    t3, y3, e3 = t.copy(), y.copy(), e.copy()
    for a, b in zip(offs[:-1], offs[1:]):
        pi = a + rng.permutation(b - a)
        t3[a:b], y3[a:b], e3[a:b] = t[pi], y[pi], e[pi]
    p, _ = oracle.periodogram(method, offs, t3, y3, e3, *grid)
    np.testing.assert_allclose(p, p0, rtol=0, atol=1e-12)


def test_constant_phase_trial_scores_zero():
    # every time a multiple of the trial period: all phases 0
    t = np.arange(20) * 0.5
    y = 15 + np.random.default_rng(0).normal(0, 0.1, 20)
    e = np.full(20, 0.1)
    st, tt, w, _, chi0 = oracle.prep(t, y, e)
    for m in (oracle.SS, oracle.SSSP):
        assert abs(oracle.trial(m, tt, y, w, chi0, 2.0)) < 1e-12


# ----------------------------------------------------------------- prep, grid, sort, argmax

def test_prep_statuses():
    t = np.linspace(0, 10, 8)
    y = np.linspace(1, 2, 8)
    e = np.full(8, 0.1)
    assert oracle.prep(t[:4], y[:4], e[:4])[0] == oracle.STATUS_TOO_FEW
    y2 = y.copy(); y2[3] = np.nan
    assert oracle.prep(t, y2, e)[0] == oracle.STATUS_NONFINITE
    e2 = e.copy(); e2[2] = 0.0
    assert oracle.prep(t, y, e2)[0] == oracle.STATUS_BAD_ERR
    assert oracle.prep(t, np.full(8, 3.0), e)[0] == oracle.STATUS_CONST_MAG
    st, tt, w, ybar, chi0 = oracle.prep(t + 5.0, y, e)
    assert st == 0
    np.testing.assert_allclose(tt, t, atol=1e-14)
    np.testing.assert_allclose(w, 100.0, rtol=1e-14)
    assert abs(ybar - 1.5) < 1e-14
    assert abs(chi0 - 100.0 * np.sum((y - 1.5) ** 2)) < 1e-10


def test_grid_numbers_from_table2():
    rows = json.load(open(os.path.join(GOLDEN, "table2_grid.json")))["rows"]
    for r in rows:
        assert oracle.grid_nfreq(0.1 / r["df"], r["fmin"], r["fmax"]) == r["n_freq"], r["dataset"]


def test_grid_half_open():
    n = 2000
    assert oracle.freq(0.1, 10.0, n, 0) == 0.1
    assert abs(oracle.freq(0.1, 10.0, n, n - 1) - (10.0 - 9.9 / n)) < 1e-12
    assert abs(oracle.freq(0.1, 10.0, n, 1) - 0.1 - 0.00495) < 1e-15


def test_fold_exact_on_dyadic_times():
    tt = np.array([0.0, 0.25, 1.5, 7.75, 100.125])
    np.testing.assert_array_equal(oracle.fold(tt, 2.0), [0.0, 0.5, 0.0, 0.5, 0.25])
    np.testing.assert_array_equal(oracle.fold(tt, 0.5), [0.0, 0.125, 0.75, 0.875, 0.0625])


def test_argsort_is_stable():
    key = np.array([0.5, 0.1, 0.5, 0.0, 0.1, 0.5])
    np.testing.assert_array_equal(oracle.argsort(key), np.argsort(key, kind="stable"))


def test_best_lowest_index_and_nan():
    assert oracle.best(np.array([0.1, 0.5, np.nan, 0.5, 0.2])) == 1
    assert oracle.best(np.array([np.nan, np.nan])) == -1


# ----------------------------------------------------------------- phase dispersion

def test_pdm_equals_anova_between_groups():
    # equal weights: the score is the between-group sum of squares over the
    # total, which follows from scipy's one-way ANOVA F statistic
    from scipy.stats import f_oneway
    rng = np.random.default_rng(8)
    n, B = 97, 7
    t = np.sort(rng.uniform(0, 80, n))
    y = rng.normal(size=n)
    e = np.full(n, 0.3)
    f = 0.731
    st, tt, w, ybar, chi0 = oracle.prep(t, y, e)
    p = oracle.pdm_periodogram(np.array([0, n]), t, y, e, f, 2 * f, 1, n_bins=B)[0, 0]
    ph = oracle.fold(tt, f)
    g = np.minimum(B - 1, np.floor(ph * B).astype(int))
    groups = [y[g == b] for b in range(B) if np.any(g == b)]
    F = f_oneway(*groups).statistic
    k = len(groups)
    sst = np.sum((y - y.mean()) ** 2)
    ssb = sst * F * (k - 1) / (F * (k - 1) + (n - k))
    assert p == pytest.approx(ssb / sst, rel=1e-10)


def test_pdm_step_curve_scores_one_and_constant_zero():
    n, B = 40, 8
    t = np.arange(n) * 2.0 ** -5          # exact phases j/40 at f = 0.8
    y = np.where(np.arange(n) < 5, 1.0, 0.0) + 3.0
    e = np.ones(n)
    f0 = 1.0 / (n * 2.0 ** -5)
    p = oracle.pdm_periodogram(np.array([0, n]), t, y, e, f0, 2 * f0, 1, n_bins=B)[0, 0]
    assert p == pytest.approx(1.0, abs=1e-12)
    e2 = oracle.pdm_periodogram(np.array([0, n]), t, np.full(n, 2.0), e, f0, 2 * f0, 1)
    assert np.isnan(e2).all()  # constant magnitudes: bad status, NaN row


def test_pdm_bins_rule():
    assert [oracle.pdm_bins(n) for n in (5, 20, 21, 100, 160, 161, 5000)] == \
        [4, 4, 4, 20, 32, 32, 32]
    assert oracle.pdm_bins(100, 9) == 9


# ----------------------------------------------------------------- variable span, exact

def _n8_case():
    from fractions import Fraction as Q
    g = json.load(open(os.path.join(GOLDEN, "supsmu_n8.json")))
    x = [Q(v, 64) for v in g["x_num_over_64"]]
    y = [Q(v, 8) for v in g["y_num_over_8"]]
    w = [Q(v) for v in g["w"]]
    spans = tuple(Q(v, 10) for v in g["spans_num_over_10"])
    return x, y, w, spans, g["alphas"]


def test_supsmu_n8_points_choose_different_spans_exact():
    # every step of the driver in exact rationals (tests/bruteforce.py) on an
    # 8-point case where half the points take the tweeter and half the
    # midrange: a misreading confined to points with differing choices (the
    # span smooth, the bass shift, the clip or the mixing) shows up here
    x, y, w, spans, alphas = _n8_case()
    xf = np.array([float(v) for v in x])
    yf = np.array([float(v) for v in y])
    wf = np.array([float(v) for v in w])
    for alpha in alphas:
        smo, chosen = bf.exact_supsmu(x, y, w, spans, alpha)
        assert chosen.count(spans[0]) >= 3 and chosen.count(spans[1]) >= 3, chosen
        ref = np.array([float(v) for v in smo])
        got = oracle.supsmu(xf, yf, wf, spans=[float(s) for s in spans], alpha=float(alpha))
        np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13, err_msg=f"alpha={alpha}")
    # the bass shift matters here: alpha 0 and 10 give different curves
    s0, _ = bf.exact_supsmu(x, y, w, spans, 0)
    s10, _ = bf.exact_supsmu(x, y, w, spans, 10)
    assert max(abs(float(a - b)) for a, b in zip(s0, s10)) > 1e-3


def test_supsmu_random_exact_with_other_spans():
    # the same exact statement on random rational inputs, other span triples
    from fractions import Fraction as Q
    rng = np.random.default_rng(31)
    for spans in [(Q(1, 20), Q(1, 5), Q(1, 2)), (Q(1, 10), Q(3, 10), Q(3, 5)),
                  (Q(1, 50), Q(1, 10), Q(3, 10)), (Q(1, 20), Q(1, 5), Q(1))]:
        for n in (9, 14, 23):
            xi = np.sort(rng.choice(256, n, replace=False))
            x = [Q(int(v), 256) for v in xi]
            y = [Q(int(v), 16) for v in rng.integers(-16, 17, n)]
            w = [Q(int(v)) for v in rng.integers(1, 6, n)]
            smo, _ = bf.exact_supsmu(x, y, w, spans, 9)
            got = oracle.supsmu(np.array([float(v) for v in x]), np.array([float(v) for v in y]),
                                np.array([float(v) for v in w]),
                                spans=[float(s) for s in spans], alpha=9.0)
            np.testing.assert_allclose(got, [float(v) for v in smo], rtol=0, atol=1e-12,
                                       err_msg=f"spans={spans} n={n}")


# ----------------------------------------------------------------- closed forms at other spans

OTHER_SPANS = [(0.02, 0.1, 0.3), (0.1, 0.3, 0.6), (0.05, 0.2, 1.0)]


def _gains(spans, n=64):
    m = [2 * oracle.halfwidth(n, s) + 1 for s in spans]
    D = [bf.dirichlet_gain(mm, n) for mm in m]
    return m, D


def _mix_gain(spans, c, D, alpha):
    # span from the per-point error ratios c_k (the same at every point of the
    # sinusoid), bass, clip; the mixed fit is (returned gain) times y
    k = int(np.argmin(c))
    span = spans[k]
    if 0 < alpha <= 10 and c[k] < c[2]:
        span += (spans[2] - span) * max(c[k] / c[2], 1e-7) ** (10 - alpha)
    span = min(max(span, spans[0]), spans[2])
    f = span - spans[1]
    if f < 0:
        f /= spans[0] - spans[1]
        return (1 - f) * D[1] + f * D[0]
    f /= spans[2] - spans[1]
    return (1 - f) * D[1] + f * D[2]


@pytest.mark.parametrize("spans", OTHER_SPANS)
@pytest.mark.parametrize("alpha", [0.0, 7.3, 9.0])
def test_trial_closed_forms_at_other_spans(spans, alpha):
    # sinusoid on exact phases: every smooth is D_m y, the smoothed CV error of
    # span k is c_k |y| D_mid-free (a constant multiple at every point), so the
    # whole driver, both single-pass readings and the fixed span have closed
    # forms for any span triple
    t, y, e = _sinusoid_object()
    st, tt, w, ybar, chi0 = oracle.prep(t, y, e)
    m, D = _gains(spans)
    c = [(1 - D[k]) / (1 - 1.0 / m[k]) for k in range(3)]
    B = _mix_gain(spans, c, D, alpha)
    p = oracle.trial(oracle.SS, tt, y, w, chi0, 1.0, spans=spans, alpha=alpha)
    assert abs(p - (1 - (1 - D[0] * B) ** 2)) < 1e-12
    p2 = oracle.trial(oracle.SSSP2, tt, y, w, chi0, 1.0, spans=spans, alpha=alpha)
    assert abs(p2 - (1 - (1 - B) ** 2)) < 1e-12
    gcv = [(1 - D[k]) ** 2 / (1 - 1.0 / m[k]) ** 2 for k in range(3)]
    k = int(np.argmin(gcv))
    p1 = oracle.trial(oracle.SSSP, tt, y, w, chi0, 1.0, spans=spans)
    assert abs(p1 - (1 - (1 - D[k]) ** 2)) < 1e-12
    for s in spans:
        mm = 2 * oracle.halfwidth(64, s) + 1
        pf = oracle.trial(oracle.SS, tt, y, w, chi0, 1.0, spans=spans, fixed_span=s)
        assert abs(pf - (1 - (1 - bf.dirichlet_gain(mm, 64)) ** 2)) < 1e-12


def test_span_one_window_is_clamped():
    # span 1.0 on 64 points: b = 32 would hold a point twice; clamped to 31
    assert oracle.halfwidth(64, 1.0) == 31
    assert oracle.halfwidth(65, 1.0) == 32
