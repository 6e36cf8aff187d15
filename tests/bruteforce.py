"""Brute-force reference for the running-line smoother, used only to pin the
oracle on tiny inputs.

Every window is fitted from scratch as a weighted least-squares problem in
matrix form (design matrix [1, x], normal equations solved by
numpy.linalg.solve), and the leverage term is read off the inverse normal
matrix.  This is a different computation from the oracle's two-pass centred
sums, so a dropped term, a wrong sign or a wrong window index in either shows
up as a mismatch.
"""
import numpy as np


def halfwidth(n, span):
    b = int(np.floor(0.5 * span * n + 0.5))
    b = max(b, 2)
    if 2 * b + 1 > n:
        b = (n - 1) // 2
    return b


def window(n, j, b, periodic):
    """(indices, x-shifts) of the window of point j."""
    if periodic:
        i = np.arange(j - b, j + b + 1)
        return np.mod(i, n), np.floor_divide(i, n).astype(float)
    lo = min(max(j - b, 0), n - 1 - 2 * b)
    return np.arange(lo, lo + 2 * b + 1), np.zeros(2 * b + 1)


def smooth(x, v, w, span, periodic=True, cv=True, vsmlsq=0.0):
    x = np.asarray(x, float)
    v = np.asarray(v, float)
    w = np.asarray(w, float)
    n = x.size
    b = halfwidth(n, span)
    s = np.zeros(n)
    r = np.zeros(n)
    lev = np.zeros(n)
    for j in range(n):
        idx, sh = window(n, j, b, periodic)
        xs = x[idx] + sh
        ws = w[idx]
        X = np.stack([np.ones_like(xs), xs], axis=1)
        A = X.T @ (ws[:, None] * X)
        xbar = np.sum(ws * xs) / np.sum(ws)
        V = np.sum(ws * (xs - xbar) ** 2)
        if V > vsmlsq:
            Ainv = np.linalg.inv(A)
            coef = np.linalg.solve(A, X.T @ (ws * v[idx]))
            s[j] = coef[0] + coef[1] * x[j]
            lev[j] = np.array([1.0, x[j]]) @ Ainv @ np.array([1.0, x[j]])
        else:
            s[j] = np.sum(ws * v[idx]) / np.sum(ws)
            lev[j] = 1.0 / np.sum(ws)
        if cv:
            d = 1.0 - w[j] * lev[j]
            r[j] = abs(v[j] - s[j]) / d if d > 0 else (r[j - 1] if j > 0 else 0.0)
    # weighted average over runs of tied x
    j = 0
    while j < n:
        j1 = j
        while j1 + 1 < n and x[j1 + 1] <= x[j1]:
            j1 += 1
        if j1 > j:
            sl = slice(j, j1 + 1)
            s[sl] = np.sum(w[sl] * s[sl]) / np.sum(w[sl])
        j = j1 + 1
    return s, r, lev


def dirichlet_gain(m, n):
    """Mean of cos(2 pi i/n) over i = -(m-1)/2 .. (m-1)/2: the factor by which
    an m-point centred moving average scales a sinusoid sampled n times per
    cycle."""
    return np.sin(np.pi * m / n) / (m * np.sin(np.pi / n))


# ----------------------------------------------------------------- exact rationals
# A second, independent statement of the whole variable-span driver in exact
# rational arithmetic (fractions.Fraction), for tiny inputs with rational x, y,
# w and a whole-number bass exponent.  Each window's line comes from the 2x2
# normal equations solved by Cramer's rule; no rounding anywhere, so the
# oracle must agree to its own rounding error.
from fractions import Fraction as _Q


def _exact_window_fit(x, v, w, j, b, periodic, vsmlsq):
    n = len(x)
    idx, sh = window(n, j, b, periodic)
    W = Sx = Sxx = Sv = Sxv = _Q(0)
    for i, d in zip(idx, sh):
        xi = x[i] + int(d)
        W += w[i]
        Sx += w[i] * xi
        Sxx += w[i] * xi * xi
        Sv += w[i] * v[i]
        Sxv += w[i] * xi * v[i]
    det = W * Sxx - Sx * Sx
    xj = x[j]
    if det / W > vsmlsq:
        a = (Sxx * Sv - Sx * Sxv) / det
        c = (W * Sxv - Sx * Sv) / det
        return a + c * xj, (Sxx - 2 * xj * Sx + xj * xj * W) / det
    return Sv / W, 1 / W


def exact_smooth(x, v, w, span, periodic, cv, vsmlsq):
    """(s, r) of the running-line smoother in exact arithmetic; the half-width
    rule is the float one (it only rounds span n/2)."""
    n = len(x)
    b = halfwidth(n, float(span))
    s, r = [], []
    for j in range(n):
        sj, h = _exact_window_fit(x, v, w, j, b, periodic, vsmlsq)
        s.append(sj)
        if cv:
            d = 1 - w[j] * h
            r.append(abs(v[j] - sj) / d if d > 0 else (r[j - 1] if j > 0 else _Q(0)))
    j = 0
    while j < n:
        j1 = j
        while j1 + 1 < n and x[j1 + 1] <= x[j1]:
            j1 += 1
        if j1 > j:
            m = sum(w[i] * s[i] for i in range(j, j1 + 1)) / sum(w[j:j1 + 1])
            for i in range(j, j1 + 1):
                s[i] = m
        j = j1 + 1
    return s, r


def exact_supsmu(x, y, w, spans, alpha, periodic=True):
    """Variable-span smoother in exact arithmetic.  Returns (smo, chosen)
    where chosen[j] is the span point j selects before the bass shift (None
    when no error is below the 1e20 cap)."""
    n = len(x)
    q = n // 4
    vsmlsq = _Q(1, 10 ** 6) * (x[3 * q - 1] - x[q - 1]) ** 2
    tw, mid, wo = spans
    fits, errs = [], []
    for sp in spans:
        f, r = exact_smooth(x, y, w, sp, periodic, True, vsmlsq)
        e, _ = exact_smooth(x, r, w, mid, periodic, False, vsmlsq)
        fits.append(f)
        errs.append(e)
    expo = 10 - alpha
    assert float(expo) == int(expo) and 0 <= expo <= 10
    cap = _Q(10) ** 20
    chosen, pts = [], []
    for j in range(n):
        es = [errs[k][j] for k in range(3)]
        least = min(es)
        k = es.index(least) if least < cap else None
        sp = spans[k] if k is not None else _Q(0)
        chosen.append(spans[k] if k is not None else None)
        e = least if k is not None else cap
        if 0 < alpha <= 10 and 0 < e < es[2]:
            ratio = max(e / es[2], _Q(1, 10 ** 7))
            sp = sp + (wo - sp) * ratio ** int(expo)
        pts.append(sp)
    sm, _ = exact_smooth(x, pts, w, mid, periodic, False, vsmlsq)
    mixed = []
    for j in range(n):
        s = min(max(sm[j], tw), wo)
        if s < mid:
            g = (mid - s) / (mid - tw)
            mixed.append(fits[1][j] + g * (fits[0][j] - fits[1][j]))
        else:
            g = (s - mid) / (wo - mid)
            mixed.append(fits[1][j] + g * (fits[2][j] - fits[1][j]))
    smo, _ = exact_smooth(x, mixed, w, tw, periodic, False, vsmlsq)
    return smo, chosen
