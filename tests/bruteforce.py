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
