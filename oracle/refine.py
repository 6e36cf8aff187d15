"""FP64 reference of search-and-refine (test infrastructure only).

The paper proposes (Sec. 6) to search a cheap proposal first and run the
exact Super Smoother only around the proposed frequencies.  Here the proposal
is a score per log-spaced frequency bin (the set encoder's logits); this
module defines, as plainly as possible, which fine-grid frequencies a given
score vector selects and what the exact search over them returns.

  bins       bin b = 0..1023 holds grid index k when E_b <= f_k < E_{b+1},
             E_b = f_min * (f_max / f_min) ** (b / 1024), f_k = f_min + k df
  selection  the top_k bins by score (NaN lowest; equal scores: lower bin
             first), each widened by `margin` bins on both sides
  result     the first maximum of the exact periodogram over the selected
             indices in increasing k (NaN skipped), as for the full grid
"""
from __future__ import annotations

import numpy as np

from . import periodogram

BINS = 1024


def grid_f(fmin, fmax, n_freq, k):
    df = (fmax - fmin) / n_freq
    return fmin + np.asarray(k, dtype=np.float64) * df


def bin_edges(fmin, fmax):
    ratio = fmax / fmin
    return np.array([fmin * ratio ** (b / BINS) for b in range(BINS + 1)])


def bin_table(fmin, fmax, n_freq):
    """First grid index of every bin (entry 1024 = n_freq), by direct search:
    the number of grid frequencies below each edge."""
    f = grid_f(fmin, fmax, n_freq, np.arange(n_freq))
    edges = bin_edges(fmin, fmax)
    tab = np.searchsorted(f, edges[1:BINS], side="left")
    return np.concatenate([[0], tab, [n_freq]]).astype(np.int64)


def top_bins(scores, top_k):
    s = np.where(np.isnan(scores), -np.inf, np.asarray(scores, dtype=np.float64))
    order = sorted(range(BINS), key=lambda b: (-s[b], b))
    return order[:top_k]


def refine_set(scores, top_k, margin, table):
    sel = np.zeros(BINS, dtype=bool)
    for b in top_bins(scores, top_k):
        sel[max(0, b - margin):min(BINS, b + margin + 1)] = True
    ks = [np.arange(table[b], table[b + 1]) for b in range(BINS) if sel[b]]
    return np.concatenate(ks).astype(np.int64) if ks else np.zeros(0, dtype=np.int64)


def refine_best(method, offsets, t, y, e, grid, scores, top_k, margin, alpha=9.0, full_below=0):
    """(best_idx, best_power) per object; -1 / NaN for objects with a bad
    status or an empty selection.  Objects with fewer than full_below points
    are searched on the whole grid."""
    fmin, fmax, n_freq = grid
    table = bin_table(fmin, fmax, n_freq)
    n_obj = len(offsets) - 1
    bi = np.full(n_obj, -1, dtype=np.int64)
    bp = np.full(n_obj, np.nan)
    for o in range(n_obj):
        a, b = offsets[o], offsets[o + 1]
        if b - a < full_below:
            ks = np.arange(n_freq, dtype=np.int64)
        else:
            ks = refine_set(scores[o], top_k, margin, table)
        if ks.size == 0:
            continue
        pg, st = periodogram(method, np.array([0, b - a]), t[a:b], y[a:b], e[a:b], fmin, fmax,
                             n_freq, ks=ks, alpha=alpha)
        if st[0] != 0:
            continue
        row = pg[0]
        best = -1
        for i in range(ks.size):
            if not np.isnan(row[i]) and (best < 0 or row[i] > row[best]):
                best = i
        if best >= 0:
            bi[o] = ks[best]
            bp[o] = row[best]
    return bi, bp


def bin_scores(t, y, e, grid):
    """Cheap exact-grid proposal score per log bin (zeros for a bad object):
    at every grid frequency the fraction of chi0 explained by the weighted
    means of B = clamp(n // 5, 4, 32) equal phase bins, phase = frac(tt f) in
    FP64, bin = min(B - 1, floor(phase B)); each log bin takes the maximum
    over its grid frequencies (0 when it holds none)."""
    from . import prep
    fmin, fmax, n_freq = grid
    st, tt, w, ybar, chi0 = prep(t, y, e)
    out = np.zeros(BINS)
    if st != 0:
        return out
    n = len(t)
    B = min(32, max(4, n // 5))
    yc = np.asarray(y, dtype=np.float64) - ybar
    f = grid_f(fmin, fmax, n_freq, np.arange(n_freq))
    score = np.empty(n_freq)
    for k0 in range(0, n_freq, 512):
        q = np.outer(f[k0:k0 + 512], tt)
        jb = np.minimum(B - 1, np.floor((q - np.floor(q)) * B).astype(np.int64))
        for r in range(jb.shape[0]):
            W = np.bincount(jb[r], weights=w, minlength=B)
            S = np.bincount(jb[r], weights=w * yc, minlength=B)
            ok = W > 0
            score[k0 + r] = np.sum(S[ok] ** 2 / W[ok]) / chi0
    tab = bin_table(fmin, fmax, n_freq)
    for b in range(BINS):
        if tab[b + 1] > tab[b]:
            out[b] = score[tab[b]:tab[b + 1]].max()
    return out
