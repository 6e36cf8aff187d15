"""Seeded synthetic light-curve catalogs.

This module only draws random catalogs; it holds none of the period-search
arithmetic, so both the HIP path and the CPU oracle can take their inputs from
it.  The paper's own datasets (Stripe82, TESS, LINEAR, ObjSmall, ObjLarge,
Syn3k; Sec. 5.2) are not available, so these catalogs stand in for them with
the same kind of shapes: tens to thousands of points per object, periods of
hours to days, non-sinusoidal light curves, photometric error bars.

A catalog is CSR: ``offsets`` (int64, n_obj+1), and per-point ``t`` (days),
``y`` (magnitudes) and ``e`` (error bars), all float64 and contiguous per
object, times sorted within an object.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

SHAPES = ("sawtooth", "sinusoid", "eclipse")


@dataclass
class Catalog:
    offsets: np.ndarray  # int64 [n_obj + 1]
    t: np.ndarray  # float64 [total]
    y: np.ndarray  # float64 [total]
    e: np.ndarray  # float64 [total]
    period: np.ndarray  # float64 [n_obj], true period (days)
    shape: np.ndarray  # int32 [n_obj], index into SHAPES

    @property
    def n_obj(self) -> int:
        return int(self.offsets.size - 1)

    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets)

    def subset(self, idx) -> "Catalog":
        idx = np.asarray(idx, dtype=np.int64)
        lens = self.lengths()[idx]
        offs = np.zeros(idx.size + 1, dtype=np.int64)
        offs[1:] = np.cumsum(lens)
        sl = [slice(self.offsets[i], self.offsets[i + 1]) for i in idx]
        cat = lambda a: np.concatenate([a[s] for s in sl]) if sl else np.zeros(0)
        return Catalog(offs, cat(self.t), cat(self.y), cat(self.e), self.period[idx].copy(),
                       self.shape[idx].copy())


def _shape_values(kind: int, u: np.ndarray) -> np.ndarray:
    if kind == 0:  # sawtooth, 0.3 mag peak to peak
        return 0.3 * (u - 0.5)
    if kind == 1:  # sinusoid, 0.15 mag semi-amplitude
        return 0.15 * np.sin(2.0 * np.pi * u)
    # eclipsing binary: two Gaussian dips (depths 0.5 and 0.2 mag, width 0.03 in phase)
    def dip(c):
        d = u - c
        d = d - np.round(d)
        return np.exp(-0.5 * (d / 0.03) ** 2)
    return -0.5 * dip(0.0) - 0.2 * dip(0.5)


def make_catalog(seed: int, n_obj: int, n_points, t_span: float, period_range, sigma: float,
                 shapes=(0, 1, 2), base_mag: float = 15.0) -> Catalog:
    """Draws ``n_obj`` light curves.

    n_points: an int (every object), a (lo, hi) tuple for uniform integers in
    [lo, hi], or ("loguniform", lo, hi) for round(exp(U[ln lo, ln hi])).
    Times are sorted U[0, t_span]; the period is log-uniform over
    ``period_range``; the phase offset is U[0, 1); the shape cycles through
    ``shapes`` in equal parts (drawn at random); magnitudes are base_mag +
    shape + N(0, sigma) with error bar sigma.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    if isinstance(n_points, (int, np.integer)):
        lens = np.full(n_obj, int(n_points), dtype=np.int64)
    elif n_points[0] == "loguniform":
        lo, hi = n_points[1], n_points[2]
        lens = np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), n_obj))).astype(np.int64)
    else:
        lens = rng.integers(n_points[0], n_points[1] + 1, n_obj).astype(np.int64)
    offsets = np.zeros(n_obj + 1, dtype=np.int64)
    offsets[1:] = np.cumsum(lens)
    total = int(offsets[-1])
    t = np.empty(total)
    y = np.empty(total)
    e = np.full(total, float(sigma))
    lo, hi = period_range
    periods = np.exp(rng.uniform(np.log(lo), np.log(hi), n_obj))
    phase0 = rng.uniform(0.0, 1.0, n_obj)
    kinds = np.asarray(shapes, dtype=np.int32)[rng.integers(0, len(shapes), n_obj)]
    for o in range(n_obj):
        a, b = offsets[o], offsets[o + 1]
        tt = np.sort(rng.uniform(0.0, t_span, b - a))
        u = np.mod(tt / periods[o] + phase0[o], 1.0)
        t[a:b] = tt
        y[a:b] = base_mag + _shape_values(int(kinds[o]), u) + rng.normal(0.0, sigma, b - a)
    return Catalog(offsets, t, y, e, periods, kinds)


# --- the workloads ---------------------------------------------------------
# Each returns (catalog, grid) with grid = (fmin, fmax, n_freq).

def single_small(seed: int = 1):
    """1 object, N=100 over 1,000 d, 0.3-mag sawtooth, P log-U[0.2, 10] d,
    noise 0.05; 2,000 frequencies on [0.1, 10) c/d; run in FP64."""
    return make_catalog(seed, 1, 100, 1000.0, (0.2, 10.0), 0.05, shapes=(0,)), (0.1, 10.0, 2000)


def catalog_uneven(seed: int = 2, n_obj: int = 10_000):
    """10,000 objects, N U_int[50, 400] over 1,000 d, sawtooth/sinusoid/eclipse
    in equal parts, noise 0.05; 20,000 frequencies on [0.1, 10) c/d."""
    return (make_catalog(seed, n_obj, (50, 400), 1000.0, (0.2, 10.0), 0.05),
            (0.1, 10.0, 20_000))


def catalog_n200(seed: int = 7, n_obj: int = 10_000):
    """The headline workload: the uneven-catalog generator with every object at
    N=200; 10,000 objects x 20,000 frequencies on [0.1, 10) c/d."""
    return (make_catalog(seed, n_obj, 200, 1000.0, (0.2, 10.0), 0.05),
            (0.1, 10.0, 20_000))


def single_dense(seed: int = 3):
    """1 object, N=3,000 over 3,000 d, eclipsing binary (dips 0.5/0.2 mag)
    + N(0, 0.02); 500,000 frequencies on [0.01, 20) c/d."""
    return make_catalog(seed, 1, 3000, 3000.0, (0.2, 10.0), 0.02, shapes=(2,)), \
        (0.01, 20.0, 500_000)


def training_set(seed: int = 4, n_obj: int = 200_000):
    """Learned-proposal training curves: N U_int[50, 400] over 1,000 d,
    periods log-U[0.1, 100] d, the three shapes; labels are taken on the
    mixed-stream grid (50,000 frequencies on [0.05, 20) c/d)."""
    return (make_catalog(seed, n_obj, (50, 400), 1000.0, (0.1, 100.0), 0.05),
            (0.05, 20.0, 50_000))


def catalog_mixed(seed: int = 5, n_obj: int = 1_000_000):
    """Mixed stream: N log-uniform on [20, 1000] over 1,000 d, periods
    log-U[0.05, 20] d, the three shapes, noise 0.05; 50,000 frequencies on
    [0.05, 20) c/d."""
    return (make_catalog(seed, n_obj, ("loguniform", 20, 1000), 1000.0, (0.05, 20.0), 0.05),
            (0.05, 20.0, 50_000))
