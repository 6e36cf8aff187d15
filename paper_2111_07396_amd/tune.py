"""Autotuner for the trial-group shape and the frequency tile.

For every light-curve length range present in a catalog it times each
trial-group shape (waves per group x points per thread) that holds the range's
longest curve, on a sample of that range's objects and a slice of the
frequency grid, with the library's own kernel timer (HIP events around the
trial kernels), then installs the fastest shape for that range in the context
(`Context.set_shape`).  With the shapes installed it times the frequency
tile T_f (trial frequencies per work item) on the whole sample and installs
the fastest (`Context.set_tile`).  Results are cached in a JSON file keyed by
device, precision, method, spans, the kernel sources and the length range
(or the catalog's length mix for the tile), so a later process reuses them
without timing.
"""
from __future__ import annotations

import hashlib
import json
import os
import re

import numpy as np

from . import OBJ_TOO_LONG, DeviceCatalog, Params, SSError, SS_METHOD_SS, shapes

# Length ranges tuned separately: (lo, hi] of points per object.
RANGES = ((0, 64), (64, 128), (128, 192), (192, 256), (256, 384), (384, 512), (512, 1024),
          (1024, 2048), (2048, 3072), (3072, 4096))
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "ssgpu_tune.json")
TILES = (16, 32, 64, 128, 256)


def source_key() -> str:
    """Hash of the HIP kernel sources without comments: a tuned choice is
    reused only for the kernels it was measured on."""
    d = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(d)):
        if name.endswith((".hip", ".hpp")):
            src = open(os.path.join(d, name)).read()
            src = re.sub(r"//[^\n]*|/\*.*?\*/", "", src, flags=re.S)
            h.update(name.encode() + b"\0" + "".join(src.split()).encode())
    return h.hexdigest()[:16]


def _device_key():
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{p.name}|{getattr(p, 'gcnArchName', '')}|{p.multi_processor_count}"


def _sub(offsets, t, y, e, idx):
    lens = np.diff(offsets)[idx]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    pick = np.concatenate([np.arange(offsets[i], offsets[i + 1]) for i in idx])
    return offs, t[pick], y[pick], e[pick]


def tune(ctx, offsets, t, y, e, grid, params: Params | None = None, method=SS_METHOD_SS,
         sample_objects=256, sample_freqs=2048, cache_path=DEFAULT_CACHE, verbose=False,
         tile=True):
    """Chooses a shape per length range for the catalog (host numpy arrays)
    and, with tile=True, the frequency tile, and installs the choices in
    `ctx`.  Returns ({range: (nw, ppl, trials_per_s)}, (tile, trials_per_s) or
    None)."""
    import torch

    params = params or Params()
    offsets = np.asarray(offsets, dtype=np.int64)
    lens = np.diff(offsets)
    cache = {}
    if cache_path and os.path.exists(cache_path):
        with open(cache_path) as f:
            cache = json.load(f)
    dev = _device_key()
    spans = f"s{params.span_min:g},{params.span_mid:g},{params.span_max:g},f{params.fixed_span:g}"
    base_key = f"{dev}|p{params.precision}|m{method}|{spans}|k{source_key()}"
    chosen = {}
    ctx.set_shape(0, 0, 0)
    ctx.set_timing(True)
    fmin, fmax, nf = grid
    nf_s = int(min(nf, sample_freqs))
    g_s = (fmin, fmin + (fmax - fmin) * nf_s / nf, nf_s)
    for lo, hi in RANGES:
        members = np.nonzero((lens > lo) & (lens <= hi))[0]
        if members.size == 0:
            continue
        key = f"{base_key}|{lo}-{hi}"
        if key in cache:
            nw, ppl, rate = cache[key]
        else:
            idx = members[:sample_objects]
            n_max = int(lens[idx].max())
            sub = _sub(offsets, t, y, e, idx)
            dc = DeviceCatalog.from_numpy(*sub)
            best = None
            for nw_c, ppl_c in shapes():
                if 64 * nw_c * ppl_c < hi or 64 * nw_c * ppl_c > 4 * max(hi, 64):
                    continue
                try:
                    ctx.set_shape(0, 0, 0)
                    ctx.set_shape(max(n_max, 1), nw_c, ppl_c)
                    out = ctx.ss_best_period(method, dc, g_s, params)
                    torch.cuda.synchronize()
                    out = ctx.ss_best_period(method, dc, g_s, params, out=out)
                    ms, _ = ctx.trial_kernel_ms()
                except SSError:  # shape rejected for this range
                    continue
                # a shape whose LDS does not hold the spans marks its objects too long
                # and returns at once: never a candidate
                if bool((out[3] == OBJ_TOO_LONG).any()):
                    continue
                rate = idx.size * nf_s / (ms * 1e-3)
                if verbose:
                    print(f"tune {lo}-{hi}: {nw_c}x{ppl_c} {rate:.3e} trials/s", flush=True)
                if best is None or rate > best[2]:
                    best = (nw_c, ppl_c, rate)
            if best is None:
                continue
            nw, ppl, rate = best
            cache[key] = [nw, ppl, rate]
        chosen[(lo, hi)] = (nw, ppl, rate)
    ctx.set_shape(0, 0, 0)
    for (lo, hi), (nw, ppl, _) in sorted(chosen.items()):
        ctx.set_shape(hi, nw, ppl)
    tile_choice = None
    if tile and chosen:
        # the tile, on a sample of the whole catalog with the shapes installed
        mix = ",".join(f"{lo}-{hi}:{int(((lens > lo) & (lens <= hi)).sum())}"
                       for lo, hi in sorted(chosen))
        key = f"{base_key}|tile|{mix}"
        if key in cache:
            tile_choice = tuple(cache[key])
        else:
            rng = np.random.default_rng(0)
            idx = np.sort(rng.choice(lens.size, min(lens.size, sample_objects), replace=False))
            dc = DeviceCatalog.from_numpy(*_sub(offsets, t, y, e, idx))
            for tf in TILES:
                ctx.set_tile(tf)
                out = ctx.ss_best_period(method, dc, g_s, params)
                torch.cuda.synchronize()
                ctx.ss_best_period(method, dc, g_s, params, out=out)
                ms, _ = ctx.trial_kernel_ms()
                rate = idx.size * nf_s / (ms * 1e-3)
                if verbose:
                    print(f"tune tile {tf}: {rate:.3e} trials/s", flush=True)
                if tile_choice is None or rate > tile_choice[1]:
                    tile_choice = (tf, rate)
            cache[key] = list(tile_choice)
        ctx.set_tile(int(tile_choice[0]))
    if cache_path:
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        with open(cache_path, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
    ctx.set_timing(False)
    return chosen, tile_choice
