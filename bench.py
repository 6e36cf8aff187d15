#!/usr/bin/env python3
"""Throughput of the Super Smoother period search on one MI355X.

Workload: the N=200 catalog -- 10,000 synthetic light curves of 200 points
each (sawtooth / sinusoid / eclipsing-binary shapes, random periods and
phases, 0.05 mag noise), searched on 20,000 trial frequencies over
[0.1, 10) c/d.  One step is one pass of the whole hot path over that catalog
for both methods: per-object prep, then for every (object, frequency) trial
fold -> sort -> smoother -> chi^2 -> P -> best period, once with the
cross-validated Super Smoother (Listing 1) and once with the single-pass
generalized-validation variant (Sec. 3).  Inputs are resident in HBM before
the timed region starts.

value = (object, frequency) trials completed per second, summed over the two
methods.  The JSON line also carries each method's own rate, the roofline of
the dominant kernel (the fused Super Smoother trial kernel, timed with HIP
events on the stream it runs on), the CPU oracle timed on a bounded sample,
and -- measured after the timed region -- the other precision, the other
catalogs (single small object, uneven catalog with its FP32c-vs-FP64 error,
single dense object) and the learned-proposal comparison.
"""
from __future__ import annotations

import argparse
import hashlib
import re
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic floating-point operations per point of one trial (each add,
# multiply, divide, compare or abs counted once), from the running-line
# smoother's sliding-window form.
SS_FLOPS_PER_POINT = 385
SSSP_FLOPS_PER_POINT = 156
# MI355X: 256 CUs x 64 FP32/FP64 FMA lanes per clock x 2.4 GHz x 2 flops.
PEAK_VALU_TFLOPS = 78.6
ENCODER_WEIGHTS = os.path.join(ROOT, "paper_2111_07396_amd", "weights", "encoder_c5.npy")


def _code_only(src: bytes) -> bytes:
    """C++ source without comments, whitespace runs collapsed (so that an edit
    of a comment does not count as a change of the kernel)."""
    src = re.sub(rb"/\*.*?\*/", b" ", src, flags=re.S)
    src = re.sub(rb"//[^\n]*", b" ", src)
    return b" ".join(src.split())


def _src_hash(csrc: str = "") -> str:
    """Hash of the code the trial kernel is built from (its own file, the
    arithmetic and wavefront helpers, and the launch structures that precede
    the learned-proposal declarations in the internal header), comments and
    layout ignored."""
    csrc = csrc or os.path.join(ROOT, "paper_2111_07396_amd", "csrc")
    h = hashlib.sha256()
    for name in ("trial_impl.hpp", "trial_f64.hip", "trial_f32c.hip", "numeric.hpp", "wave.hpp"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(_code_only(f.read()))
    with open(os.path.join(csrc, "ssgpu_internal.hpp"), "rb") as f:
        h.update(_code_only(f.read().split(b"// ---- learned frequency proposal")[0]))
    return h.hexdigest()[:16]


def _traffic(precision: str):
    """HBM bytes per SS trial-kernel launch from the committed rocprofv3 PMC
    summary, or None if it is missing or was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_ss_trial_n200_{precision}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("src_hash") != _src_hash():
        return None
    return d.get("bytes_per_launch")


def _best_rates(ctx, dc, grid, params, steps, methods):
    """Wall-clock trials/s and trial-kernel ms per method (`steps` calls each)."""
    import torch
    out = {}
    n = dc.n_obj * int(grid[2])
    for m in methods:
        r = ctx.ss_best_period(m, dc, grid, params)
        torch.cuda.synchronize()
        ms = []
        t0 = time.perf_counter()
        for _ in range(steps):
            r = ctx.ss_best_period(m, dc, grid, params, out=r)
            ms.append(ctx.trial_kernel_ms()[0])
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        out[m] = {"trials_per_s": n / dt, "wall_ms": dt * 1e3, "trial_kernel_ms": min(ms)}
    return out


# BF16 dense matrix-core peak of MI355X (TFLOP/s).
PEAK_BF16_TFLOPS = 2500.0


def _proposal_kernels(ctx, ssg, dc, grid, cat):
    """Rates of the proposal's own kernels on the mixed-stream sample: the
    set encoder forward (per-point layers on the BF16 matrix cores) and one
    training gradient, and the exact-grid bin scores."""
    import numpy as np
    import torch
    from paper_2111_07396_amd import learn
    n_pts = int(cat.offsets[-1])
    w = torch.tensor(learn.init_params(0), dtype=torch.float32, device="cuda")
    lab = torch.zeros(dc.n_obj, dtype=torch.int32, device="cuda")

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps

    t_fwd = timed(lambda: ctx.enc_forward(dc, grid, w))
    t_grad = timed(lambda: ctx.enc_train_grad(dc, grid, w, lab))
    t_sc = timed(lambda: ctx.bin_scores(dc, grid))
    # matrix-core work: 80x64 + 64x128 MACs per point (32-point tiles, padding counted as
    # algorithmic zero work: only real points); the head's 128x1024 per object is FP32 VALU
    mac_pts = (80 * 64 + 64 * 128) * n_pts
    tflops = 2.0 * mac_pts / t_fwd / 1e12
    return {"encoder_forward_ms": t_fwd * 1e3, "encoder_obj_per_s": dc.n_obj / t_fwd,
            "encoder_mfma_tflops": tflops, "encoder_frac_bf16_peak": tflops / PEAK_BF16_TFLOPS,
            "encoder_train_grad_ms": t_grad * 1e3,
            "bin_scores_ms": t_sc * 1e3,
            "bin_scores_trials_per_s": dc.n_obj * int(grid[2]) / t_sc,
            "points": n_pts, "objects": dc.n_obj}


def _extras(ctx, ssg, synth, args):
    """Measurements outside the timed region (each run once after a warm-up)."""
    import numpy as np
    import torch
    ex = {}
    names = {ssg.SS_METHOD_SS: "ss", ssg.SS_METHOD_SSSP: "sssp"}
    both = (ssg.SS_METHOD_SS, ssg.SS_METHOD_SSSP)
    # the other precision on the benchmark catalog
    other = "fp32c" if args.precision == "fp64" else "fp64"
    cat, grid = synth.catalog_n200(n_obj=args.n_obj)
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    prm = ssg.Params(precision=ssg.SS_FP32C if other == "fp32c" else ssg.SS_FP64)
    r = _best_rates(ctx, dc, grid, prm, 1, both)
    ex[f"n200_{other}"] = {names[m]: r[m]["trials_per_s"] for m in both}
    # single small object (N=100, 2,000 frequencies, FP64)
    cat1, grid1 = synth.single_small()
    dc1 = ssg.DeviceCatalog.from_numpy(cat1.offsets, cat1.t, cat1.y, cat1.e)
    r = _best_rates(ctx, dc1, grid1, ssg.Params(), 3, both)
    ex["single_small_fp64"] = {names[m]: {"ms": r[m]["wall_ms"], "trials_per_s":
                                          r[m]["trials_per_s"]} for m in both}
    # uneven catalog (N U[50,400]): rates in both precisions and the FP32c error
    cat2, grid2 = synth.catalog_uneven(n_obj=args.n_obj)
    dc2 = ssg.DeviceCatalog.from_numpy(cat2.offsets, cat2.t, cat2.y, cat2.e)
    ex["uneven"] = {}
    for pn, pv in (("fp64", ssg.SS_FP64), ("fp32c", ssg.SS_FP32C)):
        r = _best_rates(ctx, dc2, grid2, ssg.Params(precision=pv), 1, both)
        ex["uneven"][pn] = {names[m]: r[m]["trials_per_s"] for m in both}
    sub = cat2.subset(np.arange(min(500, cat2.n_obj)))
    dsub = ssg.DeviceCatalog.from_numpy(sub.offsets, sub.t, sub.y, sub.e)
    err = {}
    for m, fn in ((ssg.SS_METHOD_SS, ctx.ss_periodogram), (ssg.SS_METHOD_SSSP,
                                                             ctx.sssp_periodogram)):
        p64, _ = fn(dsub, grid2, ssg.Params(precision=ssg.SS_FP64))
        p32, _ = fn(dsub, grid2, ssg.Params(precision=ssg.SS_FP32C))
        d = (p32.double() - p64).abs()
        rel = d / (1.0 - p64).clamp_min(1e-12)
        ok = torch.isfinite(p64)
        rel = rel[ok]
        b64 = torch.nan_to_num(p64, nan=-1e300).argmax(1)
        b32 = torch.nan_to_num(p32.double(), nan=-1e300).argmax(1)
        err[names[m]] = {"max_abs_dP": float(d[ok].max()), "max_rel_chi2": float(rel.max()),
                         "p99_rel_chi2": float(torch.quantile(rel.float()[:2_000_000], 0.99)),
                         "frac_rel_over_1e-4": float((rel > 1e-4).double().mean()),
                         "best_index_agreement": float((b64 == b32).double().mean())}
    ex["uneven"]["fp32c_vs_fp64_first500"] = err
    # single dense object (N=3,000, 500,000 frequencies)
    cat3, grid3 = synth.single_dense()
    dc3 = ssg.DeviceCatalog.from_numpy(cat3.offsets, cat3.t, cat3.y, cat3.e)
    ex["single_dense"] = {}
    for pn, pv in (("fp64", ssg.SS_FP64), ("fp32c", ssg.SS_FP32C)):
        r = _best_rates(ctx, dc3, grid3, ssg.Params(precision=pv), 1, both)
        ex["single_dense"][pn] = {names[m]: {"ms": r[m]["wall_ms"], "trials_per_s":
                                             r[m]["trials_per_s"]} for m in both}
    ex["method_accuracy"] = _method_accuracy(ctx, ssg, synth)
    ex["shared_sampling"] = _shared_sampling(ctx, ssg, synth)
    ex.update(_proposal(ctx, ssg, synth, args))
    return ex


def _method_accuracy(ctx, ssg, synth, n_obj=2000):
    """Period recovery of the three methods on the uneven-catalog generator
    (the analog of the paper's SS-vs-single-pass comparison): the fraction
    of objects whose best frequency is within 1.5e-3 c/d of the true one,
    and within that of a harmonic or subharmonic (2f, f/2, 3f, f/3)."""
    import numpy as np
    import torch
    cat, grid = synth.catalog_uneven(n_obj=n_obj)
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e)
    f_true = 1.0 / cat.period
    out = {"sample": f"{n_obj} objects of the uneven-catalog generator, {grid[2]} frequencies"}
    for name, m in (("ss", ssg.SS_METHOD_SS), ("sssp_gcv", ssg.SS_METHOD_SSSP),
                    ("sssp_gv", ssg.SS_METHOD_SSSP_GV)):
        r = ctx.ss_best_period(m, dc, grid)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ctx.ss_best_period(m, dc, grid, out=r)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        fb = 1.0 / r[1].cpu().numpy()
        tol = 1.5e-3
        exact = np.abs(fb - f_true) <= tol
        harm = np.zeros_like(exact)
        for h in (2.0, 0.5, 3.0, 1.0 / 3.0):
            harm |= np.abs(fb - h * f_true) <= tol
        out[name] = {"recovered": float(exact.mean()), "harmonic": float((harm & ~exact).mean()),
                     "trials_per_s": n_obj * grid[2] / dt}
        for k, kind in enumerate(("sawtooth", "sinusoid", "eclipse")):
            sel = cat.shape == k
            out[name][f"recovered_{kind}"] = float(exact[sel].mean())
    return out


def _proposal(ctx, ssg, synth, args):
    """Proposal + exact refine against the full grid on a mixed-stream sample."""
    import numpy as np
    import torch
    from paper_2111_07396_amd import learn
    ex = {}
    cat5, grid5 = synth.catalog_mixed(n_obj=args.learned_objects)
    dc5 = ssg.DeviceCatalog.from_numpy(cat5.offsets, cat5.t, cat5.y, cat5.e)
    full5 = ctx.ss_best_period(ssg.SS_METHOD_SS, dc5, grid5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    full5 = ctx.ss_best_period(ssg.SS_METHOD_SS, dc5, grid5, out=full5)
    torch.cuda.synchronize()
    t_full = time.perf_counter() - t0
    pol = dict(learn.POLICY)
    rl = {"sample": f"{cat5.n_obj} objects of the mixed-stream generator (N log-uniform "
                    f"[20, 1000]), {grid5[2]} frequencies on [{grid5[0]}, {grid5[1]}), SS FP64",
          "policy": pol}
    rl["bin_scores_then_refine"] = learn.compare(ctx, dc5, grid5, None, full=full5,
                                                 t_full=t_full, **pol)
    # the same comparison in the compensated-FP32 precision of the mixed stream's
    # configuration (full grid and refine both in FP32c)
    rl["bin_scores_then_refine_fp32c"] = learn.compare(ctx, dc5, grid5, None,
                                                       precision=ssg.SS_FP32C, **pol)
    if os.path.exists(ENCODER_WEIGHTS):
        w = torch.tensor(np.load(ENCODER_WEIGHTS), dtype=torch.float32, device="cuda")
        rl["encoder_plus_100x_bin_scores"] = learn.compare(
            ctx, dc5, grid5, w, 100.0, pol["top_k"], pol["margin"], pol["full_below"], full=full5,
            t_full=t_full)
        rl["encoder_only"] = learn.compare(ctx, dc5, grid5, w, 0.0, pol["top_k"], pol["margin"],
                                           pol["full_below"], full=full5, t_full=t_full)
    bs = rl["bin_scores_then_refine"]
    rl["target_10x_at_99pct"] = {
        "met_by_bin_scores": bool(bs["agreement"] >= 0.99 and bs["speedup"] >= 10.0),
        "met_by_learned_network": False,
        "note": "the set encoder alone agrees on ~36 % of objects; added to the bin scores it "
                "does not raise the agreement, so the >= 10x at >= 99 % result comes from the "
                "non-learned exact-grid bin scores, not from the network"}
    ex["proposal_vs_full"] = rl
    ex["proposal_kernels"] = _proposal_kernels(ctx, ssg, dc5, grid5, cat5)
    return ex


def _host_cpu():
    """CPU model, logical CPUs and physical cores of this host (Linux)."""
    model, phys = "unknown", set()
    try:
        cur = {}
        with open("/proc/cpuinfo") as f:
            for line in f:
                if ":" not in line:
                    if cur:
                        phys.add((cur.get("physical id"), cur.get("core id")))
                    cur = {}
                    continue
                k, v = [x.strip() for x in line.split(":", 1)]
                cur[k] = v
                if k == "model name":
                    model = v
        if cur:
            phys.add((cur.get("physical id"), cur.get("core id")))
    except OSError:
        pass
    return model, os.cpu_count(), len(phys)


def _cpu_baseline(cat, grid, n_sample):
    """The FP64 C oracle on the host cores: the first n_sample objects of the
    benchmark catalog on the whole grid, both methods (OpenMP over trials)."""
    import numpy as np
    import oracle
    sub = cat.subset(np.arange(min(n_sample, cat.n_obj)))
    n_freq = int(grid[2])
    c0 = time.perf_counter()
    for m in (oracle.SS, oracle.SSSP):
        oracle.periodogram(m, sub.offsets, sub.t, sub.y, sub.e, *grid)
    c1 = time.perf_counter()
    model, logical, physical = _host_cpu()
    return {"value": 2 * sub.n_obj * n_freq / (c1 - c0), "unit": "trials/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"first {sub.n_obj} objects x all {n_freq} frequencies, SS and SSSP, "
                      f"FP64 C oracle ({c1 - c0:.1f} s)",
            "cpu_model": model, "logical_cpus": logical, "physical_cores": physical}


def _oracle_configs(synth):
    """The oracle on the single small object in full and on a sample of the
    dense object's grid (the oracle fits every window explicitly, O(n b) per
    smooth: the dense object's full grid would take hours)."""
    import numpy as np
    import oracle
    out = {}
    cat1, grid1 = synth.single_small()
    c0 = time.perf_counter()
    for m in (oracle.SS, oracle.SSSP):
        oracle.periodogram(m, cat1.offsets, cat1.t, cat1.y, cat1.e, *grid1)
    dt = time.perf_counter() - c0
    out["single_small_full"] = {"s": dt, "trials_per_s": 2 * grid1[2] / dt,
                                "trials": 2 * grid1[2], "threads": oracle.num_threads()}
    cat3, grid3 = synth.single_dense()
    ks = np.linspace(0, grid3[2] - 1, 48).astype(np.int64)
    c0 = time.perf_counter()
    for m in (oracle.SS, oracle.SSSP):
        oracle.periodogram(m, cat3.offsets, cat3.t, cat3.y, cat3.e, *grid3, ks=ks)
    dt = time.perf_counter() - c0
    rate = 2 * ks.size / dt
    out["single_dense_sample"] = {"s": dt, "trials_per_s": rate, "frequencies": int(ks.size),
                                  "full_grid_s_extrapolated": 2 * grid3[2] / rate,
                                  "threads": oracle.num_threads()}
    return out


def _shared_sampling(ctx, ssg, synth, n_obj=1000, n=200):
    """Objects that share one time sampling: the shared-catalog call (one
    fold and sort per frequency and batch) against the ordinary call on the
    same objects, FP64, 20,000 frequencies, both methods."""
    import numpy as np
    import torch
    rng = np.random.default_rng(17)
    t = np.sort(rng.uniform(0, 1000.0, n))
    cat = synth.make_catalog(17, n_obj, n, 1000.0, (0.2, 10.0), 0.05)
    y = cat.y.reshape(n_obj, n)
    e = cat.e.reshape(n_obj, n)
    grid = (0.1, 10.0, 20_000)
    sc = ssg.SharedCatalog.from_numpy(t, y, e)
    dc = ssg.DeviceCatalog.from_numpy(np.arange(n_obj + 1, dtype=np.int64) * n,
                                      np.tile(t, n_obj), y.ravel(), e.ravel())
    out = {"catalog": f"{n_obj} objects x {n} points at one set of times, {grid[2]} "
                      f"frequencies, FP64"}
    for m, name in ((ssg.SS_METHOD_SS, "ss"), (ssg.SS_METHOD_SSSP, "sssp")):
        r = {}
        for label, fn in (("shared", lambda: ctx.shared_best_period(m, sc, grid)),
                          ("ordinary", lambda: ctx.ss_best_period(m, dc, grid))):
            res = fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = fn()
            torch.cuda.synchronize()
            r[label] = n_obj * grid[2] / (time.perf_counter() - t0)
        same = torch.equal(ctx.shared_best_period(m, sc, grid)[0],
                           ctx.ss_best_period(m, dc, grid)[0])
        out[name] = {"shared_trials_per_s": r["shared"], "ordinary_trials_per_s": r["ordinary"],
                     "speedup": r["shared"] / r["ordinary"], "same_best_index": bool(same)}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=("fp64", "fp32c"), default="fp64")
    ap.add_argument("--n-obj", type=int, default=10_000)
    ap.add_argument("--cpu-sample-objects", type=int, default=100)
    ap.add_argument("--learned-objects", type=int, default=2000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--proposal-only", action="store_true",
                    help="measure only the proposal + refine comparison and print it")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              "(objects shard across GPUs with no exchange).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2111_07396_amd as ssg
    from paper_2111_07396_amd import synth

    if args.proposal_only:
        ctx = ssg.Context(0)
        print(json.dumps(_proposal(ctx, ssg, synth, args)), flush=True)
        ctx.close()
        return 0
    cat, grid = synth.catalog_n200(n_obj=args.n_obj)
    n_obj, n_freq = cat.n_obj, int(grid[2])
    npts = int(cat.lengths()[0])
    prec = ssg.SS_FP32C if args.precision == "fp32c" else ssg.SS_FP64
    params = ssg.Params(precision=prec)
    dev = torch.device("cuda:0")
    dc = ssg.DeviceCatalog.from_numpy(cat.offsets, cat.t, cat.y, cat.e, device=dev)
    ctx = ssg.Context(0)
    ctx.set_timing(True)
    outs = {m: None for m in (ssg.SS_METHOD_SS, ssg.SS_METHOD_SSSP)}
    kern_ms = {m: [] for m in outs}

    def step(record: bool):
        for m in (ssg.SS_METHOD_SS, ssg.SS_METHOD_SSSP):
            outs[m] = ctx.ss_best_period(m, dc, grid, params, out=outs[m])
            if record:
                kern_ms[m].append(ctx.trial_kernel_ms()[0])

    for _ in range(args.warmup):
        step(False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    print(f"timed {args.steps} steps in {t1 - t0:.2f} s", file=sys.stderr, flush=True)
    elapsed = t1 - t0
    trials = n_obj * n_freq
    value = 2 * trials * args.steps / elapsed

    per_method = {}
    for m, name, fpp in ((ssg.SS_METHOD_SS, "ss", SS_FLOPS_PER_POINT),
                         (ssg.SS_METHOD_SSSP, "sssp", SSSP_FLOPS_PER_POINT)):
        avg_ms = float(np.mean(kern_ms[m]))
        per_method[name] = {
            "trials_per_s_kernel": trials / (avg_ms * 1e-3),
            "trial_kernel_ms": avg_ms,
            "tflops_algorithmic": trials * npts * fpp / (avg_ms * 1e-3) / 1e12,
        }
    ss_ms = per_method["ss"]["trial_kernel_ms"]
    achieved = trials * npts * SS_FLOPS_PER_POINT / (ss_ms * 1e-3) / 1e12
    roofline = {"bound": "alu", "kernel": "fused Super Smoother trial kernel",
                "achieved": achieved, "peak": PEAK_VALU_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / PEAK_VALU_TFLOPS, "traffic": _traffic(args.precision)}

    extras = None
    if not args.no_extras:
        extras = _extras(ctx, ssg, synth, args)
        print("extras done", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        cpu = _cpu_baseline(cat, grid, args.cpu_sample_objects)

    rec = {
        "metric": "obj*freq trials/s (SS & SSSP, N=200)",
        "value": value,
        "unit": "trials/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if prec == ssg.SS_FP32C else "f64",
        "data": "synthetic",
        "config": {"workload": f"catalog of {n_obj} light curves x {npts} points, {n_freq} "
                               f"frequencies on [{grid[0]}, {grid[1]}) c/d, best period by SS "
                               f"and by SSSP", "n_obj": n_obj, "n_points": npts,
                   "n_freq": n_freq, "precision": args.precision},
        "per_method": per_method,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "extras": extras,
    }
    if not args.no_cpu_baseline and not args.no_extras:
        from paper_2111_07396_amd import synth as _s
        rec["extras"]["oracle_configs"] = _oracle_configs(_s)
    print(json.dumps(rec), flush=True)
    ctx.close()
    return 0


if __name__ == "__main__":
    sys.exit(main())
