"""Writes dense_c3_peaks.json: the CPU oracle's full-grid periodogram of the
dense single object (synth.single_dense: one light curve of 3,000 points over
3,000 d, 500,000 frequencies on [0.01, 20) c/d), for the Super Smoother
(Listing 1) and the single-pass reading R1 (Sec. 3), reduced to its best index
and its 64 highest trials.  Every value comes from oracle/ on the seeded
synthetic input; run from the repository root:

    python tests/golden/make_dense_c3.py [--npz PATH]

(--npz also keeps the two full periodograms; about 80 min on 8 cores.)"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)
import oracle  # noqa: E402
from paper_2111_07396_amd import synth  # noqa: E402  (seeded input generator only)

TOP = 64


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--npz", default=None)
    a = ap.parse_args()
    cat, grid = synth.single_dense()
    out = {"what": "CPU oracle, full grid of the dense single object (3,000 points, "
                   "500,000 frequencies on [0.01, 20) c/d): best index and the 64 "
                   "highest trials per method",
           "grid": list(grid), "methods": {}}
    full = {}
    for m, name in ((oracle.SS, "ss"), (oracle.SSSP, "sssp")):
        t0 = time.perf_counter()
        pg, st = oracle.periodogram(m, cat.offsets, cat.t, cat.y, cat.e, *grid)
        dt = time.perf_counter() - t0
        p = pg[0]
        kb = oracle.best(p)
        order = np.argsort(-p, kind="stable")[:TOP]
        out["methods"][name] = {"status": int(st[0]), "best": kb, "p_best": float(p[kb]),
                                "top": [[int(k), float(p[k])] for k in order],
                                "seconds": round(dt, 1), "threads": os.cpu_count()}
        full[name] = p
        print(f"{name}: best {kb} P {p[kb]:.12f} in {dt:.0f} s", flush=True)
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "dense_c3_peaks.json"), "w") as f:
        json.dump(out, f, indent=1)
    if a.npz:
        np.savez(a.npz, **full)


if __name__ == "__main__":
    main()
