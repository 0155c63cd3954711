"""Choose eps for the large synthetic workloads and store them in
tests/golden/eps_calibration.json.

Uses only the brute-force oracle (oracle.reference.count_rows_multi) on a
seeded sample of query rows against all n points:
  * uniform, n = 10,000,000, d = 3..6: eps whose MEAN neighbour count
    (excluding the point itself) is k = 32 and k = 256;
  * clustered, n = 5,000,000, d = 2, 3: eps whose MEDIAN neighbour count
    (excluding the point itself) is 50.
Two passes per workload: a coarse geometric grid around a starting guess,
then a fine grid around the interpolated value. Values are rounded to five
significant digits.

    python tests/golden/calibrate_eps.py            # all workloads
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle import reference  # noqa: E402
from paper_1803_04120_amd import datagen  # noqa: E402

OUT = os.path.join(HERE, "eps_calibration.json")
SAMPLE_ROWS = 4096
SAMPLE_SEED = 99


def ball(d):
    return math.pi ** (d / 2) / math.gamma(d / 2 + 1)


def stat_curve(pts, rows, eps_grid, stat):
    counts = reference.count_rows_multi(pts, eps_grid, rows) - 1  # exclude the point itself
    if stat == "mean":
        return counts.mean(axis=0)
    return np.median(counts, axis=0)


def solve(pts, rows, guess, target, stat):
    eps = guess
    for lo, hi, num in ((0.6, 1.6, 81), (0.985, 1.015, 61)):
        grid = eps * np.geomspace(lo, hi, num)
        curve = stat_curve(pts, rows, grid, stat)
        if not (curve[0] <= target <= curve[-1]):
            raise RuntimeError(f"target {target} outside [{curve[0]}, {curve[-1]}] around eps={eps}")
        k = int(np.searchsorted(curve, target))
        k = min(max(k, 1), num - 1)
        c0, c1 = curve[k - 1], curve[k]
        t = 0.0 if c1 == c0 else (target - c0) / (c1 - c0)
        eps = float(np.exp(np.log(grid[k - 1]) + t * (np.log(grid[k]) - np.log(grid[k - 1]))))
    return float(f"{eps:.5g}")


def main():
    out = {"citation": "Section VI-A shapes (uniform in [0,100]^d, FP64); eps chosen by "
                       "tests/golden/calibrate_eps.py with the brute-force oracle on "
                       f"{SAMPLE_ROWS} sampled query rows (seed {SAMPLE_SEED})",
           "uniform_n10M": {}, "clustered_n5M": {}}
    for d in (3, 4, 5, 6):
        t0 = time.time()
        n = 10_000_000
        pts = datagen.uniform(n, d, seed=30 + d)
        rows = np.random.default_rng(SAMPLE_SEED).choice(n, SAMPLE_ROWS, replace=False)
        for k in (32, 256):
            guess = (k * 100.0 ** d / (n * ball(d))) ** (1.0 / d)
            eps = solve(pts, rows, guess, float(k), "mean")
            out["uniform_n10M"][f"d{d}_k{k}"] = {"n": n, "d": d, "seed": 30 + d, "k_mean": k, "eps": eps}
            print(f"uniform d={d} k={k}: eps={eps} ({time.time() - t0:.0f}s)", flush=True)
        del pts
    for d in (2, 3):
        t0 = time.time()
        n = 5_000_000
        pts = datagen.clustered(n, d, seed=40 + d)
        rows = np.random.default_rng(SAMPLE_SEED).choice(n, SAMPLE_ROWS, replace=False)
        guess = {2: 0.09, 3: 0.49}[d]
        eps = solve(pts, rows, guess, 50.0, "median")
        out["clustered_n5M"][f"d{d}"] = {"n": n, "d": d, "seed": 40 + d, "k_median": 50, "eps": eps}
        print(f"clustered d={d}: eps={eps} ({time.time() - t0:.0f}s)", flush=True)
        del pts
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", OUT)


if __name__ == "__main__":
    main()
