"""Shared helpers for the tests (inputs only; no expected values)."""
from __future__ import annotations

import json
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name: str):
    with open(os.path.join(GOLDEN, name)) as f:
        return json.load(f)


def worked_example_points():
    """Point set realising the index example of Section IV-D (eps = 1).

    Point 0 sits at (0, 0), the minimum of both coordinates, so the padded
    grid starts one cell below it and cell column/row c covers coordinates
    [c - 1, c) (up to the slightly wider cell). Points 7 and 36 are the only
    points of cell (1, 3); the other ids are spread over the other ten
    occupied cells.
    """
    ex = golden("worked_index_example.json")
    cells = [tuple(c) for c in ex["occupied_cells_xy"]]
    n = ex["n_points"]
    special = tuple(ex["c6_point_ids"])
    pts = np.zeros((n, 2), dtype=np.float64)
    others = [c for c in cells if c != (1, 3)]
    fracs = [0.2, 0.5, 0.8, 0.35, 0.65]
    k = 0
    for pid in range(n):
        if pid == 0:
            pts[pid] = (0.0, 0.0)
            continue
        if pid in special:
            f = 0.3 if pid == special[0] else 0.7
            pts[pid] = (1 - 1 + f, 3 - 1 + (1 - f))
            continue
        cx, cy = others[k % len(others)]
        fx, fy = fracs[k % 5], fracs[(k // 5) % 5]
        pts[pid] = (cx - 1 + fx, cy - 1 + fy)
        k += 1
    return pts


def sorted_pairs(a) -> np.ndarray:
    """(P, 2) int64 array sorted by (i, j)."""
    a = np.asarray(a, dtype=np.int64).reshape(-1, 2)
    if a.shape[0] == 0:
        return a
    order = np.lexsort((a[:, 1], a[:, 0]))
    return a[order]


def pairs_from_unordered(n: int, unordered) -> np.ndarray:
    out = [(i, i) for i in range(n)]
    for i, j in unordered:
        out.append((i, j))
        out.append((j, i))
    return sorted_pairs(out)


def ordered_square_sum(dv):
    """sum_j dv_j^2 as the pair predicate defines it: each square rounded,
    then added left to right with one rounding per addition (Python floats
    are IEEE doubles and are never contracted)."""
    s = 0.0
    for v in dv:
        s = s + v * v
    return s


def fused_square_sum(dv):
    """sum_j dv_j^2 by fused multiply-adds: F_1 = fl(dv_1^2), then
    F_j = fl(dv_j^2 + F_{j-1}) with one rounding each (exact rational
    arithmetic, then a correctly rounded conversion to double)."""
    from fractions import Fraction
    f = float(Fraction(dv[0]) * Fraction(dv[0]))
    for v in dv[1:]:
        f = float(Fraction(v) * Fraction(v) + Fraction(f))
    return f


def straddling_points(d: int, eps: float, count: int, seed: int):
    """Pairs of points whose squared distance the two sums above decide
    differently against eps^2 (one <= eps^2 < the other), plus points at
    exactly eps along an axis. Base points x lie in [4, 64)^d and their
    partners y within eps, so x - y is exact (Sterbenz) and the rounded
    differences are the chosen ones. Returns (points, number of straddling
    pairs)."""
    g = np.random.default_rng(seed)
    eps2 = eps * eps
    pts = []
    found = 0
    for _ in range(400 * count):
        if found >= count:
            break
        x = g.uniform(4.0, 64.0, size=d)
        v = g.normal(size=d)
        v *= eps / np.linalg.norm(v)
        y = x + v
        # step y_0 by its ulp around the point where the ordered sum crosses
        # eps^2 (vectorised), then test the neighbours of the crossing
        ulp = np.spacing(y[0])
        k = np.arange(-48, 49, dtype=np.float64)
        ys0 = y[0] + k * ulp
        dv = x[None, :] - np.concatenate([ys0[:, None], np.repeat(y[None, 1:], k.size, 0)], axis=1)
        s = np.zeros(k.size)
        for j in range(d):
            s = s + dv[:, j] * dv[:, j]
        inside = s <= eps2
        flips = np.nonzero(inside[1:] != inside[:-1])[0]
        for f in flips[:1]:
            for idx in range(max(0, f - 2), min(k.size, f + 4)):
                row = [float(t) for t in dv[idx]]
                S = ordered_square_sum(row)
                F = fused_square_sum(row)
                if (S <= eps2) != (F <= eps2):
                    yy = y.copy()
                    yy[0] = ys0[idx]
                    pts.extend([x, yy])
                    found += 1
                    break
    # axis-aligned partners at exactly eps and one ulp beyond
    for _ in range(count):
        x = g.uniform(4.0, 64.0, size=d)
        a = int(g.integers(d))
        for off in (eps, np.nextafter(eps, 1.0)):
            y = x.copy()
            y[a] = x[a] + off
            pts.extend([x.copy(), y])
    return np.ascontiguousarray(np.array(pts, dtype=np.float64)), found
