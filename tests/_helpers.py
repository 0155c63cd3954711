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
