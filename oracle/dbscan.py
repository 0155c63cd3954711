"""Oracle for DBSCAN over the self-join's neighbour table.

TEST INFRASTRUCTURE ONLY: imported by tests/ (and nothing on the product
path). Shares no code with the HIP implementation.

The paper presents the self-join as a building block of DBSCAN (Section I,
citing Ester, Kriegel, Sander and Xu, KDD 1996), and its result batching
comes from an earlier GPU DBSCAN neighbourhood computation (Section V-A).
This module writes that clustering out from its definitions:

  N_eps(p)   the points within eps of p -- here the oracle's pair test
             d2(p, q) <= fl(eps * eps), p itself included (row p of the
             self-join result);
  core       |N_eps(p)| >= min_pts;
  cluster    a maximal set of points that are density-connected; for core
             points this is the connected component of the graph whose
             edges join core points within eps of each other, and every
             non-core point within eps of a core point (a border point)
             belongs to a cluster of one of those core points;
  noise      a point in no cluster (not core, no core point in N_eps).

The definition leaves open which cluster a border point joins when core
points of several clusters are within eps of it. The labels fixed here:
  core point   the smallest index of the core points of its cluster;
  border point the label of the smallest-index core point in N_eps(p);
  noise        -1.

Two spellings: labels_bfs (pure Python, breadth-first search over core
points, small inputs) and labels_components (numpy, with scipy's connected
components as the graph step).
"""
from __future__ import annotations

from collections import deque

import numpy as np

from . import reference


def neighbour_table(points, eps: float):
    """CSR table of the self-join: (row offsets (n + 1,), neighbours), each
    row ascending, from the brute-force oracle."""
    return reference.rows_neighbors(points, eps)


def labels_bfs(off, cols, min_pts: int) -> np.ndarray:
    """Labels from a neighbour table by breadth-first search over core
    points, visiting start points in ascending index (so each cluster is
    first reached at its smallest core index)."""
    off = np.asarray(off, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    n = off.shape[0] - 1
    core = [(off[i + 1] - off[i]) >= min_pts for i in range(n)]
    labels = [-1] * n
    for s in range(n):
        if not core[s] or labels[s] != -1:
            continue
        labels[s] = s
        queue = deque([s])
        while queue:
            p = queue.popleft()
            for q in cols[off[p]:off[p + 1]]:
                q = int(q)
                if core[q] and labels[q] == -1:
                    labels[q] = s
                    queue.append(q)
    for p in range(n):
        if core[p]:
            continue
        best = None
        for q in cols[off[p]:off[p + 1]]:
            q = int(q)
            if core[q] and (best is None or q < best):
                best = q
        if best is not None:
            labels[p] = labels[best]
    return np.asarray(labels, dtype=np.int64)


def labels_components(off, cols, min_pts: int) -> np.ndarray:
    """The same labels with the core graph's connected components computed
    by scipy (a library primitive for the graph step)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components

    off = np.asarray(off, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    n = off.shape[0] - 1
    if n == 0:
        return np.zeros(0, dtype=np.int64)
    core = np.diff(off) >= min_pts
    rows = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    keep = core[rows] & core[cols]
    g = csr_matrix((np.ones(int(keep.sum()), dtype=np.int8), (rows[keep], cols[keep])), shape=(n, n))
    _, comp = connected_components(g, directed=False)
    labels = np.full(n, -1, dtype=np.int64)
    core_idx = np.nonzero(core)[0]
    if core_idx.size:
        # smallest core index of every component that holds a core point
        first = np.full(n, n, dtype=np.int64)
        np.minimum.at(first, comp[core_idx], core_idx)
        labels[core_idx] = first[comp[core_idx]]
    # border points: the label of the smallest-index core point in the row
    cand = np.where(core[cols], cols, n)
    best = np.full(n, n, dtype=np.int64)
    np.minimum.at(best, rows, cand)
    border = (~core) & (best < n)
    labels[border] = labels[best[border]]
    return labels


def dbscan(points, eps: float, min_pts: int) -> np.ndarray:
    """Labels of DBSCAN(points, eps, min_pts) under the conventions above."""
    off, cols = neighbour_table(points, eps)
    return labels_components(off, cols, min_pts)
