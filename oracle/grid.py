"""Oracle for the grid index and its cell searches (numpy, step by step).

TEST INFRASTRUCTURE ONLY (tests, smoke check, benchmark baseline); shares no
code with the HIP implementation.

Follows Section IV-B (grid bounds and cell sizes), IV-C (index components
B, G, A, M), IV-D (adjacent-cell search with the masks) and Section V-B /
Algorithm 2 (unicomp), with these readings where the paper is silent or
assumes exact arithmetic:

* Cell width w = eps * (1 + 2^-16), rounded once more towards +inf. The paper
  uses cells of side exactly eps and assumes eps divides the range; a width
  a little above eps keeps every pair within eps in cells that differ by at
  most one in every dimension even after the rounding of the coordinate
  computation (any w >= eps is exact; only the candidate count grows).
* g_j^min = min_j - w (the paper's one-cell padding); the number of cells
  |g_j| = floor((max_j - g_j^min) / w) + 2; a point's coordinate is
  c_j = clamp(floor((x_j - g_j^min) / w), 0, |g_j| - 1). If prod |g_j|
  reaches 2^63, or some |g_j| reaches 2^31, the width is doubled until
  neither holds (ids fit 63 bits, coordinates 31 bits).
* Linear id (from the worked example of Section IV-D, where 30 = 2 + 7 * 4):
  dimension 0 varies fastest, id = c_0 + |g_0| * (c_1 + |g_1| * (c_2 + ...)).
* B = ascending distinct ids of non-empty cells; G[h] = [start, end) range in
  A (the paper's inclusive [A_h^min, A_h^max]); A = point ids ordered by
  cell id, ties by point id; M_j = sorted distinct occupied c_j.
* unicomp (Algorithm 2): block k is gated on the parity of the source cell's
  own k-th coordinate (the printed algorithm tests the y coordinate for the
  z block, which contradicts the text; the text's reading is used). Block k
  probes the cells whose k-th coordinate differs from the source's, whose
  coordinates below k range over the masked adjacent range, and whose
  coordinates above k equal the source's.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

WIDTH_INFLATION = 2.0 ** -16


def cell_width(eps: float) -> float:
    return float(np.nextafter(np.float64(eps) * np.float64(1.0 + WIDTH_INFLATION), np.inf))


def grid_params(points, eps: float):
    """(gmin[d], w, dims[d]) for the point set."""
    x = np.asarray(points, dtype=np.float64)
    mins = x.min(axis=0)
    maxs = x.max(axis=0)
    w = cell_width(eps)
    while True:
        gmin = mins - w
        cells = np.floor((maxs - gmin) / w) + 2.0
        if np.all(cells < 2.0 ** 31):
            dims = cells.astype(np.int64)
            if math.prod(int(v) for v in dims) < 2 ** 63:
                return gmin, w, dims
        w = w * 2.0


def cell_coords(points, gmin, w, dims) -> np.ndarray:
    x = np.asarray(points, dtype=np.float64)
    c = np.floor((x - gmin) / w).astype(np.int64)
    return np.clip(c, 0, np.asarray(dims, dtype=np.int64) - 1)


def linear_ids(coords, dims) -> np.ndarray:
    """Linearised cell ids (uint64), dimension 0 fastest."""
    c = np.asarray(coords, dtype=np.uint64)
    ids = np.zeros(c.shape[0], dtype=np.uint64)
    stride = 1
    for j in range(c.shape[1]):
        ids += c[:, j] * np.uint64(stride)
        stride *= int(dims[j])
    return ids


def coords_of(lin_id: int, dims):
    out = []
    for g in dims:
        out.append(int(lin_id) % int(g))
        lin_id = int(lin_id) // int(g)
    return tuple(out)


def id_of(coords, dims) -> int:
    lin, stride = 0, 1
    for c, g in zip(coords, dims):
        lin += int(c) * stride
        stride *= int(g)
    return lin


class GridIndex:
    """The index of Section IV-C built with plain numpy operations."""

    def __init__(self, points, eps: float):
        x = np.asarray(points, dtype=np.float64)
        self.n, self.d = x.shape
        self.eps = float(eps)
        self.gmin, self.w, self.dims = grid_params(x, eps)
        self.coords = cell_coords(x, self.gmin, self.w, self.dims)
        self.keys = linear_ids(self.coords, self.dims)
        self.A = np.argsort(self.keys, kind="stable").astype(np.int64)
        sorted_keys = self.keys[self.A]
        self.B, first = np.unique(sorted_keys, return_index=True)
        self.G = np.stack([first, np.append(first[1:], self.n)], axis=1).astype(np.int64)
        self.M = [np.unique(self.coords[:, j]) for j in range(self.d)]

    # -- Section IV-D: masked adjacent ranges and probes ------------------
    def filtered_ranges(self, c):
        """O_j intersected with M_j and the grid, per dimension (sorted lists)."""
        out = []
        for j in range(self.d):
            lo, hi = max(c[j] - 1, 0), min(c[j] + 1, int(self.dims[j]) - 1)
            occ = self.M[j]
            out.append([v for v in range(lo, hi + 1) if v in set(occ.tolist())])
        return out

    def probes_full(self, c):
        """Linear ids probed for a query cell (all masked adjacent cells)."""
        rngs = self.filtered_ranges(c)
        ids = [id_of(t, self.dims) for t in itertools.product(*rngs)]
        return sorted(ids)

    def probes_unicomp(self, c):
        """Linear ids probed by unicomp for a query cell (own cell excluded)."""
        rngs = self.filtered_ranges(c)
        ids = []
        for k in range(self.d):
            if c[k] % 2 == 0:
                continue
            axes = []
            for j in range(self.d):
                if j < k:
                    axes.append(rngs[j])
                elif j == k:
                    axes.append([v for v in rngs[j] if v != c[k]])
                else:
                    axes.append([c[j]])
            ids.extend(id_of(t, self.dims) for t in itertools.product(*axes))
        return sorted(ids)

    def hits(self, probe_ids):
        b = set(int(v) for v in self.B.tolist())
        return [p for p in probe_ids if p in b]

    def cell_points(self, lin_id):
        h = int(np.searchsorted(self.B, np.uint64(lin_id)))
        if h >= len(self.B) or int(self.B[h]) != int(lin_id):
            return []
        s, e = self.G[h]
        return [int(v) for v in self.A[s:e]]

    # -- distance evaluations (the counters the paper's factor ~2 is about) --
    def evaluations(self, unicomp: bool) -> int:
        """Distance evaluations of the search: every point against every
        point of every hit cell (full), or the unicomp subset with the own
        cell counted as one triangle including the diagonal."""
        sizes = {int(k): int(g[1] - g[0]) for k, g in zip(self.B.tolist(), self.G)}
        total = 0
        for key, size in sizes.items():
            c = coords_of(key, self.dims)
            if unicomp:
                total += size * (size + 1) // 2
                probes = self.probes_unicomp(c)
            else:
                probes = self.probes_full(c)
            for p in self.hits(probes):
                if unicomp or p != key:
                    total += size * sizes[p]
                else:
                    total += size * size
        return total


def unicomp_blocks_literal(c, rngs):
    """Algorithm 2 as printed for three dimensions, including its third test
    on the y coordinate (kept only so a test can show that it is wrong)."""
    out = []
    x, y, z = c
    if x % 2 == 1:
        out += [(a, y, z) for a in rngs[0] if a != x]
    if y % 2 == 1:
        out += [(a, b, z) for a in rngs[0] for b in rngs[1] if b != y]
    if y % 2 == 1:
        out += [(a, b, e) for a in rngs[0] for b in rngs[1] for e in rngs[2] if e != z]
    return out


def unicomp_blocks(c, rngs):
    """unicomp probe cells (coordinate tuples) for a source cell with the
    given per-dimension ranges; block k gated on c[k] odd."""
    d = len(c)
    out = []
    for k in range(d):
        if c[k] % 2 == 0:
            continue
        axes = [rngs[j] if j < k else ([v for v in rngs[j] if v != c[k]] if j == k else [c[j]])
                for j in range(d)]
        out += list(itertools.product(*axes))
    return out
