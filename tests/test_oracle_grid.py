"""Pins for the grid-index oracle and the unicomp cell rule (CPU only).

* The worked example of Section IV-D (tests/golden/worked_index_example.json).
* numpy's unique/argsort as the definition of B, G and A.
* The adjacency claim of the cell-width reading: every pair of the brute
  force result lies in cells that differ by at most one in every dimension,
  also for pairs placed exactly at eps and on cell boundaries.
* unicomp (Section V-B, Algorithm 2): every unordered pair of adjacent cells
  is probed exactly once, the printed version (third test on y) is not, and
  the evaluation counts obey U = (T + n) / 2.
"""
from __future__ import annotations

import itertools

import numpy as np
import pytest

from oracle import grid as og
from oracle import reference as ref
from paper_1803_04120_amd import datagen
from tests._helpers import golden, worked_example_points


@pytest.fixture(autouse=True, scope="module")
def _built(oracle_lib):
    return oracle_lib


def test_worked_example_index():
    ex = golden("worked_index_example.json")
    pts = worked_example_points()
    g = og.GridIndex(pts, ex["eps"])
    assert list(g.dims) == ex["dims"]
    assert len(g.B) == ex["n_nonempty"]
    assert int(g.B[5]) == ex["C6_linear_id"]      # C_6, 1-based in the paper
    assert int(g.B[6]) == ex["C7_linear_id"]      # C_7
    c = og.coords_of(ex["query_cell"], g.dims)
    assert list(c) == ex["query_coords"]
    rngs = g.filtered_ranges(c)
    assert rngs == ex["masked_ranges"]
    assert g.probes_full(c) == ex["probes"]
    assert g.hits(g.probes_full(c)) == ex["hits"]
    assert sorted(g.cell_points(ex["C6_linear_id"])) == sorted(ex["c6_point_ids"])
    assert g.cell_points(ex["C6_linear_id"]) == sorted(ex["c6_point_ids"])  # A is stable


@pytest.mark.parametrize("kind,d", [("uniform", 2), ("uniform", 3), ("clustered", 2), ("uniform", 6)])
def test_index_components(kind, d):
    pts = datagen.make(kind, 5000, d, seed=11 + d)
    g = og.GridIndex(pts, 2.0 if d < 6 else 25.0)
    # A is a permutation that orders points by cell id, stable in point id
    assert np.array_equal(np.sort(g.A), np.arange(g.n))
    k = g.keys[g.A]
    assert np.all(np.diff(k.astype(np.float64)) >= 0)
    same = k[1:] == k[:-1]
    assert np.all(g.A[1:][same] > g.A[:-1][same])
    # B are the distinct ids; G partitions [0, n)
    np.testing.assert_array_equal(g.B, np.unique(g.keys))
    assert g.G[0, 0] == 0 and g.G[-1, 1] == g.n
    np.testing.assert_array_equal(g.G[1:, 0], g.G[:-1, 1])
    assert np.all(g.G[:, 1] > g.G[:, 0])
    for h in range(0, len(g.B), max(1, len(g.B) // 50)):
        s, e = g.G[h]
        assert np.all(g.keys[g.A[s:e]] == g.B[h])
    # coordinates stay inside the grid; the minimum sits at or next to the
    # padding cell (rounding of g_min may put it in cell 0, which the clamp
    # and the adjacency argument allow)
    assert np.all(g.coords >= 0) and np.all(g.coords < g.dims)
    assert np.all(g.coords.min(axis=0) <= 1) and np.all(g.coords.max(axis=0) >= g.dims - 3)


@pytest.mark.parametrize("d", [2, 3, 4])
def test_pairs_lie_in_adjacent_cells(d):
    eps = 1.0
    pts = datagen.uniform(1500, d, seed=20 + d) * (8.0 / 100.0)
    # pairs placed exactly at eps along each axis, starting on cell boundaries
    g0 = og.GridIndex(pts, eps)
    extra = []
    for axis in range(d):
        a = g0.gmin + g0.w * 3.0
        b = a.copy()
        b[axis] += eps
        extra += [a, b]
    pts = np.concatenate([pts, np.asarray(extra)], axis=0)
    g = og.GridIndex(pts, eps)
    p = ref.pairs(pts, eps)
    diff = np.abs(g.coords[p[:, 0]] - g.coords[p[:, 1]])
    assert diff.max() <= 1
    n0 = 1500
    for axis in range(d):
        assert (n0 + 2 * axis, n0 + 2 * axis + 1) in set(map(tuple, p.tolist()))


@pytest.mark.parametrize("d", [2, 3, 4, 5, 6])
def test_unicomp_probes_each_adjacent_pair_once(d):
    side = 5 if d <= 4 else 4
    cells = list(itertools.product(range(side), repeat=d))
    full = [list(range(side))] * d
    seen = {}
    for c in cells:
        rngs = [[v for v in range(max(c[j] - 1, 0), min(c[j] + 1, side - 1) + 1)] for j in range(d)]
        for o in og.unicomp_blocks(c, rngs):
            key = (min(c, o), max(c, o))
            seen[key] = seen.get(key, 0) + 1
    adjacent = {(min(a, b), max(a, b)) for a in cells for b in cells
                if a != b and max(abs(x - y) for x, y in zip(a, b)) <= 1}
    assert set(seen) == adjacent
    assert all(v == 1 for v in seen.values())
    del full


def test_printed_algorithm_2_is_not_exactly_once():
    side, wrong = 5, 0
    cells = list(itertools.product(range(side), repeat=3))
    seen = {}
    for c in cells:
        rngs = [[v for v in range(max(c[j] - 1, 0), min(c[j] + 1, side - 1) + 1)] for j in range(3)]
        for o in og.unicomp_blocks_literal(c, rngs):
            key = (min(c, o), max(c, o))
            seen[key] = seen.get(key, 0) + 1
    adjacent = {(min(a, b), max(a, b)) for a in cells for b in cells
                if a != b and max(abs(x - y) for x, y in zip(a, b)) <= 1}
    wrong = sum(1 for k in adjacent if seen.get(k, 0) != 1)
    assert wrong > 0


@pytest.mark.parametrize("kind,d,eps", [("uniform", 2, 3.0), ("clustered", 2, 1.0),
                                        ("uniform", 3, 6.0), ("uniform", 4, 15.0)])
def test_unicomp_evaluation_identity(kind, d, eps):
    pts = datagen.make(kind, 3000, d, seed=5 + d)
    g = og.GridIndex(pts, eps)
    T = g.evaluations(unicomp=False)
    U = g.evaluations(unicomp=True)
    assert 2 * U == T + g.n
    # the full search covers every true pair: T >= P
    assert T >= int(ref.count_rows(pts, eps).sum())
