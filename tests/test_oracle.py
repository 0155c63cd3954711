"""Pins for the brute-force oracle (CPU only).

Each pin is something other than the oracle itself: hand-worked squared
distances (tests/golden/hand_small.json), closed-form lattice counts derived
with integer arithmetic, scipy's KD-tree pair query, and exact invariants of
the definition. A final group plants plausible mistakes in copies of the
oracle and checks that the pins catch them.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import pytest

from oracle import reference as ref
from paper_1803_04120_amd import datagen
from tests._helpers import golden, pairs_from_unordered, sorted_pairs


@pytest.fixture(autouse=True, scope="module")
def _built(oracle_lib):
    return oracle_lib


# ---------------------------------------------------------------- hand pins
@pytest.mark.parametrize("case", golden("hand_small.json")["cases"], ids=lambda c: c["name"])
def test_hand_enumeration(case):
    pts = np.asarray(case["points"], dtype=np.float64)
    expect = pairs_from_unordered(pts.shape[0], case["unordered_within"])
    assert expect.shape[0] == case["P"]
    for impl in (lambda: ref.pairs_python(pts, case["eps"]),
                 lambda: ref.pairs_numpy(pts, case["eps"]),
                 lambda: ref.pairs(pts, case["eps"])):
        got = sorted_pairs(impl())
        np.testing.assert_array_equal(got, expect)
    for key, sq in case.get("hand_sq_dist", {}).items():
        i, j = map(int, key.split("-"))
        assert ref.d2(pts, i, j) == float(sq)


# ------------------------------------------------------- lattice closed forms
def lattice_count(k: int, d: int, eps2_num: int, eps2_den: int = 1) -> int:
    """Ordered pairs of the k^d unit lattice with |v|^2 <= eps2 (a rational),
    counted over offset vectors v: each v occurs prod_j (k - |v_j|) times."""
    r = int(math.isqrt(eps2_num // eps2_den)) + 1
    total = 0
    for v in itertools.product(range(-r, r + 1), repeat=d):
        if sum(c * c for c in v) * eps2_den <= eps2_num:
            total += math.prod(max(k - abs(c), 0) for c in v)
    return total


@pytest.mark.parametrize("d,k", [(2, 9), (3, 6), (4, 4), (5, 3), (6, 3)])
@pytest.mark.parametrize("eps", [1.0, 1.5, 2.0, 2.25])
def test_lattice_closed_form(d, k, eps):
    pts = datagen.lattice(k, d)
    # eps^2 as an exact rational (all eps here are dyadic)
    num, den = (eps * eps).as_integer_ratio()
    expect = lattice_count(k, d, num, den)
    assert int(ref.count_rows(pts, eps).sum()) == expect
    # power-of-two scaling of coordinates and eps leaves the pair set unchanged
    a = ref.pairs(pts, eps)
    b = ref.pairs(pts * 0.25, eps * 0.25)
    np.testing.assert_array_equal(a, b)


def test_lattice_boundary_inclusive():
    # distance exactly 1 is in, sqrt(2) is out, for eps = 1 (Section III uses <=)
    pts = datagen.lattice(3, 2)
    got = set(map(tuple, ref.pairs(pts, 1.0).tolist()))
    centre = 4  # (1, 1)
    assert (centre, 1) in got and (centre, 3) in got and (centre, 5) in got and (centre, 7) in got
    assert (centre, 0) not in got and (centre, 8) not in got


def test_axis_pair_at_exact_eps():
    for eps in (0.1, 0.3, 1.0 / 3.0, 0.04, 0.2, 13.0564, 9.4959):
        for d in (2, 3, 6):
            for axis in range(d):
                pts = np.zeros((3, d))
                pts[1, axis] = eps            # difference is exactly eps
                pts[2, axis] = -eps * 1.0000001
                got = set(map(tuple, ref.pairs(pts, eps).tolist()))
                assert (0, 1) in got and (1, 0) in got
                assert (0, 2) not in got and (2, 0) not in got


# --------------------------------------------------------------- library pin
@pytest.mark.parametrize("d,n,eps", [(2, 4000, 1.2), (3, 3000, 4.0), (4, 2000, 12.0),
                                     (5, 2000, 20.0), (6, 1500, 30.0)])
def test_against_scipy_kdtree(d, n, eps):
    scipy_spatial = pytest.importorskip("scipy.spatial")
    pts = datagen.uniform(n, d, seed=100 + d)
    tree = scipy_spatial.cKDTree(pts)
    und = tree.query_pairs(r=eps, p=2.0, output_type="ndarray")
    expect = pairs_from_unordered(n, und.tolist())
    got = ref.pairs(pts, eps)
    assert got.shape[0] > n  # the radius gives real neighbours
    np.testing.assert_array_equal(got, expect)


# -------------------------------------------------- three spellings agree
@pytest.mark.parametrize("seed", [1, 2, 3])
def test_spellings_agree(seed):
    g = np.random.default_rng(seed)
    n, d = 60, int(g.integers(2, 7))
    pts = g.uniform(0, 10, size=(n, d))
    pts[5] = pts[17]  # a duplicate point
    eps = 3.0
    a = np.asarray(ref.pairs_python(pts, eps), dtype=np.int64)
    b = ref.pairs_numpy(pts, eps)
    c = ref.pairs(pts, eps)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(b, c)
    assert (5, 17) in set(map(tuple, c.tolist()))


# ---------------------------------------------------------------- invariants
def test_invariants_uniform():
    pts = datagen.uniform(3000, 3, seed=7)
    eps = 3.0
    p = ref.pairs(pts, eps)
    s = set(map(tuple, p.tolist()))
    # symmetry and self pairs
    assert all((j, i) in s for i, j in s)
    assert all((i, i) in s for i in range(pts.shape[0]))
    # sorted by (i, j), no duplicates
    np.testing.assert_array_equal(p, sorted_pairs(p))
    assert len(s) == p.shape[0]
    # monotone in eps as set inclusion
    q = set(map(tuple, ref.pairs(pts, 2.5).tolist()))
    assert q <= s and len(q) < len(s)
    # permutation equivariance
    perm = np.random.default_rng(3).permutation(pts.shape[0])
    pp = ref.pairs(pts[perm], eps)
    relabel = sorted_pairs(np.stack([perm[pp[:, 0]], perm[pp[:, 1]]], axis=1))
    np.testing.assert_array_equal(relabel, p)
    # an appended constant coordinate adds exact zeros at the end
    pc = ref.pairs(np.concatenate([pts, np.full((pts.shape[0], 1), 42.0)], axis=1), eps)
    np.testing.assert_array_equal(pc, p)


def test_row_counts_match_pairs_and_sampled_rows():
    pts = datagen.clustered(4000, 2, seed=41)
    eps = 0.5
    p = ref.pairs(pts, eps)
    counts = ref.count_rows(pts, eps)
    np.testing.assert_array_equal(np.bincount(p[:, 0], minlength=4000), counts)
    rows = np.array([0, 17, 3999, 17])
    off, js = ref.rows_neighbors(pts, eps, rows)
    for r, i in enumerate(rows):
        np.testing.assert_array_equal(js[off[r]:off[r + 1]], p[p[:, 0] == i, 1])
    multi = ref.count_rows_multi(pts, [0.25, 0.5, 1.0], rows)
    np.testing.assert_array_equal(multi[:, 1], counts[rows])
    assert np.all(np.diff(multi, axis=1) >= 0)


def test_empty_and_single():
    assert ref.pairs(np.zeros((0, 3)), 1.0).shape == (0, 2)
    np.testing.assert_array_equal(ref.pairs(np.ones((1, 4)), 1e-9), [[0, 0]])


# ------------------------------------------------- planted-mistake checks
def _mutant(kind):
    def pairs(points, eps):
        x = np.asarray(points, dtype=np.float64)
        n, d = x.shape
        eps2 = float(eps) * float(eps)
        out = []
        for i in range(n):
            acc = np.zeros(n)
            dims = range(d - 1) if kind == "drop_last_dim" else range(d)
            for k in dims:
                t = x[i, k] + x[:, k] if kind == "sign" else x[i, k] - x[:, k]
                acc = acc + (np.abs(t) if kind == "abs" else t * t)
            hit = acc < eps2 if kind == "strict" else acc <= eps2
            if kind == "no_self":
                hit[i] = False
            js = np.nonzero(hit)[0]
            if kind == "half" :
                js = js[js >= i]
            out += [(i, int(j)) for j in js]
        return sorted_pairs(out)
    return pairs


@pytest.mark.parametrize("kind", ["strict", "drop_last_dim", "sign", "abs", "no_self", "half"])
def test_pins_catch_planted_mistakes(kind):
    bad = _mutant(kind)
    failures = 0
    for case in golden("hand_small.json")["cases"]:
        pts = np.asarray(case["points"], dtype=np.float64)
        expect = pairs_from_unordered(pts.shape[0], case["unordered_within"])
        got = bad(pts, case["eps"])
        if got.shape != expect.shape or not np.array_equal(got, expect):
            failures += 1
    for d, k in [(2, 5), (3, 4)]:
        pts = datagen.lattice(k, d)
        num, den = (2.25).as_integer_ratio()
        if bad(pts, 1.5).shape[0] != lattice_count(k, d, num, den):
            failures += 1
    assert failures > 0, f"planted mistake {kind!r} went unnoticed"


# ----------------------------------------------------- CPU grid-join baseline
@pytest.mark.parametrize("kind,d,n,eps", [("uniform", 2, 20011, 0.6), ("clustered", 2, 20011, 0.3),
                                          ("clustered", 3, 15013, 0.9), ("uniform", 4, 12007, 9.0),
                                          ("uniform", 6, 7919, 22.0), ("uniform", 1, 5003, 0.05),
                                          ("uniform", 8, 3001, 40.0)])
def test_cpu_grid_join_equals_brute_force(kind, d, n, eps):
    """The host-core grid join (the baseline the GPU is reported against)
    gives the brute force's pairs in the same (i, j) order."""
    pts = datagen.make(kind, n, d, seed=77 + d)
    counts, got = ref.grid_join(pts, eps)
    want = ref.pairs(pts, eps)
    assert np.array_equal(got.astype(np.int64), want)
    assert np.array_equal(counts, ref.count_rows(pts, eps))


def test_cpu_grid_join_lattice_boundaries():
    """Lattice points at spacing 1 with eps exactly 1: every axis neighbour
    sits on a cell boundary and must be found."""
    for d in (1, 2, 3):
        g = np.stack(np.meshgrid(*[np.arange(6, dtype=np.float64)] * d, indexing="ij"), -1).reshape(-1, d)
        _, got = ref.grid_join(g, 1.0)
        assert np.array_equal(got.astype(np.int64), ref.pairs(g, 1.0))
        assert got.shape[0] == g.shape[0] * (1 + 2 * d) - 2 * d * 6 ** (d - 1)


# ------------------------------------------------ distance join of two sets
def test_join_rs_hand_example():
    """R = {(0,0), (3,4)}, S = {(0,1), (3,0), (6,8)}, eps = 5: squared
    distances 1, 9, 100 from the first query and 18, 16, 25 from the second;
    25 sits exactly on eps^2 and is included."""
    R = np.array([[0.0, 0.0], [3.0, 4.0]])
    S = np.array([[0.0, 1.0], [3.0, 0.0], [6.0, 8.0]])
    got = ref.join_rs_numpy(R, S, 5.0)
    np.testing.assert_array_equal(got, np.array([[0, 0], [0, 1], [1, 0], [1, 1], [1, 2]]))


def test_join_rs_special_cases():
    pts = datagen.uniform(700, 3, seed=41)
    # R = S is the self-join (the C brute force, an independent spelling)
    np.testing.assert_array_equal(ref.join_rs_numpy(pts, pts, 6.0), ref.pairs(pts, 6.0))
    # swapping the sets transposes every pair
    R, S = pts[:300], pts[300:]
    a = ref.join_rs_numpy(R, S, 7.0)
    b = ref.join_rs_numpy(S, R, 7.0)
    assert a.shape[0] > 0
    np.testing.assert_array_equal(sorted_pairs(b[:, ::-1]), a)
    # empty sides
    assert ref.join_rs_numpy(R[:0], S, 7.0).shape == (0, 2)
    assert ref.join_rs_numpy(R, S[:0], 7.0).shape == (0, 2)


def test_join_rs_against_scipy_kdtree():
    scipy_spatial = pytest.importorskip("scipy.spatial")
    R = datagen.uniform(1500, 2, seed=42)
    S = datagen.uniform(2500, 2, seed=43)
    want = scipy_spatial.cKDTree(R).query_ball_tree(scipy_spatial.cKDTree(S), r=1.5, p=2.0)
    expect = np.array(sorted((i, j) for i, js in enumerate(want) for j in js), dtype=np.int64).reshape(-1, 2)
    np.testing.assert_array_equal(ref.join_rs_numpy(R, S, 1.5), expect)
