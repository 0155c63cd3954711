"""Pins of the DBSCAN oracle (CPU): hand-worked labels, the two spellings
against each other, and scikit-learn's DBSCAN (an independent library
implementation of Ester et al.'s algorithm) on the parts of the result that
the definition fixes -- the core points, the noise, the partition of the core
points into clusters -- plus the validity of every border label."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import dbscan as odb
from paper_1803_04120_amd import datagen


def _labels(pts, eps, min_pts):
    off, cols = odb.neighbour_table(pts, eps)
    a = odb.labels_bfs(off, cols, min_pts)
    b = odb.labels_components(off, cols, min_pts)
    np.testing.assert_array_equal(a, b)
    return a


def test_hand_example_two_clusters_and_noise(oracle_lib):
    # 1-D, eps = 1, min_pts = 3: points 1 and 11 are core (three points
    # within 1 each, themselves included); 0, 2 and 10, 12 are their border
    # points; 20, 30, 31 have fewer than three points within 1 and no core
    # neighbour: noise.
    pts = np.array([[0.0], [1.0], [2.0], [10.0], [11.0], [12.0], [20.0], [30.0], [31.0]])
    np.testing.assert_array_equal(_labels(pts, 1.0, 3), [1, 1, 1, 4, 4, 4, -1, -1, -1])
    # min_pts = 2: every point with a neighbour is core; 0-1-2 chain into one
    # cluster, 30-31 form a second one, 20 is alone
    np.testing.assert_array_equal(_labels(pts, 1.0, 2), [0, 0, 0, 3, 3, 3, -1, 7, 7])
    # min_pts = 1: every point is core
    np.testing.assert_array_equal(_labels(pts, 1.0, 1), [0, 0, 0, 3, 3, 3, 6, 7, 7])


def test_border_point_between_two_clusters(oracle_lib):
    # eps = 10, min_pts = 4: 8 (index 2) and 28 (index 4) are the only core
    # points and lie 20 apart, so they form two clusters; 18 (index 3) is
    # within 10 of both and takes the label of the smaller index, 2.
    pts = np.array([[0.0], [4.0], [8.0], [18.0], [28.0], [32.0], [36.0]])
    np.testing.assert_array_equal(_labels(pts, 10.0, 4), [2, 2, 2, 2, 4, 4, 4])


def test_empty_and_single(oracle_lib):
    assert _labels(np.zeros((0, 2)), 1.0, 2).shape == (0,)
    np.testing.assert_array_equal(_labels(np.zeros((1, 2)), 1.0, 1), [0])
    np.testing.assert_array_equal(_labels(np.zeros((1, 2)), 1.0, 2), [-1])


def _check_against_sklearn(pts, eps, min_pts):
    from sklearn.cluster import DBSCAN
    lab = _labels(pts, eps, min_pts)
    off, cols = odb.neighbour_table(pts, eps)
    counts = np.diff(off)
    core = counts >= min_pts
    sk = DBSCAN(eps=eps, min_samples=min_pts, algorithm="brute").fit(pts)
    sk_core = np.zeros(pts.shape[0], dtype=bool)
    sk_core[sk.core_sample_indices_] = True
    np.testing.assert_array_equal(core, sk_core)
    # noise is fixed by the definition
    np.testing.assert_array_equal(lab == -1, sk.labels_ == -1)
    # the core points' partition is fixed: same clusters up to renaming
    pairs = {}
    for a, b in zip(lab[core], sk.labels_[core]):
        assert pairs.setdefault(a, b) == b
    assert len(set(pairs.values())) == len(pairs)
    # core labels are the smallest core index of their cluster
    for c in np.unique(lab[core]):
        assert c == np.nonzero(core & (lab == c))[0].min()
    # a border point carries the label of its smallest-index core neighbour,
    # which is one of the clusters sklearn could have chosen
    for p in np.nonzero(~core & (lab != -1))[0]:
        nb = cols[off[p]:off[p + 1]].astype(np.int64)
        nbc = nb[core[nb]]
        assert lab[p] == lab[nbc.min()]
        assert sk.labels_[p] in set(sk.labels_[nbc])
    return lab


@pytest.mark.parametrize("d,n,eps,min_pts", [(2, 3000, 1.2, 5), (2, 3000, 2.5, 12), (3, 2500, 3.0, 6),
                                             (5, 2000, 14.0, 4)])
def test_matches_sklearn_on_clustered_points(oracle_lib, d, n, eps, min_pts):
    pts = datagen.clustered(n, d, seed=300 + d)
    lab = _check_against_sklearn(pts, eps, min_pts)
    assert (lab >= 0).sum() > 0 and (lab == -1).sum() > 0  # clusters and noise both present


def test_planted_mistakes_are_caught(oracle_lib):
    """A core test with '>' instead of '>=', or neighbourhoods without the
    point itself, change the hand example's labels."""
    pts = np.array([[0.0], [1.0], [2.0], [10.0], [11.0], [12.0], [20.0], [30.0], [31.0]])
    off, cols = odb.neighbour_table(pts, 1.0)
    want = [1, 1, 1, 4, 4, 4, -1, -1, -1]
    strict = odb.labels_bfs(off, cols, 4)  # '>' 3 is '>=' 4
    assert not np.array_equal(strict, want)
    keep = cols != np.repeat(np.arange(9), np.diff(off))
    off2 = np.concatenate([[0], np.cumsum(np.bincount(np.repeat(np.arange(9), np.diff(off))[keep], minlength=9))])
    no_self = odb.labels_bfs(off2, cols[keep], 3)
    assert not np.array_equal(no_self, want)
