"""CSR neighbour-table output, unsorted rows, and the DBSCAN consumer on the
GPU, against the oracle.

- The CSR fill must hold exactly the pair form's rows (offsets and column
  ids), sorted or -- with sort_output off -- as the same sets per row.
- DBSCAN labels must equal the oracle's (oracle/dbscan.py, pinned against
  hand-worked cases and scikit-learn) exactly: core points carry the
  smallest core index of their cluster, border points the label of their
  smallest-index core neighbour, noise -1. The oracle's neighbour tables come
  from the brute force or, at larger sizes, the host-core grid join -- never
  from the GPU.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import dbscan as odb
from oracle import reference as ref
from paper_1803_04120_amd import datagen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def sj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1803_04120_amd as m
    m._lib.load()
    return m


def _say(msg):
    print(f"[case] {msg}", flush=True)


CASES = [("uniform", 2, 20011, 0.9), ("clustered", 2, 15013, 0.25), ("clustered", 3, 12007, 1.1),
         ("uniform", 4, 9001, 14.0), ("clustered", 5, 8009, 4.0), ("uniform", 6, 6007, 30.0)]


@pytest.mark.parametrize("kind,d,n,eps", CASES)
@pytest.mark.parametrize("unicomp", [True, False])
def test_csr_equals_pairs(sj, kind, d, n, eps, unicomp):
    pts = datagen.make(kind, n, d, seed=500 + d)
    x = torch.from_numpy(pts).cuda()
    _say(f"csr {kind} d={d} n={n} eps={eps} unicomp={unicomp}")
    with sj.Index(x, eps) as ix:
        P = ix.count(unicomp=unicomp)
        pairs = ix.fill().cpu().numpy().astype(np.int64)
        off_pairs = ix.export(sj._lib.SJ_EXPORT_ROW_OFFSETS).astype(np.int64)
        ix.count(unicomp=unicomp)
        row_off, cols = ix.fill_csr()
    row_off = row_off.cpu().numpy()
    cols = cols.cpu().numpy().astype(np.int64)
    assert cols.shape[0] == P == pairs.shape[0]
    np.testing.assert_array_equal(row_off, off_pairs)
    np.testing.assert_array_equal(cols, pairs[:, 1])
    want = ref.pairs(pts, eps)
    np.testing.assert_array_equal(pairs, want)


def _row_sorted(off, js):
    out = js.copy()
    for i in range(off.shape[0] - 1):
        out[off[i]:off[i + 1]] = np.sort(out[off[i]:off[i + 1]])
    return out


@pytest.mark.parametrize("kind,d,n,eps", CASES + [("clustered", 3, 30011, 2.5)])
def test_unsorted_rows_hold_the_same_sets(sj, kind, d, n, eps):
    """sort_output off: the rows keep their offsets and hold the same j, in
    any order (pairs and CSR forms)."""
    pts = datagen.make(kind, n, d, seed=600 + d)
    x = torch.from_numpy(pts).cuda()
    _say(f"unsorted {kind} d={d} n={n} eps={eps}")
    with sj.Index(x, eps) as ix:
        ix.count(sort_output=True)
        want = ix.fill().cpu().numpy().astype(np.int64)
        off = ix.export(sj._lib.SJ_EXPORT_ROW_OFFSETS).astype(np.int64)
        ix.count(sort_output=False)
        got = ix.fill().cpu().numpy().astype(np.int64)
        ix.count(sort_output=False)
        row_off, cols = ix.fill_csr()
    np.testing.assert_array_equal(got[:, 0], want[:, 0])
    np.testing.assert_array_equal(_row_sorted(off, got[:, 1]), want[:, 1])
    np.testing.assert_array_equal(row_off.cpu().numpy(), off)
    np.testing.assert_array_equal(_row_sorted(off, cols.cpu().numpy().astype(np.int64)), want[:, 1])


DB_CASES = [("clustered", 2, 20011, 0.3, 8), ("clustered", 2, 20011, 0.6, 40), ("clustered", 3, 15013, 1.2, 10),
            ("uniform", 2, 20011, 0.9, 4), ("clustered", 4, 10007, 4.0, 6), ("clustered", 6, 8009, 12.0, 5)]


@pytest.mark.parametrize("kind,d,n,eps,min_pts", DB_CASES)
def test_dbscan_matches_oracle(sj, kind, d, n, eps, min_pts):
    pts = datagen.make(kind, n, d, seed=700 + d)
    _say(f"dbscan {kind} d={d} n={n} eps={eps} min_pts={min_pts}")
    want = odb.dbscan(pts, eps, min_pts)
    x = torch.from_numpy(pts).cuda()
    labels, nc = sj.dbscan(x, eps, min_pts)
    got = labels.cpu().numpy().astype(np.int64)
    np.testing.assert_array_equal(got, want)
    assert nc == len(np.unique(want[want >= 0]))
    assert nc > 0
    # the same from an explicit CSR table
    with sj.Index(x, eps) as ix:
        ix.count(sort_output=False)
        row_off, cols = ix.fill_csr()
    labels2, nc2 = sj.dbscan_csr(row_off, cols, min_pts)
    np.testing.assert_array_equal(labels2.cpu().numpy().astype(np.int64), want)
    assert nc2 == nc


def test_dbscan_edges(sj):
    _say("dbscan edges")
    labels, nc = sj.dbscan(torch.zeros((0, 2), dtype=torch.float64, device="cuda"), 1.0, 3)
    assert labels.shape == (0,) and nc == 0
    pts = datagen.uniform(5000, 2, seed=3)
    x = torch.from_numpy(pts).cuda()
    # min_pts = 1: every point is core
    labels, nc = sj.dbscan(x, 0.5, 1)
    np.testing.assert_array_equal(labels.cpu().numpy(), odb.dbscan(pts, 0.5, 1))
    # eps tiny: every point alone -> all noise at min_pts 2
    labels, nc = sj.dbscan(x, 1e-9, 2)
    assert nc == 0 and bool((labels == -1).all())
    # identical points: one cluster labelled 0
    labels, nc = sj.dbscan(torch.full((3000, 3), 2.5, dtype=torch.float64, device="cuda"), 0.1, 10)
    assert nc == 1 and bool((labels == 0).all())
    with pytest.raises(sj.SjError):
        sj.dbscan(x, 0.5, 0)


def test_dbscan_clustered_500k_vs_cpu_grid_join(sj):
    """Half a million clustered 3-D points: the oracle's labels from the
    host-core grid join's neighbour table."""
    n, d, eps, min_pts = 500_000, 3, 0.3, 20
    pts = datagen.clustered(n, d, seed=743)
    _say(f"dbscan clustered 3d n={n}")
    counts, pairs = ref.grid_join(pts, eps)
    off = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    want = odb.labels_components(off, pairs[:, 1].astype(np.int64), min_pts)
    del pairs
    labels, nc = sj.dbscan(torch.from_numpy(pts).cuda(), eps, min_pts)
    np.testing.assert_array_equal(labels.cpu().numpy().astype(np.int64), want)
    assert nc == len(np.unique(want[want >= 0]))
