"""GPU distance join of a query set R with an indexed set S (sj_join_rs)
against the oracle's two-set join (oracle.reference.join_rs_numpy), element
by element."""
from __future__ import annotations

import numpy as np
import pytest

from oracle import reference as ref
from paper_1803_04120_amd import datagen
from tests._helpers import straddling_points

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
    print(f"[rs] {msg}", flush=True)


def assert_same(got, want, what):
    assert got.shape == want.shape, f"{what}: {got.shape[0]} pairs vs oracle {want.shape[0]}"
    if not np.array_equal(got, want):
        bad = np.nonzero(np.any(got != want, axis=1))[0][:5]
        raise AssertionError(f"{what}: first differing rows {bad.tolist()}: "
                             f"got {got[bad].tolist()} want {want[bad].tolist()}")


def rs_pairs(sj, S, R, eps, host_queries=False):
    with sj.Index(torch.from_numpy(S).cuda(), eps) as ix:
        q = R if host_queries else torch.from_numpy(R).cuda()
        return ix.join_rs(q).cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("kind,d,ns,nr,eps", [("uniform", 1, 3001, 2003, 0.05), ("uniform", 2, 20011, 7001, 0.9),
                                              ("clustered", 2, 15013, 9001, 0.3), ("uniform", 3, 12007, 5003, 4.0),
                                              ("clustered", 4, 8009, 4001, 2.5), ("uniform", 6, 4001, 2003, 30.0)])
def test_join_rs_matches_oracle(sj, kind, d, ns, nr, eps):
    _say(f"{kind} d={d} ns={ns} nr={nr} eps={eps}")
    S = datagen.make(kind, ns, d, seed=500 + d)
    # clustered: the same clusters (same seed, other n); uniform: independent
    R = datagen.make(kind, nr, d, seed=500 + d if kind == "clustered" else 600 + d)
    want = ref.join_rs_numpy(R, S, eps)
    assert want.shape[0] > nr // 4  # real neighbours
    assert_same(rs_pairs(sj, S, R, eps), want, f"R x S {kind} d={d}")


@pytest.mark.parametrize("d", [4, 6, 8])
def test_join_rs_straddling_pairs(sj, d):
    """Query/point pairs that a fused multiply-add sum and the predicate's
    left-to-right sum decide differently: the two-set join's fused-square
    filter must hand them to the exact sum."""
    _say(f"straddling pairs d={d}")
    eps = 0.7
    pts, found = straddling_points(d, eps, 40, seed=50 + d)
    assert found == 40
    R = np.ascontiguousarray(pts[0::2])
    S = np.ascontiguousarray(pts[1::2])
    assert_same(rs_pairs(sj, S, R, eps), ref.join_rs_numpy(R, S, eps), f"straddling R x S d={d}")


def test_join_rs_queries_outside_the_index_box(sj):
    """Queries just outside S's bounding box (within eps of its points),
    one cell out, far away, and non-finite-free extremes."""
    _say("queries outside the box")
    S = datagen.uniform(5000, 2, seed=71)
    lo, hi = S.min(axis=0), S.max(axis=0)
    R = np.array([[lo[0] - 0.3, lo[1] + 10.0], [hi[0] + 0.2, hi[1] + 0.2], [lo[0] - 1.5, lo[1]],
                  [1e9, -1e9], [-1e300, 1e300], [50.0, 50.0], [hi[0] + 0.7, 50.0]], dtype=np.float64)
    want = ref.join_rs_numpy(R, S, 0.75)
    assert want.shape[0] > 0
    assert_same(rs_pairs(sj, S, R, 0.75), want, "outside the box")


def test_join_rs_self_and_edges(sj):
    _say("R = S, host queries, empty R, dimension mismatch, capacity")
    S = datagen.uniform(6007, 3, seed=73)
    # R = S gives the self-join
    np.testing.assert_array_equal(rs_pairs(sj, S, S, 3.0), ref.pairs(S, 3.0))
    # queries from host memory
    R = datagen.uniform(1003, 3, seed=74)
    np.testing.assert_array_equal(rs_pairs(sj, S, R, 3.0, host_queries=True), ref.join_rs_numpy(R, S, 3.0))
    with sj.Index(torch.from_numpy(S).cuda(), 3.0) as ix:
        assert ix.join_rs(torch.zeros((0, 3), dtype=torch.float64, device="cuda")).shape[0] == 0
        with pytest.raises(ValueError):
            ix.join_rs(torch.zeros((5, 2), dtype=torch.float64, device="cuda"))
        from paper_1803_04120_amd import _lib
        import ctypes
        q = torch.from_numpy(R).cuda()
        total = ctypes.c_uint64(0)
        buf = torch.empty((4, 2), dtype=torch.int32, device="cuda")
        rc = _lib.load().sj_join_rs(ix._h, ctypes.c_void_p(q.data_ptr()), R.shape[0], 1,
                                    ctypes.c_void_p(buf.data_ptr()), 4, None, ctypes.byref(total))
        assert rc == _lib.SJ_ECAPACITY
        want = ref.join_rs_numpy(R, S, 3.0)
        assert total.value == want.shape[0]
        # caller buffers: too small raises, large enough is filled in one call
        with pytest.raises(ValueError):
            ix.join_rs(q, out=buf)
        big = torch.empty((want.shape[0] + 100, 2), dtype=torch.int32, device="cuda")
        got = ix.join_rs(q, out=big).cpu().numpy().astype(np.int64)
        np.testing.assert_array_equal(got, want)


def test_join_rs_count_then_fill(sj):
    """The two-call form: the count keeps the sorted queries and offsets, the
    fill writes the pairs from them (host queries are copied by the count);
    a fill with no count, or into a buffer below P, is refused."""
    import ctypes
    from paper_1803_04120_amd import _lib
    L = _lib.load()
    _say("two-set join count then fill")
    S = datagen.clustered(8009, 3, seed=75)
    R = datagen.uniform(3001, 3, seed=76)
    want = ref.join_rs_numpy(R, S, 1.5)
    with sj.Index(torch.from_numpy(S).cuda(), 1.5) as ix:
        buf = torch.empty((want.shape[0], 2), dtype=torch.int32, device="cuda")
        assert L.sj_join_rs_fill(ix._h, ctypes.c_void_p(buf.data_ptr()), want.shape[0], None) == _lib.SJ_ESTATE
        for host in (True, False):
            q = R if host else torch.from_numpy(R).cuda()
            ptr = ctypes.c_void_p(q.ctypes.data if host else q.data_ptr())
            total = ctypes.c_uint64(0)
            _lib.check(L.sj_join_rs_count(ix._h, ptr, R.shape[0], 0 if host else 1, None, ctypes.byref(total)))
            assert total.value == want.shape[0]
            assert L.sj_join_rs_fill(ix._h, ctypes.c_void_p(buf.data_ptr()), total.value - 1, None) == _lib.SJ_ECAPACITY
            _lib.check(L.sj_join_rs_fill(ix._h, ctypes.c_void_p(buf.data_ptr()), total.value, None))
            np.testing.assert_array_equal(buf.cpu().numpy().astype(np.int64), want)


@pytest.mark.parametrize("kind,d,ns,nr,eps", [("uniform", 1, 4001, 3001, 0.05), ("uniform", 2, 20011, 6007, 4.0),
                                              ("clustered", 2, 12007, 5003, 2.0), ("clustered", 3, 9001, 4001, 3.0),
                                              ("uniform", 4, 6007, 3001, 14.0), ("uniform", 5, 5003, 2003, 20.0),
                                              ("uniform", 7, 3001, 1009, 40.0), ("uniform", 8, 2003, 1009, 45.0)])
def test_tiled_and_per_query_kernels_agree(sj, kind, d, ns, nr, eps, monkeypatch):
    """The grid-row tiled kernel (default) and the per-query kernel
    (SJ_JOIN_KERNEL=ranges) give the oracle's pairs, with rows from a few
    entries to hundreds (the fused row sort's LDS slot, the wave and block
    row sorts in 1..3-D), 1..8-D, a third of the queries outside S's box."""
    _say(f"tiled vs per-query {kind} d={d} ns={ns} nr={nr} eps={eps}")
    S = datagen.make(kind, ns, d, seed=800 + d)
    R = datagen.make(kind, nr, d, seed=800 + d if kind == "clustered" else 900 + d)
    R[: nr // 3] = R[: nr // 3] * 1.2 - 10.0  # some beyond the box, some far out
    want = ref.join_rs_numpy(R, S, eps)
    assert want.shape[0] > nr
    got_tiled = rs_pairs(sj, S, R, eps)
    monkeypatch.setenv("SJ_JOIN_KERNEL", "ranges")
    got_pq = rs_pairs(sj, S, R, eps)
    monkeypatch.delenv("SJ_JOIN_KERNEL")
    assert_same(got_tiled, want, f"tiled R x S {kind} d={d}")
    assert_same(got_pq, want, f"per-query R x S {kind} d={d}")


def test_join_rs_nonfinite_and_far_queries(sj):
    """Queries with a NaN or infinite coordinate, or more than a cell outside
    S's grid in one dimension, have no neighbours; the rest of the rows are
    unaffected. All queries far away: an empty result."""
    _say("non-finite and far queries")
    S = datagen.uniform(7001, 3, seed=77)
    R = datagen.uniform(2003, 3, seed=78)
    R[5, 1] = np.nan
    R[17, 0] = np.inf
    R[29, 2] = -np.inf
    R[31] = [np.nan, np.nan, np.nan]
    R[40, 2] = 1e12
    want = ref.join_rs_numpy(R, S, 2.5)
    got = rs_pairs(sj, S, R, 2.5)
    assert_same(got, want, "non-finite queries")
    assert not np.isin(got[:, 0], [5, 17, 29, 31, 40]).any()
    far = np.full((100, 3), 1e6)
    assert rs_pairs(sj, S, far, 2.5).shape[0] == 0


def test_join_rs_run_statistics(sj):
    """sj_last_run_stats after a two-set join: the query rows as n, the pairs
    and longest row of the result, S's cells, and the tiled kernel's
    distance evaluations (at least one per pair)."""
    from paper_1803_04120_amd import _lib
    S = datagen.uniform(6007, 3, seed=79)
    R = datagen.uniform(2003, 3, seed=80)
    want = ref.join_rs_numpy(R, S, 4.0)
    with sj.Index(torch.from_numpy(S).cuda(), 4.0) as ix:
        got = ix.join_rs(torch.from_numpy(R).cuda())
        cells = ix.stats()["cells"]
    st = _lib.last_run_stats()
    assert st["n"] == R.shape[0] and st["d"] == 3
    assert st["pairs"] == got.shape[0] == want.shape[0]
    assert st["max_row_pairs"] == int(np.bincount(want[:, 0]).max())
    assert st["cells"] == cells
    assert st["evals"] >= st["pairs"] and st["batches"] == 1
