"""GPU parity: the HIP path against the CPU oracle, pair set by pair set.

Every pair set must be bit-exact: same (i, j) pairs in the same (i, j)
order. Inputs are seeded synthetic point sets shaped like the paper's
workloads at sizes the brute force finishes in seconds, spanning many
workgroups and ragged tails, plus the degenerate cases of the method.
"""
from __future__ import annotations

import numpy as np
import pytest

from oracle import grid as og
from oracle import reference as ref
from paper_1803_04120_amd import datagen
from tests._helpers import golden, straddling_points, worked_example_points

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


def gpu_pairs(sj, pts, eps, **kw):
    x = torch.from_numpy(np.ascontiguousarray(pts)).to("cuda")
    out = sj.selfjoin(x, eps, **kw)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.int64)


def assert_same(got, want, what):
    assert got.shape == want.shape, f"{what}: {got.shape[0]} pairs vs oracle {want.shape[0]}"
    if not np.array_equal(got, want):
        bad = np.nonzero(np.any(got != want, axis=1))[0][:5]
        raise AssertionError(f"{what}: first differing rows {bad.tolist()}: "
                             f"got {got[bad].tolist()} want {want[bad].tolist()}")


# ---------------------------------------------------------- small workload
MODES = [dict(unicomp=u, precision=p) for u in (True, False) for p in ("fp64", "fp32_band")]


@pytest.mark.parametrize("mode", MODES, ids=lambda m: f"uni{int(m['unicomp'])}-{m['precision']}")
def test_uniform_2d_10k_eps1(sj, mode):
    """The small 2-D workload: n = 10,000 uniform in [0,100]^2, eps = 1."""
    _say(f"uniform 2d n=10000 eps=1 {mode}")
    pts = datagen.uniform(10000, 2, seed=1)
    want = ref.pairs(pts, 1.0)
    assert_same(gpu_pairs(sj, pts, 1.0, **mode), want, f"2d-10k {mode}")


CASES = [
    ("uniform", 2, 20011, 0.6), ("uniform", 3, 15013, 3.0), ("uniform", 4, 12007, 9.0),
    ("uniform", 5, 9001, 16.0), ("uniform", 6, 7919, 22.0), ("clustered", 2, 20011, 0.3),
    ("clustered", 3, 15013, 0.9), ("uniform", 1, 5003, 0.05), ("uniform", 8, 3001, 40.0),
]


@pytest.mark.parametrize("kind,d,n,eps", CASES)
@pytest.mark.parametrize("mode", MODES, ids=lambda m: f"uni{int(m['unicomp'])}-{m['precision']}")
def test_parity_small(sj, kind, d, n, eps, mode):
    _say(f"{kind} d={d} n={n} eps={eps} {mode}")
    pts = datagen.make(kind, n, d, seed=1000 + d)
    want = ref.pairs(pts, eps)
    assert_same(gpu_pairs(sj, pts, eps, **mode), want, f"{kind}-{d}d {mode}")


@pytest.fixture(params=["tiled", "ranges"])
def join_kernel(request, monkeypatch):
    """Run a test with each refine kernel (grid-row tiled, per-point ranges)."""
    monkeypatch.setenv("SJ_JOIN_KERNEL", request.param)
    return request.param


@pytest.mark.parametrize("kind,d,n,eps", [("uniform", 2, 30011, 0.35), ("clustered", 2, 30011, 0.2),
                                          ("uniform", 3, 20011, 3.5), ("clustered", 3, 15013, 0.7),
                                          ("uniform", 5, 9001, 18.0), ("uniform", 1, 4001, 0.02)])
@pytest.mark.parametrize("mode", MODES, ids=lambda m: f"uni{int(m['unicomp'])}-{m['precision']}")
def test_parity_both_kernels(sj, join_kernel, kind, d, n, eps, mode):
    _say(f"{join_kernel} {kind} d={d} n={n} eps={eps} {mode}")
    pts = datagen.make(kind, n, d, seed=2000 + d)
    want = ref.pairs(pts, eps)
    assert_same(gpu_pairs(sj, pts, eps, **mode), want, f"{join_kernel} {kind}-{d}d {mode}")


@pytest.mark.parametrize("slot", ["16", "24", "32"])
@pytest.mark.parametrize("kind,d,n,eps", [("uniform", 2, 30011, 1.8), ("clustered", 2, 30011, 0.25),
                                          ("uniform", 3, 20011, 6.8)])
def test_fused_fill_slot_sizes(sj, monkeypatch, slot, kind, d, n, eps):
    """The fused fill with each LDS row-slot size: rows that fit are sorted in
    registers, longer ones (up to 64) by the wave, longer still by the row-sort
    kernels; all must give the oracle's pairs."""
    monkeypatch.setenv("SJ_FUSED_NS", slot)
    _say(f"fused slot {slot} {kind} d={d} n={n} eps={eps}")
    pts = datagen.make(kind, n, d, seed=3000 + d)
    want = ref.pairs(pts, eps)
    lens = np.bincount(want[:, 0], minlength=n)
    assert lens.max() > 64 or kind == "uniform"
    assert (lens > int(slot)).any()
    assert_same(gpu_pairs(sj, pts, eps, unicomp=False), want, f"slot {slot} {kind}-{d}d")


@pytest.mark.parametrize("slot", ["16", "24", "32"])
@pytest.mark.parametrize("d", [2, 3])
def test_fused_fill_row_lengths_at_every_boundary(sj, monkeypatch, slot, d):
    """Groups of k coincident points, far apart, give rows of exactly k
    entries: k at and around the slot size (kept in the slot / first entries
    in the slot and the rest spilled), around 64 (sorted by the wave / by the
    row-sort kernels after the slot entries are copied out) and beyond."""
    monkeypatch.setenv("SJ_FUSED_NS", slot)
    ks = [1, 2, 15, 16, 17, 23, 24, 25, 31, 32, 33, 63, 64, 65, 66, 100, 129]
    rng = np.random.default_rng(77 + d)
    groups = []
    for g, k in enumerate(ks):
        centre = np.zeros(d)
        centre[0] = 10.0 * g
        centre[1] = 5.0 * (g % 3)
        groups.append(np.repeat(centre[None, :], k, axis=0))
    pts = np.concatenate(groups)
    pts = pts[rng.permutation(len(pts))]  # rows in random original order
    _say(f"row-length boundaries slot {slot} d={d} n={len(pts)}")
    want = ref.pairs(pts, 0.5)
    lens = np.bincount(want[:, 0], minlength=len(pts))
    assert sorted(set(lens.tolist())) == sorted(set(ks))
    assert_same(gpu_pairs(sj, pts, 0.5, unicomp=False), want, f"row boundaries slot {slot} d={d}")


@pytest.mark.parametrize("fused", ["0", "1"])
@pytest.mark.parametrize("kind,d,n,eps", [("uniform", 4, 12007, 14.0), ("clustered", 5, 9001, 3.0),
                                          ("uniform", 2, 20011, 1.5)])
def test_fused_and_unfused_fill(sj, monkeypatch, fused, kind, d, n, eps):
    """The row sort fused into the fill (default up to 3-D) and run after it
    (default from 4-D) give the same pairs, forced either way."""
    monkeypatch.setenv("SJ_FUSED_SORT", fused)
    _say(f"fused={fused} {kind} d={d} n={n} eps={eps}")
    pts = datagen.make(kind, n, d, seed=4000 + d)
    want = ref.pairs(pts, eps)
    assert_same(gpu_pairs(sj, pts, eps, unicomp=False), want, f"fused={fused} {kind}-{d}d")


# ---------------------------------------------------------------- edges
def test_empty_and_single(sj):
    _say("empty and single point")
    for d in (2, 5):
        out = gpu_pairs(sj, np.zeros((0, d)), 1.0)
        assert out.shape == (0, 2)
        out = gpu_pairs(sj, np.full((1, d), 3.0), 1.0)
        np.testing.assert_array_equal(out, [[0, 0]])


@pytest.mark.parametrize("n,d", [(1, 3), (63, 3), (64, 3), (65, 3), (1024, 3), (1025, 3), (3000, 3), (16385, 3),
                                 (17000, 3), (65, 6), (1025, 6), (3000, 6)])
def test_identical_points_one_cell(sj, n, d):
    """All points equal: one cell, every row has n entries (exercises every
    row-sort size class, including rows longer than a workgroup's LDS; in
    6-D windows of many tiles with hit bits)."""
    _say(f"identical points n={n} d={d}")
    x = torch.full((n, d), 7.25, dtype=torch.float64, device="cuda")
    for uni in (True, False):
        got = sj.selfjoin(x, 0.5, unicomp=uni)
        assert got.shape[0] == n * n
        k = torch.arange(n * n, dtype=torch.int64, device="cuda")
        assert torch.equal(got[:, 0].long(), k // n)
        assert torch.equal(got[:, 1].long(), k % n)
        del got, k


@pytest.mark.parametrize("d", [2, 3, 4])
def test_lattice_boundaries(sj, d):
    """Integer lattice with eps = 1 (distance 1 in, sqrt 2 out) and points on
    cell boundaries; also a power-of-two scaled copy."""
    _say(f"lattice d={d}")
    k = {2: 40, 3: 14, 4: 7}[d]
    pts = datagen.lattice(k, d)
    for scale in (1.0, 0.125):
        want = ref.pairs(pts * scale, 1.0 * scale)
        for uni in (True, False):
            for prec in ("fp64", "fp32_band"):
                got = gpu_pairs(sj, pts * scale, 1.0 * scale, unicomp=uni, precision=prec)
                assert_same(got, want, f"lattice d={d} scale={scale} uni={uni} {prec}")


@pytest.mark.parametrize("d", [3, 4, 5, 6, 7, 8])
def test_fused_filter_straddling_pairs(sj, d):
    """Pairs whose squared distance a fused multiply-add sum and the
    predicate's left-to-right sum put on different sides of eps^2: the FP64
    grid-row kernel's fused-square filter (4-D and up) must send them to the
    exact sum and count them as re-decisions."""
    _say(f"fused-filter straddling pairs d={d}")
    eps = 0.7
    pts, found = straddling_points(d, eps, 40, seed=d)
    assert found == 40
    want = ref.pairs(pts, eps)
    for uni in (True, False):
        got = gpu_pairs(sj, pts, eps, unicomp=uni, precision="fp64")
        assert_same(got, want, f"straddling d={d} uni={uni}")
        if d >= 4:  # the filter's dimensions (below them the exact sum runs directly)
            assert sj.last_run_stats()["band_rechecks"] >= found


@pytest.mark.parametrize("d", [4, 6])
@pytest.mark.parametrize("scale,eps", [(2e-160, 1.5e-160), (1e151, 3.3e150)])
def test_fused_filter_extreme_eps(sj, d, scale, eps):
    """eps^2 below 2^-900 (subnormal squares) or above 2^1000: the fused-square
    filter's band cannot be trusted there, so every candidate goes to the
    exact sum; the pair set must still be the oracle's."""
    _say(f"extreme eps d={d} scale={scale:g} eps={eps:g}")
    g = np.random.default_rng(d)
    pts = g.uniform(0.0, 1.0, size=(1500, d)) * scale
    want = ref.pairs(pts, eps)
    assert 1500 < want.shape[0] < 1500 * 1500  # neither only the self pairs nor every pair
    for uni in (True, False):
        got = gpu_pairs(sj, pts, eps, unicomp=uni, precision="fp64")
        assert_same(got, want, f"extreme eps d={d} scale={scale:g} uni={uni}")
        st = sj.last_run_stats()
        assert st["band_rechecks"] == st["evals"]  # every candidate to the exact sum


@pytest.mark.parametrize("d,uni,prec", [(5, True, "fp64"), (6, False, "fp64"), (8, True, "fp64")])
def test_hit_bits_replay_matches_recompute(sj, d, uni, prec, monkeypatch):
    """From 5-D on the count pass records hit bits and the fill replays
    them: the pair set must be the oracle's with and without them
    (SJ_HIT_BITS=0), and the statistics must say which ran."""
    n, eps = {5: (9001, 16.0), 6: (7919, 22.0), 8: (3001, 40.0)}[d]
    _say(f"hit bits d={d} uni={uni} {prec}")
    pts = datagen.uniform(n, d, seed=3000 + d)
    want = ref.pairs(pts, eps)
    got = gpu_pairs(sj, pts, eps, unicomp=uni, precision=prec)
    assert sj.last_run_stats()["hit_bit_bytes"] > 0
    assert_same(got, want, f"hit bits d={d} uni={uni} {prec}")
    monkeypatch.setenv("SJ_HIT_BITS", "0")
    got0 = gpu_pairs(sj, pts, eps, unicomp=uni, precision=prec)
    assert sj.last_run_stats()["hit_bit_bytes"] == 0
    assert_same(got0, want, f"no hit bits d={d} uni={uni} {prec}")


def test_fp32_band_request_by_dimension(sj):
    """An FP32 pre-test request runs the pre-test up to 5-D (without hit
    bits: its count would spill registers with them) and the faster FP64
    path from 6-D on; precision_used says which, and both give the oracle's
    pairs."""
    for d, n, eps in ((5, 9001, 16.0), (6, 7919, 22.0)):
        _say(f"fp32 band request d={d}")
        pts = datagen.uniform(n, d, seed=3000 + d)
        want = ref.pairs(pts, eps)
        got = gpu_pairs(sj, pts, eps, precision="fp32_band")
        st = sj.last_run_stats()
        assert_same(got, want, f"fp32 band request d={d}")
        if d <= 5:
            assert st["precision_used"] == 1 and st["hit_bit_bytes"] == 0
        else:
            assert st["precision_used"] == 0 and st["hit_bit_bytes"] > 0


def test_pairs_at_exact_eps_and_next_float(sj):
    """Pairs at exactly eps and at nextafter(eps) along every axis must be
    decided as the FP64 definition decides them, in both precisions."""
    _say("exact-eps pairs")
    g = np.random.default_rng(5)
    eps = 0.0909
    rows = []
    for d in (2, 3):
        base = g.uniform(0, 100, size=(400, d))
        for axis in range(d):
            a = base[:100].copy()
            b = a.copy()
            b[:, axis] = a[:, axis] + eps
            c = a.copy()
            c[:, axis] = a[:, axis] + np.nextafter(eps, 1.0)
            rows.append((d, np.concatenate([base, b, c], axis=0)))
    for d, pts in rows:
        want = ref.pairs(pts, eps)
        for prec in ("fp64", "fp32_band"):
            got = gpu_pairs(sj, pts, eps, precision=prec)
            assert_same(got, want, f"exact-eps d={d} {prec}")


@pytest.mark.parametrize("d", [3, 6])
def test_eps_covers_everything(sj, d):
    """eps beyond the extent: every pair, every candidate a hit (in 6-D every
    recorded hit bit set)."""
    _say(f"eps larger than the data extent d={d}")
    pts = datagen.uniform(2500, d, seed=8)
    got = gpu_pairs(sj, pts, 1000.0)
    assert got.shape[0] == 2500 * 2500
    k = np.arange(2500 * 2500, dtype=np.int64)
    assert np.array_equal(got[:, 0], k // 2500) and np.array_equal(got[:, 1], k % 2500)


def test_duplicates_and_far_outlier(sj):
    _say("duplicates and outlier")
    pts = datagen.uniform(5000, 2, seed=9)
    pts[100:200] = pts[0]
    pts[4999] = (1e6, -1e6)
    want = ref.pairs(pts, 0.7)
    assert_same(gpu_pairs(sj, pts, 0.7), want, "duplicates+outlier")


def test_invalid_inputs(sj):
    _say("invalid inputs")
    pts = datagen.uniform(100, 2, seed=1)
    pts[7, 1] = np.nan
    with pytest.raises(sj.SjError, match="NaN"):
        sj.selfjoin(torch.from_numpy(pts).cuda(), 1.0)
    ok = torch.from_numpy(datagen.uniform(100, 2, seed=1)).cuda()
    ix = sj.Index(ok, 1.0)
    with pytest.raises(RuntimeError):
        ix.fill()
    P = ix.count()
    too_small = torch.empty((max(P - 1, 1), 2), dtype=torch.int32, device="cuda")
    from paper_1803_04120_amd import _lib
    import ctypes
    rc = _lib.load().sj_join_fill(ix._h, ctypes.c_void_p(too_small.data_ptr()), P - 1, None)
    assert rc == _lib.SJ_ECAPACITY
    ix.close()


@pytest.mark.parametrize("d", range(1, 9))
def test_bbox_every_dimension_count(sj, d):
    # The bounding-box pass is compiled per dimension count, and with more
    # than four grid strides of points (1024 workgroups x 256) each thread
    # loads four points before folding them in: 1.1M points exercise both
    # that loop and the remainder loop. Exact min and the cell counts that
    # follow from the max; then a non-finite value in the last coordinate,
    # once in each loop, must be rejected.
    n = 1_100_000
    pts = datagen.uniform(n, d, seed=40 + d)
    _say(f"bbox d={d} n={n}")
    x = torch.from_numpy(pts).cuda()
    with sj.Index(x, 3.0) as ix:
        grid = ix.export(sj._lib.SJ_EXPORT_GRID)
        lo, hi = pts.min(axis=0), pts.max(axis=0)
        w = grid[16]
        # the grid of Section IV-B as the index lays it out: one spare cell
        # below the minimum, floor((max - g_min) / w) + 2 cells per dimension
        gmin = lo - w
        np.testing.assert_array_equal(grid[:d], gmin)
        np.testing.assert_array_equal(grid[8:8 + d].astype(np.int64), (np.floor((hi - gmin) / w) + 2).astype(np.int64))
    for pos, bad in ((1_050_000, np.nan), (1_099_999, np.inf), (1_050_000, -np.inf)):
        y = pts.copy()
        y[pos, d - 1] = bad
        with pytest.raises(sj.SjError, match="NaN"):
            sj.selfjoin(torch.from_numpy(y).cuda(), 3.0)


# --------------------------------------------------------- index parity
@pytest.mark.parametrize("kind,d,n,eps", [("uniform", 2, 30011, 0.5), ("clustered", 3, 20011, 0.8),
                                          ("uniform", 6, 10007, 25.0), ("uniform", 2, 5000, 1e-3),
                                          ("uniform", 1, 20011, 0.01), ("clustered", 4, 12007, 2.0),
                                          ("uniform", 5, 9001, 20.0), ("uniform", 7, 6007, 40.0),
                                          ("clustered", 8, 5003, 6.0)])
def test_index_matches_grid_oracle(sj, kind, d, n, eps):
    _say(f"index {kind} d={d} n={n} eps={eps}")
    pts = datagen.make(kind, n, d, seed=77)
    g = og.GridIndex(pts, eps)
    with sj.Index(torch.from_numpy(pts).cuda(), eps) as ix:
        grid = ix.export(sj._lib.SJ_EXPORT_GRID)
        np.testing.assert_array_equal(grid[:d], g.gmin)
        np.testing.assert_array_equal(grid[8:8 + d].astype(np.int64), g.dims)
        assert grid[16] == g.w
        np.testing.assert_array_equal(ix.export(sj._lib.SJ_EXPORT_CELL_IDS), g.B)
        # A: the paper's order by cell; inside a cell (an order the paper
        # leaves open) by the dimension-0 sub-cell floor(t * s), then by id
        s_sub = int(grid[17])
        assert s_sub in (1, 2, 4, 8)
        t = (pts[:, 0] - g.gmin[0]) / g.w
        sub = np.clip(np.floor(t * s_sub), 0, s_sub * g.dims[0] - 1).astype(np.int64) % s_sub
        key2 = g.keys.astype(np.int64) * s_sub + sub
        a_want = np.argsort(key2, kind="stable")
        a_got = ix.export(sj._lib.SJ_EXPORT_PERM).astype(np.int64)
        np.testing.assert_array_equal(a_got, a_want)
        np.testing.assert_array_equal(np.sort(g.keys[a_got]), g.keys[g.A])  # same cells as the paper's A
        starts = ix.export(sj._lib.SJ_EXPORT_CELL_START).astype(np.int64)
        np.testing.assert_array_equal(starts[:-1], g.G[:, 0])
        assert starts[-1] == n
        st = ix.stats()
        assert st["cells"] == len(g.B)
        assert st["max_cell_points"] == int((g.G[:, 1] - g.G[:, 0]).max())
        masks = ix.export(sj._lib.SJ_EXPORT_MASKS)
        off = 0
        for j in range(d):
            words = (int(g.dims[j]) + 31) // 32
            bits = np.unpackbits(masks[off:off + words].view(np.uint8), bitorder="little")
            np.testing.assert_array_equal(np.nonzero(bits)[0], g.M[j])
            off += words


def _cells_of_ranges(ix, sj, B, starts, cell):
    roff = ix.export(sj._lib.SJ_EXPORT_RANGE_OFF)
    rng = ix.export(sj._lib.SJ_EXPORT_RANGES).reshape(-1, 2)
    cells = []
    for s, e in rng[roff[cell]:roff[cell + 1]]:
        first = int(np.searchsorted(starts, s, side="right") - 1)
        last = int(np.searchsorted(starts, e, side="left") - 1)
        cells += [int(B[h]) for h in range(first, last + 1)]
    return sorted(cells)


def test_worked_example_search(sj):
    """Section IV-D's example: query cell 30 finds the occupied cells 22, 30
    and 36 among the masked probes; unicomp probes the subset of those."""
    _say("worked example")
    ex = golden("worked_index_example.json")
    pts = worked_example_points()
    g = og.GridIndex(pts, ex["eps"])
    with sj.Index(torch.from_numpy(pts).cuda(), ex["eps"]) as ix:
        B = ix.export(sj._lib.SJ_EXPORT_CELL_IDS)
        starts = ix.export(sj._lib.SJ_EXPORT_CELL_START)
        assert len(B) == ex["n_nonempty"]
        assert int(B[5]) == ex["C6_linear_id"] and int(B[6]) == ex["C7_linear_id"]
        perm = ix.export(sj._lib.SJ_EXPORT_PERM)
        assert sorted(perm[starts[5]:starts[6]].tolist()) == sorted(ex["c6_point_ids"])
        ix.search(unicomp=False)
        h = int(np.searchsorted(B, ex["query_cell"]))
        assert _cells_of_ranges(ix, sj, B, starts, h) == ex["hits"]
        for cell in range(len(B)):
            c = og.coords_of(int(B[cell]), g.dims)
            assert _cells_of_ranges(ix, sj, B, starts, cell) == g.hits(g.probes_full(c))
        ix.search(unicomp=True)
        for cell in range(len(B)):
            c = og.coords_of(int(B[cell]), g.dims)
            assert _cells_of_ranges(ix, sj, B, starts, cell) == g.hits(g.probes_unicomp(c))


@pytest.mark.parametrize("kind,d,eps", [("uniform", 2, 1.5), ("clustered", 2, 0.5),
                                        ("uniform", 3, 6.0), ("uniform", 5, 20.0)])
def test_unicomp_evaluation_counts(sj, join_kernel, kind, d, eps, monkeypatch):
    """Distance evaluations: full search = the oracle's T, unicomp = (T+n)/2
    (the per-point kernel, and the tiled kernel without dimension-0
    sub-cells). With sub-cells (the default, s of them per cell) the tiled
    kernel evaluates, for each point, the points of its adjacent cells whose
    sub-cell differs from its own by at most s (T_s, counted here by brute
    force over all ordered pairs), and unicomp (T_s + n) / 2."""
    _say(f"evaluation counts {kind} d={d}")
    n = 6000
    pts = datagen.make(kind, n, d, seed=3)
    g = og.GridIndex(pts, eps)
    T = g.evaluations(unicomp=False)
    for shift in ((None, 0) if join_kernel == "tiled" else (None,)):
        if shift is None:
            monkeypatch.delenv("SJ_SUBCELL_SHIFT", raising=False)
        else:
            monkeypatch.setenv("SJ_SUBCELL_SHIFT", str(shift))
        with sj.Index(torch.from_numpy(pts).cuda(), eps) as ix:
            s_sub = int(ix.export(sj._lib.SJ_EXPORT_GRID)[17])
            want = T
            if join_kernel == "tiled" and s_sub > 1:
                sub = np.clip(np.floor((pts[:, 0] - g.gmin[0]) / g.w * s_sub), 0,
                              s_sub * g.dims[0] - 1).astype(np.int64)
                cc = g.coords.astype(np.int64)
                want = 0
                for a in range(0, n, 500):
                    adj = np.all(np.abs(cc[a:a + 500, None, :] - cc[None, :, :]) <= 1, axis=2)
                    want += int(np.count_nonzero(adj & (np.abs(sub[a:a + 500, None] - sub[None, :]) <= s_sub)))
                assert want < T
            ix.count(unicomp=False)
            assert ix.stats()["evals"] == want
            ix.count(unicomp=True)
            assert ix.stats()["evals"] == (want + n) // 2
    monkeypatch.delenv("SJ_SUBCELL_SHIFT", raising=False)


# ---------------------------------------------------------------- batching
@pytest.mark.parametrize("cap,minb", [(0, 3), (5000, 1), (20000, 3), (777, 1)])
@pytest.mark.parametrize("uni,fill", [(True, None), (True, "whole"), (True, "runs"), (False, None)])
def test_batches_partition_the_result(sj, cap, minb, uni, fill, monkeypatch):
    """Runs partition the result, each sorted by (i, j), whether each run
    fills its own rows (SJ_BATCH_FILL=runs) or one unicomp fill of every row
    precedes the runs' sorts (whole)."""
    _say(f"batches cap={cap} min={minb} uni={uni} fill={fill}")
    if fill:
        monkeypatch.setenv("SJ_BATCH_FILL", fill)
    pts = datagen.clustered(12000, 2, seed=21)
    eps = 0.4
    want = ref.pairs(pts, eps)
    with sj.Index(torch.from_numpy(pts).cuda(), eps) as ix:
        P = ix.count(unicomp=uni)
        maxrow = ix.stats()["max_row_pairs"]
        if cap and cap < maxrow:
            with pytest.raises(sj.SjError, match="SJ_ECAPACITY"):
                ix.join_batched(unicomp=uni, batch_capacity_pairs=cap, min_batches=minb)
            return
        got, info = ix.join_batched(unicomp=uni, batch_capacity_pairs=cap, min_batches=minb)
        assert P == want.shape[0]
        assert len(info) >= minb
        assert all(npairs <= (cap or P) for _, _, _, npairs in info)
        # the runs cover the cell-ordered positions [0, n) in order
        assert info[0][1] == 0 and info[-1][2] == 12000
        assert all(info[k][2] == info[k + 1][1] for k in range(len(info) - 1))
        g = got.cpu().numpy().astype(np.int64)
        perm = ix.export(sj._lib.SJ_EXPORT_PERM).astype(np.int64)
        at = 0
        for _, r0, r1, npairs in info:
            run = g[at:at + npairs]
            at += npairs
            key = run[:, 0] * 12000 + run[:, 1]
            assert np.all(np.diff(key) > 0), "a run is not sorted by (i, j)"
            assert set(np.unique(run[:, 0])) <= set(perm[r0:r1].tolist())
        assert_same(g[np.lexsort((g[:, 1], g[:, 0]))], want, f"batched cap={cap}")


@pytest.mark.parametrize("d,eps", [(4, 14.0), (5, 20.0)])
def test_batches_whole_fill_in_high_d(sj, d, eps):
    """From 4-D on the batched join fills every row once with unicomp and
    sorts each run out of that table (the default when it fits in memory):
    the runs, merged, are the oracle's pairs."""
    _say(f"batches whole fill d={d}")
    pts = datagen.uniform(7001, d, seed=22 + d)
    want = ref.pairs(pts, eps)
    with sj.Index(torch.from_numpy(pts).cuda(), eps) as ix:
        got, info = ix.join_batched(unicomp=True, batch_capacity_pairs=max(want.shape[0] // 5, 4096), min_batches=3)
        assert ix.stats()["fill_unicomp"] == 1 and len(info) >= 3
    g = got.cpu().numpy().astype(np.int64)
    assert_same(g[np.lexsort((g[:, 1], g[:, 0]))], want, f"batched whole fill d={d}")


def test_convenience_host_and_device_output(sj):
    _say("sj_selfjoin host/device")
    import ctypes
    from paper_1803_04120_amd import _lib
    L = _lib.load()
    pts = datagen.uniform(8000, 3, seed=4)
    eps = 2.5
    want = ref.pairs(pts, eps)
    for on_dev, cap, minb in ((1, 0, 1), (0, 0, 3), (0, 4000, 1), (1, 3000, 2)):
        o = _lib.opts(True, "fp64", cap, minb)
        out = ctypes.c_void_p()
        npairs = ctypes.c_uint64()
        _lib.check(L.sj_selfjoin(ctypes.c_void_p(pts.ctypes.data), 8000, 3, eps, ctypes.byref(o), 0,
                                 on_dev, None, ctypes.byref(out), ctypes.byref(npairs)))
        P = npairs.value
        host = np.zeros(2 * P, dtype=np.uint32)
        if on_dev:
            hip = ctypes.CDLL("libamdhip64.so")
            hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
            assert hip.hipMemcpy(ctypes.c_void_p(host.ctypes.data), out, 8 * P, 2) == 0
        else:
            ctypes.memmove(host.ctypes.data, out.value, 8 * P)
        L.sj_free(out)
        assert_same(host.reshape(-1, 2).astype(np.int64), want, f"sj_selfjoin dev={on_dev} cap={cap}")


@pytest.mark.parametrize("mode", ["full", "unicomp"])
@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6])
def test_both_fill_kernels_in_every_dimension(sj, mode, d, monkeypatch):
    """The fill pass either evaluates all adjacent cells (each point writes
    its own row) or the unicomp subset (mirrored pairs placed by atomics);
    the library picks by the pairs-to-evaluations ratio, SJ_FILL_MODE forces
    one. Both must give the oracle's pairs in every dimension, and the
    statistics must say which one ran."""
    monkeypatch.setenv("SJ_FILL_MODE", mode)
    n = 9001
    pts = datagen.clustered(n, d, seed=1300 + d)
    eps = {1: 0.01, 2: 0.3, 3: 1.2, 4: 3.0, 5: 5.0, 6: 7.0}[d]
    _say(f"fill mode {mode} d={d}")
    want = ref.pairs(pts, eps)
    x = torch.from_numpy(pts).cuda()
    for prec in ("fp64", "fp32_band"):
        with sj.Index(x, eps) as ix:
            ix.count(unicomp=True, precision=prec)
            got = ix.fill().cpu().numpy().astype(np.int64)
            st = ix.stats()
        assert st["fill_unicomp"] == (1 if mode == "unicomp" else 0)
        assert_same(got, want, f"fill {mode} d={d} {prec}")
