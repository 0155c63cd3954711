"""GPU brute-force join (Section VI-B's all-pairs comparison) against the
oracle, and against the grid join where the grid degenerates.

The brute force evaluates every ordered pair with the same binary64 pair
test, so its result must equal the oracle's pair set exactly, row order
included, at every size: ragged tails of the 256-lane query blocks and
256-point candidate tiles, every dimension count 1..8, the degenerate inputs
(empty, one point, all points equal, non-finite coordinates, pairs at
exactly eps), and host or device input.
"""
from __future__ import annotations

import numpy as np
import pytest

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


def _brute(sj, pts, eps, on_device=True):
    src = torch.from_numpy(np.ascontiguousarray(pts)).cuda() if on_device else np.ascontiguousarray(pts)
    out = sj.bruteforce(src, eps)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.int64)


def _same(got, want, what):
    assert got.shape == want.shape, f"{what}: {got.shape[0]} pairs vs oracle {want.shape[0]}"
    if not np.array_equal(got, want):
        bad = np.nonzero(np.any(got != want, axis=1))[0][:5]
        raise AssertionError(f"{what}: first differing rows {bad.tolist()}: got {got[bad].tolist()} "
                             f"want {want[bad].tolist()}")


def test_uniform_2d_10k_eps1(sj):
    """The small 2-D workload (10,000 uniform points in [0,100]^2, eps 1)."""
    _say("brute uniform 2d n=10000 eps=1")
    pts = datagen.uniform(10000, 2, seed=1)
    _same(_brute(sj, pts, 1.0), ref.pairs(pts, 1.0), "brute 10k 2-D")
    st = sj.last_run_stats()
    assert st["evals"] == 10000 * 10000 and st["d"] == 2


@pytest.mark.parametrize("d", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("kind", ["uniform", "clustered"])
def test_every_dimension(sj, d, kind):
    n = 3001
    pts = datagen.make(kind, n, d, seed=100 + d)
    eps = {1: 0.05, 2: 2.0, 3: 6.0, 4: 12.0, 5: 18.0, 6: 24.0, 7: 30.0, 8: 36.0}[d]
    _say(f"brute {kind} d={d} n={n} eps={eps}")
    want = ref.pairs(pts, eps)
    assert want.shape[0] > n  # some pairs beyond the self pairs
    _same(_brute(sj, pts, eps), want, f"brute {kind} d={d}")


@pytest.mark.parametrize("n", [1, 2, 63, 255, 256, 257, 511, 512, 513, 1023, 1024, 1025, 4097])
@pytest.mark.parametrize("d", [2, 6])
def test_ragged_sizes(sj, n, d):
    """Sizes around the candidate tile (256) and the query block (1024 rows
    in 2-D, 512 in 6-D)."""
    pts = datagen.uniform(n, d, seed=n * 10 + d)
    eps = 6.0 if d == 2 else 30.0
    _say(f"brute ragged n={n} d={d}")
    _same(_brute(sj, pts, eps), ref.pairs(pts, eps), f"brute n={n} d={d}")


def test_empty(sj):
    _say("brute empty")
    got = sj.bruteforce(torch.zeros((0, 3), dtype=torch.float64, device="cuda"), 1.0)
    assert got.shape == (0, 2)


def test_all_points_equal_and_eps_covering_everything(sj):
    _say("brute identical points / eps covering all")
    pts = np.full((1500, 3), 7.25)
    n = pts.shape[0]
    got = _brute(sj, pts, 1e-9)
    assert got.shape[0] == n * n
    _same(got, ref.pairs(pts, 1e-9), "identical points")
    pts = datagen.uniform(1300, 4, seed=9)
    got = _brute(sj, pts, 1000.0)
    assert got.shape[0] == 1300 * 1300
    _same(got, ref.pairs(pts, 1000.0), "eps covering all")


def test_pairs_at_exactly_eps(sj):
    """Integer lattice with eps = 1: axis neighbours at distance exactly 1
    are pairs, diagonal ones (sqrt 2) are not; and eps just below 1."""
    g = np.arange(12, dtype=np.float64)
    pts = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
    for eps in (1.0, np.nextafter(1.0, 0.0), np.sqrt(2.0)):
        _say(f"brute lattice eps={eps!r}")
        want = np.array(ref.pairs_python(pts, eps), dtype=np.int64).reshape(-1, 2)
        _same(_brute(sj, pts, eps), want, f"lattice eps={eps!r}")


def test_non_finite_points_pair_with_nothing(sj):
    """A NaN or infinite coordinate gives a NaN or infinite distance to every
    point, itself included: such points appear in no pair (the definition,
    applied literally; the numpy oracle computes the same)."""
    pts = datagen.uniform(700, 3, seed=4)
    pts[3, 1] = np.nan
    pts[10, 0] = np.inf
    pts[11, 0] = np.inf
    pts[12, 2] = -np.inf
    _say("brute non-finite points")
    with np.errstate(invalid="ignore"):
        want = ref.pairs_numpy(pts, 9.0)
    got = _brute(sj, pts, 9.0)
    _same(got, want, "non-finite")
    assert not np.isin([3, 10, 11, 12], got[:, 0]).any()


def test_host_input_and_caller_buffer(sj):
    pts = datagen.clustered(6000, 3, seed=12)
    eps = 1.5
    _say("brute host input / caller buffer")
    want = ref.pairs(pts, eps)
    _same(_brute(sj, pts, eps, on_device=False), want, "host input")
    buf = torch.empty((want.shape[0] + 10, 2), dtype=torch.int32, device="cuda")
    got = sj.bruteforce(torch.from_numpy(pts).cuda(), eps, out=buf)
    _same(got.cpu().numpy().astype(np.int64), want, "caller buffer")
    small = torch.empty((want.shape[0] - 1, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(ValueError, match="room for"):
        sj.bruteforce(torch.from_numpy(pts).cuda(), eps, out=small)


def test_where_the_grid_degenerates(sj):
    """6-D, 200,000 points, eps a third of the range: the grid has 3..4 cells
    per dimension, so 3^d cells x points per cell is about n and the grid join
    evaluates nearly every pair -- the regime where the paper's comparison
    expects a brute force to compete. Both joins must give the same pairs,
    and sampled rows must match the oracle."""
    n, d, eps = 200_000, 6, 100.0 / 3.0
    pts = datagen.uniform(n, d, seed=61)
    x = torch.from_numpy(pts).cuda()
    _say(f"brute vs grid 6-D n={n} eps={eps:.4f}")
    got = sj.bruteforce(x, eps)
    grid = sj.selfjoin(x, eps)
    assert torch.equal(got, grid)
    g = got.cpu().numpy().astype(np.int64)
    del got, grid
    rows = np.sort(np.random.default_rng(5).choice(n, 64, replace=False))
    off, js = ref.rows_neighbors(pts, eps, rows)
    a = np.searchsorted(g[:, 0], rows, side="left")
    b = np.searchsorted(g[:, 0], rows, side="right")
    for k, i in enumerate(rows):
        np.testing.assert_array_equal(g[a[k]:b[k], 1], js[off[k]:off[k + 1]].astype(np.int64),
                                      err_msg=f"row {i}")
    torch.cuda.empty_cache()
