"""Parity at the full workload sizes (GPU).

Whole results are compared pair for pair with the host-core grid join
(oracle/cpu_grid_join.c, itself checked against the brute force) wherever
it finishes in about a minute on the host: the 2M-point 2-D sweep, the
10M-point 3..6-D joins at 32 neighbours per point, the 5M-point clustered
joins in both precisions and the two-set join. Every join is also checked
on a seeded sample of result rows that the brute-force oracle computes one
by one against all n candidates (4096 rows for the 10M-point joins at 256
neighbours, whose whole results the host join would take many minutes to
produce), plus exact equalities that hold at any size: unicomp on = off,
FP32 pre-test = FP64, batched = unbatched, unicomp evaluations = (T + n) / 2.
The joins run through the same entry points and launch configuration as
bench.py (count pass, whole-result fill).
"""
from __future__ import annotations

import json
import os

import numpy as np
import pytest

from oracle import reference as ref
from paper_1803_04120_amd import datagen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

CALIB = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "eps_calibration.json")
SAMPLE_ROWS = 256


@pytest.fixture(scope="module")
def sj():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1803_04120_amd as m
    m._lib.load()
    return m


def _say(msg):
    print(f"[case] {msg}", flush=True)


def _calib():
    with open(CALIB) as f:
        return json.load(f)


def _join(sj, x, eps, **kw):
    ix = sj.Index(x, eps)
    P = ix.count(**kw)
    out = torch.empty((P, 2), dtype=torch.int32, device="cuda")
    ix.fill(out)
    off = ix.export(sj._lib.SJ_EXPORT_ROW_OFFSETS).astype(np.int64)
    stats = ix.stats()
    ix.close()
    return out, off, stats


def _check_rows(pts, eps, out, off, seed, nrows=SAMPLE_ROWS):
    n = pts.shape[0]
    rows = np.sort(np.random.default_rng(seed).choice(n, nrows, replace=False))
    roff, js = ref.rows_neighbors(pts, eps, rows)
    host = out if isinstance(out, np.ndarray) else None
    for k, i in enumerate(rows):
        a, b = int(off[i]), int(off[i + 1])
        seg = (host[a:b] if host is not None else out[a:b].cpu().numpy()).astype(np.int64)
        want = js[roff[k]:roff[k + 1]].astype(np.int64)
        assert np.all(seg[:, 0] == i), f"row {i}: wrong row ids"
        np.testing.assert_array_equal(seg[:, 1], want, err_msg=f"row {i} differs")
    return rows


def _whole_vs_grid_join(pts, eps, got, off):
    """The whole GPU result (host copy) against the host-core grid join."""
    counts, want = ref.grid_join(pts, eps)
    np.testing.assert_array_equal(np.diff(off), counts)
    assert got.shape == want.shape
    assert np.array_equal(got, want)


def test_uniform_2d_2M_eps_sweep(sj):
    """The 2-D workload: 2,000,000 uniform points, eps 0.04 .. 0.2."""
    pts = datagen.uniform(2_000_000, 2, seed=2)
    x = torch.from_numpy(pts).cuda()
    for e in (0.04, 0.08, 0.12, 0.16, 0.2):
        _say(f"uniform 2d n=2M eps={e}")
        out, off, st = _join(sj, x, e, unicomp=True)
        assert off[-1] == out.shape[0] == st["pairs"]
        _check_rows(pts, e, out, off, seed=int(e * 1000))
        out0, off0, _ = _join(sj, x, e, unicomp=False)
        assert torch.equal(out, out0)
        np.testing.assert_array_equal(off, off0)
        del out, out0
    torch.cuda.empty_cache()


@pytest.mark.parametrize("eps", [0.04, 0.2])
def test_uniform_2d_2M_whole_result_vs_cpu_grid_join(sj, eps):
    """Whole result, not a sample: the 2M-point 2-D join against the host-core
    grid join (itself checked against the brute force), pair for pair."""
    pts = datagen.uniform(2_000_000, 2, seed=2)
    x = torch.from_numpy(pts).cuda()
    _say(f"uniform 2d n=2M eps={eps} whole result vs CPU grid join")
    out, off, _ = _join(sj, x, eps, unicomp=True)
    got = out.cpu().numpy()
    del out, x
    counts, want = ref.grid_join(pts, eps)
    assert got.shape == want.shape
    np.testing.assert_array_equal(np.diff(off), counts)
    assert np.array_equal(got, want)
    torch.cuda.empty_cache()


@pytest.mark.parametrize("key", ["d3_k32", "d3_k256", "d4_k32", "d4_k256",
                                 "d5_k32", "d5_k256", "d6_k32", "d6_k256"])
def test_uniform_10M(sj, key):
    """10,000,000 uniform points in 3..6-D at eps for mean 32 / 256
    neighbours: the whole result against the host grid join (32
    neighbours) or 4096 sampled rows against the brute force (256); unicomp
    on vs off must agree exactly."""
    c = _calib()["uniform_n10M"][key]
    _say(f"uniform n=10M {key} eps={c['eps']}")
    pts = datagen.uniform(c["n"], c["d"], seed=c["seed"])
    x = torch.from_numpy(pts).cuda()
    out, off, st = _join(sj, x, c["eps"], unicomp=True)
    assert off[-1] == out.shape[0]
    mean_k = out.shape[0] / c["n"] - 1
    assert abs(mean_k - c["k_mean"]) < 0.05 * c["k_mean"]
    out0, _, st0 = _join(sj, x, c["eps"], unicomp=False)
    assert torch.equal(out, out0)
    del out0
    # the paper's factor ~2: unicomp evaluates (T + n) / 2 candidates
    assert 2 * st["evals"] == st0["evals"] + c["n"]
    if c["k_mean"] <= 32:
        got = out.cpu().numpy()
        del out
        _check_rows(pts, c["eps"], got, off, seed=7, nrows=1024)
        _say(f"uniform n=10M {key}: whole result vs CPU grid join")
        _whole_vs_grid_join(pts, c["eps"], got, off)
        del got
    else:
        _check_rows(pts, c["eps"], out, off, seed=7, nrows=4096)
        del out
    del x
    torch.cuda.empty_cache()


@pytest.mark.parametrize("key", ["d2", "d3"])
def test_clustered_5M_fp32_band_equals_fp64(sj, key):
    """5,000,000 clustered points (median 50 neighbours): the whole FP64
    result and the whole FP32 pre-test result (FP64 band re-decision) are
    each compared with the host grid join, pair for pair."""
    c = _calib()["clustered_n5M"][key]
    _say(f"clustered n=5M {key} eps={c['eps']}")
    pts = datagen.clustered(c["n"], c["d"], seed=c["seed"])
    x = torch.from_numpy(pts).cuda()
    out, off, st = _join(sj, x, c["eps"], precision="fp64")
    got64 = out.cpu().numpy()
    del out
    out32, off32, st32 = _join(sj, x, c["eps"], precision="fp32_band")
    assert st32["precision_used"] == 1
    assert st32["band_rechecks"] > 0
    got32 = out32.cpu().numpy()
    del out32, x
    torch.cuda.empty_cache()
    rows = _check_rows(pts, c["eps"], got64, off, seed=11, nrows=1024)
    counts = np.diff(off)
    assert np.median(counts[rows] - 1) == pytest.approx(c["k_median"], rel=0.35)
    _say(f"clustered n=5M {key}: whole results vs CPU grid join")
    counts_o, want = ref.grid_join(pts, c["eps"])
    np.testing.assert_array_equal(counts, counts_o)
    np.testing.assert_array_equal(np.diff(off32), counts_o)
    assert np.array_equal(got64, want), "FP64 result differs from the grid join"
    assert np.array_equal(got32, want), "FP32+band result differs from the grid join"


def test_batched_equals_unbatched_at_scale(sj):
    """Result larger than one batch buffer (2^27 pairs): the batches'
    concatenation equals the single-buffer result."""
    c = _calib()["uniform_n10M"]["d3_k32"]
    _say("batched 10M d3 k32")
    pts = datagen.uniform(c["n"], c["d"], seed=c["seed"])
    x = torch.from_numpy(pts).cuda()
    out, off, _ = _join(sj, x, c["eps"], unicomp=True)
    with sj.Index(x, c["eps"]) as ix:
        got, info = ix.join_batched(unicomp=True, batch_capacity_pairs=1 << 27, min_batches=3)
    assert len(info) >= 3
    assert all(npairs <= (1 << 27) for _, _, _, npairs in info)
    # every run sorted within itself; the merged runs are the whole result
    key = got[:, 0].to(torch.int64) * c["n"] + got[:, 1].to(torch.int64)
    at = 0
    for _, _, _, npairs in info:
        assert bool((key[at + 1:at + npairs] > key[at:at + npairs - 1]).all())
        at += npairs
    key = torch.sort(key).values
    want = out[:, 0].to(torch.int64) * c["n"] + out[:, 1].to(torch.int64)
    assert torch.equal(key, want)
    del out, got, x
    torch.cuda.empty_cache()


def test_two_set_join_1M_queries_vs_2M_indexed(sj):
    """The two-set join at the bench's size: 10^6 uniform queries (seed 1002)
    against the 2,000,000 indexed points (seed 2), eps 0.04 .. 0.2. Sampled
    query rows are recomputed by the oracle against all of S; every reported
    pair is checked against the predicate, and the pairs must come sorted by
    (query, indexed row) with no repeats."""
    S = datagen.uniform(2_000_000, 2, seed=2)
    R = datagen.uniform(1_000_000, 2, seed=1002)
    s_dev, r_dev = torch.from_numpy(S).cuda(), torch.from_numpy(R).cuda()
    buf = None
    for e in (0.04, 0.08, 0.12, 0.16, 0.2):
        _say(f"two-set join 1M queries x 2M indexed eps={e}")
        with sj.Index(s_dev, e) as ix:
            got_t = ix.join_rs(r_dev)
            if buf is None or buf.shape[0] < got_t.shape[0]:
                buf = torch.empty((got_t.shape[0] + 1024, 2), dtype=torch.int32, device="cuda")
            # the caller-buffer form (one call, as timed) gives the same pairs
            assert torch.equal(ix.join_rs(r_dev, out=buf), got_t)
        got = got_t.cpu().numpy().astype(np.int64)
        del got_t
        assert got.shape[0] > R.shape[0]  # several neighbours per query
        key = got[:, 0] * S.shape[0] + got[:, 1]
        assert np.all(np.diff(key) > 0), "pairs not sorted or repeated"
        with np.errstate(over="ignore"):
            t0 = R[got[:, 0], 0] - S[got[:, 1], 0]
            t1 = R[got[:, 0], 1] - S[got[:, 1], 1]
            d2 = (0.0 + t0 * t0) + t1 * t1
        assert np.all(d2 <= e * e), "a reported pair is farther than eps"
        rows = np.sort(np.random.default_rng(int(e * 1000) + 7).choice(R.shape[0], 128, replace=False))
        want = ref.join_rs_numpy(R[rows], S, e)
        want[:, 0] = rows[want[:, 0]]
        a = np.searchsorted(got[:, 0], rows, side="left")
        b = np.searchsorted(got[:, 0], rows, side="right")
        seg = np.concatenate([got[x:y] for x, y in zip(a, b)], axis=0)
        np.testing.assert_array_equal(seg, want)
        if e in (0.04, 0.2):
            # whole set: the host grid join of S followed by R; its rows of
            # R's points, restricted to the columns of S, are R x S
            _say(f"two-set join eps={e}: whole result vs CPU grid join of S + R")
            ns = S.shape[0]
            _, both = ref.grid_join(np.concatenate([S, R], axis=0), e)
            both = both.astype(np.int64)
            keep = (both[:, 0] >= ns) & (both[:, 1] < ns)
            want_all = both[keep]
            del both
            want_all[:, 0] -= ns
            assert np.array_equal(got, want_all)
            del want_all
    del s_dev, r_dev, buf
    torch.cuda.empty_cache()
