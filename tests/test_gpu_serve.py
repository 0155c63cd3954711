"""Served results are the same alone and in the mix (GPU).

A set of requests of different sizes, dimensions, distributions and eps is
run through the continuous-batching server all at once (several slots, so
their work overlaps on the device) and again one by one with the plain
entry point; every served pair set must equal the solo one exactly, and the
small ones must equal the oracle.
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


def _requests():
    from paper_1803_04120_amd.serve import uniform_eps_for_k
    g = np.random.default_rng(7)
    out = []
    for r in range(14):
        n = int(np.exp(g.uniform(np.log(1e3), np.log(2e5))))
        d = int(g.integers(2, 7))
        kind = "uniform" if r % 2 == 0 else "clustered"
        k = float(np.exp(g.uniform(np.log(4), np.log(64))))
        eps = uniform_eps_for_k(n, d, k) * (0.3 if kind == "clustered" else 1.0)
        pts = datagen.make(kind, n, d, seed=100 + r)
        out.append(dict(points=torch.from_numpy(pts).cuda(), host=pts, eps=eps, n=n, d=d,
                        precision="fp32_band" if r % 3 else "fp64", unicomp=bool(r % 4),
                        expected_pairs=int(n * (k + 1))))
    return out


def test_served_equals_solo(sj):
    from paper_1803_04120_amd.serve import Server
    reqs = _requests()
    print(f"[case] serve {len(reqs)} requests", flush=True)
    solo = [sj.selfjoin(q["points"], q["eps"], unicomp=q["unicomp"], precision=q["precision"])
            for q in reqs]
    torch.cuda.synchronize()
    with Server(slots=4, mem_budget_bytes=8 << 30) as srv:
        ids = [srv.submit(q["points"], q["eps"], unicomp=q["unicomp"], precision=q["precision"],
                          expected_pairs=q["expected_pairs"]) for q in reqs]
        got = {}
        while len(got) < len(ids):
            for c in srv.poll(timeout_ms=100):
                assert c["status"] == 0, c
                got[c["req_id"]] = (c, srv.result(c))
                srv.release(c["req_id"])
        slots_used = {c["slot"] for c, _ in got.values()}
    assert len(slots_used) > 1
    for q, rid, s in zip(reqs, ids, solo):
        c, t = got[rid]
        assert torch.equal(t, s), f"served result differs for n={q['n']} d={q['d']}"
    for q, s in zip(reqs, solo):
        if q["n"] <= 20000:
            want = ref.pairs(q["host"], q["eps"])
            np.testing.assert_array_equal(s.cpu().numpy().astype(np.int64), want)


def test_small_budget_still_completes(sj):
    from paper_1803_04120_amd.serve import Server
    reqs = _requests()[:6]
    print("[case] serve with a tiny budget", flush=True)
    with Server(slots=4, mem_budget_bytes=1 << 20) as srv:
        ids = [srv.submit(q["points"], q["eps"], precision=q["precision"], expected_pairs=1)
               for q in reqs]
        got = {}
        while len(got) < len(ids):
            for c in srv.poll(timeout_ms=100):
                got[c["req_id"]] = c
                srv.release(c["req_id"])
        info = srv.info()
    assert all(c["status"] == 0 for c in got.values())
    assert info["over_estimate"] >= 1
    for q, rid in zip(reqs, ids):
        assert got[rid]["npairs"] == sj.Index(q["points"], q["eps"]).count(precision=q["precision"])


def test_open_loop_stream(sj):
    from paper_1803_04120_amd.serve import Server, run_stream
    reqs = _requests()
    print("[case] open-loop stream", flush=True)
    arrivals = datagen.poisson_arrivals(len(reqs), rate_per_s=400.0, seed=3)
    sizes = {}
    with Server(slots=4, mem_budget_bytes=8 << 30) as srv:
        done, span = run_stream(srv, reqs, arrivals,
                                on_complete=lambda r, c: sizes.__setitem__(r, c["npairs"]))
    assert all(c["status"] == 0 for c in done)
    lat = np.array([c["latency_ms"] for c in done])
    assert np.all(lat > 0) and span > 0
    assert len(sizes) == len(reqs)


def test_served_full_size_requests(sj):
    """Requests at the stream's full size range: up to 2e6 points, clustered
    4..6-D ones included, all in flight at once on four slots. Each served
    result must equal the same request run alone and the host-core grid join
    (pair for pair)."""
    from paper_1803_04120_amd.serve import Server, uniform_eps_for_k
    # (n, d, kind, k, eps factor): the clustered requests' eps is scaled down
    # from the uniform closed form so their results stay at 1e8..6e8 pairs
    specs = [(2_000_000, 4, "clustered", 40.0, 0.2), (1_200_000, 6, "clustered", 24.0, 0.1),
             (2_000_000, 5, "uniform", 64.0, 1.0), (800_000, 4, "uniform", 100.0, 1.0),
             (1_500_000, 3, "clustered", 16.0, 0.4), (300_000, 6, "uniform", 128.0, 1.0)]
    reqs = []
    for r, (n, d, kind, k, f) in enumerate(specs):
        eps = uniform_eps_for_k(n, d, k) * f
        pts = datagen.make(kind, n, d, seed=900 + r)
        reqs.append(dict(points=torch.from_numpy(pts).cuda(), host=pts, eps=eps, n=n, d=d,
                         precision="fp32_band" if r % 2 else "fp64", expected_pairs=int(n * (k + 1))))
    print(f"[case] serve {len(reqs)} full-size requests", flush=True)
    with Server(slots=4, mem_budget_bytes=96 << 30) as srv:
        ids = [srv.submit(q["points"], q["eps"], precision=q["precision"], expected_pairs=q["expected_pairs"])
               for q in reqs]
        got = {}
        while len(got) < len(ids):
            for c in srv.poll(timeout_ms=200):
                assert c["status"] == 0, c
                got[c["req_id"]] = srv.result(c).cpu().numpy()
                srv.release(c["req_id"])
    for q, rid in zip(reqs, ids):
        print(f"[case] full-size request n={q['n']} d={q['d']}: solo and CPU grid join", flush=True)
        solo = sj.selfjoin(q["points"], q["eps"], precision=q["precision"]).cpu().numpy()
        assert np.array_equal(got[rid], solo), f"served != solo for n={q['n']} d={q['d']}"
        _, want = ref.grid_join(q["host"], q["eps"])
        assert np.array_equal(solo, want), f"solo != grid join for n={q['n']} d={q['d']}"
        del solo, want
    torch.cuda.empty_cache()
