"""Scheduler of the continuous-batching server, exercised without a GPU
(dry-run backend: no device work, simulated durations and result sizes)."""
from __future__ import annotations

import time

import numpy as np
import pytest


@pytest.fixture(scope="module")
def serve():
    from paper_1803_04120_amd import _lib, serve as s
    import os
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1803_04120_amd import build
        build.build()
    return s


def _drain(srv, want):
    out = {}
    t0 = time.time()
    while len(out) < want and time.time() - t0 < 30:
        for c in srv.poll(timeout_ms=50):
            out[c["req_id"]] = c
    return out


def test_all_requests_complete_and_fifo_start(serve):
    with serve.Server(slots=1, mem_budget_bytes=1 << 40, dry_run=True) as srv:
        ids = [srv.submit(np.zeros((1000 * (k + 1), 2)), 1.0, expected_pairs=100) for k in range(12)]
        done = _drain(srv, len(ids))
        assert sorted(done) == sorted(ids)
        # one slot: start order = submit order, so queue times are non-decreasing
        q = [done[i]["queue_ms"] for i in ids]
        assert all(q[i] <= q[i + 1] + 1e-6 for i in range(len(q) - 1))
        for i in ids:
            assert done[i]["status"] == 0
            srv.release(i)
        info = srv.info()
        assert info["completed"] == 12 and info["mem_used_bytes"] == 0


def test_budget_limits_concurrency(serve):
    # each request estimates ~1 MiB + index bytes; a 3-request budget with 8 slots
    n = 20000
    with serve.Server(slots=8, mem_budget_bytes=1, dry_run=True) as srv:
        ids = [srv.submit(np.zeros((n, 3)), 1.0, expected_pairs=1000) for _ in range(6)]
        seen_running = []
        got = {}
        t0 = time.time()
        while len(got) < len(ids) and time.time() - t0 < 30:
            seen_running.append(srv.info()["running"])
            for c in srv.poll(timeout_ms=1):
                got[c["req_id"]] = c
                srv.release(c["req_id"])
        assert len(got) == 6
        # budget 1 byte: only the request admitted into an empty server may run
        assert max(seen_running) <= 1
        assert srv.info()["peak_mem_bytes"] > 0


def test_estimate_misses_are_absorbed(serve):
    with serve.Server(slots=4, mem_budget_bytes=1 << 40, dry_run=True) as srv:
        ids = [srv.submit(np.zeros((5000, 2)), 1.0, expected_pairs=5000) for _ in range(8)]
        done = _drain(srv, 8)
        # even ids report twice the expected result
        for i in ids:
            assert done[i]["npairs"] == (10000 if i % 2 == 0 else 5000)
            srv.release(i)
        assert srv.info()["over_estimate"] >= 4


def test_release_unknown_and_bad_options(serve):
    from paper_1803_04120_amd import _lib
    with serve.Server(slots=2, mem_budget_bytes=1 << 30, dry_run=True) as srv:
        with pytest.raises(_lib.SjError):
            srv.release(12345)
    with pytest.raises(_lib.SjError):
        serve.Server(slots=0, mem_budget_bytes=1 << 30, dry_run=True)


def test_open_loop_stream_latency_accounting(serve):
    from paper_1803_04120_amd import datagen
    reqs = [{"points": np.zeros((int(n), 2)), "eps": 1.0, "expected_pairs": int(n)}
            for n in np.exp(np.random.default_rng(1).uniform(np.log(1e3), np.log(2e5), 40))]
    arr = datagen.poisson_arrivals(len(reqs), rate_per_s=2000.0, seed=5)
    with serve.Server(slots=4, mem_budget_bytes=1 << 40, dry_run=True) as srv:
        done, span = serve.run_stream(srv, reqs, arr)
    assert all(c is not None and c["status"] == 0 for c in done)
    for c in done:
        assert c["latency_ms"] >= c["service_ms"] >= 0
        assert abs(c["latency_ms"] - c["queue_ms"] - c["service_ms"]) < 1e-6
    assert span > 0


def test_no_deadlock_when_every_running_request_waits_for_memory(serve):
    # four equal requests whose estimates exactly fill the budget; the even
    # ids then need twice their estimated result and nobody releases until
    # all are done: the waiting requests must still make progress
    n, exp = 20000, 200000
    per = None
    with serve.Server(slots=4, mem_budget_bytes=1 << 40, dry_run=True) as probe:
        rid = probe.submit(np.zeros((n, 2)), 1.0, expected_pairs=exp)
        _drain(probe, 1)
        per = probe.info()["peak_mem_bytes"]
        probe.release(rid)
    with serve.Server(slots=4, mem_budget_bytes=4 * per, dry_run=True) as srv:
        ids = [srv.submit(np.zeros((n, 2)), 1.0, expected_pairs=exp) for _ in range(4)]
        done = _drain(srv, 4)
        assert sorted(done) == sorted(ids)
        assert srv.info()["over_estimate"] >= 2
        for i in ids:
            srv.release(i)


def test_release_before_poll(serve):
    """A request released as soon as it has completed, before any poll
    reported it, is never reported afterwards (and polling does not touch
    the freed record)."""
    with serve.Server(slots=2, mem_budget_bytes=1 << 40, dry_run=True) as srv:
        a = srv.submit(np.zeros((2000, 2)), 1.0, expected_pairs=10)
        b = srv.submit(np.zeros((2000, 2)), 1.0, expected_pairs=10)
        t0 = time.time()
        while srv.info()["completed"] < 2 and time.time() - t0 < 30:
            time.sleep(0.005)
        assert srv.info()["completed"] == 2
        srv.release(a)
        got = _drain(srv, 1)
        assert list(got) == [b]
        assert srv.poll(timeout_ms=20) == []
        srv.release(b)
