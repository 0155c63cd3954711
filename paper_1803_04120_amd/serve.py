"""Continuous-batching self-join server (Python face of sj_server_* in libsj).

    srv = Server(slots=4, mem_budget_bytes=32 << 30)
    rid = srv.submit(points_cuda_f64, eps, precision="fp32_band", expected_pairs=n * 17)
    for c in srv.poll(timeout_ms=-1):
        pairs = srv.result(c)          # (P, 2) int32 device tensor (a copy)
        srv.release(c["req_id"])

`run_stream` replays a timed request stream (open loop: each request is
submitted at its arrival time whatever is still running) and reports
latency percentiles and throughput.
"""
from __future__ import annotations

import ctypes
import math
import time

import numpy as np

from . import _lib

__all__ = ["Server", "run_stream", "uniform_eps_for_k"]


class SjServerOpts(ctypes.Structure):
    _fields_ = [("slots", ctypes.c_uint32), ("flags", ctypes.c_uint32),
                ("mem_budget_bytes", ctypes.c_uint64)]


class SjCompletion(ctypes.Structure):
    _fields_ = [("req_id", ctypes.c_uint64), ("status", ctypes.c_int32), ("slot", ctypes.c_uint32),
                ("pairs_dev", ctypes.c_void_p), ("npairs", ctypes.c_uint64),
                ("queue_ms", ctypes.c_double), ("service_ms", ctypes.c_double),
                ("latency_ms", ctypes.c_double), ("evals", ctypes.c_uint64),
                ("band_rechecks", ctypes.c_uint64)]


class SjServerInfo(ctypes.Structure):
    _fields_ = [("queued", ctypes.c_uint64), ("running", ctypes.c_uint64),
                ("mem_used_bytes", ctypes.c_uint64), ("peak_mem_bytes", ctypes.c_uint64),
                ("over_estimate", ctypes.c_uint64), ("completed", ctypes.c_uint64)]


def _bind():
    L = _lib.load()
    if getattr(L, "_sj_server_bound", False):
        return L
    vp = ctypes.c_void_p
    L.sj_server_create.restype = ctypes.c_int
    L.sj_server_create.argtypes = [ctypes.POINTER(SjServerOpts), ctypes.POINTER(vp)]
    L.sj_server_submit.restype = ctypes.c_int
    L.sj_server_submit.argtypes = [vp, vp, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_double, ctypes.c_int,
                                   ctypes.POINTER(_lib.SjJoinOpts), ctypes.c_uint64,
                                   ctypes.POINTER(ctypes.c_uint64)]
    L.sj_server_poll.restype = ctypes.c_int
    L.sj_server_poll.argtypes = [vp, ctypes.POINTER(SjCompletion), ctypes.c_uint32,
                                 ctypes.POINTER(ctypes.c_uint32), ctypes.c_int32]
    L.sj_server_release.restype = ctypes.c_int
    L.sj_server_release.argtypes = [vp, ctypes.c_uint64]
    L.sj_server_info.restype = ctypes.c_int
    L.sj_server_info.argtypes = [vp, ctypes.POINTER(SjServerInfo)]
    L.sj_server_destroy.restype = None
    L.sj_server_destroy.argtypes = [vp]
    L._sj_server_bound = True
    return L


class Server:
    def __init__(self, slots: int = 4, mem_budget_bytes: int = 32 << 30, dry_run: bool = False):
        L = _bind()
        o = SjServerOpts(slots=int(slots), flags=1 if dry_run else 0,
                         mem_budget_bytes=int(mem_budget_bytes))
        h = ctypes.c_void_p()
        _lib.check(L.sj_server_create(ctypes.byref(o), ctypes.byref(h)))
        self._h = h
        self._keep = {}  # req_id -> input kept alive until completion

    def submit(self, points, eps: float, *, unicomp: bool = True, precision: str = "fp32_band",
               expected_pairs: int = 0, sync: bool = True) -> int:
        """Queue a request. The server reads device points on its own streams,
        so with sync (the default) torch's current stream is synchronised first;
        pass sync=False when the points are known to be complete."""
        try:
            import torch
            is_tensor = isinstance(points, torch.Tensor)
        except ImportError:  # pragma: no cover
            is_tensor = False
        if is_tensor:
            t = points.contiguous()
            if t.dtype != torch.float64 or t.dim() != 2:
                raise ValueError("points must be a (n, d) float64 tensor")
            ptr, n, d, on_dev, keep = t.data_ptr(), t.shape[0], t.shape[1], int(t.is_cuda), t
            if on_dev and sync:
                torch.cuda.current_stream(t.device).synchronize()
        else:
            a = np.ascontiguousarray(np.asarray(points, dtype=np.float64))
            ptr, n, d, on_dev, keep = a.ctypes.data, a.shape[0], a.shape[1], 0, a
        o = _lib.opts(unicomp, precision)
        rid = ctypes.c_uint64(0)
        _lib.check(_bind().sj_server_submit(self._h, ctypes.c_void_p(ptr), n, d, float(eps), on_dev,
                                            ctypes.byref(o), int(expected_pairs), ctypes.byref(rid)))
        self._keep[rid.value] = keep
        return int(rid.value)

    def poll(self, timeout_ms: int = 0, cap: int = 64):
        recs = (SjCompletion * cap)()
        cnt = ctypes.c_uint32(0)
        _lib.check(_bind().sj_server_poll(self._h, recs, cap, ctypes.byref(cnt), int(timeout_ms)))
        out = []
        for k in range(cnt.value):
            r = recs[k]
            out.append({"req_id": int(r.req_id), "status": int(r.status), "slot": int(r.slot),
                        "pairs_dev": int(r.pairs_dev or 0), "npairs": int(r.npairs),
                        "queue_ms": r.queue_ms, "service_ms": r.service_ms,
                        "latency_ms": r.latency_ms, "evals": int(r.evals),
                        "band_rechecks": int(r.band_rechecks)})
            self._keep.pop(int(r.req_id), None)
        return out

    def result(self, completion):
        """Copy of a completed request's pairs as a (P, 2) int32 device tensor."""
        import torch
        from . import _copy_d2d
        P = completion["npairs"]
        t = torch.empty((P, 2), dtype=torch.int32, device="cuda")
        if P:
            _copy_d2d(t.data_ptr(), completion["pairs_dev"], P * 8)
        return t

    def release(self, req_id: int):
        _lib.check(_bind().sj_server_release(self._h, int(req_id)))

    def info(self) -> dict:
        i = SjServerInfo()
        _lib.check(_bind().sj_server_info(self._h, ctypes.byref(i)))
        return {k: int(getattr(i, k)) for k, _ in SjServerInfo._fields_}

    def close(self):
        if getattr(self, "_h", None):
            _bind().sj_server_destroy(self._h)
            self._h = None
            self._keep.clear()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass


def unit_ball_volume(d: int) -> float:
    return math.pi ** (d / 2) / math.gamma(d / 2 + 1)


def uniform_eps_for_k(n: int, d: int, k: float, box: float = 100.0) -> float:
    """eps giving about k neighbours per point for n uniform points in
    [0, box]^d, ignoring the boundary: n V_d eps^d / box^d = k."""
    return (k * box ** d / (n * unit_ball_volume(d))) ** (1.0 / d)


def run_stream(server: Server, requests, arrivals_s, on_complete=None, poll_ms: int = 1):
    """Open-loop replay: request r is submitted at arrivals_s[r] (seconds from
    the start) regardless of what is running. requests[r] is a dict with
    points, eps, precision, unicomp, expected_pairs; device points must be
    complete before the call (they are submitted without synchronising). on_complete(r_index,
    completion) may inspect the result before it is released.
    Returns per-request completions (in request order) and the makespan."""
    order = np.argsort(np.asarray(arrivals_s))
    t0 = time.perf_counter()
    pending = {}
    done = [None] * len(requests)
    nxt = 0
    while nxt < len(order) or pending:
        now = time.perf_counter() - t0
        while nxt < len(order) and arrivals_s[order[nxt]] <= now:
            r = int(order[nxt])
            q = requests[r]
            rid = server.submit(q["points"], q["eps"], unicomp=q.get("unicomp", True),
                                precision=q.get("precision", "fp32_band"),
                                expected_pairs=q.get("expected_pairs", 0), sync=False)
            pending[rid] = r
            nxt += 1
        wait = poll_ms
        if nxt < len(order):
            wait = max(0, min(poll_ms, int(1e3 * (arrivals_s[order[nxt]] - (time.perf_counter() - t0)))))
        for c in server.poll(timeout_ms=wait if pending else 0):
            r = pending.pop(c["req_id"])
            if on_complete is not None:
                on_complete(r, c)
            server.release(c["req_id"])
            done[r] = c
        if not pending and nxt < len(order):
            dt = arrivals_s[order[nxt]] - (time.perf_counter() - t0)
            if dt > 0:
                time.sleep(min(dt, 0.002))
    return done, time.perf_counter() - t0
