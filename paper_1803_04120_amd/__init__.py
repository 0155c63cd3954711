"""MI355X-native epsilon-distance similarity self-join (Gowanlock & Karsin).

Python face of libsj.so. PyTorch supplies device memory and the current
stream; the grid index, the adjacent-cell search and refine, the pair
emission and the sorts all run in the HIP library.

    import torch, paper_1803_04120_amd as sj
    pts = torch.rand(10000, 2, dtype=torch.float64, device="cuda") * 100
    pairs = sj.selfjoin(pts, 1.0)          # (P, 2) int32, sorted by (i, j)
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import SjError  # noqa: F401

__all__ = ["Index", "selfjoin", "bruteforce", "dbscan", "dbscan_csr", "band_thresholds", "last_run_stats",
           "SjError", "version"]


def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    if stream is None:
        if torch.cuda.is_available():
            return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
        return ctypes.c_void_p(0)
    if isinstance(stream, int):
        return ctypes.c_void_p(stream)
    return ctypes.c_void_p(stream.cuda_stream)


def _points_arg(points):
    """(pointer, n, d, on_device, keepalive) for a float64 (n, d) tensor/array."""
    torch = _torch()
    if isinstance(points, torch.Tensor):
        if points.dtype != torch.float64:
            raise TypeError("points must be float64")
        if points.dim() != 2:
            raise ValueError("points must have shape (n, d)")
        t = points.contiguous()
        return ctypes.c_void_p(t.data_ptr()), t.shape[0], t.shape[1], int(t.is_cuda), t
    a = np.ascontiguousarray(np.asarray(points, dtype=np.float64))
    if a.ndim != 2:
        raise ValueError("points must have shape (n, d)")
    return ctypes.c_void_p(a.ctypes.data), a.shape[0], a.shape[1], 0, a


class Index:
    """Device-resident grid index of Section IV-C (B, G, A, M and the
    cell-ordered coordinates). Build once, join many times."""

    def __init__(self, points, eps: float, stream=None):
        L = _lib.load()
        ptr, n, d, on_dev, keep = _points_arg(points)
        self._stream = stream
        self.n, self.d, self.eps = int(n), int(d), float(eps)
        h = ctypes.c_void_p()
        _lib.check(L.sj_build_index(ptr, n, d, float(eps), on_dev, _stream_handle(stream),
                                    ctypes.byref(h)))
        del keep
        self._h = h
        self._device = points.device if hasattr(points, "device") and getattr(points, "is_cuda", False) else None
        self._counted = None

    # ---------------------------------------------------------------- join
    def count(self, unicomp: bool = True, precision: str = "fp64", sort_output: bool = True) -> int:
        """Count pass: result size P (rows and offsets stay on the device).
        sort_output=False lets the fill leave each row's j unsorted."""
        L = _lib.load()
        o = _lib.opts(unicomp, precision, sort_output=sort_output)
        total = ctypes.c_uint64(0)
        _lib.check(L.sj_join_count(self._h, ctypes.byref(o), _stream_handle(self._stream),
                                   ctypes.byref(total)))
        self._counted = int(total.value)
        return self._counted

    def fill(self, out=None):
        """Fill pass after count(): (P, 2) int32 device tensor sorted by (i, j)."""
        torch = _torch()
        if self._counted is None:
            raise RuntimeError("fill() needs count() first")
        P = self._counted
        if out is None:
            dev = self._device or torch.device("cuda")
            out = torch.empty((P, 2), dtype=torch.int32, device=dev)
        if out.dtype != torch.int32 or not out.is_contiguous() or out.numel() < 2 * P:
            raise ValueError("out must be a contiguous int32 tensor with room for P pairs")
        L = _lib.load()
        _lib.check(L.sj_join_fill(self._h, ctypes.c_void_p(out.data_ptr() if P else 0),
                                  P, _stream_handle(self._stream)))
        return out[:P] if out.shape[0] != P else out

    def fill_csr(self):
        """Fill pass after count() into a CSR neighbour table: (row_off int64
        (n + 1,), cols int32 (P,)) device tensors; row i's neighbours are
        cols[row_off[i]:row_off[i + 1]]."""
        torch = _torch()
        if self._counted is None:
            raise RuntimeError("fill_csr() needs count() first")
        P = self._counted
        dev = self._device or torch.device("cuda")
        row_off = torch.empty((self.n + 1,), dtype=torch.int64, device=dev)
        cols = torch.empty((max(P, 1),), dtype=torch.int32, device=dev)
        _lib.check(_lib.load().sj_join_fill_csr(self._h, ctypes.c_void_p(row_off.data_ptr()),
                                                ctypes.c_void_p(cols.data_ptr()), P,
                                                _stream_handle(self._stream)))
        return row_off, cols[:P]

    def join_rs(self, queries, out=None):
        """Distance join of the query rows (float64 (nr, d), host or device)
        with the indexed set: (P, 2) int32 device tensor of (query row,
        indexed row) pairs sorted by (i, j), at the index's eps."""
        torch = _torch()
        L = _lib.load()
        ptr, nr, d, on_dev, keep = _points_arg(queries)
        if nr and d != self.d:
            raise ValueError(f"queries have {d} dimensions, the index {self.d}")
        total = ctypes.c_uint64(0)
        if out is not None:
            # one call when the buffer is large enough
            if out.dtype != torch.int32 or not out.is_contiguous():
                raise ValueError("out must be a contiguous int32 tensor")
            rc = L.sj_join_rs(self._h, ptr, nr, on_dev, ctypes.c_void_p(out.data_ptr()), out.numel() // 2,
                              _stream_handle(self._stream), ctypes.byref(total))
            if rc == _lib.SJ_ECAPACITY:
                raise ValueError(f"out has room for {out.numel() // 2} pairs, the result has {total.value}")
            _lib.check(rc)
            P = int(total.value)
            del keep
            return out[:P] if out.shape[0] != P else out
        # count once, allocate the exact result, fill from the count's state
        _lib.check(L.sj_join_rs_count(self._h, ptr, nr, on_dev, _stream_handle(self._stream),
                                      ctypes.byref(total)))
        P = int(total.value)
        dev = self._device or torch.device("cuda")
        out = torch.empty((P, 2), dtype=torch.int32, device=dev)
        if P:
            _lib.check(L.sj_join_rs_fill(self._h, ctypes.c_void_p(out.data_ptr()), P,
                                         _stream_handle(self._stream)))
        del keep
        return out

    def join(self, unicomp: bool = True, precision: str = "fp64"):
        self.count(unicomp, precision)
        return self.fill()

    def batches(self, callback, unicomp: bool = True, precision: str = "fp64",
                batch_capacity_pairs: int = 0, min_batches: int = 1) -> int:
        """Batched join: callback(pairs_ptr, npairs, batch_id, row_begin, row_end)
        is called per run with a device pointer valid during the call. A run
        holds the rows of the cell-ordered positions [row_begin, row_end),
        sorted by (i, j) within the run; the runs partition the result.
        Returns the total number of pairs."""
        L = _lib.load()
        o = _lib.opts(unicomp, precision, batch_capacity_pairs, min_batches)
        err = []

        def _cb(user, ptr, npairs, bid, r0, r1):
            try:
                callback(int(ptr or 0), int(npairs), int(bid), int(r0), int(r1))
                return 0
            except Exception as e:  # noqa: BLE001
                err.append(e)
                return 1
        cfun = _lib.RUN_CB(_cb)
        total = ctypes.c_uint64(0)
        rc = L.sj_selfjoin_index(self._h, ctypes.byref(o), cfun, None,
                                 _stream_handle(self._stream), ctypes.byref(total))
        if err:
            raise err[0]
        _lib.check(rc)
        return int(total.value)

    def join_batched(self, unicomp: bool = True, precision: str = "fp64",
                     batch_capacity_pairs: int = 0, min_batches: int = 1):
        """Batched join gathered into one (P, 2) int32 device tensor, the runs
        one after another (each sorted by (i, j) within itself); also returns
        the list of (batch_id, row_begin, row_end, npairs)."""
        torch = _torch()
        chunks, info = [], []

        def cb(ptr, npairs, bid, r0, r1):
            t = torch.empty((npairs, 2), dtype=torch.int32, device=self._device or "cuda")
            if npairs:
                _copy_d2d(t.data_ptr(), ptr, npairs * 8)
            chunks.append(t)
            info.append((bid, r0, r1, npairs))
        self.batches(cb, unicomp, precision, batch_capacity_pairs, min_batches)
        out = torch.cat(chunks, 0) if chunks else torch.empty((0, 2), dtype=torch.int32,
                                                               device=self._device or "cuda")
        return out, info

    # ------------------------------------------------------------- inspect
    def search(self, unicomp: bool):
        _lib.check(_lib.load().sj_index_search(self._h, 1 if unicomp else 0,
                                               _stream_handle(self._stream)))

    def stats(self) -> dict:
        st = _lib.SjStats()
        _lib.check(_lib.load().sj_index_stats(self._h, ctypes.byref(st)))
        return _lib.stats_dict(st)

    def export(self, what: int) -> np.ndarray:
        L = _lib.load()
        size = ctypes.c_uint64(0)
        _lib.check(L.sj_index_export_size(self._h, what, ctypes.byref(size)))
        dtype = {
            _lib.SJ_EXPORT_CELL_IDS: np.uint64, _lib.SJ_EXPORT_CELL_START: np.uint32,
            _lib.SJ_EXPORT_PERM: np.uint32, _lib.SJ_EXPORT_MASKS: np.uint32,
            _lib.SJ_EXPORT_RANGE_OFF: np.uint64, _lib.SJ_EXPORT_RANGES: np.uint32,
            _lib.SJ_EXPORT_GRID: np.float64, _lib.SJ_EXPORT_ROW_OFFSETS: np.uint64}[what]
        out = np.zeros(int(size.value) // np.dtype(dtype).itemsize, dtype=dtype)
        _lib.check(L.sj_index_export(self._h, what,
                                     ctypes.c_void_p(out.ctypes.data) if out.size else None,
                                     size.value))
        return out

    def close(self):
        if getattr(self, "_h", None):
            _lib.load().sj_destroy_index(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


_hip = None


def _copy_d2d(dst: int, src: int, nbytes: int):
    """Device-to-device copy on torch's current stream (HIP runtime call)."""
    global _hip
    torch = _torch()
    if _hip is None:
        _hip = ctypes.CDLL("libamdhip64.so")
        _hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                        ctypes.c_int, ctypes.c_void_p]
        _hip.hipMemcpyAsync.restype = ctypes.c_int
    s = torch.cuda.current_stream()
    rc = _hip.hipMemcpyAsync(ctypes.c_void_p(dst), ctypes.c_void_p(src), ctypes.c_size_t(nbytes),
                             3, ctypes.c_void_p(s.cuda_stream))  # 3 = hipMemcpyDeviceToDevice
    if rc != 0:
        raise RuntimeError(f"hipMemcpyAsync failed ({rc})")
    s.synchronize()


def selfjoin(points, eps: float, *, unicomp: bool = True, precision: str = "fp64",
             stream=None):
    """All pairs (i, j) with d2(p_i, p_j) <= eps^2 as a (P, 2) int32 device
    tensor sorted by (i, j). points: (n, d) float64 CUDA tensor."""
    with Index(points, eps, stream=stream) as ix:
        return ix.join(unicomp=unicomp, precision=precision)


def bruteforce(points, eps: float, *, out=None, stream=None):
    """All-pairs join (no index, n^2 evaluations of the same pair test):
    (P, 2) int32 device tensor sorted by (i, j). points: (n, d) float64,
    host or device. With `out` (a contiguous int32 device tensor) the pairs
    go there in one call when it has room; without it the count pass runs
    twice (once to size the result)."""
    torch = _torch()
    L = _lib.load()
    ptr, n, d, on_dev, keep = _points_arg(points)
    total = ctypes.c_uint64(0)
    sh = _stream_handle(stream)
    if out is not None:
        if out.dtype != torch.int32 or not out.is_contiguous():
            raise ValueError("out must be a contiguous int32 tensor")
        rc = L.sj_bruteforce(ptr, n, d, float(eps), on_dev, ctypes.c_void_p(out.data_ptr()),
                             out.numel() // 2, sh, ctypes.byref(total))
        if rc == _lib.SJ_ECAPACITY:
            raise ValueError(f"out has room for {out.numel() // 2} pairs, the result has {total.value}")
        _lib.check(rc)
        P = int(total.value)
        del keep
        return out[:P] if out.shape[0] != P else out
    _lib.check(L.sj_bruteforce(ptr, n, d, float(eps), on_dev, None, 0, sh, ctypes.byref(total)))
    P = int(total.value)
    dev = points.device if getattr(points, "is_cuda", False) else torch.device("cuda")
    res = torch.empty((P, 2), dtype=torch.int32, device=dev)
    if P:
        _lib.check(L.sj_bruteforce(ptr, n, d, float(eps), on_dev, ctypes.c_void_p(res.data_ptr()), P, sh,
                                   ctypes.byref(total)))
    del keep
    return res


def dbscan_csr(row_off, cols, min_pts: int, stream=None):
    """DBSCAN labels (int32 device tensor, -1 = noise; a cluster is labelled
    by its smallest core index) and the cluster count, from a CSR neighbour
    table (row_off int64 (n + 1,), cols int32, device tensors)."""
    torch = _torch()
    n = int(row_off.shape[0]) - 1
    labels = torch.empty((max(n, 0),), dtype=torch.int32, device=row_off.device)
    nc = ctypes.c_uint64(0)
    _lib.check(_lib.load().sj_dbscan_csr(ctypes.c_void_p(row_off.data_ptr()), ctypes.c_void_p(cols.data_ptr()),
                                         n, int(min_pts), ctypes.c_void_p(labels.data_ptr()),
                                         _stream_handle(stream), ctypes.byref(nc)))
    return labels, int(nc.value)


def dbscan(points, eps: float, min_pts: int, stream=None):
    """DBSCAN of (n, d) float64 points (host or device) at radius eps:
    (labels int32 device tensor, number of clusters)."""
    torch = _torch()
    ptr, n, d, on_dev, keep = _points_arg(points)
    dev = points.device if getattr(points, "is_cuda", False) else torch.device("cuda")
    labels = torch.empty((n,), dtype=torch.int32, device=dev)
    nc = ctypes.c_uint64(0)
    _lib.check(_lib.load().sj_dbscan(ptr, n, d, float(eps), int(min_pts), on_dev,
                                     ctypes.c_void_p(labels.data_ptr()), _stream_handle(stream),
                                     ctypes.byref(nc)))
    del keep
    return labels, int(nc.value)


def last_run_stats() -> dict:
    """Statistics of the last join run on the calling thread."""
    return _lib.last_run_stats()


def band_thresholds(d: int, eps: float, extent: float):
    """(lo, hi) FP32 thresholds of the pre-test, or None if not usable."""
    lo, hi = ctypes.c_float(0), ctypes.c_float(0)
    rc = _lib.load().sj_band_thresholds(int(d), float(eps), float(extent), ctypes.byref(lo),
                                        ctypes.byref(hi))
    if rc != _lib.SJ_OK:
        return None
    return np.float32(lo.value), np.float32(hi.value)


def version() -> str:
    return _lib.load().sj_version().decode()
