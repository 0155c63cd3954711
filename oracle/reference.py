"""Oracle for the epsilon self-join: the problem's definition written out.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU-baseline leg, never by the product path. Shares no code with
the HIP implementation.

Definition followed (Section III, problem statement; both orders of a pair
are reported as in Section V-B): R(X, eps) is the set of ordered pairs (i, j)
of row indices with

    d2(i, j) <= fl(eps * eps),
    d2(i, j) = (...(t_0*t_0 + t_1*t_1) + ...) + t_{d-1}*t_{d-1},
    t_k = X[i, k] - X[j, k],

evaluated in binary64, dimension order 0..d-1, each operation rounded
separately. The paper states the test as sqrt(sum) <= eps; the oracle uses
the squared form, which is its reading of that test (the two can differ only
when d2 and eps^2 are within an ulp of each other). Pairs are returned sorted
by (i, j) as an (P, 2) int64 array.

Three independent spellings are provided:
  * pairs_python: pure Python floats and loops (tiny inputs only);
  * pairs_numpy:  numpy, vectorised over candidates (small inputs);
  * pairs / count_rows / rows_pairs: the C brute force in sj_oracle.c
    (OpenMP), for anything bigger.

join_rs_numpy is the same predicate between two sets, R x S (the join the
self-join specialises, Section II), for the two-set join to come.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        lib = ctypes.CDLL(_LIB_PATH)
        i64, dbl, vp = ctypes.c_int64, ctypes.c_double, ctypes.c_void_p
        lib.sjo_count_rows.restype = i64
        lib.sjo_count_rows.argtypes = [vp, i64, i64, dbl, vp, i64, vp]
        lib.sjo_fill_rows.restype = None
        lib.sjo_fill_rows.argtypes = [vp, i64, i64, dbl, vp, i64, vp, vp]
        lib.sjo_count_rows_multi.restype = None
        lib.sjo_count_rows_multi.argtypes = [vp, i64, i64, vp, i64, vp, i64, vp]
        lib.sjo_d2.restype = dbl
        lib.sjo_d2.argtypes = [vp, i64, i64, i64]
        lib.sjg_grid_join.restype = i64
        lib.sjg_grid_join.argtypes = [vp, i64, i64, dbl, vp, vp]
        _lib = lib
    return _lib


def _as_points(x) -> np.ndarray:
    x = np.ascontiguousarray(np.asarray(x, dtype=np.float64))
    if x.ndim != 2:
        raise ValueError("points must be an (n, d) array")
    return x


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


# --------------------------------------------------------------------------
# pure Python: the definition with plain floats
# --------------------------------------------------------------------------
def d2_python(a, b) -> float:
    acc = 0.0
    for ak, bk in zip(a, b):
        t = float(ak) - float(bk)
        acc = acc + t * t
    return acc


def pairs_python(points, eps: float):
    """Sorted list of (i, j) with d2 <= eps*eps, by two nested loops."""
    pts = [tuple(float(v) for v in row) for row in np.asarray(points, dtype=np.float64)]
    eps2 = float(eps) * float(eps)
    out = []
    for i, a in enumerate(pts):
        for j, b in enumerate(pts):
            if d2_python(a, b) <= eps2:
                out.append((i, j))
    return out


# --------------------------------------------------------------------------
# numpy: same definition, vectorised over the candidate j
# --------------------------------------------------------------------------
def pairs_numpy(points, eps: float) -> np.ndarray:
    x = _as_points(points)
    n, d = x.shape
    eps2 = float(eps) * float(eps)
    rows = []
    for i in range(n):
        acc = np.zeros(n, dtype=np.float64)
        for k in range(d):
            t = x[i, k] - x[:, k]
            acc = acc + t * t
        js = np.nonzero(acc <= eps2)[0]
        rows.append(np.stack([np.full(js.shape, i, dtype=np.int64), js.astype(np.int64)], axis=1))
    if not rows:
        return np.zeros((0, 2), dtype=np.int64)
    return np.concatenate(rows, axis=0)


# --------------------------------------------------------------------------
# C brute force
# --------------------------------------------------------------------------
def count_rows(points, eps: float, rows=None) -> np.ndarray:
    """Neighbour count (self included) of each query row (all rows if None)."""
    x = _as_points(points)
    n, d = x.shape
    r = None if rows is None else np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    nrows = n if r is None else r.shape[0]
    counts = np.zeros(nrows, dtype=np.int64)
    if nrows:
        _load().sjo_count_rows(_ptr(x), n, d, float(eps), _ptr(r), nrows, _ptr(counts))
    return counts


def rows_neighbors(points, eps: float, rows=None):
    """(row_offsets[nrows+1], neighbours) for the query rows, each row's
    neighbours ascending. Memory is sum of counts * 4 bytes."""
    x = _as_points(points)
    n, d = x.shape
    r = None if rows is None else np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    nrows = n if r is None else r.shape[0]
    counts = count_rows(x, eps, r)
    off = np.zeros(nrows + 1, dtype=np.int64)
    np.cumsum(counts, out=off[1:])
    out_j = np.zeros(int(off[-1]), dtype=np.uint32)
    if nrows:
        _load().sjo_fill_rows(_ptr(x), n, d, float(eps), _ptr(r), nrows, _ptr(off), _ptr(out_j))
    return off, out_j


def pairs(points, eps: float) -> np.ndarray:
    """All pairs sorted by (i, j) as an (P, 2) int64 array (C brute force)."""
    x = _as_points(points)
    n = x.shape[0]
    off, js = rows_neighbors(x, eps)
    ii = np.repeat(np.arange(n, dtype=np.int64), np.diff(off))
    return np.stack([ii, js.astype(np.int64)], axis=1)


def count_rows_multi(points, eps_list, rows) -> np.ndarray:
    """counts[r, e] = neighbours of rows[r] within eps_list[e] (ascending)."""
    x = _as_points(points)
    n, d = x.shape
    e = np.ascontiguousarray(np.asarray(eps_list, dtype=np.float64))
    if np.any(np.diff(e) < 0):
        raise ValueError("eps_list must be ascending")
    r = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    counts = np.zeros((r.shape[0], e.shape[0]), dtype=np.int64)
    _load().sjo_count_rows_multi(_ptr(x), n, d, _ptr(e), e.shape[0], _ptr(r), r.shape[0], _ptr(counts))
    return counts


def d2(points, i: int, j: int) -> float:
    x = _as_points(points)
    return float(_load().sjo_d2(_ptr(x), x.shape[1], int(i), int(j)))


# --------------------------------------------------------------------------
# CPU grid join (host-core baseline; checked against the brute force)
# --------------------------------------------------------------------------
def grid_join(points, eps: float, with_pairs: bool = True):
    """The grid self-join of cpu_grid_join.c on the host's cores:
    (row counts, pairs sorted by (i, j) as (P, 2) int32 or None)."""
    x = _as_points(points)
    n, d = x.shape
    counts = np.zeros(n, dtype=np.int64)
    if n == 0:
        return counts, (np.zeros((0, 2), dtype=np.int32) if with_pairs else None)
    total = _load().sjg_grid_join(_ptr(x), n, d, float(eps), _ptr(counts), None)
    if total < 0:
        raise MemoryError("grid join: allocation failed")
    if not with_pairs:
        return counts, None
    out = np.zeros((int(total), 2), dtype=np.int32)
    got = _load().sjg_grid_join(_ptr(x), n, d, float(eps), _ptr(counts), _ptr(out))
    if got != total:
        raise RuntimeError("grid join: count and fill disagree")
    return counts, out


# --------------------------------------------------------------------------
# distance join of two sets (the operation the self-join specialises)
# --------------------------------------------------------------------------
def join_rs_numpy(r_points, s_points, eps: float) -> np.ndarray:
    """Sorted (i, j) pairs, i a row of R and j a row of S, with the same
    predicate as the self-join (d2 in binary64, dimension order 0..d-1, each
    operation rounded, d2 <= fl(eps * eps)). Section II places the self-join
    as the special case R = S of this join; Section III gives the predicate.
    Vectorised over the rows of S (small inputs)."""
    r = _as_points(r_points)
    s = _as_points(s_points)
    if r.shape[0] and s.shape[0] and r.shape[1] != s.shape[1]:
        raise ValueError("R and S must have the same dimension")
    eps2 = float(eps) * float(eps)
    rows = []
    for i in range(r.shape[0]):
        acc = np.zeros(s.shape[0], dtype=np.float64)
        with np.errstate(over="ignore"):  # a far query's d2 is +inf: not within eps
            for k in range(r.shape[1]):
                t = r[i, k] - s[:, k]
                acc = acc + t * t
        js = np.nonzero(acc <= eps2)[0]
        rows.append(np.stack([np.full(js.shape, i, dtype=np.int64), js.astype(np.int64)], axis=1))
    if not rows:
        return np.zeros((0, 2), dtype=np.int64)
    return np.concatenate(rows, axis=0)

