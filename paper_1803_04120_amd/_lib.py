"""ctypes binding of libsj.so (the C ABI declared in include/sj.h).

Argument marshalling only: every step of the join runs in the HIP library.
If the library has not been built the import of a function fails loudly;
there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsj.so")

SJ_OK = 0
SJ_EINVAL = -1
SJ_ENOMEM = -2
SJ_EGRID = -3
SJ_EDEVICE = -4
SJ_ESTATE = -5
SJ_ECAPACITY = -6

SJ_FP64 = 0
SJ_FP32_BAND = 1

SJ_EXPORT_CELL_IDS = 1
SJ_EXPORT_CELL_START = 2
SJ_EXPORT_PERM = 3
SJ_EXPORT_MASKS = 4
SJ_EXPORT_RANGE_OFF = 5
SJ_EXPORT_RANGES = 6
SJ_EXPORT_GRID = 7
SJ_EXPORT_ROW_OFFSETS = 8

_ERRNAMES = {SJ_EINVAL: "SJ_EINVAL", SJ_ENOMEM: "SJ_ENOMEM", SJ_EGRID: "SJ_EGRID",
             SJ_EDEVICE: "SJ_EDEVICE", SJ_ESTATE: "SJ_ESTATE", SJ_ECAPACITY: "SJ_ECAPACITY"}


class SjJoinOpts(ctypes.Structure):
    _fields_ = [("unicomp", ctypes.c_int32),
                ("precision", ctypes.c_int32),
                ("batch_capacity_pairs", ctypes.c_uint64),
                ("min_batches", ctypes.c_uint32),
                ("sort_output", ctypes.c_int32)]


class SjStats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64),
                ("d", ctypes.c_uint32),
                ("key_bits", ctypes.c_uint32),
                ("cells", ctypes.c_uint64),
                ("grid_dims", ctypes.c_uint64 * 8),
                ("eps", ctypes.c_double),
                ("cell_width", ctypes.c_double),
                ("max_cell_points", ctypes.c_uint32),
                ("precision_used", ctypes.c_uint32),
                ("ranges", ctypes.c_uint64),
                ("evals", ctypes.c_uint64),
                ("band_rechecks", ctypes.c_uint64),
                ("pairs", ctypes.c_uint64),
                ("max_row_pairs", ctypes.c_uint64),
                ("batches", ctypes.c_uint32),
                ("unicomp_used", ctypes.c_uint32),
                ("ms_build", ctypes.c_double),
                ("ms_count", ctypes.c_double),
                ("ms_fill", ctypes.c_double),
                ("chunks", ctypes.c_uint64),
                ("fill_unicomp", ctypes.c_uint32),
                ("reserved0", ctypes.c_uint32),
                ("hit_bit_bytes", ctypes.c_uint64)]


class SjKernelTime(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48),
                ("launches", ctypes.c_uint64),
                ("total_ms", ctypes.c_double)]


RUN_CB = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64,
                          ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64)

_lib = None


class SjError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


def load():
    """Load libsj.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -c 'import __graft_entry__ as g; g.build()'`")
    L = ctypes.CDLL(LIB_PATH)
    vp, u64, u32, i32, dbl = (ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32,
                              ctypes.c_int32, ctypes.c_double)
    pidx = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "sj_default_opts": (None, [ctypes.POINTER(SjJoinOpts)]),
        "sj_build_index": (ctypes.c_int, [vp, u64, u32, dbl, ctypes.c_int, vp, pidx]),
        "sj_destroy_index": (None, [vp]),
        "sj_join_count": (ctypes.c_int, [vp, ctypes.POINTER(SjJoinOpts), vp,
                                         ctypes.POINTER(ctypes.c_uint64)]),
        "sj_join_fill": (ctypes.c_int, [vp, vp, u64, vp]),
        "sj_join_fill_csr": (ctypes.c_int, [vp, vp, vp, u64, vp]),
        "sj_dbscan_csr": (ctypes.c_int, [vp, vp, u64, u32, vp, vp, ctypes.POINTER(u64)]),
        "sj_dbscan": (ctypes.c_int, [vp, u64, u32, dbl, u32, ctypes.c_int, vp, vp, ctypes.POINTER(u64)]),
        "sj_join_rs": (ctypes.c_int, [vp, vp, u64, ctypes.c_int, vp, u64, vp, ctypes.POINTER(u64)]),
        "sj_join_rs_count": (ctypes.c_int, [vp, vp, u64, ctypes.c_int, vp, ctypes.POINTER(u64)]),
        "sj_join_rs_fill": (ctypes.c_int, [vp, vp, u64, vp]),
        "sj_selfjoin_index": (ctypes.c_int, [vp, ctypes.POINTER(SjJoinOpts), RUN_CB, vp, vp,
                                             ctypes.POINTER(ctypes.c_uint64)]),
        "sj_selfjoin": (ctypes.c_int, [vp, u64, u32, dbl, ctypes.POINTER(SjJoinOpts), ctypes.c_int,
                                       ctypes.c_int, vp, ctypes.POINTER(ctypes.c_void_p),
                                       ctypes.POINTER(ctypes.c_uint64)]),
        "sj_free": (None, [vp]),
        "sj_index_stats": (ctypes.c_int, [vp, ctypes.POINTER(SjStats)]),
        "sj_last_run_stats": (ctypes.c_int, [ctypes.POINTER(SjStats)]),
        "sj_bruteforce": (ctypes.c_int, [vp, u64, u32, dbl, ctypes.c_int, vp, u64, vp, ctypes.POINTER(u64)]),
        "sj_bruteforce_noalloc": (ctypes.c_int, [vp, u64, u32, dbl, vp, u64, vp, ctypes.POINTER(u64)]),
        "sj_index_export_size": (ctypes.c_int, [vp, ctypes.c_int, ctypes.POINTER(ctypes.c_uint64)]),
        "sj_index_export": (ctypes.c_int, [vp, ctypes.c_int, vp, u64]),
        "sj_index_search": (ctypes.c_int, [vp, ctypes.c_int, vp]),
        "sj_band_thresholds": (ctypes.c_int, [u32, dbl, dbl, ctypes.POINTER(ctypes.c_float),
                                              ctypes.POINTER(ctypes.c_float)]),
        "sj_memory_info": (ctypes.c_int, [ctypes.POINTER(u64), ctypes.POINTER(u64)]),
        "sj_release_cached_memory": (ctypes.c_int, []),
        "sj_profile_enable": (ctypes.c_int, [ctypes.c_int]),
        "sj_profile_select": (ctypes.c_int, [ctypes.c_char_p]),
        "sj_profile_read": (ctypes.c_int, [ctypes.POINTER(SjKernelTime), u32,
                                           ctypes.POINTER(ctypes.c_uint32)]),
        "sj_last_error": (ctypes.c_char_p, []),
        "sj_version": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    del i32
    _lib = L
    return L


def check(rc: int):
    if rc != SJ_OK:
        msg = load().sj_last_error().decode(errors="replace")
        raise SjError(rc, msg)


def opts(unicomp: bool = True, precision: str = "fp64", batch_capacity_pairs: int = 0,
         min_batches: int = 1, sort_output: bool = True) -> SjJoinOpts:
    o = SjJoinOpts()
    load().sj_default_opts(ctypes.byref(o))
    o.unicomp = 1 if unicomp else 0
    if precision in ("fp64", SJ_FP64):
        o.precision = SJ_FP64
    elif precision in ("fp32_band", "fp32", SJ_FP32_BAND):
        o.precision = SJ_FP32_BAND
    else:
        raise ValueError(f"unknown precision {precision!r}")
    o.batch_capacity_pairs = int(batch_capacity_pairs or 0)
    o.min_batches = int(max(1, min_batches))
    o.sort_output = 1 if sort_output else 0
    return o


def stats_dict(st: SjStats) -> dict:
    out = {}
    for name, _ in SjStats._fields_:
        v = getattr(st, name)
        if name == "grid_dims":
            v = [int(x) for x in v][: st.d]
        out[name] = v
    return out


def last_run_stats() -> dict:
    """Statistics of the last join run on this thread (sj_last_run_stats)."""
    st = SjStats()
    check(load().sj_last_run_stats(ctypes.byref(st)))
    return stats_dict(st)


def memory_info() -> dict:
    """Device bytes the library holds: cached for reuse and live."""
    c, l = ctypes.c_uint64(0), ctypes.c_uint64(0)
    check(load().sj_memory_info(ctypes.byref(c), ctypes.byref(l)))
    return {"cached_bytes": int(c.value), "live_bytes": int(l.value)}


def release_cached_memory():
    """Free the library's cached device blocks (waits for the device)."""
    check(load().sj_release_cached_memory())


def profile_enable(on: bool = True):
    load().sj_profile_enable(1 if on else 0)


def profile_select(prefix: str = ""):
    """Time only kernels whose name starts with prefix ("" = all)."""
    load().sj_profile_select(prefix.encode() if prefix else None)


def profile_read() -> dict:
    """{kernel name: (launches, total_ms)} recorded since profile_enable."""
    L = load()
    cnt = ctypes.c_uint32(0)
    L.sj_profile_read(None, 0, ctypes.byref(cnt))
    recs = (SjKernelTime * max(1, cnt.value))()
    L.sj_profile_read(recs, cnt.value, ctypes.byref(cnt))
    return {recs[i].name.decode(): (int(recs[i].launches), float(recs[i].total_ms))
            for i in range(cnt.value)}
