"""The C ABI library loads and exports every symbol include/sj.h declares;
host-only entry points behave as documented (CPU, no device calls)."""
from __future__ import annotations

import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sj.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = set(re.findall(r"\b(sj_[a-z_0-9]+)\s*\(", text))
    names.discard("sj_run_cb")
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1803_04120_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_1803_04120_amd import build
        build.build()
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 15
    for name in names:
        assert hasattr(lib, name), f"{name} declared in sj.h but not exported"


def test_default_opts(lib):
    from paper_1803_04120_amd import _lib
    o = _lib.SjJoinOpts()
    lib.sj_default_opts(ctypes.byref(o))
    assert (o.unicomp, o.precision, o.batch_capacity_pairs, o.min_batches, o.sort_output) == (1, 0, 0, 1, 1)


@pytest.mark.parametrize("d,eps,extent", [(2, 0.04, 50.0), (2, 0.2, 50.0), (3, 0.9142, 50.0),
                                          (6, 13.0564, 50.0), (2, 0.0909, 67.0), (3, 0.491, 70.0)])
def test_band_thresholds_match_oracle_reading(lib, d, eps, extent):
    import paper_1803_04120_amd as sj
    from oracle import band
    got = sj.band_thresholds(d, eps, extent)
    want = band.thresholds(eps, d, extent)
    assert got is not None and want is not None
    assert got[0] == want[0] and got[1] == want[1]
    assert float(got[0]) < eps * eps < float(got[1])


def test_band_thresholds_unusable(lib):
    import paper_1803_04120_amd as sj
    assert sj.band_thresholds(3, 1e-9, 1e6) is None


@pytest.mark.parametrize("n,d,eps,msg", [(10, 0, 1.0, "d must be"), (10, 9, 1.0, "d must be"),
                                         (10, 2, 0.0, "eps"), (10, 2, float("nan"), "eps"),
                                         (10, 2, float("inf"), "eps"), (2 ** 32, 2, 1.0, "n must")])
def test_argument_errors_before_device_work(lib, n, d, eps, msg):
    from paper_1803_04120_amd import _lib
    h = ctypes.c_void_p()
    dummy = np.zeros(16)
    rc = lib.sj_build_index(ctypes.c_void_p(dummy.ctypes.data), n, d, eps, 0, None, ctypes.byref(h))
    assert rc == _lib.SJ_EINVAL
    assert msg in lib.sj_last_error().decode()
    assert not h.value


def test_null_arguments(lib):
    from paper_1803_04120_amd import _lib
    assert lib.sj_build_index(None, 10, 2, 1.0, 0, None, None) == _lib.SJ_EINVAL
    assert lib.sj_index_stats(None, None) == _lib.SJ_EINVAL
    lib.sj_destroy_index(None)
    lib.sj_free(None)


def test_profile_select_and_read_without_device_work(lib):
    from paper_1803_04120_amd import _lib
    _lib.profile_select("tiled_")
    _lib.profile_enable(True)
    assert _lib.profile_read() == {}
    _lib.profile_enable(False)
    _lib.profile_select("")
    assert lib.sj_profile_select(None) == 0
