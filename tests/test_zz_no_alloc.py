"""The allocation-free brute force (sj_bruteforce_noalloc), called through
the C ABI, against the allocating entry point (sj_bruteforce) on the same
inputs: bit-exact pairs on two calls in a row, the second smaller (the
fixed scratch array keeps the first call's contents, which must not leak
into the second), plus its documented errors."""
from __future__ import annotations

import ctypes

import numpy as np
import pytest

from paper_1803_04120_amd import datagen

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def lib():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1803_04120_amd import _lib
    return _lib.load()


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _noalloc(lib, x, eps, out):
    total = ctypes.c_uint64(0)
    rc = lib.sj_bruteforce_noalloc(ctypes.c_void_p(x.data_ptr()), x.shape[0], x.shape[1], float(eps),
                                   ctypes.c_void_p(out.data_ptr()), out.shape[0], _stream(), ctypes.byref(total))
    return rc, int(total.value)


def test_noalloc_equals_allocating_on_two_calls(lib):
    import paper_1803_04120_amd as sj
    for n, d, eps, seed in ((300_000, 3, 1.2, 801), (40_000, 5, 14.0, 802)):
        print(f"[case] noalloc brute n={n} d={d} eps={eps}", flush=True)
        x = torch.from_numpy(datagen.uniform(n, d, seed)).cuda()
        want = sj.bruteforce(x, eps)
        P = want.shape[0]
        out = torch.full((P + 257, 2), -7, dtype=torch.int32, device="cuda")
        rc, total = _noalloc(lib, x, eps, out)
        assert rc == 0, lib.sj_last_error().decode()
        torch.cuda.synchronize()
        assert total == P
        assert torch.equal(out[:P], want)
        assert bool((out[P:] == -7).all())  # nothing written past the result


def test_noalloc_errors(lib):
    from paper_1803_04120_amd import _lib
    x = torch.from_numpy(datagen.uniform(5000, 2, 803)).cuda()
    out = torch.empty((4, 2), dtype=torch.int32, device="cuda")
    rc, total = _noalloc(lib, x, 3.0, out)  # more pairs than the buffer holds
    assert rc == _lib.SJ_ECAPACITY and total > 5000
    big = ctypes.c_uint64(0)
    rc = lib.sj_bruteforce_noalloc(ctypes.c_void_p(x.data_ptr()), (1 << 21) + 1, 2, 1.0,
                                   ctypes.c_void_p(out.data_ptr()), 4, _stream(), ctypes.byref(big))
    assert rc == _lib.SJ_EINVAL and "at most" in lib.sj_last_error().decode()
    rc = lib.sj_bruteforce_noalloc(ctypes.c_void_p(x.data_ptr()), 5000, 9, 1.0,
                                   ctypes.c_void_p(out.data_ptr()), 4, _stream(), ctypes.byref(big))
    assert rc == _lib.SJ_EINVAL
