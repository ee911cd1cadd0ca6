"""The allocation-free exchange-rule entry point (re_test_exchange_noalloc),
called through the C ABI: its decisions equal re_test_exchange's on the same
inputs, on two calls in a row (the second with fewer replicas, so that its
staging holds values of the first call past its own end), and a ladder past
its static limit is rejected."""
import ctypes as C

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def lib():
    from paper_0812_1633_amd import re as R
    L = R.lib()
    f = L.re_test_exchange_noalloc
    f.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_int, C.c_uint64, C.c_int64, C.c_int, C.c_void_p]
    f.restype = C.c_int
    return R, f


def ladder_case(g, R):
    T = np.cumsum(g.uniform(1e-3, 0.05, R)) + 0.5
    slot = g.permutation(R).astype(np.int32)
    U = g.normal(-3000, 2.0, R)
    return U, T, slot


def call(f, U, T, slot, seed, k, maxd):
    R = U.size
    dec = np.zeros(max(1, R - 1), np.uint8)
    rc = f(U.ctypes.data, T.ctypes.data, slot.ctypes.data, R, seed, k, maxd, dec.ctypes.data)
    return rc, dec[: R - 1]


def test_noalloc_matches_allocating_entry_point(lib):
    R, f = lib
    g = np.random.default_rng(123)
    for Rn, maxd in ((4096, 1), (37, 3)):
        U, T, slot = ladder_case(g, Rn)
        for k in (0, 1, 12345):
            rc, dec = call(f, U, T, slot, 99, k, maxd)
            assert rc == 0, R.lib().re_last_error(None)
            ref = R.re_test_exchange(U, T, slot, 99, k, maxd)
            assert np.array_equal(dec, ref), (Rn, k)
            assert set(np.unique(dec).tolist()) <= {0, 1, 255}


def test_noalloc_rejects_past_its_limit(lib):
    R, f = lib
    g = np.random.default_rng(5)
    U, T, slot = ladder_case(g, 4097)
    rc, _ = call(f, U, T, slot, 1, 0, 1)
    assert rc == R.RE_EINVAL
    assert b"4096" in R.lib().re_last_error(None)
