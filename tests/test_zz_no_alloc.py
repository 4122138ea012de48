"""The allocation-free spectrum entry point (chfpe_spectrum_2d_noalloc)
against the allocating one (chfpe_spectrum_2d), through the C ABI: two
calls in a row on the same device scratch, the second with a smaller
input, each equal to the allocating call bit for bit (same kernels, same
summation order); sizes past the scratch are refused."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


@pytest.fixture(scope="module")
def abi():
    import torch
    import paper_2509_25840_amd as pk
    assert torch.cuda.is_available(), "GPU tests need a visible GPU"
    L = ctypes.CDLL(pk.LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    for name in ("chfpe_spectrum_2d_noalloc", "chfpe_spectrum_2d"):
        fn = getattr(L, name)
        fn.argtypes = [dp, ctypes.c_int64, ctypes.c_int64, ctypes.c_double, ctypes.c_double, dp, ctypes.c_void_p]
        fn.restype = ctypes.c_int
    return L


def test_noalloc_spectrum_equals_the_allocating_entry_point(abi):
    rng = np.random.default_rng(5)
    for n2, n1 in ((256, 128), (17, 9)):  # the second call is smaller
        R = np.ascontiguousarray(rng.standard_normal((n2, n1)))
        got = np.full_like(R, np.nan)
        ref = np.full_like(R, np.nan)
        print(f"[no-alloc] {n2} x {n1}", flush=True)
        assert abi.chfpe_spectrum_2d_noalloc(_dp(R), n1, n2, 0.005, 0.01, _dp(got), None) == 0
        assert abi.chfpe_spectrum_2d(_dp(R), n1, n2, 0.005, 0.01, _dp(ref), None) == 0
        assert np.all(np.isfinite(got))
        assert np.array_equal(got, ref)


def test_noalloc_spectrum_refuses_sizes_past_its_scratch(abi):
    R = np.zeros((1024, 129))
    I = np.zeros_like(R)
    assert abi.chfpe_spectrum_2d_noalloc(_dp(R), 129, 1024, 0.005, 0.01, _dp(I), None) == -1  # EINVAL
    assert not I.any()
