"""CPU-side checks of the C ABI: the library loads, exports every declared
symbol, sizes workspaces and rejects invalid parameters before any device
call (no GPU is needed for any of this)."""
import ctypes
import os
import re

import pytest

import workloads as wl

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "chfpe.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(chfpe_[a-z0-9_]+)\s*\(", txt)))


@pytest.fixture(scope="module")
def binding():
    import paper_2509_25840_amd as pk
    if not os.path.exists(pk.LIB_PATH):
        pytest.fail("libchfpe.so is not built (run __graft_entry__.build())")
    return pk


def test_header_declares_the_boundary():
    names = declared_functions()
    for fn in ("chfpe_setup", "chfpe_equilibrate", "chfpe_propagate", "chfpe_response_1d",
               "chfpe_response_2d", "chfpe_destroy", "chfpe_workspace_bytes"):
        assert fn in names


def test_library_exports_every_declared_symbol(binding):
    L = ctypes.CDLL(binding.LIB_PATH)
    missing = [fn for fn in declared_functions() if not hasattr(L, fn)]
    assert not missing, missing


def test_workspace_bytes_covers_eight_states(binding):
    w = wl.workload("two_mode_32")
    p = binding.params_from_workload(w)
    n = binding.workspace_bytes(p)
    state_bytes = 10 * 32 ** 4 * 8
    assert 7 * state_bytes <= n < 8 * state_bytes + (1 << 24)


@pytest.mark.parametrize("field,value", [
    ("M", 0), ("M", 4), ("K", -1), ("beta", 0.0), ("beta", -1.0), ("precision", 7),
])
def test_invalid_parameters_are_rejected_without_a_device(binding, field, value):
    w = wl.workload("two_mode_32")
    p = binding.params_from_workload(w)
    setattr(p, field, value)
    assert binding.workspace_bytes(p) == 0
    L = binding.lib()
    ctx = ctypes.c_void_p()
    rc = L.chfpe_setup(ctypes.byref(p), None, 0, None, ctypes.byref(ctx))
    assert rc == binding.CHFPE_EINVAL
    assert ctx.value is None
    assert len(L.chfpe_last_error(None)) > 0


def test_invalid_grid_sizes_are_rejected(binding):
    w = wl.workload("two_mode_32")
    for bad in ([4, 32], [32, 49]):
        p = binding.params_from_workload(w)
        p.Nq[0], p.Nq[1] = bad
        assert binding.workspace_bytes(p) == 0
    p = binding.params_from_workload(w)
    p.Lp[1] = 0.0
    assert binding.workspace_bytes(p) == 0
    p = binding.params_from_workload(w)
    p.g2[0][1] = float("nan")
    assert binding.workspace_bytes(p) == 0


def test_small_workspace_is_rejected(binding):
    w = wl.workload("one_mode_48")
    p = binding.params_from_workload(w)
    L = binding.lib()
    ctx = ctypes.c_void_p()
    fake = ctypes.c_void_p(1 << 20)  # never dereferenced: the size check comes first
    rc = L.chfpe_setup(ctypes.byref(p), fake, 16, None, ctypes.byref(ctx))
    assert rc == binding.CHFPE_ENOMEM


def test_null_context_calls_are_rejected(binding):
    L = binding.lib()
    assert L.chfpe_equilibrate(None, 1, 0.1) == binding.CHFPE_EINVAL
    assert L.chfpe_propagate(None, 1, 0.1) == binding.CHFPE_EINVAL
    assert L.chfpe_state_count(None) == 0
    assert L.chfpe_autotune(None, 1) == binding.CHFPE_EINVAL
    buf = (ctypes.c_int32 * 6)()
    assert L.chfpe_tile_config(None, buf, 6) == binding.CHFPE_EINVAL
    L.chfpe_destroy(None)
