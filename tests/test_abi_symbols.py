"""The C-ABI library loads on the host and exports every entry point the header
declares (no compute calls: those need a GPU)."""
import ctypes
import os
import re

import pytest

from paper_2605_25346_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "diffreach.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(dr_[a-z_]+)\s*\(", src)))


def test_header_declares_binding_names():
    assert declared_symbols() == sorted(binding.EXPORTED)


def test_library_exports_every_symbol():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built in this checkout (run __graft_entry__.build())")
    lib = ctypes.CDLL(binding.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    binding.load()


def test_struct_layouts():
    # dr_network: int, ptr, int, ptr, ptr, ptr, ptr, int, ptr, int (LP64 natural alignment)
    assert ctypes.sizeof(binding.dr_network) == 80
    assert ctypes.sizeof(binding.dr_batch) == 48
    assert ctypes.sizeof(binding.dr_options) == 28


def test_last_error_without_context():
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = binding.load()
    assert isinstance(lib.dr_last_error(None), bytes)
    # argument validation happens before any device call
    st = lib.dr_create(None, None, 0, None, None)
    assert st == binding.DR_EINVAL
    assert b"NULL" in lib.dr_last_error(None)


def test_null_context_is_rejected_before_any_device_call():
    """Every entry point that takes a context returns DR_EINVAL for a NULL one (and
    the size query 0) without touching a device."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = binding.load()
    N = None
    assert lib.dr_bound_init(N, N, N, N) == binding.DR_EINVAL
    assert lib.dr_propagate_backward(N, N, N, N, N, N) == binding.DR_EINVAL
    assert lib.dr_optimize_duals(N, 0, 0.0, 0, N, N, N, N, N, N, N, N) == binding.DR_EINVAL
    assert lib.dr_param_grad(N, N, N, 0, N, N, N, N, N, N, N, N, N, 0, N, N) == binding.DR_EINVAL
    assert lib.dr_param_grad_static(N, N, N, 0, N, N, N, N, N, N, N, N, N, N) == binding.DR_EINVAL
    assert lib.dr_set_weights(N, 0, N, N) == binding.DR_EINVAL
    assert lib.dr_param_grad_workspace(N, 16) == 0
    assert lib.dr_reach_dt(N, N, 1, N, N, N) == binding.DR_EINVAL
    assert lib.dr_reach_dt_joint(N, N, 1, N, N, N, N, N) == binding.DR_EINVAL
    assert lib.dr_reach_dt_grad(N, N, 1, N, N, N, N, N, N, N, N, N, N, N, 0, N, N) == binding.DR_EINVAL
    assert lib.dr_reach_grad_workspace(N, 4, 2) == 0
    assert lib.dr_hidden_max(N) == 0 and lib.dr_spec_rows(N) == 0
