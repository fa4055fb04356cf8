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
    # dr_ct_field: int, int, 4 ptr; dr_ct_options: double, 4 int, double
    assert ctypes.sizeof(binding.dr_ct_field) == 40
    assert ctypes.sizeof(binding.dr_ct_options) == 32


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
    assert lib.dr_reach_ct(N, N, N, N, N, N, N, N) == binding.DR_EINVAL


def test_ct_arguments_are_checked_before_any_device_call():
    """dr_flowpipe_ct validates the field and the options on the host (the device
    pointers are only passed on, never read here)."""
    if not os.path.exists(binding.LIB_PATH):
        pytest.skip("library not built")
    lib = binding.load()
    fake = 0x1000
    f = binding.dr_ct_field(n=3, n_u=0, a=fake, F=fake, G=None, Q=None)
    o = binding.dr_ct_options(h=0.1, steps=2, intervals=1, tries=40, rounds=3, eps=1e-9)
    call = lambda f, o: lib.dr_flowpipe_ct(ctypes.byref(f), ctypes.byref(o), 0, None, None, None, None, None, None)
    assert lib.dr_flowpipe_ct(None, None, 0, None, None, None, None, None, None) == binding.DR_EINVAL
    assert call(f, o) == binding.DR_OK                       # an empty batch launches nothing
    bad = [("h", -1.0, binding.DR_EINVAL), ("h", float("inf"), binding.DR_EINVAL), ("steps", 0, binding.DR_EINVAL),
           ("intervals", -1, binding.DR_EINVAL), ("tries", 0, binding.DR_EINVAL), ("rounds", 101, binding.DR_EINVAL),
           ("eps", 0.0, binding.DR_EINVAL)]
    for name, v, want in bad:
        o2 = binding.dr_ct_options(h=0.1, steps=2, intervals=1, tries=40, rounds=3, eps=1e-9)
        setattr(o2, name, v)
        assert call(f, o2) == want, name
        assert name.encode() in lib.dr_last_error(None)
    for kw, want in ((dict(n=17), binding.DR_ESHAPE), (dict(n=0), binding.DR_ESHAPE), (dict(n_u=1), binding.DR_EINVAL),
                     (dict(F=None), binding.DR_EINVAL)):
        f2 = binding.dr_ct_field(n=3, n_u=0, a=fake, F=fake, G=None, Q=None)
        for k, v in kw.items():
            setattr(f2, k, v)
        assert call(f2, o) == want, kw
    f3 = binding.dr_ct_field(n=3, n_u=1, a=fake, F=fake, G=fake, Q=None)
    assert call(f3, o) == binding.DR_EINVAL                  # the flowpipe takes no input
    assert b"n_u = 0" in lib.dr_last_error(None)
