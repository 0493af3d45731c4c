"""CPU-side checks of the C-ABI library: it loads, and it exports every
function that include/sf_grav.h declares (no compute call without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "sf_grav.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(sf_grav_\w+)\s*\(", src)))


def test_header_declares_entry_points():
    names = _declared()
    for required in ("sf_grav_build_tree", "sf_grav_accel", "sf_grav_accel_backward",
                     "sf_grav_tree_free"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2010_11254_amd import _lib
    L = _lib.lib()
    for name in _declared():
        assert hasattr(L, name), name
        assert isinstance(getattr(L, name), ctypes._CFuncPtr)


def test_opts_layout_and_defaults():
    from paper_2010_11254_amd import _lib
    o = _lib.make_opts()
    assert o.struct_size == ctypes.sizeof(_lib.sf_grav_opts) == 64
    assert (o.theta, o.order, o.leaf_cap, o.group_cap, o.form) == (0.5, 2, 32, 32, 0)
    assert o.alpha == -1.0          # relative criterion off by default
    assert ctypes.sizeof(_lib.sf_grav_stats) == 8 + 5 * 8 + 32 * 8 + 8


def test_strerror_and_invalid_arguments_without_device():
    from paper_2010_11254_amd import _lib
    L = _lib.lib()
    assert L.sf_grav_strerror(1) == b"invalid argument"
    o = _lib.make_opts()
    h = ctypes.c_void_p()
    # argument checks happen before anything touches the device
    st = L.sf_grav_build_tree(None, None, None, 10, 0, ctypes.byref(o), None, ctypes.byref(h))
    assert st == _lib.SF_E_INVALID and not h.value
    assert b"non-NULL" in L.sf_grav_last_error()
    p = ctypes.c_void_p(16)
    st = L.sf_grav_build_tree(p, p, p, 0, 0, ctypes.byref(o), None, ctypes.byref(h))
    assert st == _lib.SF_E_INVALID
    bad = _lib.make_opts(theta=-1.0)
    st = L.sf_grav_build_tree(p, p, p, 10, 0, ctypes.byref(bad), None, ctypes.byref(h))
    assert st == _lib.SF_E_INVALID and b"theta" in L.sf_grav_last_error()
    bad = _lib.make_opts(leaf_cap=65)
    assert L.sf_grav_build_tree(p, p, p, 10, 0, ctypes.byref(bad), None, ctypes.byref(h)) == 1
    bad = _lib.make_opts(order=1)
    assert L.sf_grav_accel(None, p, p, p, 10, 0, ctypes.byref(bad), p, p, None) == 1
    bad = _lib.make_opts(n_gas=11)
    assert L.sf_grav_accel(None, p, p, p, 10, 0, ctypes.byref(bad), p, p, None) == 1
    o2 = _lib.make_opts()
    o2.struct_size = 8
    assert L.sf_grav_accel(None, p, p, p, 10, 0, ctypes.byref(o2), p, p, None) == 1
    assert L.sf_grav_accel(None, p, p, p, 10, 7, ctypes.byref(o), p, p, None) == 1
    assert L.sf_grav_accel(None, p, p, p, 10, 0, ctypes.byref(o), None, p, None) == 1
    assert L.sf_grav_tree_free(None) == 0
    bad = _lib.make_opts(alpha=float("nan"))
    assert L.sf_grav_accel(None, p, p, p, 10, 0, ctypes.byref(bad), p, p, None) == 1
    assert b"alpha" in L.sf_grav_last_error()
    # the new handle calls reject NULL before touching anything
    assert L.sf_grav_tree_set_field(None, p, None) == 1
    assert L.sf_grav_tree_refit(None, p, p, p, None) == 1
    assert L.sf_grav_get_stats(None, None) == 1
