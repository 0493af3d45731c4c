"""Error paths of the C ABI on the device: input validation, handle state, and
that a failed call leaves the library usable (no sticky device error)."""
import ctypes

import numpy as np
import pytest
import torch

from synth import clustered_cloud

pytestmark = pytest.mark.gpu

SF_E_INVALID, SF_E_STATE = 1, 4


def _lib():
    from paper_2010_11254_amd import _lib as L
    return L


def _say(*a):
    print("[gpu]", *a, flush=True)


def _cloud(dtype=np.float32):
    ps = clustered_cloud(3000, 8, seed=31, dtype=dtype)
    return ps, [torch.as_tensor(np.ascontiguousarray(v)).cuda() for v in (ps.x, ps.m, ps.h)]


def _status(fn):
    L = _lib()
    with pytest.raises(L.SfGravError) as ei:
        fn()
    return ei.value.status


@pytest.mark.parametrize("what", ["nan_pos", "inf_pos", "zero_h", "neg_h", "neg_m"])
def test_validate_rejects_bad_inputs(what):
    L = _lib()
    _say("validate", what)
    ps, (x, m, h) = _cloud()
    k = 1234
    if what == "nan_pos":
        x[k, 1] = float("nan")
    elif what == "inf_pos":
        x[k, 0] = float("inf")
    elif what == "zero_h":
        h[k] = 0.0
    elif what == "neg_h":
        h[k] = -1e-3
    else:
        m[k] = -1e-6
    o = L.make_opts(form="fp32c", n_gas=ps.n_gas, validate=True)
    assert _status(lambda: L.sf_grav_build_tree(x, m, h, o)) == SF_E_INVALID
    assert _status(lambda: L.sf_grav_accel(None, x, m, h, o)) == SF_E_INVALID
    ga = torch.ones((ps.n, 3), dtype=torch.float32, device="cuda")
    assert _status(lambda: L.sf_grav_accel_backward(None, x, m, h, o, ga)) == SF_E_INVALID
    torch.cuda.synchronize()


def test_library_usable_after_errors():
    # a rejected call, then the same valid evaluation twice: identical results
    L = _lib()
    _say("valid evaluation after a rejected one")
    ps, (x, m, h) = _cloud()
    o = L.make_opts(form="fp32c", n_gas=ps.n_gas, validate=True)
    t = L.sf_grav_build_tree(x, m, h, o)
    a0, p0 = L.sf_grav_accel(t, None, None, None, o)
    torch.cuda.synchronize()
    L.sf_grav_tree_free(t)
    hb = h.clone()
    hb[7] = 0.0
    assert _status(lambda: L.sf_grav_build_tree(x, m, hb, o)) == SF_E_INVALID
    t = L.sf_grav_build_tree(x, m, h, o)
    a1, p1 = L.sf_grav_accel(t, None, None, None, o)
    torch.cuda.synchronize()
    L.sf_grav_tree_free(t)
    assert torch.equal(a0, a1) and torch.equal(p0, p1)


def test_handle_state_errors():
    L = _lib()
    _say("handle state")
    ps, (x, m, h) = _cloud()
    o = L.make_opts(form="fp32c", n_gas=ps.n_gas)
    t = L.sf_grav_build_tree(x, m, h, o)
    acc = torch.empty((ps.n + 1, 3), dtype=torch.float32, device="cuda")
    pot = torch.empty((ps.n + 1,), dtype=torch.float32, device="cuda")
    st = L.lib().sf_grav_accel(t.handle, None, None, None, ctypes.c_int64(ps.n + 1), L.SF_F32,
                               ctypes.byref(o), ctypes.c_void_p(acc.data_ptr()),
                               ctypes.c_void_p(pot.data_ptr()), L._stream())
    assert st == SF_E_STATE
    st = L.lib().sf_grav_accel(t.handle, None, None, None, ctypes.c_int64(ps.n), L.SF_F64,
                               ctypes.byref(o), ctypes.c_void_p(acc.data_ptr()),
                               ctypes.c_void_p(pot.data_ptr()), L._stream())
    assert st == SF_E_STATE
    # interaction counts exist only when the walk collected them
    L.sf_grav_accel(t, None, None, None, o)
    assert _status(lambda: L.sf_grav_tree_export(t, "group_npc")) == SF_E_STATE
    # the handle still evaluates normally
    a, p = L.sf_grav_accel(t, None, None, None, o)
    torch.cuda.synchronize()
    assert torch.isfinite(a).all() and torch.isfinite(p).all()
    L.sf_grav_tree_free(t)
