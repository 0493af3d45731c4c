"""The allocation-free direct entry point against sf_grav_accel's direct path.

sf_grav_accel_direct_noalloc runs the same kernels with its scratch in a
fixed device array, so its outputs must equal the allocating entry point's
bit for bit; two calls in a row (the second smaller) check that nothing
left in the shared array by the first call leaks into the second.
"""
import ctypes

import numpy as np
import pytest
import torch

from synth import clustered_cloud, uniform_sphere

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2010_11254_amd import _lib
    return _lib


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(ps):
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    return d(ps.x), d(ps.m), d(ps.h)


def _both(ps, form):
    L = _lib()
    x, m, h = _dev(ps)
    o = L.make_opts(form=form, n_gas=ps.n_gas)
    a0, p0 = L.sf_grav_accel(None, x, m, h, o)
    a1 = torch.full_like(a0, float("nan"))
    p1 = torch.full_like(p0, float("nan"))
    st = L.lib().sf_grav_accel_direct_noalloc(
        ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(m.data_ptr()), ctypes.c_void_p(h.data_ptr()),
        ps.n, L._dt(x), ctypes.byref(o), ctypes.c_void_p(a1.data_ptr()),
        ctypes.c_void_p(p1.data_ptr()), L._stream())
    assert st == L.SF_OK, L.lib().sf_grav_last_error()
    torch.cuda.synchronize()
    return (a0.cpu().numpy(), p0.cpu().numpy()), (a1.cpu().numpy(), p1.cpu().numpy())


@pytest.mark.parametrize("form,dtype", [("fp32c", np.float32), ("fp32", np.float32),
                                        ("fp64", np.float64)])
def test_noalloc_equals_direct_two_calls(form, dtype):
    # first call larger, with sinks; second smaller, without
    for ps in (clustered_cloud(30000, 57, seed=41, dtype=dtype),
               uniform_sphere(1000, seed=42, dtype=dtype)):
        _say("noalloc", form, "n =", ps.n, "sinks", ps.n_sink)
        ref, got = _both(ps, form)
        assert np.array_equal(ref[0], got[0]) and np.array_equal(ref[1], got[1])


def test_noalloc_largest_size():
    # n = 2^19 in the form with the largest scratch (FP64 inputs and form,
    # half sinks) fits the fixed array; compared on a sample of rows
    n = 1 << 19
    ps = uniform_sphere(n, seed=43, dtype=np.float64, h=0.01)
    ps.n_gas = n // 2
    _say("noalloc fp64 n =", n)
    L = _lib()
    x, m, h = _dev(ps)
    o = L.make_opts(form="fp64", n_gas=ps.n_gas)
    a1, p1 = L.sf_grav_accel_direct_noalloc(x, m, h, o)
    a0, p0 = L.sf_grav_accel(None, x, m, h, o)
    torch.cuda.synchronize()
    assert torch.equal(a0, a1) and torch.equal(p0, p1)


def test_noalloc_rejects_oversize():
    L = _lib()
    o = L.make_opts()
    p = ctypes.c_void_p(16)
    st = L.lib().sf_grav_accel_direct_noalloc(p, p, p, (1 << 19) + 1, 0, ctypes.byref(o), p, p, None)
    assert st == L.SF_E_UNSUPPORTED
    assert b"allocation-free maximum" in L.lib().sf_grav_last_error()
