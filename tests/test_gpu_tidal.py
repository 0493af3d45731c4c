"""GPU parity of the tidal tensor and jerk (sf_grav_accel_tidal) against the
oracle: the tree's frozen-list evaluation (monopole node terms, softened
pairs, exact sink-sink sums) on the same lists, and the direct sum at
theta = 0.  Velocities are seeded normals; the previous field of the
relative criterion is the oracle's direct field."""
import numpy as np
import pytest
import torch

from oracle import direct as odirect
from oracle import tree as otree
from synth import clustered_cloud, uniform_sphere

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2010_11254_amd import _lib
    return _lib


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a)).cuda() for a in arrs]


def _rowerr(a, ref):
    return np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)


def gpu_tidal(ps, v, form, theta, order=2, alpha=None, field=None, leaf_cap=16, group_cap=32):
    L = _lib()
    x, m, h, vv = _dev(ps.x, ps.m, ps.h, v)
    o = L.make_opts(form=form, theta=theta, order=order, leaf_cap=leaf_cap, group_cap=group_cap,
                    n_gas=ps.n_gas, alpha=alpha)
    t = L.sf_grav_build_tree(x, m, h, o)
    if alpha is not None:
        L.sf_grav_tree_set_field(t, _dev(field)[0])
    a, p, tid, jerk = L.sf_grav_accel_tidal(t, o, vel=vv)
    a0, p0 = L.sf_grav_accel(t, None, None, None, o)
    torch.cuda.synchronize()
    L.sf_grav_tree_free(t)
    out = [u.double().cpu().numpy() for u in (a, p, tid, jerk, a0, p0)]
    return out


@pytest.mark.parametrize("form,order,alpha", [("fp64", 2, None), ("fp64", 0, 0.002),
                                              ("fp32c", 2, 0.005), ("fp32", 2, None)])
def test_tidal_tree_matches_oracle_lists(form, order, alpha):
    _say("tidal tree", form, "order", order, "alpha", alpha)
    dtype = np.float64 if form == "fp64" else np.float32
    ps = clustered_cloud(12000, 23, seed=61, dtype=dtype)
    v = np.random.default_rng(62).standard_normal((ps.n, 3)).astype(dtype)
    field = None
    if alpha is not None:
        field, _ = odirect.direct(ps.x.astype(float), ps.m.astype(float), ps.h.astype(float))
        field = field.astype(dtype)
    a, p, tid, jerk, a0, p0 = gpu_tidal(ps, v, form, 0.5, order, alpha, field)
    x, m, h = (u.astype(np.float64) for u in (ps.x, ps.m, ps.h))
    lists = otree.tree_lists(x, m, h, ps.n_gas, 0.5, 16, 32, alpha=alpha,
                             field=None if field is None else field.astype(np.float64))
    Tr, Jr = otree.tree_tidal(x, m, h, v.astype(np.float64), ps.n_gas, lists)
    eT, eJ = _rowerr(tid, Tr), _rowerr(jerk, Jr)
    ea = _rowerr(a, a0)
    print(f"{form}: T err median {np.median(eT):.2e} p99 {np.quantile(eT, 0.99):.2e}; "
          f"j err median {np.median(eJ):.2e} p99 {np.quantile(eJ, 0.99):.2e}; "
          f"a vs sf_grav_accel max {ea.max():.2e}", flush=True)
    if form == "fp64":
        assert np.quantile(eT, 0.99) < 1e-10 and np.quantile(eJ, 0.99) < 1e-10
        assert ea.max() < 1e-12
    elif form == "fp32c":
        assert np.median(eT) < 1e-5 and np.median(eJ) < 1e-5
        assert np.quantile(eT, 0.99) < 2e-4 and np.quantile(eJ, 0.99) < 2e-4
        assert np.quantile(ea, 0.99) < 1e-5
    else:   # plain FP32: absolute coordinates, uncompensated sums
        assert np.median(eT) < 1e-4 and np.median(eJ) < 1e-4
        assert np.quantile(ea, 0.99) < 1e-4


def test_tidal_theta_zero_is_direct_sum():
    _say("tidal theta 0")
    ps = clustered_cloud(6000, 13, seed=63, dtype=np.float64)
    v = np.random.default_rng(64).standard_normal((ps.n, 3))
    a, p, tid, jerk, _, _ = gpu_tidal(ps, v, "fp64", 0.0)
    Tr, Jr = odirect.direct_tidal(ps.x, ps.m, ps.h, v)
    ar, pr = odirect.direct(ps.x, ps.m, ps.h)
    assert np.max(_rowerr(tid, Tr)) < 1e-10
    assert np.max(_rowerr(jerk, Jr)) < 1e-10
    assert np.max(_rowerr(a, ar)) < 1e-10
    assert np.max(np.abs(p - pr) / np.abs(pr)) < 1e-12


def test_tidal_edge_sizes_and_optional_outputs():
    L = _lib()
    for n, ns in ((1, 0), (2, 1), (65, 3), (200, 5)):
        _say("tidal edge n =", n, "sinks", ns)
        ps = uniform_sphere(n, seed=700 + n, h=0.3)
        ps.n_gas = n - ns
        v = np.random.default_rng(800 + n).standard_normal((n, 3))
        x, m, h, vv = _dev(ps.x, ps.m, ps.h, v)
        o = L.make_opts(form="fp64", theta=0.0, order=2, leaf_cap=4, group_cap=8, n_gas=ps.n_gas)
        t = L.sf_grav_build_tree(x, m, h, o)
        a, p, tid, jerk = L.sf_grav_accel_tidal(t, o, vel=vv)
        a2, p2, tid2, jerk2 = L.sf_grav_accel_tidal(t, o, vel=None, want_pot=False)
        torch.cuda.synchronize()
        L.sf_grav_tree_free(t)
        assert jerk2 is None and p2 is None
        assert torch.equal(tid, tid2) and torch.equal(a, a2)
        if n == 1:
            assert torch.all(tid == 0) and torch.all(jerk == 0)
            continue
        Tr, Jr = odirect.direct_tidal(ps.x, ps.m, ps.h, v)
        assert np.allclose(tid.cpu().numpy(), Tr, rtol=1e-10, atol=1e-12 * np.abs(Tr).max())
        assert np.allclose(jerk.cpu().numpy(), Jr, rtol=1e-10, atol=1e-12 * np.abs(Jr).max())
