"""GPU parity of the adjoint (sf_grav_accel_backward) against the oracle.

Direct path: the oracle's exact analytic VJP (itself pinned to torch autograd
and central differences).  Tree path: torch autograd of the oracle's frozen-list
tree evaluation, i.e. the derivative of the tree approximation with opening
decisions held fixed -- what the library's tree adjoint is specified to be.
"""
import numpy as np
import pytest
import torch

from oracle import direct as odirect
from oracle import tree as otree
from synth import clustered_cloud, cotangents, differentiation_cloud, uniform_sphere

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2010_11254_amd import _lib
    return _lib


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a)).cuda() for a in arrs]


def gpu_backward(ps, ga, gp, form, path, theta=0.5, order=2, leaf_cap=16, group_cap=64):
    L = _lib()
    x, m, h = _dev(ps.x, ps.m, ps.h)
    g_a, g_p = _dev(ga.astype(ps.x.dtype), gp.astype(ps.x.dtype))
    o = L.make_opts(form=form, theta=theta, order=order, leaf_cap=leaf_cap, group_cap=group_cap,
                    n_gas=ps.n_gas)
    if path == "tree":
        t = L.sf_grav_build_tree(x, m, h, o)
        gx, gm, gh = L.sf_grav_accel_backward(t, None, None, None, o, g_a, g_p)
        torch.cuda.synchronize()
        L.sf_grav_tree_free(t)
    else:
        gx, gm, gh = L.sf_grav_accel_backward(None, x, m, h, o, g_a, g_p)
        torch.cuda.synchronize()
    return [v.double().cpu().numpy() for v in (gx, gm, gh)]


def _close(got, ref, rtol, name):
    scale = np.abs(ref).max()
    err = np.abs(got - ref) / (np.abs(ref) + 1e-3 * scale)
    assert np.quantile(err, 0.99) <= rtol and np.median(err) <= rtol / 10, \
        (name, float(np.median(err)), float(np.quantile(err, 0.99)), float(err.max()))


def oracle_tree_vjp(ps, ga, gp, theta=0.5, order=2, leaf_cap=16, group_cap=64):
    lists = otree.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta, leaf_cap, group_cap)
    X = torch.tensor(ps.x, dtype=torch.float64, requires_grad=True)
    M = torch.tensor(ps.m, dtype=torch.float64, requires_grad=True)
    H = torch.tensor(ps.h, dtype=torch.float64, requires_grad=True)
    a, p = otree.tree_eval(X, M, H, ps.n_gas, lists, 1.0, order)
    ((a * torch.tensor(ga)).sum() + (p * torch.tensor(gp)).sum()).backward()
    return X.grad.numpy(), M.grad.numpy(), H.grad.numpy()


# ---------------------------------------------------------------- direct

@pytest.mark.parametrize("form,rtol", [("fp64", 1e-9), ("fp32", 1e-3), ("fp32c", 2e-4)])
def test_direct_adjoint_matches_oracle(form, rtol):
    _say("direct adjoint", form)
    ps = clustered_cloud(6000, 20, seed=12, dtype=np.float64 if form == "fp64" else np.float32)
    ga, gp = cotangents(ps.n, seed=12)
    got = gpu_backward(ps, ga, gp, form, "direct")
    ref = odirect.direct_vjp(ps.x.astype(float), ps.m.astype(float), ps.h.astype(float), ga, gp)
    for g, r, name in zip(got, ref, ("x", "m", "h")):
        _close(g, r, rtol, name)


@pytest.mark.parametrize("form,rtol", [("fp64", 1e-9), ("fp32c", 2e-4)])
def test_direct_adjoint_edge_sizes(form, rtol):
    # single particle, pairs, ragged 64-particle tiles, sinks at the end of
    # the order (gas-sink and sink-sink pairs)
    dt = np.float64 if form == "fp64" else np.float32
    for n, n_sink in ((1, 0), (2, 1), (3, 0), (63, 2), (64, 0), (65, 3), (130, 5)):
        _say("direct adjoint", form, "n =", n, "sinks", n_sink)
        ps = uniform_sphere(n, seed=500 + n, dtype=dt)
        rng = np.random.default_rng(600 + n)
        ps.h = (ps.h * (1.0 + 0.5 * rng.random(n))).astype(dt)
        ps.n_gas = n - n_sink
        ga, gp = cotangents(ps.n, seed=500 + n)
        got = gpu_backward(ps, ga, gp, form, "direct")
        if n == 1:
            assert all(np.all(g == 0.0) for g in got)
            continue
        ref = odirect.direct_vjp(ps.x.astype(float), ps.m.astype(float), ps.h.astype(float), ga,
                                 gp)
        for g, r, name in zip(got, ref, ("x", "m", "h")):
            _close(g, r, rtol, (n, name))


def test_direct_adjoint_dense_torch_reference_2048():
    # the differentiation workload's dense reference: N = 2048 clustered gas
    _say("direct adjoint vs dense torch, 2048")
    ps = differentiation_cloud(2048, seed=7, dtype=np.float64)
    ga, gp = cotangents(ps.n, seed=7)
    got = gpu_backward(ps, ga, gp, "fp64", "direct")
    X = torch.tensor(ps.x, requires_grad=True)
    M = torch.tensor(ps.m, requires_grad=True)
    H = torch.tensor(ps.h, requires_grad=True)
    from test_oracle_direct import _torch_dense
    a, p = _torch_dense(X, M, H, 1.0)
    ((a * torch.tensor(ga)).sum() + (p * torch.tensor(gp)).sum()).backward()
    for g, r, name in zip(got, (X.grad.numpy(), M.grad.numpy(), H.grad.numpy()), ("x", "m", "h")):
        _close(g, r, 1e-9, name)


# ---------------------------------------------------------------- tree

@pytest.mark.parametrize("order", [0, 2])
def test_tree_adjoint_fp64_matches_oracle(order):
    _say("tree adjoint fp64, order", order)
    ps = clustered_cloud(5000, 12, seed=13, dtype=np.float64)
    ga, gp = cotangents(ps.n, seed=13)
    got = gpu_backward(ps, ga, gp, "fp64", "tree", order=order)
    ref = oracle_tree_vjp(ps, ga, gp, order=order)
    for g, r, name in zip(got, ref, ("x", "m", "h")):
        _close(g, r, 1e-8, name)


def test_tree_adjoint_fp32c_matches_oracle():
    _say("tree adjoint fp32c")
    ps = clustered_cloud(5000, 12, seed=14)
    ga, gp = cotangents(ps.n, seed=14)
    got = gpu_backward(ps, ga, gp, "fp32c", "tree")
    ref = oracle_tree_vjp(ps, ga, gp)
    for g, r, name in zip(got, ref, ("x", "m", "h")):
        _close(g, r, 2e-4, name)


@pytest.mark.parametrize("form,rtol,dtype", [("fp64", 1e-8, np.float64), ("fp32c", 2e-4, np.float32)])
def test_tree_adjoint_gas_only_matches_oracle(form, rtol, dtype):
    # no sinks: the gas-only node adjoints are neither allocated nor walked
    _say("tree adjoint gas only", form)
    ps = differentiation_cloud(3000, seed=21, dtype=dtype)
    ga, gp = cotangents(ps.n, seed=21)
    got = gpu_backward(ps, ga, gp, form, "tree")
    ref = oracle_tree_vjp(ps, ga, gp)
    for g, r, name in zip(got, ref, ("x", "m", "h")):
        _close(g, r, rtol, name)


@pytest.mark.parametrize("form,rtol", [("fp64", 1e-8), ("fp32", 1e-3), ("fp32c", 2e-4)])
def test_tree_adjoint_edge_sizes(form, rtol):
    # tiny trees (one leaf, one split, group and batch boundaries) with mixed
    # softening radii, against the oracle tree's adjoint on the same lists
    dt = np.float64 if form == "fp64" else np.float32
    for n in (1, 2, 3, 17, 33, 65, 200):
        _say("tree adjoint", form, "n =", n)
        ps = uniform_sphere(n, seed=300 + n, dtype=dt)   # about 32 neighbours within h
        rng = np.random.default_rng(400 + n)
        ps.h = (ps.h * (1.0 + 0.5 * rng.random(n))).astype(dt)
        ga, gp = cotangents(ps.n, seed=300 + n)
        got = gpu_backward(ps, ga, gp, form, "tree", leaf_cap=16, group_cap=32)
        if n == 1:
            assert all(np.all(g == 0.0) for g in got)
            continue
        ref = oracle_tree_vjp(ps, ga, gp, leaf_cap=16, group_cap=32)
        for g, r, name in zip(got, ref, ("x", "m", "h")):
            _close(g, r, rtol, (n, name))


def test_tree_adjoint_theta_zero_is_direct_adjoint():
    _say("tree adjoint theta 0 == direct oracle")
    ps = clustered_cloud(3000, 10, seed=15, dtype=np.float64)
    ga, gp = cotangents(ps.n, seed=15)
    got = gpu_backward(ps, ga, gp, "fp64", "tree", theta=0.0)
    ref = odirect.direct_vjp(ps.x, ps.m, ps.h, ga, gp)
    for g, r, name in zip(got, ref, ("x", "m", "h")):
        _close(g, r, 1e-9, name)


# ---------------------------------------------------------------- autograd

def test_autograd_function_gradcheck_direct():
    _say("gradcheck SFGravity direct fp64")
    from paper_2010_11254_amd import gravity
    ps = clustered_cloud(48, 4, seed=16, dtype=np.float64)
    x, m, h = (torch.tensor(v, device="cuda", requires_grad=True) for v in (ps.x, ps.m, ps.h))
    f = lambda x, m, h: gravity(x, m, h, path="direct", form="fp64", n_gas=ps.n_gas)
    assert torch.autograd.gradcheck(f, (x, m, h), eps=1e-7, atol=1e-6, rtol=1e-5)


def test_autograd_function_tree_backward():
    _say("SFGravity tree backward vs oracle")
    from paper_2010_11254_amd import gravity
    ps = clustered_cloud(3000, 8, seed=17, dtype=np.float64)
    ga, gp = cotangents(ps.n, seed=17)
    x, m, h = (torch.tensor(v, device="cuda", requires_grad=True) for v in (ps.x, ps.m, ps.h))
    a, p = gravity(x, m, h, path="tree", form="fp64", n_gas=ps.n_gas, leaf_cap=16, group_cap=64)
    ((a * torch.tensor(ga, device="cuda")).sum() + (p * torch.tensor(gp, device="cuda")).sum()).backward()
    ref = oracle_tree_vjp(ps, ga, gp)
    for g, r, name in zip((x.grad, m.grad, h.grad), ref, ("x", "m", "h")):
        _close(g.cpu().numpy(), r, 1e-8, name)


@pytest.mark.parametrize("n_gas,form", [(20000, "fp32c"), (1 << 20, "fp32c"), (1 << 20, "fp64")])
def test_tree_adjoint_independent_of_task_order(n_gas, form):
    # before any forward on the handle the adjoint takes its groups in Morton
    # order; after one, in the cost order the forward recorded (exact at
    # 20000 particles, cost classes at 2^20): the same gradients up to the
    # summation order of its FP64 accumulations
    L = _lib()
    _say("tree adjoint task order", form, "n_gas", n_gas)
    ps = clustered_cloud(n_gas, 64, seed=51)
    ga, gp = cotangents(ps.n, seed=51, dtype=np.float32)
    x, m, h, g_a, g_p = _dev(ps.x, ps.m, ps.h, ga, gp)
    o = L.make_opts(form=form, n_gas=ps.n_gas)
    t = L.sf_grav_build_tree(x, m, h, o)
    first = L.sf_grav_accel_backward(t, None, None, None, o, g_a, g_p)
    L.sf_grav_accel(t, None, None, None, o)
    second = L.sf_grav_accel_backward(t, None, None, None, o, g_a, g_p)
    torch.cuda.synchronize()
    L.sf_grav_tree_free(t)
    for a, b, name in zip(first, second, ("x", "m", "h")):
        scale = b.abs().max().item()
        assert torch.allclose(a, b, rtol=1e-5, atol=1e-6 * scale), name


def test_tree_adjoint_theta_zero_deep_stack():
    _say("tree adjoint theta 0, leaf 1, uniform 20000: deep stack")
    from synth import uniform_sphere
    ps = uniform_sphere(20000, seed=3)
    ga, gp = cotangents(ps.n, seed=18)
    got = gpu_backward(ps, ga, gp, "fp64", "tree", theta=0.0, leaf_cap=1, group_cap=8)
    ref = odirect.direct_vjp(ps.x, ps.m, ps.h, ga, gp)
    for g, r, name in zip(got, ref, ("x", "m", "h")):
        _close(g, r, 1e-9, name)
