"""GPU parity: the HIP library (through its C ABI) against the CPU oracle.

Inputs are seeded synthetic clouds (uniform sphere, clustered clouds with
sinks on gas positions).  Bars:
  * Morton order, topology and groups: bit-exact with the oracle's spec;
  * direct path: FP64 form to 1e-12, FP32C median relative error <= 1e-6;
  * tree path: the FP64 form reproduces the oracle's tree (same opening
    decisions, same interaction counts per group) to 1e-10; FP32C to 1e-5;
    theta = 0 reproduces the direct sum.
"""
import numpy as np
import pytest
import torch

from oracle import direct as odirect
from oracle import tree as otree
from synth import ParticleSet, clustered_cloud, uniform_sphere

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2010_11254_amd import _lib
    return _lib


def _dev(ps):
    d = lambda a: torch.as_tensor(np.ascontiguousarray(a)).cuda()
    return d(ps.x), d(ps.m), d(ps.h)


def _say(*a):
    print("[case]", *a, flush=True)


def _relerr(a, ref):
    return np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)


def gpu_direct(ps, form, G=1.0):
    L = _lib()
    x, m, h = _dev(ps)
    o = L.make_opts(form=form, G=G, n_gas=ps.n_gas)
    a, p = L.sf_grav_accel(None, x, m, h, o)
    torch.cuda.synchronize()
    return a.double().cpu().numpy(), p.double().cpu().numpy()


def gpu_tree(ps, form, theta=0.5, order=2, leaf_cap=16, group_cap=64, stats=False, keep=False):
    L = _lib()
    x, m, h = _dev(ps)
    o = L.make_opts(form=form, theta=theta, order=order, leaf_cap=leaf_cap, group_cap=group_cap,
                    n_gas=ps.n_gas, collect_stats=stats)
    t = L.sf_grav_build_tree(x, m, h, o)
    a, p = L.sf_grav_accel(t, None, None, None, o)
    torch.cuda.synchronize()
    out = a.double().cpu().numpy(), p.double().cpu().numpy()
    if keep:
        return out + (t,)
    L.sf_grav_tree_free(t)
    return out


# ---------------------------------------------------------------- direct

def test_direct_fp64_uniform_sphere():
    _say("direct fp64 uniform4k")
    ps = uniform_sphere(4096, seed=0)
    a, p = gpu_direct(ps, "fp64")
    ar, pr = odirect.direct(ps.x, ps.m, ps.h)
    assert np.max(_relerr(a, ar)) < 1e-11
    assert np.max(np.abs(p - pr) / np.abs(pr)) < 1e-12


@pytest.mark.parametrize("form", ["fp32c", "fp32"])
def test_direct_fp32_forms_uniform_sphere(form):
    _say("direct", form, "uniform4k")
    ps = uniform_sphere(4096, seed=0)
    a, p = gpu_direct(ps, form)
    ar, pr = odirect.direct(ps.x, ps.m, ps.h)
    e = _relerr(a, ar)
    assert np.median(e) <= 1e-6, np.median(e)
    assert np.median(np.abs(p - pr) / np.abs(pr)) <= 1e-6


@pytest.mark.parametrize("form,tol_med,dtype", [("fp64", 1e-12, np.float64),
                                                 ("fp32c", 1e-6, np.float32)])
def test_direct_clustered_with_sinks(form, tol_med, dtype):
    # outputs come back in the input dtype, so the FP64 form is checked on
    # FP64 inputs
    _say("direct", form, "clustered 20000+37 sinks")
    ps = clustered_cloud(20000, 37, seed=11, dtype=dtype)   # ragged tiles, coincident sinks
    a, p = gpu_direct(ps, form)
    x, m, h = (v.astype(np.float64) for v in (ps.x, ps.m, ps.h))
    ar, pr = odirect.direct(x, m, h)
    e = _relerr(a, ar)
    assert np.median(e) <= tol_med, np.median(e)
    assert np.median(e[ps.n_gas:]) <= max(tol_med, 1e-6)
    ep = np.abs(p - pr) / np.abs(pr)
    assert np.median(ep) <= tol_med


def test_direct_edge_sizes():
    for n in (1, 2, 63, 64, 65):
        _say("direct fp32c n =", n)
        ps = uniform_sphere(n, seed=n, dtype=np.float32, h=0.3)
        a, p = gpu_direct(ps, "fp32c")
        ar, pr = odirect.direct(ps.x.astype(float), ps.m.astype(float), ps.h.astype(float))
        assert np.allclose(a, ar, rtol=1e-5, atol=1e-5 * (np.abs(ar).max() + 1e-30))
        assert np.allclose(p, pr, rtol=1e-5, atol=1e-7)


def test_direct_momentum_fp64():
    _say("direct fp64 momentum")
    ps = clustered_cloud(5000, 20, seed=2, dtype=np.float64)
    a, _ = gpu_direct(ps, "fp64")
    net = (ps.m[:, None] * a).sum(0)
    assert np.all(np.abs(net) <= 1e-12 * (ps.m * np.linalg.norm(a, axis=1)).sum())


# ---------------------------------------------------------------- tree build

@pytest.mark.parametrize("leaf_cap,group_cap", [(16, 64), (4, 16), (1, 8)])
def test_tree_build_bit_exact(leaf_cap, group_cap):
    _say("tree build bit-exact", leaf_cap, group_cap)
    L = _lib()
    ps = clustered_cloud(30000, 50, seed=3)
    x, m, h = _dev(ps)
    o = L.make_opts(leaf_cap=leaf_cap, group_cap=group_cap, n_gas=ps.n_gas)
    t = L.sf_grav_build_tree(x, m, h, o)
    ref = otree.build_tree(ps.x.astype(np.float64), leaf_cap)
    keys = L.sf_grav_tree_export(t, "keys").numpy().view(np.uint64)
    assert np.array_equal(keys, ref.keys)
    assert np.array_equal(L.sf_grav_tree_export(t, "order").numpy(), ref.order)
    for name, arr in [("node_level", ref.level), ("node_first", ref.first),
                      ("node_count", ref.count), ("node_parent", ref.parent),
                      ("node_child", ref.child_first), ("node_nchild", ref.n_child)]:
        got = L.sf_grav_tree_export(t, name).numpy()
        assert np.array_equal(got, arr), name
    g = otree.make_groups(ref, group_cap)
    assert np.array_equal(L.sf_grav_tree_export(t, "group_first").numpy(), g[:, 0])
    assert np.array_equal(L.sf_grav_tree_export(t, "group_count").numpy(), g[:, 1])
    mom = otree.node_moments(ref, ps.x, ps.m, ps.h)
    gm = L.sf_grav_tree_export(t, "node_mass").numpy()
    assert np.allclose(gm, mom["M"], rtol=1e-12)
    com = L.sf_grav_tree_export(t, "node_com").numpy()
    assert np.allclose(com, mom["com"], rtol=0, atol=1e-12)
    q = L.sf_grav_tree_export(t, "node_quad").numpy()
    qref = mom["Q"][:, [0, 1, 2, 0, 0, 1], [0, 1, 2, 1, 2, 2]]
    # Q of a one-particle node is 0 in exact arithmetic and rounding noise
    # after the FP64 parallel-axis shifts, so scale by M L^2 of the node
    side = float(np.max(ps.x.max(0).astype(float) - ps.x.min(0).astype(float)))
    scale = (mom["M"] * (side * np.ldexp(1.0, -ref.level)) ** 2)[:, None]
    assert np.all(np.abs(q - qref) <= 1e-12 * scale)
    L.sf_grav_tree_free(t)


def test_tree_build_identical_points_depth_limit():
    _say("tree build identical points")
    L = _lib()
    xh = np.zeros((200, 3))
    xh[100:] = 1.0
    xh[150:] = [1.0, 0.5, 0.25]
    x = torch.tensor(xh).cuda()
    m = torch.full((200,), 1.0 / 200, dtype=torch.float64).cuda()
    h = torch.full((200,), 0.01, dtype=torch.float64).cuda()
    o = L.make_opts(leaf_cap=8, group_cap=16)
    t = L.sf_grav_build_tree(x, m, h, o)
    ref = otree.build_tree(xh, 8)
    assert np.array_equal(L.sf_grav_tree_export(t, "node_count").numpy(), ref.count)
    a, p = L.sf_grav_accel(t, None, None, None, o)
    ar, pr = odirect.direct(xh, m.cpu().numpy(), h.cpu().numpy())
    assert np.allclose(a.cpu().numpy(), ar, rtol=1e-5, atol=1e-6 * np.abs(ar).max())
    L.sf_grav_tree_free(t)


# ---------------------------------------------------------------- tree eval

@pytest.mark.parametrize("order", [0, 2])
def test_tree_fp64_matches_tree_oracle(order):
    _say("tree fp64 vs oracle tree, order", order)
    ps = clustered_cloud(12000, 30, seed=4, dtype=np.float64)
    a, p, t = gpu_tree(ps, "fp64", order=order, stats=True, keep=True)
    ar, pr, lists = otree.tree_forward(ps.x, ps.m, ps.h, ps.n_gas, theta=0.5, order=order)
    L = _lib()
    npc = L.sf_grav_tree_export(t, "group_npc").numpy()
    npp = L.sf_grav_tree_export(t, "group_npp").numpy()
    for g, (pc, pp) in lists.gas_lists.items():
        assert npc[g] == pc.size and npp[g] == pp.size, g
    L.sf_grav_tree_free(t)
    assert np.max(_relerr(a, ar)) < 1e-10
    assert np.max(np.abs(p - pr) / np.abs(pr)) < 1e-10


@pytest.mark.parametrize("form,tol", [("fp32c", 2e-5), ("fp32", 2e-4)])
def test_tree_fp32_forms_match_tree_oracle(form, tol):
    _say("tree", form, "vs oracle tree")
    ps = clustered_cloud(12000, 30, seed=4)
    a, p = gpu_tree(ps, form)
    ar, pr, _ = otree.tree_forward(ps.x, ps.m, ps.h, ps.n_gas, theta=0.5, order=2)
    e = _relerr(a, ar)
    assert np.median(e) < tol / 10 and np.quantile(e, 0.99) < tol, (np.median(e), np.quantile(e, 0.99))


def test_tree_theta_zero_is_direct():
    _say("tree theta 0 fp64 == direct")
    ps = clustered_cloud(6000, 12, seed=5, dtype=np.float64)
    a, p = gpu_tree(ps, "fp64", theta=0.0)
    ar, pr = odirect.direct(ps.x, ps.m, ps.h)
    assert np.max(_relerr(a, ar)) < 1e-11


def test_tree_uniform_sphere_monopole_error():
    _say("tree monopole uniform4k theta 0.5")
    ps = uniform_sphere(4096, seed=0)
    a, p = gpu_tree(ps, "fp32c", order=0)
    ar, pr, _ = otree.tree_forward(ps.x, ps.m, ps.h, ps.n_gas, theta=0.5, order=0)
    assert np.median(_relerr(a, ar)) < 1e-6


def test_tree_theta_zero_deep_stack_is_direct():
    # leaf capacity 1 on a uniform cloud makes a near-full octree: a walk at
    # theta 0 then holds more stack entries than the LDS window and moves the
    # oldest ones out to device memory and back
    _say("tree theta 0, leaf 1, uniform 20000: deep stack")
    ps = uniform_sphere(20000, seed=3)
    a, p = gpu_tree(ps, "fp64", theta=0.0, leaf_cap=1, group_cap=8)
    ar, pr = odirect.direct(ps.x, ps.m, ps.h)
    assert np.max(_relerr(a, ar)) < 1e-11
    assert np.max(np.abs(p - pr) / np.abs(pr)) < 1e-11


def _lattice(side, h_cells, jitter, seed, dtype):
    """side^3 lattice points at multiples of 1/16 (exact in FP32), masses
    around 1/n, softening h_cells/16 times (1 + jitter * U(-1, 1))."""
    rng = np.random.default_rng(seed)
    g = np.arange(side, dtype=np.float64) / 16.0
    x = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    n = x.shape[0]
    m = rng.uniform(0.5, 1.5, n) / n
    h = (h_cells / 16.0) * (1.0 + jitter * rng.uniform(-1.0, 1.0, n))
    return ParticleSet(x=x.astype(dtype), m=m.astype(dtype), h=h.astype(dtype), n_gas=n)


@pytest.mark.parametrize("h_cells,jitter", [(1.0, 0.0), (2.5, 0.3)])
def test_tree_lattice_softening_boundary(h_cells, jitter):
    # A lattice puts many pairs exactly at (h_cells = 1) or around the
    # softening radius and many near-leaf particles right at max(h) from a
    # group box, where the walk decides per particle between the softened
    # and the Newtonian-only evaluation; both forms must match the oracle
    # tree, and the same lists must be formed.
    _say("tree lattice 12^3, h =", h_cells, "cells, jitter", jitter)
    for form, dt, tol in (("fp64", np.float64, 1e-10), ("fp32c", np.float32, 2e-5)):
        ps = _lattice(12, h_cells, jitter, seed=11, dtype=dt)
        a, p, t = gpu_tree(ps, form, leaf_cap=8, group_cap=32, stats=True, keep=True)
        x64, m64, h64 = (v.astype(np.float64) for v in (ps.x, ps.m, ps.h))
        ar, pr, lists = otree.tree_forward(x64, m64, h64, ps.n_gas, theta=0.5, order=2,
                                           leaf_cap=8, group_cap=32)
        L = _lib()
        npc = L.sf_grav_tree_export(t, "group_npc").numpy()
        npp = L.sf_grav_tree_export(t, "group_npp").numpy()
        L.sf_grav_tree_free(t)
        for g, (pc, pp) in lists.gas_lists.items():
            assert npc[g] == pc.size and npp[g] == pp.size, (form, g)
        # errors against the RMS field (lattice symmetry leaves some targets
        # with a nearly cancelled acceleration)
        e = np.linalg.norm(a - ar, axis=1) / np.sqrt(np.mean(np.sum(ar * ar, axis=1)))
        ep = np.abs(p - pr) / np.sqrt(np.mean(pr * pr))
        assert np.max(e) < tol and np.max(ep) < tol, (form, np.max(e), np.max(ep))


@pytest.mark.parametrize("form", ["fp64", "fp32c"])
def test_tree_edge_sizes(form):
    # tiny trees: a single leaf (n <= leaf capacity), one split, a few
    # levels, the group and particle-batch boundaries; topology bit-exact
    # and forces against the oracle tree (same lists)
    L = _lib()
    dt = np.float64 if form == "fp64" else np.float32
    tol = 1e-10 if form == "fp64" else 2e-5
    for n in (1, 2, 3, 16, 17, 33, 65, 129, 200):
        _say("tree", form, "n =", n)
        ps = uniform_sphere(n, seed=100 + n, dtype=dt, h=0.05)
        a, p, t = gpu_tree(ps, form, leaf_cap=16, group_cap=32, stats=True, keep=True)
        x64, m64, h64 = (v.astype(np.float64) for v in (ps.x, ps.m, ps.h))
        ref = otree.build_tree(x64, 16)
        for name, arr in [("node_level", ref.level), ("node_first", ref.first),
                          ("node_count", ref.count), ("node_parent", ref.parent),
                          ("node_child", ref.child_first), ("node_nchild", ref.n_child)]:
            assert np.array_equal(L.sf_grav_tree_export(t, name).numpy(), arr), (n, name)
        L.sf_grav_tree_free(t)
        if n == 1:
            assert np.all(a == 0.0)
            continue
        ar, pr, _ = otree.tree_forward(x64, m64, h64, ps.n_gas, theta=0.5, order=2, leaf_cap=16,
                                       group_cap=32)
        e = np.linalg.norm(a - ar, axis=1) / np.sqrt(np.mean(np.sum(ar * ar, axis=1)))
        ep = np.abs(p - pr) / np.sqrt(np.mean(pr * pr))
        assert np.max(e) < tol and np.max(ep) < tol, (n, np.max(e), np.max(ep))

