"""GPU parity at the workloads' full sizes, in the launch configuration the
benchmark times (leaf 32, group 32, theta 0.5, quadrupole), on outputs the
oracle computes one by one (sampled groups and targets), plus properties that
hold at any size: determinism of the forward pass and translation invariance.

precision4m = 4,194,304 clustered gas + 2048 sink binaries (seed 2);
clustered1m = 1,048,576 clustered gas + 256 sinks on gas positions (seed 1);
fractal16m = 16,777,216 gas in a three-level Plummer-in-Plummer hierarchy +
10,000 sinks (seed 4), the largest workload (742,488 groups).
"""
import numpy as np
import pytest
import torch

from oracle import direct as odirect
from oracle import tree as otree
from synth import clustered_cloud, make_config, precision_cloud, subsample

pytestmark = pytest.mark.gpu

LEAF, GROUP = 32, 32   # the benchmark's capacities


def _lib():
    from paper_2010_11254_amd import _lib
    return _lib


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a)).cuda() for a in arrs]


def _relerr(a, ref):
    return np.linalg.norm(a - ref, axis=1) / np.linalg.norm(ref, axis=1)


@pytest.fixture(scope="module")
def c2():
    _say("generating precision4m")
    return precision_cloud(1 << 22, 2048, seed=2)


@pytest.fixture(scope="module")
def c1():
    _say("generating clustered1m")
    return clustered_cloud(1 << 20, 256, seed=1)


def _pick_groups(groups, sink_sorted, k_rand, k_sink, seed):
    rng = np.random.default_rng(seed)
    with_sink = [g for g in range(groups.shape[0])
                 if sink_sorted[groups[g, 0]:groups[g, 0] + groups[g, 1]].any()]
    sel = set(rng.choice(groups.shape[0], k_rand, replace=False).tolist())
    sel |= set(rng.choice(with_sink, min(k_sink, len(with_sink)), replace=False).tolist())
    return sorted(sel)


def _sampled_field(ps, x64, m64, h64, tgt, seed):
    """Previous field for the relative criterion: the oracle's exact direct
    field on the sampled targets (so their groups' g_min has its true size),
    seeded Gaussian vectors of the same median magnitude elsewhere.  Rounded
    to FP32 so that both handles and the oracle see the same values."""
    f_t, _ = odirect.direct(x64, m64, h64, targets=tgt)
    rng = np.random.default_rng([seed, 77])
    field = rng.standard_normal((ps.n, 3))
    field *= np.median(np.linalg.norm(f_t, axis=1)) / np.sqrt(3.0)
    field[tgt] = f_t
    return field.astype(np.float32).astype(np.float64)


def _tree_sampled(ps, k_rand, k_sink, seed, alpha=None):
    """GPU tree (FP64 form on FP64 copies of the inputs, FP32C on the FP32
    inputs) against the oracle's frozen-list evaluation of sampled groups;
    with `alpha` the relative opening criterion is on, driven by the field of
    `_sampled_field` on both sides."""
    L = _lib()
    x64, m64, h64 = (v.astype(np.float64) for v in (ps.x, ps.m, ps.h))
    _say("oracle tree lists", ps.n, "alpha", alpha)
    tree = otree.build_tree(x64, LEAF)
    groups = otree.make_groups(tree, GROUP)
    sink_sorted = (tree.order >= ps.n_gas)
    sel = _pick_groups(groups, sink_sorted, k_rand, k_sink, seed)
    tgt = np.concatenate([tree.order[groups[g, 0]:groups[g, 0] + groups[g, 1]] for g in sel])
    field = None if alpha is None else _sampled_field(ps, x64, m64, h64, tgt, seed)
    lists = otree.tree_lists(x64, m64, h64, ps.n_gas, 0.5, LEAF, GROUP, groups_sel=sel, lazy=True,
                             alpha=alpha, field=field)
    t64 = lambda v: torch.as_tensor(v)
    with torch.no_grad():
        ar, pr = otree.tree_eval(t64(x64), t64(m64), t64(h64), ps.n_gas, lists, 1.0, 2, targets=tgt)
    ar, pr = ar.numpy(), pr.numpy()
    out = {}
    for form, arrs in (("fp64", (x64, m64, h64)), ("fp32c", (ps.x, ps.m, ps.h))):
        _say("gpu tree", form, ps.n)
        x, m, h = _dev(*arrs)
        o = L.make_opts(form=form, n_gas=ps.n_gas, collect_stats=True, leaf_cap=LEAF,
                        group_cap=GROUP, alpha=alpha)
        t = L.sf_grav_build_tree(x, m, h, o)
        if alpha is not None:
            L.sf_grav_tree_set_field(t, _dev(field.astype(arrs[0].dtype))[0])
        a, p = L.sf_grav_accel(t, None, None, None, o)
        torch.cuda.synchronize()
        npc = L.sf_grav_tree_export(t, "group_npc").numpy()
        npp = L.sf_grav_tree_export(t, "group_npp").numpy()
        L.sf_grav_tree_free(t)
        for g, (pc, pp) in lists.gas_lists.items():   # same opening decisions
            assert npc[g] == pc.size and npp[g] == pp.size, (form, g)
        out[form] = (a.double().cpu().numpy()[tgt], p.double().cpu().numpy()[tgt])
    e64 = _relerr(out["fp64"][0], ar)
    assert e64.max() < 1e-10, e64.max()
    assert np.max(np.abs(out["fp64"][1] - pr) / np.abs(pr)) < 1e-10
    e32 = _relerr(out["fp32c"][0], ar)
    assert np.median(e32) < 2e-6 and np.quantile(e32, 0.99) < 2e-5, (np.median(e32), e32.max())
    return tgt.size, lists, sel


def _direct_sampled(ps, k, seed):
    L = _lib()
    x, m, h = _dev(ps.x, ps.m, ps.h)
    _say("gpu direct fp32c", ps.n)
    a, p = L.sf_grav_accel(None, x, m, h, L.make_opts(form="fp32c", n_gas=ps.n_gas))
    torch.cuda.synchronize()
    idx = subsample(ps.n, k, seed)
    ar, pr = odirect.direct(ps.x.astype(float), ps.m.astype(float), ps.h.astype(float),
                            targets=idx)
    e = _relerr(a.double().cpu().numpy()[idx], ar)
    ep = np.abs(p.double().cpu().numpy()[idx] - pr) / np.abs(pr)
    assert np.median(e) <= 1e-6 and np.median(ep) <= 1e-6, (np.median(e), np.median(ep))
    assert np.quantile(e, 0.99) < 1e-3, np.quantile(e, 0.99)


# ---------------------------------------------------------------- precision4m

def test_precision4m_build_bit_exact(c2):
    _say("precision4m build bit-exact")
    L = _lib()
    x, m, h = _dev(c2.x, c2.m, c2.h)
    t = L.sf_grav_build_tree(x, m, h, L.make_opts(n_gas=c2.n_gas, leaf_cap=LEAF, group_cap=GROUP))
    ref = otree.build_tree(c2.x.astype(np.float64), LEAF)
    assert np.array_equal(L.sf_grav_tree_export(t, "keys").numpy().view(np.uint64), ref.keys)
    assert np.array_equal(L.sf_grav_tree_export(t, "order").numpy(), ref.order)
    for name, arr in [("node_level", ref.level), ("node_first", ref.first),
                      ("node_count", ref.count), ("node_parent", ref.parent),
                      ("node_child", ref.child_first), ("node_nchild", ref.n_child)]:
        assert np.array_equal(L.sf_grav_tree_export(t, name).numpy(), arr), name
    g = otree.make_groups(ref, GROUP)
    assert np.array_equal(L.sf_grav_tree_export(t, "group_first").numpy(), g[:, 0])
    assert np.array_equal(L.sf_grav_tree_export(t, "group_count").numpy(), g[:, 1])
    # moments of sampled nodes (every level) against the oracle's sums
    lazy = otree.LazyMoments(ref, c2.x, c2.m, c2.h)
    rng = np.random.default_rng(9)
    nodes = np.unique(np.concatenate([rng.choice(ref.n_nodes, 3000, replace=False),
                                      np.arange(64)]))
    gm = L.sf_grav_tree_export(t, "node_mass").numpy()[nodes]
    gc = L.sf_grav_tree_export(t, "node_com").numpy()[nodes]
    assert np.allclose(gm, lazy["M"][nodes], rtol=1e-12, atol=0)
    assert np.allclose(gc, lazy["com"][nodes], rtol=0, atol=1e-12)
    L.sf_grav_tree_free(t)


def test_precision4m_tree_sampled_groups(c2):
    _say("precision4m tree, sampled groups")
    assert _tree_sampled(c2, k_rand=16, k_sink=8, seed=2)[0] > 400


def test_precision4m_tree_sampled_groups_relative(c2):
    """The benchmark's opening rule: theta 0.5 with the relative criterion at
    alpha = 0.003; the criterion must actually open nodes here."""
    _say("precision4m tree relative, sampled groups")
    n_t, rel, sel = _tree_sampled(c2, k_rand=16, k_sink=8, seed=12, alpha=0.003)
    assert n_t > 400
    x64, m64, h64 = (v.astype(np.float64) for v in (c2.x, c2.m, c2.h))
    ang = otree.tree_lists(x64, m64, h64, c2.n_gas, 0.5, LEAF, GROUP, groups_sel=sel, lazy=True)
    work = lambda ls: sum(pc.size + pp.size for pc, pp in ls.gas_lists.values())
    assert work(rel) > work(ang), (work(rel), work(ang))


def test_precision4m_direct_sampled(c2):
    _say("precision4m direct, sampled targets")
    _direct_sampled(c2, 256, seed=2)


# ---------------------------------------------------------------- clustered1m

def test_clustered1m_tree_sampled_groups(c1):
    _say("clustered1m tree, sampled groups")
    assert _tree_sampled(c1, k_rand=16, k_sink=6, seed=1)[0] > 400


def test_clustered1m_tree_sampled_groups_relative(c1):
    _say("clustered1m tree relative, sampled groups")
    assert _tree_sampled(c1, k_rand=16, k_sink=6, seed=11, alpha=0.003)[0] > 400


def test_clustered1m_direct_sampled(c1):
    _say("clustered1m direct, sampled targets")
    _direct_sampled(c1, 256, seed=1)


# ---------------------------------------------------------------- properties

def test_forward_is_deterministic(c1):
    _say("forward determinism, clustered1m tree + direct subset")
    L = _lib()
    x, m, h = _dev(c1.x, c1.m, c1.h)
    runs = []
    for _ in range(2):
        o = L.make_opts(form="fp32c", n_gas=c1.n_gas)
        t = L.sf_grav_build_tree(x, m, h, o)
        a, p = L.sf_grav_accel(t, None, None, None, o)
        L.sf_grav_tree_free(t)
        k = 65536
        ad, pd = L.sf_grav_accel(None, x[:k].contiguous(), m[:k].contiguous(), h[:k].contiguous(),
                                 L.make_opts(form="fp32c", n_gas=k))
        torch.cuda.synchronize()
        runs.append([v.cpu().numpy() for v in (a, p, ad, pd)])
    for u, v in zip(*runs):
        assert np.array_equal(u, v)


def test_translation_invariance_fp32c():
    _say("translation invariance, fp32c tree and direct")
    L = _lib()
    ps = clustered_cloud(60000, 40, seed=8)
    x0 = ps.x.astype(np.float64)
    shift = np.array([0.5, -0.25, 0.125])
    x1 = x0 + shift
    assert np.array_equal(x1 - shift, x0)    # the shift is exact in FP64
    m, h = ps.m.astype(np.float64), ps.h.astype(np.float64)
    res = []
    for xx in (x0, x1):
        x, mm, hh = _dev(xx, m, h)
        o = L.make_opts(form="fp32c", n_gas=ps.n_gas)
        t = L.sf_grav_build_tree(x, mm, hh, o)
        a, p = L.sf_grav_accel(t, None, None, None, o)
        L.sf_grav_tree_free(t)
        ad, pd = L.sf_grav_accel(None, x, mm, hh, o)
        torch.cuda.synchronize()
        res.append([v.cpu().numpy() for v in (a, ad)])
    for k in range(2):
        e = _relerr(res[1][k], res[0][k])
        assert np.median(e) <= 1e-6 and np.quantile(e, 0.99) <= 1e-5, (k, np.median(e), e.max())


# ---------------------------------------------------------------- fractal16m

def test_fractal16m_tree_sampled_groups():
    _say("generating fractal16m")
    c4 = make_config("fractal16m")
    _say("fractal16m tree, sampled groups")
    assert _tree_sampled(c4, k_rand=4, k_sink=2, seed=4)[0] > 100
