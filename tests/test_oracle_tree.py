"""Pins of the oracle's octree path (Sec. 2.2) against independent facts.

* Morton keys against a bit-by-bit string construction;
* the topology against its defining invariants (occupied cells, split rule,
  breadth-first order) -- these determine the tree uniquely;
* groups against their defining invariants;
* theta = 0 opens every node, so the tree must reproduce the direct sum
  (independent C code), for gas and sink targets;
* multipole truncation error falls as (L/r)^2 for monopoles and (L/r)^3 for
  quadrupoles;
* the adjoint of the frozen-list tree (autograd) reduces to the independent
  C adjoint at theta = 0 and matches central differences at theta = 0.5.
"""
import numpy as np
import pytest
import torch

from oracle import direct
from oracle import tree as T
from synth import clustered_cloud, uniform_sphere


def _keys_bruteforce(x):
    x = np.asarray(x, dtype=np.float64)
    lo, hi = x.min(0), x.max(0)
    side = max(hi - lo) or 1.0
    out = []
    for p in x:
        q = [min(max(int(np.floor((p[d] - lo[d]) * (2.0 ** 21 / side))), 0), 2 ** 21 - 1)
             for d in range(3)]
        bits = "".join(format(q[0], "021b")[b] + format(q[1], "021b")[b] + format(q[2], "021b")[b]
                       for b in range(21))
        out.append(int(bits, 2))
    return np.array(out, dtype=np.uint64)


def test_morton_keys_bit_layout():
    rng = np.random.default_rng(0)
    x = rng.uniform(-1, 2, (500, 3))
    x[3] = x.max(0)                     # a point on the upper corner clamps
    key, lo, side = T.morton_keys(x)
    assert np.array_equal(key, _keys_bruteforce(x))
    assert side == float(np.max(x.max(0) - x.min(0)))


def _check_topology(tr, leaf_cap):
    n = tr.keys.shape[0]
    assert tr.level[0] == 0 and tr.first[0] == 0 and tr.count[0] == n
    # BFS order: level non-decreasing, first increasing within a level
    lv = tr.level
    assert np.all(np.diff(lv) >= 0)
    for l in np.unique(lv):
        f = tr.first[lv == l]
        assert np.all(np.diff(f) > 0)
    covered = np.zeros(n, dtype=int)
    for k in range(tr.n_nodes):
        l, f, c = int(tr.level[k]), int(tr.first[k]), int(tr.count[k])
        shift = np.uint64(3 * (21 - l))
        pre = tr.keys[f:f + c] >> shift
        assert np.all(pre == pre[0])                          # one cell
        if f > 0:
            assert (tr.keys[f - 1] >> shift) != pre[0]        # maximal range
        if f + c < n:
            assert (tr.keys[f + c] >> shift) != pre[0]
        split = c > leaf_cap and l < 21
        assert (tr.n_child[k] > 0) == split
        if split:
            ch = np.arange(tr.child_first[k], tr.child_first[k] + tr.n_child[k])
            assert np.all(tr.parent[ch] == k)
            assert tr.first[ch[0]] == f
            assert np.all(tr.first[ch[1:]] == tr.first[ch[:-1]] + tr.count[ch[:-1]])
            assert tr.first[ch[-1]] + tr.count[ch[-1]] == f + c
        else:
            covered[f:f + c] += 1
        if k > 0:
            assert tr.count[tr.parent[k]] > leaf_cap
    assert np.all(covered == 1)                               # leaves partition


@pytest.mark.parametrize("leaf_cap", [1, 4, 16])
def test_topology_invariants(leaf_cap):
    ps = clustered_cloud(3000, 8, seed=5, dtype=np.float32)
    x = ps.x.astype(np.float64)
    x[10] = x[11]                                             # identical keys
    x[12] = x[11]
    tr = T.build_tree(x, leaf_cap)
    assert np.all(np.diff(tr.keys.astype(np.float64)) >= 0)
    _check_topology(tr, leaf_cap)


def test_topology_depth_limit_identical_points():
    x = np.zeros((40, 3))
    x[20:] = 1.0
    tr = T.build_tree(x, leaf_cap=4)
    _check_topology(tr, 4)
    leaves = tr.n_child == 0
    assert set(tr.level[leaves]) == {21}
    assert sorted(tr.count[leaves]) == [20, 20]


@pytest.mark.parametrize("cap", [8, 64])
def test_groups_invariants(cap):
    ps = clustered_cloud(4000, 8, seed=6)
    tr = T.build_tree(ps.x.astype(np.float64), 16)
    g = T.make_groups(tr, cap)
    assert g[0, 0] == 0 and np.all(g[1:, 0] == g[:-1, 0] + g[:-1, 1])
    assert g[-1, 0] + g[-1, 1] == ps.n
    assert np.all((g[:, 1] >= 1) & (g[:, 1] <= cap))
    # each group is one node, a slice of an over-full leaf, or a run of
    # consecutive whole small siblings that is greedy (the next small sibling
    # would not have fitted)
    ends = tr.first + tr.count
    for f, c in g:
        inside = np.nonzero((tr.first <= f) & (f + c <= ends))[0]
        k = inside[np.argmin(tr.count[inside])]
        if tr.n_child[k] == 0 and tr.count[k] > cap:
            assert (f - tr.first[k]) % cap == 0 and c == min(cap, ends[k] - f)
        elif tr.count[k] <= cap:
            assert f == tr.first[k] and c == tr.count[k]
        else:
            ch = np.arange(tr.child_first[k], tr.child_first[k] + tr.n_child[k])
            run = ch[(tr.first[ch] >= f) & (ends[ch] <= f + c)]
            assert tr.first[run[0]] == f and ends[run[-1]] == f + c
            assert np.all(tr.count[run] <= cap) and run.size >= 2
            nxt = run[-1] + 1
            if nxt < ch[-1] + 1 and tr.count[nxt] <= cap:
                assert c + tr.count[nxt] > cap


def test_theta_zero_reproduces_direct_with_sinks():
    ps = clustered_cloud(3000, 24, seed=9, dtype=np.float64)
    a, p, _ = T.tree_forward(ps.x, ps.m, ps.h, ps.n_gas, theta=0.0, order=2, leaf_cap=8, group_cap=32)
    ar, pr = direct.direct(ps.x, ps.m, ps.h)
    assert np.allclose(a, ar, rtol=1e-11, atol=1e-12 * np.abs(ar).max())
    assert np.allclose(p, pr, rtol=1e-12)


def test_no_target_inside_accepted_node():
    ps = uniform_sphere(2000, seed=1)
    L = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=0.9, leaf_cap=8, group_cap=32)
    tr = L.tree
    for g, (pc, pp) in L.gas_lists.items():
        f, c = L.groups[g]
        ff, cc = tr.first[pc], tr.count[pc]
        assert not np.any((ff < f + c) & (f < ff + cc))
        # opened-leaf particles plus accepted-node particles cover each target once
        cover = np.zeros(ps.n, dtype=int)
        for k in pc:
            cover[tr.first[k]:tr.first[k] + tr.count[k]] += 1
        cover[pp] += 1
        assert np.all(cover == 1)


def test_error_falls_with_theta_and_order():
    ps = uniform_sphere(4096, seed=0)
    ar, _ = direct.direct(ps.x, ps.m, ps.h)
    err = {}
    for order in (0, 2):
        for th in (0.3, 0.5, 0.8):
            a, _, _ = T.tree_forward(ps.x, ps.m, ps.h, ps.n_gas, theta=th, order=order)
            e = np.linalg.norm(a - ar, axis=1) / np.linalg.norm(ar, axis=1)
            err[order, th] = np.median(e)
    for order in (0, 2):
        assert err[order, 0.3] < err[order, 0.5] < err[order, 0.8]
    for th in (0.3, 0.5, 0.8):
        assert err[2, th] < 0.5 * err[0, th]


def test_multipole_truncation_scaling():
    rng = np.random.default_rng(4)
    k = 64
    cl = rng.uniform(0, 1, (k, 3)) * 0.1 + 0.45
    m = rng.uniform(0.5, 1.5, k)
    h = np.full(k, 1e-3)
    tr = T.build_tree(cl, leaf_cap=k)      # single leaf: root holds the cluster
    mom = T.node_moments(tr, cl, m, h)
    errs = {0: [], 2: []}
    for D in (1.0, 2.0, 4.0):
        tgt = np.array([0.5 + D, 0.5, 0.5 + 0.3 * D])
        xs = torch.tensor(np.vstack([cl[tr.order], tgt[None]]))
        ms = torch.tensor(np.concatenate([m[tr.order], [0.0]]))
        hs = torch.tensor(np.concatenate([h, [1e-3]]))
        ex, _ = direct.direct(np.vstack([cl, tgt[None]]), np.concatenate([m, [0.0]]),
                              np.concatenate([h, [1e-3]]), targets=[k])
        for order in (0, 2):
            M = torch.tensor(mom["M"])
            com = torch.tensor(mom["com"])
            Q = torch.tensor(mom["Q"])
            a, _ = T._eval_group(xs, ms, hs, np.array([k]), np.array([0]), np.zeros(0, np.int64),
                                 M, com, Q, np.array([0]), order, 1.0)
            errs[order].append(np.linalg.norm(a.numpy()[0] - ex[0]) / np.linalg.norm(ex[0]))
    r0 = np.array(errs[0])
    r2 = np.array(errs[2])
    # doubling the distance divides the relative error by ~4 (mono), ~8 (quad)
    assert np.all((r0[:-1] / r0[1:] > 3.2) & (r0[:-1] / r0[1:] < 4.8))
    assert np.all((r2[:-1] / r2[1:] > 6.0) & (r2[:-1] / r2[1:] < 10.0))


def _tree_loss(ps, lists, ga, gp, order, xt, mt, ht):
    a, p = T.tree_eval(xt, mt, ht, ps.n_gas, lists, 1.0, order)
    return (a * torch.tensor(ga)).sum() + (p * torch.tensor(gp)).sum()


def test_tree_adjoint_theta_zero_equals_direct_adjoint():
    ps = clustered_cloud(600, 6, seed=3, dtype=np.float64)
    ga = np.random.default_rng(1).standard_normal((ps.n, 3))
    gp = np.random.default_rng(2).standard_normal(ps.n)
    lists = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=0.0, leaf_cap=8, group_cap=32)
    xt = torch.tensor(ps.x, requires_grad=True)
    mt = torch.tensor(ps.m, requires_grad=True)
    ht = torch.tensor(ps.h, requires_grad=True)
    _tree_loss(ps, lists, ga, gp, 2, xt, mt, ht).backward()
    gx, gm, gh = direct.direct_vjp(ps.x, ps.m, ps.h, ga, gp)
    assert np.allclose(xt.grad.numpy(), gx, rtol=1e-8, atol=1e-9 * np.abs(gx).max())
    assert np.allclose(mt.grad.numpy(), gm, rtol=1e-8, atol=1e-9 * np.abs(gm).max())
    # sinks share one radius: ties split half/half in both oracles
    assert np.allclose(ht.grad.numpy(), gh, rtol=1e-8, atol=1e-9 * np.abs(gh).max())


def test_tree_adjoint_matches_frozen_list_differences():
    ps = clustered_cloud(800, 4, seed=4, dtype=np.float64)
    rng = np.random.default_rng(3)
    ga = rng.standard_normal((ps.n, 3))
    gp = rng.standard_normal(ps.n)
    lists = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=0.5, leaf_cap=8, group_cap=32)
    xt = torch.tensor(ps.x, requires_grad=True)
    mt = torch.tensor(ps.m, requires_grad=True)
    ht = torch.tensor(ps.h, requires_grad=True)
    _tree_loss(ps, lists, ga, gp, 2, xt, mt, ht).backward()
    eps = 1e-6
    for k in [0, 5, 400, ps.n - 1]:
        for d in range(3):
            xp = ps.x.copy()
            xp[k, d] += eps
            xm = ps.x.copy()
            xm[k, d] -= eps
            with torch.no_grad():
                lp = _tree_loss(ps, lists, ga, gp, 2, torch.tensor(xp), torch.tensor(ps.m), torch.tensor(ps.h))
                lm = _tree_loss(ps, lists, ga, gp, 2, torch.tensor(xm), torch.tensor(ps.m), torch.tensor(ps.h))
            fd = float(lp - lm) / (2 * eps)
            assert fd == pytest.approx(float(xt.grad[k, d]), rel=1e-5, abs=1e-7 * float(xt.grad.abs().max()))
        mp = ps.m.copy()
        mp[k] += eps
        mm = ps.m.copy()
        mm[k] -= eps
        with torch.no_grad():
            lp = _tree_loss(ps, lists, ga, gp, 2, torch.tensor(ps.x), torch.tensor(mp), torch.tensor(ps.h))
            lm = _tree_loss(ps, lists, ga, gp, 2, torch.tensor(ps.x), torch.tensor(mm), torch.tensor(ps.h))
        fd = float(lp - lm) / (2 * eps)
        assert fd == pytest.approx(float(mt.grad[k]), rel=1e-5, abs=1e-7 * float(mt.grad.abs().max()))


def test_lazy_moments_equal_eager_and_lists_agree():
    # the lazily computed moments are the same sums; walks over a few groups
    # give the same lists either way
    ps = clustered_cloud(6000, 20, seed=21, dtype=np.float64)
    tree = T.build_tree(ps.x, 16)
    eager = T.node_moments(tree, ps.x, ps.m, ps.h)
    lazy = T.LazyMoments(tree, ps.x, ps.m, ps.h)
    idx = np.array([0, 5, 17, tree.n_nodes - 1, 5])
    for name in ("M", "com", "Q", "hmax"):
        assert np.array_equal(lazy[name][idx], eager[name][idx])
    sel = [0, 3, 11]
    a = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, groups_sel=sel)
    b = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, groups_sel=sel, lazy=True)
    assert a.gas_lists.keys() == b.gas_lists.keys()
    for g in a.gas_lists:
        for u, v in zip(a.gas_lists[g], b.gas_lists[g]):
            assert np.array_equal(u, v)


def test_differentiable_moments_equal_plain_sums():
    # the torch moments that the adjoint differentiates are the same M, centre
    # of mass and traceless Q as the plain FP64 node sums (with and without a
    # particle selection)
    ps = clustered_cloud(3000, 12, seed=8, dtype=np.float64)
    tree = T.build_tree(ps.x, 8)
    xs = torch.tensor(ps.x[tree.order])
    ms = torch.tensor(ps.m[tree.order])
    nodes = np.arange(tree.n_nodes)
    for sel in (None, np.arange(ps.n) < ps.n_gas):
        mom = T.node_moments(tree, ps.x, ps.m, ps.h, sel=sel)
        ok = mom["M"] > 0
        M, com, Q = T._moments_torch(tree, xs, ms, nodes[ok], None if sel is None else sel[tree.order])
        assert np.allclose(M.numpy(), mom["M"][ok], rtol=1e-13, atol=0)
        scale = np.abs(ps.x).max()
        assert np.allclose(com.numpy(), mom["com"][ok], rtol=0, atol=1e-13 * scale)
        qs = (mom["M"][ok] * (tree.side / 2.0 ** tree.level[ok]) ** 2)[:, None, None]
        assert np.all(np.abs(Q.numpy() - mom["Q"][ok]) <= 1e-13 * qs)
