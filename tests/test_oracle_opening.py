"""Pins of the oracle's opening rule (Sec. 2.2) against the per-target rule.

The paper states its criteria for one target point x_t and one node of cube
side L, mass M and centre of mass c: the node may be used as a multipole only
if L <= Theta |c - x_t| (Barnes-Hut) and, with the acceleration-based
criterion, G M L^2 / |c - x_t|^4 <= alpha |g_t| (g_t the target's previous
field).  The group walk makes one decision for a set of targets; these tests
re-derive, by brute force over every target and every node, that

  * every accepted node passes both per-target tests for EVERY gas target of
    the group, contains no target and holds no pair inside the softening
    radius max(h_t, h_j) (Sec. 2.2.1), and has positive mass;
  * every opened node fails at least one of the group-level tests;
  * accepted nodes and opened leaves partition the particles.

L is recomputed here from the root side and the node level (side / 2^level)
and r from a projection of c onto the group box, not from the oracle's own
expressions.  Two planted mistakes in the oracle (cube side halved; distance
measured from the group centre) must be caught.
"""
import numpy as np
import pytest
import torch

from oracle import direct
from oracle import tree as T
from synth import clustered_cloud, uniform_sphere


def _opened_nodes(tree, pc, pp):
    """Nodes the walk opened: ancestors of accepted nodes and of opened
    leaves, plus the opened leaves themselves."""
    leaf_of = np.full(tree.keys.shape[0], -1, dtype=np.int64)
    for k in np.nonzero(tree.n_child == 0)[0]:
        leaf_of[tree.first[k]:tree.first[k] + tree.count[k]] = k
    leaves = np.unique(leaf_of[pp]) if pp.size else np.zeros(0, np.int64)
    opened = set(int(k) for k in leaves)
    for k in list(pc) + list(leaves):
        p = tree.parent[k]
        while p >= 0:
            opened.add(int(p))
            p = tree.parent[p]
    return np.array(sorted(opened), dtype=np.int64), leaves


def check_lists(x, m, h, n_gas, lists, theta, alpha=None, field=None, G=1.0):
    """Violations of the per-target rule (a list of strings; empty = pass)."""
    tree = lists.tree
    xs = np.asarray(x, np.float64)[tree.order]
    hs = np.asarray(h, np.float64)[tree.order]
    ms = np.asarray(m, np.float64)[tree.order]
    gmag = None if alpha is None else np.linalg.norm(np.asarray(field, np.float64), axis=1)[tree.order]
    L_of = tree.side / 2.0 ** tree.level.astype(np.float64)
    # cube corners from the integer cell coordinates of the first key
    bad = []
    for g, (pc, pp) in lists.gas_lists.items():
        f, c = lists.groups[g]
        mem = np.arange(f, f + c)
        tg = mem[~lists.is_sink_sorted[mem]]
        blo, bhi = xs[mem].min(0), xs[mem].max(0)
        hg = hs[mem].max()
        # partition
        cover = np.zeros(xs.shape[0], dtype=int)
        for k in pc:
            cover[tree.first[k]:tree.first[k] + tree.count[k]] += 1
        cover[pp] += 1
        if not np.all(cover == 1):
            bad.append(f"group {g}: accepted nodes and opened leaves do not partition")
        for k in pc:
            kf, kc = tree.first[k], tree.count[k]
            Mk = ms[kf:kf + kc].sum()
            if not Mk > 0:
                bad.append(f"group {g}: accepted node {k} has no mass")
                continue
            ck = (ms[kf:kf + kc, None] * xs[kf:kf + kc]).sum(0) / Mk
            r = np.linalg.norm(ck[None, :] - xs[tg], axis=1)
            L = L_of[k]
            if np.any(L > theta * r * (1 + 1e-12)):
                bad.append(f"group {g}: node {k} accepted with L/r > theta for a target")
            if alpha is not None:
                lhs = G * Mk * L * L / r ** 4
                if np.any(lhs > alpha * gmag[tg] * (1 + 1e-12)):
                    bad.append(f"group {g}: node {k} accepted with G M L^2/r^4 > alpha |g|")
            if np.any((tg >= kf) & (tg < kf + kc)):
                bad.append(f"group {g}: node {k} contains a target")
            d = np.linalg.norm(xs[kf:kf + kc][None, :, :] - xs[tg][:, None, :], axis=2)
            if np.any(d < np.maximum(hs[tg][:, None], hs[kf:kf + kc][None, :])):
                bad.append(f"group {g}: node {k} holds a softened pair")
        opened, _ = _opened_nodes(tree, pc, pp)
        clo, chi, _ = tree.cube()
        gmin = None if alpha is None else gmag[mem].min()
        for k in opened:
            kf, kc = tree.first[k], tree.count[k]
            Mk = ms[kf:kf + kc].sum()
            if not Mk > 0:
                continue
            ck = (ms[kf:kf + kc, None] * xs[kf:kf + kc]).sum(0) / Mk
            r = np.linalg.norm(ck - np.clip(ck, blo, bhi))
            L = L_of[k]
            near = (kf < f + c) and (f < kf + kc)
            near |= bool(np.all((clo[k] <= bhi) & (blo <= chi[k])))
            gapv = np.maximum(np.maximum(clo[k] - bhi, blo - chi[k]), 0.0)
            near |= np.linalg.norm(gapv) < max(hs[kf:kf + kc].max(), hg) * (1 + 1e-12)
            why = near or L > theta * r * (1 - 1e-12)
            if alpha is not None:
                why = why or G * Mk * L * L > alpha * gmin * r ** 4 * (1 - 1e-12)
            if not why:
                bad.append(f"group {g}: node {k} opened without a reason")
    return bad


@pytest.fixture(scope="module")
def cloud():
    ps = clustered_cloud(2500, 6, seed=31, dtype=np.float64)
    field, _ = direct.direct(ps.x, ps.m, ps.h)
    return ps, field


@pytest.mark.parametrize("theta", [0.3, 0.5, 0.9])
def test_barnes_hut_rule_per_target(cloud, theta):
    ps, _ = cloud
    lists = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=theta, leaf_cap=8, group_cap=32)
    assert sum(v[0].size for v in lists.gas_lists.values()) > 0   # some nodes accepted
    bad = check_lists(ps.x, ps.m, ps.h, ps.n_gas, lists, theta)
    assert not bad, bad[:5]


@pytest.mark.parametrize("theta,alpha", [(0.5, 0.01), (0.7, 0.002), (0.9, 0.05)])
def test_relative_rule_per_target(cloud, theta, alpha):
    ps, field = cloud
    lists = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=theta, leaf_cap=8, group_cap=32,
                         alpha=alpha, field=field)
    bad = check_lists(ps.x, ps.m, ps.h, ps.n_gas, lists, theta, alpha, field)
    assert not bad, bad[:5]


def test_checker_catches_half_side(cloud, monkeypatch):
    # planted mistake: the walk sees cube sides half as long as they are
    ps, _ = cloud
    orig = T.Tree.cube

    def half(self):
        clo, chi, cell = orig(self)
        return clo, chi, 0.5 * cell

    monkeypatch.setattr(T.Tree, "cube", half)
    lists = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=0.5, leaf_cap=8, group_cap=32)
    monkeypatch.undo()
    bad = check_lists(ps.x, ps.m, ps.h, ps.n_gas, lists, 0.5)
    assert any("L/r > theta" in b for b in bad)


def test_checker_catches_distance_from_group_centre(cloud):
    # planted mistake: r measured from the centre of the group box, i.e. the
    # walk run with a box shrunk to its centre (guards kept on the true box
    # would hide nothing: the per-target test is what must fail)
    ps, _ = cloud
    lists = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=0.5, leaf_cap=8, group_cap=32)
    tree = lists.tree
    xs = ps.x[tree.order]
    clo, chi, cell = tree.cube()
    for g in list(lists.gas_lists):
        f, c = lists.groups[g]
        cen = 0.5 * (xs[f:f + c].min(0) + xs[f:f + c].max(0))
        lists.gas_lists[g] = T.walk(tree, tree.mom["all"], clo, chi, cell, cen, cen,
                                    ps.h[tree.order][f:f + c].max(), f, c, 0.5)
    bad = check_lists(ps.x, ps.m, ps.h, ps.n_gas, lists, 0.5)
    assert any("L/r > theta" in b for b in bad)


def test_checker_catches_relative_rule_on_group_mean(cloud):
    # planted mistake: the relative test fed the group's mean |g| instead of
    # the smallest -- some member's accuracy demand is then violated
    ps, field = cloud
    alpha = 0.002
    lists = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=0.9, leaf_cap=8, group_cap=32)
    tree = lists.tree
    xs, hs = ps.x[tree.order], ps.h[tree.order]
    gmag = np.linalg.norm(field, axis=1)[tree.order]
    clo, chi, cell = tree.cube()
    for g in list(lists.gas_lists):
        f, c = lists.groups[g]
        lists.gas_lists[g] = T.walk(tree, tree.mom["all"], clo, chi, cell, xs[f:f + c].min(0),
                                    xs[f:f + c].max(0), hs[f:f + c].max(), f, c, 0.9,
                                    alpha * gmag[f:f + c].mean())
    bad = check_lists(ps.x, ps.m, ps.h, ps.n_gas, lists, 0.9, alpha, field)
    assert any("alpha |g|" in b for b in bad)


def test_alpha_infinite_gives_barnes_hut_lists(cloud):
    ps, field = cloud
    a = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=0.5, leaf_cap=8, group_cap=32)
    for alpha in (np.inf, 1e300):
        b = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=0.5, leaf_cap=8, group_cap=32,
                         alpha=alpha, field=field)
        assert a.gas_lists.keys() == b.gas_lists.keys()
        for g in a.gas_lists:
            for u, v in zip(a.gas_lists[g], b.gas_lists[g]):
                assert np.array_equal(u, v)
        for p in a.sink_lists:
            for u, v in zip(a.sink_lists[p], b.sink_lists[p]):
                assert np.array_equal(u, v)


def test_alpha_zero_gives_direct_sum(cloud):
    # every node of positive mass fails G M L^2 <= 0: the tree opens
    # everything and reproduces the (independent, C) direct sum
    ps, field = cloud
    a, p, lists = T.tree_forward(ps.x, ps.m, ps.h, ps.n_gas, theta=0.5, order=2, leaf_cap=8,
                                 group_cap=32, alpha=0.0, field=field)
    assert all(v[0].size == 0 for v in lists.gas_lists.values())
    ar, pr = direct.direct(ps.x, ps.m, ps.h)
    assert np.allclose(a, ar, rtol=1e-11, atol=1e-12 * np.abs(ar).max())
    assert np.allclose(p, pr, rtol=1e-12)


def test_error_falls_with_alpha():
    # uniform sphere, monopole: the relative criterion tightens the accuracy
    # of the lowest-|g| targets (near the centre) that theta alone leaves worst
    ps = uniform_sphere(4096, seed=0)
    ar, _ = direct.direct(ps.x, ps.m, ps.h)
    p99 = []
    for alpha in (None, 0.02, 0.005, 0.001):
        a, _, _ = T.tree_forward(ps.x, ps.m, ps.h, ps.n_gas, theta=0.5, order=0, alpha=alpha,
                                 field=ar)
        e = np.linalg.norm(a - ar, axis=1) / np.linalg.norm(ar, axis=1)
        p99.append(np.quantile(e, 0.99))
    assert all(p99[i + 1] < p99[i] for i in range(len(p99) - 1)), p99


def test_massless_nodes_are_opened_not_skipped():
    # a cluster of massless tracers far from the massive particles: its nodes
    # have M = 0 and must reach the lists as particle pairs, so the tree's
    # mass derivative at theta = 0.5 (autograd of the frozen-list sum) equals
    # the direct sum's for the tracers
    rng = np.random.default_rng(5)
    xa = rng.standard_normal((400, 3)) * 0.05
    xb = rng.standard_normal((100, 3)) * 0.02 + np.array([2.0, 0.0, 0.0])
    x = np.vstack([xa, xb])
    m = np.concatenate([np.full(400, 1.0 / 400), np.zeros(100)])
    h = np.full(500, 0.01)
    lists = T.tree_lists(x, m, h, 500, theta=0.5, leaf_cap=8, group_cap=32)
    pp_all = np.concatenate([v[1] for v in lists.gas_lists.values()])
    tracer_sorted = np.nonzero(lists.tree.order >= 400)[0]
    assert np.isin(tracer_sorted, pp_all).all()
    xt = torch.tensor(x, requires_grad=True)
    mt = torch.tensor(m, requires_grad=True)
    ht = torch.tensor(h, requires_grad=True)
    rng = np.random.default_rng(6)
    ga, gp = rng.standard_normal((500, 3)), rng.standard_normal(500)
    a, p = T.tree_eval(xt, mt, ht, 500, lists, 1.0, 2)
    ((a * torch.tensor(ga)).sum() + (p * torch.tensor(gp)).sum()).backward()
    # the tracers' own mass derivative: only pair terms with every target
    # (accepted massive nodes never involve a tracer as a source)
    _, gm_direct, _ = direct.direct_vjp(x, m, h, ga, gp)
    gm_tree = mt.grad.numpy()
    # the direct sum's derivative differs from the tree's by the tree's
    # truncation error only; at a distance of 2 with theta 0.5 that is small
    rel = np.abs(gm_tree[400:] - gm_direct[400:]) / np.abs(gm_direct[400:]).max()
    assert np.max(rel) < 2e-3
    assert np.all(gm_tree[400:] != 0.0)
