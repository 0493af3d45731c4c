"""oracle/tree.py -- TEST INFRASTRUCTURE ONLY (never imported by the library).

A slow, plain CPU Barnes-Hut octree for the softened self-gravity of the paper
(Sec. 2.2 "Gravity"; softening rules of Sec. 2.2.1), written to define exactly
what the GPU tree path must produce:

* the octree (Sec. 2.2: the domain is subdivided recursively into octants).
  Cells are cubes addressed by 21-bit-per-axis Morton keys; a cell is split
  while it holds more than `leaf_cap` particles and is above level 21;
* node moments: mass, centre of mass and the traceless quadrupole about it
  (the paper uses monopoles; quadrupoles are an option of this library),
  accumulated by plain FP64 sums over each node's particles;
* target groups and the group walk with the Barnes-Hut opening angle
  theta = L/r (Sec. 2.2; the paper's fiducial value is 0.5);
* the evaluation: multipole terms for accepted nodes, softened particle pairs
  for opened leaves.

Reading of the paper used throughout (its text gives the criterion for one
target point; a group walk must make one decision for a set of targets):
a node is opened for a group when ANY of these holds, else it is accepted as
a multipole:
  (a) L^2 > theta^2 r^2, r = distance from the node centre of mass to the
      group's bounding box (0 if inside) -- the per-target test made safe for
      every target of the group;
  (r) only when a relative tolerance alpha is given: G M L^2 > alpha g r^4,
      with g the smallest previous field magnitude |g| among the group's
      members and r as in (a) -- Sec. 2.2's acceleration-based criterion (the
      node's quadrupole-order error G M L^2 / r^4 must stay below a fraction
      alpha of the target's total field), which the paper always combines
      with (a); taking the smallest r and the smallest |g| makes it hold for
      every member;
  (b) the node's cube meets the group's bounding box, or the node holds one of
      the group's particles -- a target never sits inside an accepted node;
  (c) the gap between cube and bounding box is below the larger of the two
      maximum softening radii -- every softened pair (r < max(S_i,S_j),
      Sec. 2.2.1) is summed particle by particle, so nodes carry no softening;
  (z) the node's mass is zero: it has no centre of mass to expand about, so
      its (massless) particles are summed as pairs, which keeps the mass
      derivative of the frozen-list approximation equal to the direct sum's.
All decisions are taken in FP64 with separate multiply and add steps.

Sink particles: targets that are sinks see gas through the tree (node moments
over gas only) and other sinks through an exact FP64 direct sum.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import torch

LEVELS = 21
KEY_BITS = 3 * LEVELS


# --------------------------------------------------------------- Morton keys

def _spread(q):
    k = np.zeros(q.shape, dtype=np.uint64)
    for b in range(LEVELS):
        k |= ((q >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return k


def morton_keys(x):
    """Root cube and 63-bit keys, x-bit most significant in each triple.

    lo = per-axis minimum, side = largest extent (1 if all points coincide),
    s = 2^21/side, q_d = floor((x_d - lo_d) * s) clamped to [0, 2^21 - 1].
    """
    x = np.asarray(x, dtype=np.float64)
    lo = x.min(axis=0)
    hi = x.max(axis=0)
    side = float(np.max(hi - lo))
    if side == 0.0:
        side = 1.0
    s = float(2.0 ** LEVELS) / side
    q = np.floor((x - lo) * s)
    q = np.clip(q, 0.0, float(2 ** LEVELS - 1)).astype(np.uint64)
    key = (_spread(q[:, 0]) << np.uint64(2)) | (_spread(q[:, 1]) << np.uint64(1)) | _spread(q[:, 2])
    return key, lo, side


def deinterleave(code, level):
    """Integer cube coordinates of a level-`level` prefix (x, y, z)."""
    code = np.asarray(code, dtype=np.uint64)
    out = []
    for axis_shift in (2, 1, 0):
        v = np.zeros(code.shape, dtype=np.uint64)
        for b in range(level):
            v |= ((code >> np.uint64(3 * b + axis_shift)) & np.uint64(1)) << np.uint64(b)
        out.append(v.astype(np.int64))
    return np.stack(out, axis=-1)


# --------------------------------------------------------------- topology

@dataclasses.dataclass
class Tree:
    keys: np.ndarray      # sorted keys (uint64)
    order: np.ndarray     # sorted position -> input index
    lo: np.ndarray
    side: float
    level: np.ndarray
    first: np.ndarray
    count: np.ndarray
    parent: np.ndarray
    child_first: np.ndarray
    n_child: np.ndarray
    leaf_cap: int
    # moments (filled by node_moments)
    mom: dict = dataclasses.field(default_factory=dict)

    @property
    def n_nodes(self):
        return int(self.level.shape[0])

    def is_leaf(self):
        return self.n_child == 0

    def cube(self):
        """Per-node cube (lo corner, hi corner, side) in FP64."""
        lvl = self.level
        pref = self.keys[self.first] >> (np.uint64(3) * (np.uint64(LEVELS) - lvl.astype(np.uint64)))
        ij = np.zeros((lvl.shape[0], 3), dtype=np.int64)
        for l in np.unique(lvl):
            sel = lvl == l
            ij[sel] = deinterleave(pref[sel], int(l))
        cell = self.side * np.ldexp(1.0, -lvl.astype(np.int64))
        clo = self.lo[None, :] + ij.astype(np.float64) * cell[:, None]
        chi = self.lo[None, :] + (ij + 1).astype(np.float64) * cell[:, None]
        return clo, chi, cell


def build_topology(keys_sorted, leaf_cap):
    """Breadth-first octree over sorted keys.

    Node = occupied cell.  A node is split into its occupied octants (in
    octant order) when it holds more than leaf_cap particles and its level is
    below 21.  The node array lists level 0, then level 1, ..., each level in
    particle order; children of a node are therefore contiguous.
    """
    n = keys_sorted.shape[0]
    level, first, count, parent = [0], [0], [n], [-1]
    child_first, n_child = [], []
    i = 0
    while i < len(level):
        l, f, c = level[i], first[i], count[i]
        if c > leaf_cap and l < LEVELS:
            shift = np.uint64(3 * (LEVELS - l - 1))
            dig = ((keys_sorted[f:f + c] >> shift) & np.uint64(7)).astype(np.int64)
            bounds = np.searchsorted(dig, np.arange(9), side="left")
            child_first.append(len(level))
            nc = 0
            for o in range(8):
                cnt = int(bounds[o + 1] - bounds[o])
                if cnt:
                    level.append(l + 1)
                    first.append(f + int(bounds[o]))
                    count.append(cnt)
                    parent.append(i)
                    nc += 1
            n_child.append(nc)
        else:
            child_first.append(-1)
            n_child.append(0)
        i += 1
    a = lambda v, t=np.int64: np.asarray(v, dtype=t)
    return a(level), a(first), a(count), a(parent), a(child_first), a(n_child)


def build_tree(x, leaf_cap=16):
    key, lo, side = morton_keys(x)
    order = np.argsort(key, kind="stable")          # ties keep input order
    ks = key[order]
    level, first, count, parent, cf, nc = build_topology(ks, leaf_cap)
    return Tree(ks, order.astype(np.int64), lo, side, level, first, count, parent,
                cf, nc, leaf_cap)


# --------------------------------------------------------------- moments

def _sorted_fields(tree, x, m, h, sel):
    xs = np.asarray(x, dtype=np.float64)[tree.order]
    ms = np.asarray(m, dtype=np.float64)[tree.order]
    hs = np.asarray(h, dtype=np.float64)[tree.order]
    if sel is not None:
        w = np.asarray(sel, dtype=bool)[tree.order]
        ms = np.where(w, ms, 0.0)
        hs = np.where(w, hs, 0.0)
    return xs, ms, hs


def _one_node(xs, ms, hs, f, c):
    """M, centre of mass, traceless Q and max h of the particles [f, f + c)."""
    mk = ms[f:f + c]
    xk = xs[f:f + c]
    Mk = mk.sum()
    ck = np.zeros(3)
    Qk = np.zeros((3, 3))
    if Mk > 0:
        ck = (mk[:, None] * xk).sum(axis=0) / Mk
        y = xk - ck
        S = (mk[:, None, None] * y[:, :, None] * y[:, None, :]).sum(axis=0)
        Qk = 3.0 * S - np.trace(S) * np.eye(3)
    return Mk, ck, Qk, hs[f:f + c].max()


def node_moments(tree, x, m, h, sel=None):
    """M, centre of mass, traceless quadrupole Q = 3S - tr(S) I and max h.

    S = sum m (x - com)(x - com)^T over the node's particles; `sel` (bool per
    input particle) restricts the sums (e.g. gas only).  Sums are plain FP64.
    """
    xs, ms, hs = _sorted_fields(tree, x, m, h, sel)
    nn = tree.n_nodes
    M = np.zeros(nn)
    com = np.zeros((nn, 3))
    Q = np.zeros((nn, 3, 3))
    hmax = np.zeros(nn)
    for k in range(nn):
        M[k], com[k], Q[k], hmax[k] = _one_node(xs, ms, hs, tree.first[k], tree.count[k])
    return {"M": M, "com": com, "Q": Q, "hmax": hmax}


class LazyMoments:
    """The same per-node sums as node_moments, computed the first time a node
    is indexed -- for walking a few groups of a tree with millions of nodes.
    `mom["M"][idx]`, `mom["com"][idx]`, ... behave like the arrays."""

    class _Field:
        def __init__(self, owner, name):
            self.owner, self.name = owner, name

        def __getitem__(self, idx):
            self.owner._ensure(idx)
            return self.owner.arr[self.name][idx]

    def __init__(self, tree, x, m, h, sel=None):
        self.tree = tree
        self.xs, self.ms, self.hs = _sorted_fields(tree, x, m, h, sel)
        nn = tree.n_nodes
        self.done = np.zeros(nn, dtype=bool)
        self.arr = {"M": np.zeros(nn), "com": np.zeros((nn, 3)), "Q": np.zeros((nn, 3, 3)),
                    "hmax": np.zeros(nn)}

    def _ensure(self, idx):
        ks = np.unique(np.atleast_1d(np.arange(self.tree.n_nodes)[idx]))
        for k in ks[~self.done[ks]]:
            out = _one_node(self.xs, self.ms, self.hs, self.tree.first[k], self.tree.count[k])
            for name, v in zip(("M", "com", "Q", "hmax"), out):
                self.arr[name][k] = v
            self.done[k] = True

    def __getitem__(self, name):
        return LazyMoments._Field(self, name)


# --------------------------------------------------------------- groups

def make_groups(tree, group_cap=64):
    """Target groups: contiguous Morton runs of at most group_cap particles.

    Walking down from the root, a node holding at most group_cap particles is
    taken whole; consecutive such children of a split node are packed into one
    run while the run stays within group_cap; an over-full leaf (only at level
    21) is cut into consecutive slices of group_cap.  Runs are listed in
    particle order and partition all particles.
    """
    out = []

    def visit(k):
        f, c = int(tree.first[k]), int(tree.count[k])
        if c <= group_cap:
            out.append((f, c))
            return
        if tree.n_child[k] == 0:
            for s in range(f, f + c, group_cap):
                out.append((s, min(group_cap, f + c - s)))
            return
        run_f, run_c = -1, 0
        for ch in range(tree.child_first[k], tree.child_first[k] + tree.n_child[k]):
            cc = int(tree.count[ch])
            if cc > group_cap:
                if run_c:
                    out.append((run_f, run_c))
                    run_c = 0
                visit(ch)
                continue
            if run_c + cc > group_cap:
                out.append((run_f, run_c))
                run_c = 0
            if run_c == 0:
                run_f = int(tree.first[ch])
            run_c += cc
        if run_c:
            out.append((run_f, run_c))

    visit(0)
    return np.asarray(out, dtype=np.int64).reshape(-1, 2)


# --------------------------------------------------------------- walk

def field_norms(acc_prev):
    """|g| per particle from a previous field (n, 3): sqrt((gx^2 + gy^2) + gz^2)
    in FP64, each step separately rounded."""
    g = np.asarray(acc_prev, dtype=np.float64)
    return np.sqrt((g[:, 0] * g[:, 0] + g[:, 1] * g[:, 1]) + g[:, 2] * g[:, 2])


def walk(tree, mom, clo, chi, cell, blo, bhi, hg, gfirst, gcount, theta, ag=None, G=1.0):
    """Interaction lists of one group: (accepted nodes, opened-leaf particles).

    Particles are returned as sorted positions.  `ag` = alpha * (smallest
    previous |g| of the group's members) switches on the relative criterion
    (r); None leaves only the opening angle and the guards.
    """
    th2 = theta * theta
    M, com, hmax = mom["M"], mom["com"], mom["hmax"]
    front = np.array([0], dtype=np.int64)
    pc, pp = [], []
    gl = gfirst + gcount
    while front.size:
        f = tree.first[front]
        c = tree.count[front]
        overlap = (f < gl) & (gfirst < f + c)
        lo, hi = clo[front], chi[front]
        meets = np.all((lo <= bhi[None, :]) & (blo[None, :] <= hi), axis=1)
        gap = np.maximum(np.maximum(lo - bhi[None, :], blo[None, :] - hi), 0.0)
        dbb2 = (gap[:, 0] * gap[:, 0] + gap[:, 1] * gap[:, 1]) + gap[:, 2] * gap[:, 2]
        hm = np.maximum(hmax[front], hg)
        soft = dbb2 < hm * hm
        cm = com[front]
        e = np.maximum(np.maximum(blo[None, :] - cm, cm - bhi[None, :]), 0.0)
        r2 = (e[:, 0] * e[:, 0] + e[:, 1] * e[:, 1]) + e[:, 2] * e[:, 2]
        L = cell[front]
        L2 = L * L
        angle = L2 > (th2 * r2)
        Mf = M[front]
        opened = overlap | meets | soft | angle | ~(Mf > 0.0)
        if ag is not None:
            with np.errstate(invalid="ignore"):   # inf * 0 (alpha = inf, r = 0) is not open
                opened |= ((G * Mf) * L2) > (ag * (r2 * r2))
        pc.append(front[~opened])
        op = front[opened]
        leaf = tree.n_child[op] == 0
        for k in op[leaf]:
            pp.append(np.arange(tree.first[k], tree.first[k] + tree.count[k]))
        inner = op[~leaf]
        if inner.size:
            front = np.concatenate([np.arange(tree.child_first[k], tree.child_first[k] + tree.n_child[k])
                                    for k in inner])
        else:
            front = np.zeros(0, dtype=np.int64)
    pc = np.concatenate(pc) if pc else np.zeros(0, np.int64)
    pp = np.concatenate(pp) if pp else np.zeros(0, np.int64)
    return pc.astype(np.int64), pp.astype(np.int64)


# --------------------------------------------------------------- kernel (torch)

def _kernel_FP(r, h):
    """Softened force and potential factors (M4 cubic spline, support h)."""
    u = r / h
    u2, u3 = u * u, u * u * u
    u4, u5 = u3 * u, u3 * u2
    h3 = h * h * h
    safe_u = torch.where(u > 0.25, u, torch.full_like(u, 0.25))
    safe_r = torch.where(r > 0, r, torch.ones_like(r))
    Fa = (32.0 / 3.0 - 192.0 / 5.0 * u2 + 32.0 * u3) / h3
    Fb = (64.0 / 3.0 - 48.0 * u + 192.0 / 5.0 * u2 - 32.0 / 3.0 * u3
          - 1.0 / (15.0 * safe_u ** 3)) / h3
    Fn = 1.0 / safe_r ** 3
    Pa = (14.0 / 5.0 - 16.0 / 3.0 * u2 + 48.0 / 5.0 * u4 - 32.0 / 5.0 * u5) / h
    Pb = (16.0 / 5.0 - 1.0 / (15.0 * safe_u) - 32.0 / 3.0 * u2 + 16.0 * u3
          - 48.0 / 5.0 * u4 + 32.0 / 15.0 * u5) / h
    Pn = 1.0 / safe_r
    F = torch.where(u < 0.5, Fa, torch.where(u < 1.0, Fb, Fn))
    P = torch.where(u < 0.5, Pa, torch.where(u < 1.0, Pb, Pn))
    return F, P


def _safe_norm(d):
    r2 = (d * d).sum(-1)
    pos = r2 > 0
    r = torch.sqrt(torch.where(pos, r2, torch.ones_like(r2)))
    return torch.where(pos, r, torch.zeros_like(r))


# --------------------------------------------------------------- full pass

@dataclasses.dataclass
class TreeLists:
    tree: Tree
    groups: np.ndarray             # (n_groups, 2) first, count
    gas_lists: dict                # group id -> (pc, pp)
    sink_lists: dict               # sorted pos of sink -> (pc, pp) with gas moments
    is_sink_sorted: np.ndarray
    n_pc: int = 0
    n_pp: int = 0


def tree_lists(x, m, h, n_gas, theta=0.5, leaf_cap=16, group_cap=64, groups_sel=None,
               lazy=False, alpha=None, field=None, G=1.0):
    """Build the tree and every interaction list (optionally for some groups;
    `lazy` computes node moments only where the walks look).

    alpha (>= 0) with field (previous accelerations, (n, 3), input order)
    adds the relative criterion: a group uses alpha times the smallest |g| of
    its members, a sink target alpha times its own |g|.
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    tree = build_tree(x, leaf_cap)
    is_sink = np.arange(n) >= n_gas
    moments = LazyMoments if lazy else node_moments
    tree.mom["all"] = moments(tree, x, m, h)
    tree.mom["gas"] = moments(tree, x, m, h, sel=~is_sink)
    clo, chi, cell = tree.cube()
    groups = make_groups(tree, group_cap)
    xs = x[tree.order]
    hs = np.asarray(h, dtype=np.float64)[tree.order]
    sink_sorted = is_sink[tree.order]
    gmag = None
    if alpha is not None:
        if field is None:
            raise ValueError("the relative criterion needs a previous field")
        gmag = field_norms(field)[tree.order]
    gl, sl = {}, {}
    n_pc = n_pp = 0
    gsel = range(groups.shape[0]) if groups_sel is None else groups_sel
    for g in gsel:
        f, c = groups[g]
        if np.all(sink_sorted[f:f + c]):
            continue
        blo, bhi = xs[f:f + c].min(axis=0), xs[f:f + c].max(axis=0)
        hg = hs[f:f + c].max()
        ag = None if gmag is None else alpha * gmag[f:f + c].min()
        pc, pp = walk(tree, tree.mom["all"], clo, chi, cell, blo, bhi, hg, f, c, theta, ag, G)
        gl[g] = (pc, pp)
        ng = int((~sink_sorted[f:f + c]).sum())
        n_pc += ng * pc.size
        n_pp += ng * pp.size
        for p in range(f, f + c):
            if sink_sorted[p]:
                sl[p] = None
    if groups_sel is None:
        for p in np.nonzero(sink_sorted)[0]:
            sl[int(p)] = None
    for p in list(sl):
        ag = None if gmag is None else alpha * gmag[p]
        pc, pp = walk(tree, tree.mom["gas"], clo, chi, cell, xs[p], xs[p], hs[p], p, 1, theta,
                      ag, G)
        pp = pp[~sink_sorted[pp]]
        sl[p] = (pc, pp)
    return TreeLists(tree, groups, gl, sl, sink_sorted, n_pc, n_pp)


def _moments_torch(tree, xs, ms, nodes, sel_sorted):
    """Differentiable M, com, Q of `nodes` recomputed from sorted particles."""
    f = tree.first[nodes]
    c = tree.count[nodes]
    memb_node = np.repeat(np.arange(nodes.size), c)
    memb_part = np.concatenate([np.arange(a, a + b) for a, b in zip(f, c)]) if nodes.size else np.zeros(0, np.int64)
    mm = ms[memb_part]
    if sel_sorted is not None:
        mm = mm * torch.as_tensor(sel_sorted[memb_part], dtype=ms.dtype)
    xp = xs[memb_part]
    idx = torch.as_tensor(memb_node)
    M = torch.zeros(nodes.size, dtype=xs.dtype).index_add(0, idx, mm)
    mx = torch.zeros(nodes.size, 3, dtype=xs.dtype).index_add(0, idx, mm[:, None] * xp)
    com = mx / M[:, None]
    y = xp - com[idx]
    S = torch.zeros(nodes.size, 3, 3, dtype=xs.dtype).index_add(
        0, idx, mm[:, None, None] * y[:, :, None] * y[:, None, :])
    tr = S[:, 0, 0] + S[:, 1, 1] + S[:, 2, 2]
    Q = 3.0 * S - tr[:, None, None] * torch.eye(3, dtype=xs.dtype)
    return M, com, Q


def _eval_group(xs, ms, hs, tgt, pc, pp, M, com, Q, node_row, order, G, skip_self=True):
    """Accelerations and potentials of sorted targets `tgt` from one list."""
    xt = xs[tgt]
    a = torch.zeros(len(tgt), 3, dtype=xs.dtype)
    phi = torch.zeros(len(tgt), dtype=xs.dtype)
    if pc.size:
        rows = torch.as_tensor(node_row[pc])
        r = xt[:, None, :] - com[rows][None, :, :]          # target - com
        rho2 = (r * r).sum(-1)
        rho = torch.sqrt(rho2)
        irho = 1.0 / rho
        Mn = M[rows][None, :]
        a = a - G * (Mn * irho ** 3)[..., None].mul(r).sum(1)
        phi = phi - G * (Mn * irho).sum(1)
        if order == 2:
            Qn = Q[rows][None, :, :, :]
            Qr = (Qn * r[..., None, :]).sum(-1)
            rQr = (Qr * r).sum(-1)
            a = a + G * (Qr * (irho ** 5)[..., None]).sum(1)
            a = a - G * (2.5 * rQr * irho ** 7)[..., None].mul(r).sum(1)
            phi = phi - G * (0.5 * rQr * irho ** 5).sum(1)
    if pp.size:
        src = torch.as_tensor(pp)
        d = xs[src][None, :, :] - xt[:, None, :]
        r = _safe_norm(d)
        hij = torch.maximum(hs[torch.as_tensor(tgt)][:, None], hs[src][None, :])
        F, P = _kernel_FP(r, hij)
        mj = ms[src][None, :]
        keep = torch.as_tensor(np.asarray(tgt)[:, None] != pp[None, :], dtype=xs.dtype)
        a = a + G * ((keep * mj * F)[..., None] * d).sum(1)
        phi = phi - G * (keep * mj * P).sum(1)
    return a, phi


def tree_eval(x, m, h, n_gas, lists, G=1.0, order=0, targets=None):
    """Evaluate the frozen lists in FP64 torch (differentiable in x, m, h).

    x, m, h are torch tensors in input order.  Returns (acc, pot) in input
    order for every particle (or only rows `targets`, input indices).
    """
    tree = lists.tree
    n = x.shape[0]
    order_t = torch.as_tensor(tree.order)
    xs, ms, hs = x[order_t], m[order_t], h[order_t]
    inv = np.empty(n, dtype=np.int64)
    inv[tree.order] = np.arange(n)
    want = None
    if targets is not None:
        want = np.zeros(n, dtype=bool)
        want[inv[np.asarray(targets)]] = True
    sink_sorted = lists.is_sink_sorted
    acc = torch.zeros(n, 3, dtype=x.dtype)
    pot = torch.zeros(n, dtype=x.dtype)
    outs_idx, outs_a, outs_p = [], [], []

    def moments_for(nodes_needed, sel):
        uniq = np.unique(nodes_needed)
        row = np.full(tree.n_nodes, -1, dtype=np.int64)
        row[uniq] = np.arange(uniq.size)
        M, com, Q = _moments_torch(tree, xs, ms, uniq, sel)
        return M, com, Q, row

    all_pc = [v[0] for v in lists.gas_lists.values()]
    if all_pc:
        M, com, Q, row = moments_for(np.concatenate(all_pc + [np.zeros(0, np.int64)]), None)
    for g, (pc, pp) in lists.gas_lists.items():
        f, c = lists.groups[g]
        tgt = np.arange(f, f + c)
        tgt = tgt[~sink_sorted[tgt]]
        if want is not None:
            tgt = tgt[want[tgt]]
        if tgt.size == 0:
            continue
        a_g, p_g = _eval_group(xs, ms, hs, tgt, pc, pp, M, com, Q, row, order, G)
        outs_idx.append(tgt)
        outs_a.append(a_g)
        outs_p.append(p_g)
    sinks = [p for p in lists.sink_lists if want is None or want[p]]
    if sinks:
        gas_sel = ~sink_sorted
        Mg, comg, Qg, rowg = moments_for(
            np.concatenate([lists.sink_lists[p][0] for p in sinks] + [np.zeros(0, np.int64)]), gas_sel)
        sink_pos = np.nonzero(sink_sorted)[0]
        for p in sinks:
            pc, pp = lists.sink_lists[p]
            a_s, p_s = _eval_group(xs, ms, hs, np.array([p]), pc, pp, Mg, comg, Qg, rowg, order, G)
            others = sink_pos[sink_pos != p]
            if others.size:
                a_d, p_d = _eval_group(xs, ms, hs, np.array([p]), np.zeros(0, np.int64), others,
                                       Mg, comg, Qg, rowg, order, G)
                a_s, p_s = a_s + a_d, p_s + p_d
            outs_idx.append(np.array([p]))
            outs_a.append(a_s)
            outs_p.append(p_s)
    if outs_idx:
        idx_sorted = np.concatenate(outs_idx)
        rows = torch.as_tensor(tree.order[idx_sorted])
        acc = acc.index_put((rows,), torch.cat(outs_a))
        pot = pot.index_put((rows,), torch.cat(outs_p))
    if targets is not None:
        t = torch.as_tensor(np.asarray(targets))
        return acc[t], pot[t]
    return acc, pot


def tree_forward(x, m, h, n_gas, G=1.0, theta=0.5, order=0, leaf_cap=16, group_cap=64,
                 alpha=None, field=None):
    """Convenience: lists + FP64 evaluation, numpy in and out."""
    lists = tree_lists(x, m, h, n_gas, theta, leaf_cap, group_cap, alpha=alpha, field=field,
                       G=G)
    t = lambda v: torch.as_tensor(np.asarray(v, dtype=np.float64))
    with torch.no_grad():
        a, p = tree_eval(t(x), t(m), t(h), n_gas, lists, G, order)
    return a.numpy(), p.numpy(), lists


# --------------------------------------------------------------- tidal tensor and jerk

def _kernel_F_FrR(r, h):
    """F and (dF/dr)/r of the softened kernel (numpy, FP64), r >= 0."""
    u = r / h
    h3, h5 = h ** 3, h ** 5
    safe_u = np.where(u > 0.25, u, 0.25)
    safe_r = np.where(r > 0, r, 1.0)
    Fa = (32.0 / 3.0 - 192.0 / 5.0 * u ** 2 + 32.0 * u ** 3) / h3
    Fb = (64.0 / 3.0 - 48.0 * u + 192.0 / 5.0 * u ** 2 - 32.0 / 3.0 * u ** 3
          - 1.0 / (15.0 * safe_u ** 3)) / h3
    Ra = (-384.0 / 5.0 + 96.0 * u) / h5
    Rb = (-48.0 / safe_u + 384.0 / 5.0 - 32.0 * u + 1.0 / (5.0 * safe_u ** 5)) / h5
    F = np.where(u < 0.5, Fa, np.where(u < 1.0, Fb, 1.0 / safe_r ** 3))
    R = np.where(u < 0.5, Ra, np.where(u < 1.0, Rb, -3.0 / safe_r ** 5))
    return F, R


def _tidal_terms(d, w, mF, mR):
    """Sums over the last-but-one axis of -(mF I + mR d d^T) and
    mF w + mR (d.w) d, as (.., 6) and (.., 3)."""
    T = np.stack([-(mF + mR * d[..., 0] * d[..., 0]), -(mF + mR * d[..., 1] * d[..., 1]),
                  -(mF + mR * d[..., 2] * d[..., 2]), -mR * d[..., 0] * d[..., 1],
                  -mR * d[..., 0] * d[..., 2], -mR * d[..., 1] * d[..., 2]], axis=-1).sum(-2)
    J = None
    if w is not None:
        dw = (d * w).sum(-1)
        J = (mF[..., None] * w + (mR * dw)[..., None] * d).sum(-2)
    return T, J


def tree_tidal(x, m, h, v, n_gas, lists, G=1.0):
    """Tidal tensor (n, 6: xx yy zz xy xz yz) and jerk (n, 3; None without v)
    of the frozen lists (Sec. 2.2: both summed in the same pass as g, from the
    monopole contributions of accepted nodes and the softened pair kernel of
    opened particles).  Node monopole: mass M, centre of mass c and
    mass-weighted velocity V of the node's particles (gas only for sink
    targets); sinks add the exact sum over the other sinks."""
    tree = lists.tree
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    xs = x[tree.order]
    ms = np.asarray(m, np.float64)[tree.order]
    hs = np.asarray(h, np.float64)[tree.order]
    vs = None if v is None else np.asarray(v, np.float64)[tree.order]
    sink = lists.is_sink_sorted
    T = np.zeros((n, 6))
    J = np.zeros((n, 3)) if v is not None else None

    def nodes(pc, gas_only):
        """M, centre of mass and mean velocity of the nodes pc."""
        idx = np.concatenate([np.arange(tree.first[k], tree.first[k] + tree.count[k]) for k in pc])
        starts = np.concatenate([[0], np.cumsum(tree.count[pc])[:-1]])
        mk = ms[idx] * (~sink[idx] if gas_only else 1.0)
        M = np.add.reduceat(mk, starts)
        com = np.add.reduceat(mk[:, None] * xs[idx], starts) / M[:, None]
        V = None if vs is None else np.add.reduceat(mk[:, None] * vs[idx], starts) / M[:, None]
        return M, com, V

    def targets(tg, pc, pp, gas_only):
        """T and j of the sorted targets tg from one list."""
        Tt = np.zeros((tg.size, 6))
        Jt = np.zeros((tg.size, 3)) if vs is not None else None
        if pc.size:
            M, com, V = nodes(pc, gas_only)
            d = com[None, :, :] - xs[tg][:, None, :]
            r = np.sqrt((d * d).sum(-1))
            w = None if vs is None else V[None, :, :] - vs[tg][:, None, :]
            t, j = _tidal_terms(d, w, M / r ** 3, -3.0 * M / r ** 5)
            Tt += t
            if Jt is not None:
                Jt += j
        if pp.size:
            d = xs[pp][None, :, :] - xs[tg][:, None, :]
            r = np.sqrt((d * d).sum(-1))
            F, R = _kernel_F_FrR(r, np.maximum(hs[pp][None, :], hs[tg][:, None]))
            keep = tg[:, None] != pp[None, :]
            w = None if vs is None else vs[pp][None, :, :] - vs[tg][:, None, :]
            t, j = _tidal_terms(d, w, keep * ms[pp][None, :] * F, keep * ms[pp][None, :] * R)
            Tt += t
            if Jt is not None:
                Jt += j
        return Tt, Jt

    for g, (pc, pp) in lists.gas_lists.items():
        f, c = lists.groups[g]
        tg = np.arange(f, f + c)
        tg = tg[~sink[tg]]
        Tt, Jt = targets(tg, pc, pp, False)
        T[tree.order[tg]] = G * Tt
        if J is not None:
            J[tree.order[tg]] = G * Jt
    sink_pos = np.nonzero(sink)[0]
    for p, (pc, pp) in lists.sink_lists.items():
        others = sink_pos[sink_pos != p]
        Tt, Jt = targets(np.array([p]), pc, np.concatenate([pp, others]).astype(np.int64), True)
        T[tree.order[p]] = G * Tt[0]
        if J is not None:
            J[tree.order[p]] = G * Jt[0]
    return T, J
