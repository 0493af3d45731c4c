"""Finite-difference checks of both adjoints on the differentiation workload
(2^18 clustered gas, per-particle softening, seed 7; cotangents N(0, 1)).

Direct path: the GPU adjoint (FP64) against the oracle's pair-local central
differences (step 1e-6) at 64 random particles (x, y, z, m, h each).
Tree path (theta 0.5, quadrupole): the GPU adjoint against central
differences of the GPU's own FP64 forward on the frozen tree (refit to
x +- eps); a sample counts only when both perturbed walks keep every group's
list checksum (otherwise the decisions flipped: the tree approximation is not
differentiable there, and the sample is reported, not compared).
"""
import numpy as np
import pytest
import torch

from oracle import direct as odirect
from synth import cotangents, differentiation_cloud

pytestmark = pytest.mark.gpu

EPS = 1e-6


def _lib():
    from paper_2010_11254_amd import _lib
    return _lib


def _say(*a):
    print("[case]", *a, flush=True)


@pytest.fixture(scope="module")
def diff256k():
    ps = differentiation_cloud(1 << 18, seed=7)
    x, m, h = (np.asarray(v, dtype=np.float64) for v in (ps.x, ps.m, ps.h))
    ga, gp = cotangents(ps.n, seed=7)
    pick = np.random.default_rng([7, 2]).choice(ps.n, 64, replace=False)
    return x, m, h, ga, gp, pick


def _dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a)).cuda() for a in arrs]


def test_direct_adjoint_fd_diff256k(diff256k):
    _say("direct adjoint vs oracle FD, 2^18")
    x, m, h, ga, gp, pick = diff256k
    L = _lib()
    X, M, H, GA, GP = _dev(x, m, h, ga, gp)
    o = L.make_opts(form="fp64")
    gx, gm, gh = L.sf_grav_accel_backward(None, X, M, H, o, GA, GP)
    torch.cuda.synchronize()
    got = np.concatenate([gx.cpu().numpy()[pick], gm.cpu().numpy()[pick, None],
                          gh.cpu().numpy()[pick, None]], axis=1)
    fd = np.stack([odirect.fd_gradient(x, m, h, ga, gp, int(k), eps=EPS) for k in pick])
    err = np.abs(got - fd) / (np.abs(fd) + 1e-6 * np.abs(fd).max(axis=0))
    print("direct FD rel err: median %.2e p99 %.2e max %.2e" % (
        np.median(err), np.quantile(err, 0.99), err.max()), flush=True)
    assert np.median(err) < 1e-7
    assert err.max() < 1e-4


def test_tree_adjoint_frozen_fd_diff256k(diff256k):
    _say("tree adjoint vs frozen-tree FD, 2^18")
    x, m, h, ga, gp, pick = diff256k
    L = _lib()
    X, M, H, GA, GP = _dev(x, m, h, ga, gp)
    o = L.make_opts(form="fp64", theta=0.5, order=2, collect_stats=True)
    t = L.sf_grav_build_tree(X, M, H, o)
    gx, gm, gh = L.sf_grav_accel_backward(t, None, None, None, o, GA, GP)
    grad = np.concatenate([gx.cpu().numpy(), gm.cpu().numpy()[:, None], gh.cpu().numpy()[:, None]],
                          axis=1)
    acc = torch.empty_like(X)
    pot = torch.empty_like(M)

    def loss(Xv, Mv, Hv):
        L.sf_grav_tree_refit(t, Xv, Mv, Hv)
        L.sf_grav_accel(t, None, None, None, o, acc=acc, pot=pot)
        cks = L.sf_grav_tree_export(t, "group_cks").numpy()
        return float((acc * GA).sum() + (pot * GP).sum()), cks

    _, c0 = loss(X, M, H)
    errs, flips = [], 0
    for k in pick:
        for c in range(5):
            vals = []
            for sgn in (1.0, -1.0):
                Xv, Mv, Hv = X.clone(), M.clone(), H.clone()
                if c < 3:
                    Xv[k, c] += sgn * EPS
                elif c == 3:
                    Mv[k] += sgn * EPS * M[k]
                else:
                    Hv[k] += sgn * EPS * H[k]
                vals.append(loss(Xv, Mv, Hv))
            if not (np.array_equal(vals[0][1], c0) and np.array_equal(vals[1][1], c0)):
                flips += 1
                continue
            step = EPS if c < 3 else EPS * (m[k] if c == 3 else h[k])
            fd = (vals[0][0] - vals[1][0]) / (2 * step)
            g = grad[k, c]
            errs.append(abs(fd - g) / (abs(g) + 1e-6 * np.abs(grad[:, c]).max()))
    L.sf_grav_tree_free(t)
    errs = np.array(errs)
    print("tree frozen FD: %d samples, %d decision flips; rel err median %.2e p99 %.2e max %.2e"
          % (errs.size, flips, np.median(errs), np.quantile(errs, 0.99), errs.max()), flush=True)
    assert errs.size >= 0.9 * 5 * pick.size
    assert np.median(errs) < 1e-5
    assert np.quantile(errs, 0.9) < 1e-3
