"""Pins of the oracle's FP64 direct sum (Sec. 2.2, Sec. 2.2.1).

Each test checks the oracle against something it does not share code with:
a 50-digit brute force from the symbolically derived kernel, exact physics
(point-mass limit, antisymmetry => zero net force, translation invariance,
the potential of a uniform sphere), and for the adjoint central differences
and torch autograd of an independently written dense sum.
"""
import numpy as np
import pytest
import torch

from kernel_ref import mp_direct
from oracle import direct
from synth import uniform_sphere


def _tiny_set(seed=3, n=12):
    rng = np.random.default_rng(seed)
    x = rng.uniform(-0.3, 0.3, (n, 3))
    x[5] = x[4]                      # coincident distinct pair (r = 0)
    x[7] = x[6] + [0.011, 0.0, 0.0]  # inner branch for h = 0.05
    x[9] = x[8] + [0.0, 0.03, 0.0]   # outer branch
    m = rng.uniform(0.1, 2.0, n)
    h = rng.choice([0.02, 0.05, 0.2], n)
    return x, m, h


def test_brute_force_mpmath_tiny():
    x, m, h = _tiny_set()
    a, p = direct.direct(x, m, h, G=1.3)
    ar, pr = mp_direct(x, m, h, G=1.3)
    assert np.allclose(a, ar, rtol=1e-12, atol=1e-12 * np.abs(ar).max())
    assert np.allclose(p, pr, rtol=1e-13, atol=0)


def test_point_mass_limit_pair():
    # beyond max(h_i, h_j) the law is exactly Newtonian (Sec. 2.2.1)
    for r, hi, hj in [(0.5, 0.1, 0.4999), (2.0, 2.0, 1.0), (1e-3, 1e-4, 9e-4)]:
        x = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
        m = np.array([1.0, 3.0])
        h = np.array([hi, hj])
        a, p = direct.direct(x, m, h, G=2.0)
        assert a[0, 0] == pytest.approx(2.0 * 3.0 / r ** 2, rel=1e-15)
        assert a[1, 0] == pytest.approx(-2.0 * 1.0 / r ** 2, rel=1e-15)
        assert p[0] == pytest.approx(-2.0 * 3.0 / r, rel=1e-15)


def test_softening_uses_larger_radius_both_ways():
    # the pair is softened with max(h_i, h_j) in both directions (Sec. 2.2.1)
    x = np.array([[0.0, 0.0, 0.0], [0.1, 0.0, 0.0]])
    m = np.array([1.0, 1.0])
    a1, p1 = direct.direct(x, m, np.array([1e-4, 0.3]))
    a2, p2 = direct.direct(x, m, np.array([0.3, 0.3]))
    assert np.array_equal(a1, a2) and np.array_equal(p1, p2)
    assert a1[0, 0] == -a1[1, 0]


def test_compact_cluster_far_field():
    rng = np.random.default_rng(5)
    k = 200
    cl = rng.uniform(-1, 1, (k, 3)) * 0.01
    D = 3.0
    x = np.vstack([[[-D, 0, 0]], cl])
    m = np.concatenate([[1e-9], rng.uniform(0.5, 1.5, k)])
    h = np.full(k + 1, 1e-3)
    a, p = direct.direct(x, m, h, targets=[0])
    M = m[1:].sum()
    assert a[0, 0] == pytest.approx(M / D ** 2, rel=(0.02 / D) ** 2 * 10)


def test_zero_net_force():
    # antisymmetric pairs conserve momentum (Sec. 2.2.1)
    x, m, h = _tiny_set(seed=11, n=300)
    a, _ = direct.direct(x, m, h)
    net = (m[:, None] * a).sum(0)
    scale = (m * np.linalg.norm(a, axis=1)).sum()
    assert np.all(np.abs(net) <= 1e-13 * scale)


def test_translation_invariance():
    x, m, h = _tiny_set(seed=2, n=200)
    shift = np.array([0.5, -0.25, 0.125])     # exactly representable
    a1, p1 = direct.direct(x, m, h)
    a2, p2 = direct.direct(x + shift, m, h)
    assert np.allclose(a1, a2, rtol=1e-10, atol=1e-10 * np.abs(a1).max())
    assert np.allclose(p1, p2, rtol=1e-12)


def test_uniform_sphere_interior_potential():
    # Interior of a uniform sphere (radius R, mass M), >= h from the surface:
    # E[phi] = ((N-1)/N) (-G M / 2R^3) (3R^2 - r^2 - <|y|^2>_W),  <|y|^2>_W = 9/40 h^2,
    # E[a]   = -((N-1)/N) G M x / R^3.
    # The Poisson noise of one realisation shifts phi coherently by ~N^-1/2,
    # so the softening offset (9/40 h^2 GM/2R^3) is checked on the difference
    # softened - Newtonian of the same realisation, where that mode cancels.
    n, hh = 65536, 0.2
    ps = uniform_sphere(n, seed=0, h=hh)
    r = np.linalg.norm(ps.x, axis=1)
    inner = np.nonzero(r <= 1.0 - hh)[0]
    sel = inner[np.random.default_rng(0).choice(inner.size, 4096, replace=False)]
    a, p = direct.direct(ps.x, ps.m, ps.h, targets=sel)
    _, p_newton = direct.direct(ps.x, ps.m, np.full(n, 1e-12), targets=sel)
    f = (n - 1) / n
    offset = f * 0.5 * (9.0 / 40.0) * hh ** 2
    assert np.mean(p - p_newton) == pytest.approx(offset, rel=0.01)
    # the quadratic profile itself (slope and intercept, Newtonian part)
    A = np.vstack([np.ones(sel.size), r[sel] ** 2]).T
    coef, *_ = np.linalg.lstsq(A, p_newton, rcond=None)
    assert coef[0] == pytest.approx(-f * 1.5, rel=0.01)
    assert coef[1] == pytest.approx(f * 0.5, rel=0.02)
    slope = (a * ps.x[sel]).sum(1) / (r[sel] ** 2)
    assert np.median(slope) == pytest.approx(-f, rel=0.02)


# ---------------------------------------------------------------- adjoint

def _torch_dense(x, m, h, G):
    """Independent dense softened sum written with torch ops (autograd)."""
    d = x[None, :, :] - x[:, None, :]                  # d_ij = x_j - x_i
    n = x.shape[0]
    eye = torch.eye(n, dtype=torch.bool)
    r2 = (d * d).sum(-1)
    r = torch.sqrt(torch.where(eye | (r2 == 0), torch.ones_like(r2), r2))
    r = torch.where(r2 == 0, torch.zeros_like(r), r)
    H = torch.maximum(h[:, None], h[None, :])
    q = r / H
    q2, q3 = q * q, q * q * q
    qs = torch.where(q > 0.25, q, torch.full_like(q, 0.25))
    rs = torch.where(r > 0, r, torch.ones_like(r))
    Fi = (32 / 3 - 192 / 5 * q2 + 32 * q3) / H ** 3
    Fo = (64 / 3 - 48 * q + 192 / 5 * q2 - 32 / 3 * q3 - 1 / (15 * qs ** 3)) / H ** 3
    Pi = (14 / 5 - 16 / 3 * q2 + 48 / 5 * q2 * q2 - 32 / 5 * q3 * q2) / H
    Po = (16 / 5 - 1 / (15 * qs) - 32 / 3 * q2 + 16 * q3 - 48 / 5 * q2 * q2 + 32 / 15 * q3 * q2) / H
    F = torch.where(q < 0.5, Fi, torch.where(q < 1, Fo, 1 / rs ** 3))
    P = torch.where(q < 0.5, Pi, torch.where(q < 1, Po, 1 / rs))
    w = (~eye).to(x.dtype) * m[None, :]
    a = G * ((w * F)[..., None] * d).sum(1)
    phi = -G * (w * P).sum(1)
    return a, phi


def test_adjoint_matches_torch_autograd():
    rng = np.random.default_rng(21)
    n = 400
    x = rng.uniform(-0.5, 0.5, (n, 3))
    m = rng.uniform(0.5, 1.5, n) / n
    h = rng.uniform(0.05, 0.25, n)          # distinct radii: no ties
    ga = rng.standard_normal((n, 3))
    gp = rng.standard_normal(n)
    gx, gm, gh = direct.direct_vjp(x, m, h, ga, gp, G=1.0)
    X = torch.tensor(x, requires_grad=True)
    Mt = torch.tensor(m, requires_grad=True)
    Ht = torch.tensor(h, requires_grad=True)
    a, phi = _torch_dense(X, Mt, Ht, 1.0)
    a_np, p_np = direct.direct(x, m, h)
    assert np.allclose(a.detach().numpy(), a_np, rtol=1e-11, atol=1e-11 * np.abs(a_np).max())
    L = (a * torch.tensor(ga)).sum() + (phi * torch.tensor(gp)).sum()
    L.backward()
    for got, ref in [(gx, X.grad), (gm, Mt.grad), (gh, Ht.grad)]:
        ref = ref.numpy()
        assert np.allclose(got, ref, rtol=1e-9, atol=1e-10 * np.abs(ref).max())


def test_adjoint_matches_central_differences():
    rng = np.random.default_rng(8)
    n = 300
    x = rng.uniform(-0.5, 0.5, (n, 3))
    x[1] = x[0]                               # coincident pair
    m = rng.uniform(0.5, 1.5, n) / n
    h = rng.uniform(0.05, 0.3, n)
    ga = rng.standard_normal((n, 3))
    gp = rng.standard_normal(n)
    gx, gm, gh = direct.direct_vjp(x, m, h, ga, gp)
    for k in [0, 2, 17, 150, 299]:
        fd = direct.fd_gradient(x, m, h, ga, gp, k, eps=1e-6)
        an = np.array([gx[k, 0], gx[k, 1], gx[k, 2], gm[k], gh[k]])
        assert np.allclose(an, fd, rtol=2e-6, atol=2e-6 * np.abs(an).max()), (k, an, fd)


def test_sparse_cotangent_vjp_equals_dense():
    # the O(k n) form for cotangents on a few particles, used at full size,
    # against the dense VJP: the skipped pairs' terms are exact zeros
    rng = np.random.default_rng(31)
    n = 700
    x = rng.standard_normal((n, 3))
    m = rng.uniform(0.5, 1.5, n)
    h = rng.uniform(0.05, 0.4, n)
    h[::7] = h[0]   # equal radii (the split tie of dL/dh)
    ga, gp = np.zeros((n, 3)), np.zeros(n)
    act = rng.choice(n, 23, replace=False)
    ga[act] = rng.standard_normal((act.size, 3))
    gp[act] = rng.standard_normal(act.size)
    dense = direct.direct_vjp(x, m, h, ga, gp)
    sparse = direct.direct_vjp_sparse(x, m, h, ga, gp)
    for a, b in zip(dense, sparse):
        assert np.allclose(a, b, rtol=1e-13, atol=1e-13 * np.abs(a).max())
    assert np.count_nonzero(sparse[0]) > 3 * (n - act.size)   # every particle receives terms
