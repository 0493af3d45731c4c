"""Pins of the oracle's tidal tensor T = -grad grad Phi and jerk j = da/dt
(Sec. 2.2: both summed in the same pass as g, from spatial derivatives of the
same softened kernel).

* Poisson: the trace of T at a particle is -4 pi G sum_j m_j W(r_ij, h_ij),
  with W the M4 cubic spline density written out here from its definition;
  Newtonian pairs add nothing to the trace;
* central differences of the oracle's own acceleration: in the target's
  position (all nine components of d a / d x) and in time along the
  velocities (x + v t);
* a point mass: T = G m (3 n n^T - I) / r^3 outside the softening radius;
* uniform motion of every particle: j = 0 exactly;
* a uniform sphere: T averaged over the deep interior is -G M / R^3 I
  (constant, negative definite), within its sampling error;
* the tree's T and j: theta = 0 reproduces the direct sum; at theta = 0.5
  the monopole node terms stay close to it.
"""
import numpy as np

from oracle import direct
from oracle import tree as T
from synth import clustered_cloud, uniform_sphere


def _W(r, h):
    """M4 cubic spline density with compact support h, normalised to 1."""
    u = r / h
    k = np.where(u < 0.5, 1 - 6 * u ** 2 + 6 * u ** 3, np.where(u < 1, 2 * (1 - u) ** 3, 0.0))
    return 8.0 / (np.pi * h ** 3) * k


def _full(t6):
    xx, yy, zz, xy, xz, yz = t6
    return np.array([[xx, xy, xz], [xy, yy, yz], [xz, yz, zz]])


def test_trace_is_poisson():
    rng = np.random.default_rng(1)
    n = 300
    x = rng.standard_normal((n, 3)) * 0.1
    m = rng.uniform(0.5, 1.5, n) / n
    h = rng.uniform(0.02, 0.2, n)
    x[7] = x[8]                           # a coincident pair (r = 0)
    Tt, _ = direct.direct_tidal(x, m, h, G=2.0)
    tr = Tt[:, 0] + Tt[:, 1] + Tt[:, 2]
    for i in range(n):
        d = np.linalg.norm(x - x[i], axis=1)
        keep = np.arange(n) != i
        ref = -4 * np.pi * 2.0 * np.sum((m * _W(d, np.maximum(h, h[i])))[keep])
        assert abs(tr[i] - ref) <= 1e-9 * (np.abs(Tt[i, :3]).sum() + abs(ref)), (i, tr[i], ref)


def test_point_mass_tidal_tensor():
    x = np.array([[0.0, 0.0, 0.0], [0.3, -0.4, 1.2]])
    m = np.array([2.0, 0.5])
    h = np.array([0.1, 0.05])
    Tt, _ = direct.direct_tidal(x, m, h, G=1.5, targets=[1])
    d = x[0] - x[1]
    r = np.linalg.norm(d)
    nn = d / r
    ref = 1.5 * 2.0 * (3 * np.outer(nn, nn) - np.eye(3)) / r ** 3
    assert np.allclose(_full(Tt[0]), ref, rtol=1e-13, atol=1e-15)


def test_tidal_is_gradient_of_the_field():
    ps = clustered_cloud(400, 3, seed=4, dtype=np.float64)
    x, m, h = ps.x, ps.m, ps.h
    Tt, _ = direct.direct_tidal(x, m, h)
    eps = 1e-6
    for i in (0, 17, 250, ps.n - 1):
        fd = np.zeros((3, 3))
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += eps
            xm[i, c] -= eps
            ap, _ = direct.direct(xp, m, h, targets=[i])
            am, _ = direct.direct(xm, m, h, targets=[i])
            fd[:, c] = (ap[0] - am[0]) / (2 * eps)
        got = _full(Tt[i])
        assert np.allclose(got, fd, rtol=1e-5, atol=1e-6 * np.abs(got).max()), (i, got, fd)


def test_jerk_is_time_derivative_of_the_field():
    ps = clustered_cloud(400, 3, seed=5, dtype=np.float64)
    rng = np.random.default_rng(6)
    v = rng.standard_normal((ps.n, 3))
    _, J = direct.direct_tidal(ps.x, ps.m, ps.h, v)
    eps = 1e-7
    ap, _ = direct.direct(ps.x + eps * v, ps.m, ps.h)
    am, _ = direct.direct(ps.x - eps * v, ps.m, ps.h)
    fd = (ap - am) / (2 * eps)
    scale = np.abs(J).max()
    assert np.allclose(J, fd, rtol=1e-5, atol=1e-6 * scale)


def test_uniform_motion_has_no_jerk():
    ps = clustered_cloud(200, 2, seed=7, dtype=np.float64)
    v = np.tile([0.3, -1.0, 2.5], (ps.n, 1))
    _, J = direct.direct_tidal(ps.x, ps.m, ps.h, v)
    assert np.all(J == 0.0)


def test_uniform_sphere_interior_tidal_tensor():
    # uniform sphere of radius 1, mass 1: inside (away from the edge by more
    # than the softening) the expected tidal tensor is -G M (N-1)/N / R^3 I
    n = 8192
    ps = uniform_sphere(n, seed=11, h=0.1)
    r = np.linalg.norm(ps.x, axis=1)
    inner = np.nonzero(r < 0.5)[0]
    Tt, _ = direct.direct_tidal(ps.x, ps.m, ps.h, targets=inner)
    ref = -(n - 1) / n
    diag = Tt[:, :3]
    mean, se = diag.mean(0), diag.std(0) / np.sqrt(inner.size)
    assert np.all(np.abs(mean - ref) < 4 * se + 1e-3), (mean, se)
    off = Tt[:, 3:]
    assert np.all(np.abs(off.mean(0)) < 4 * off.std(0) / np.sqrt(inner.size) + 1e-3)
    ev = np.linalg.eigvalsh(_full(Tt.mean(0)))
    assert np.all(ev < 0)                  # negative definite


def test_tree_tidal_theta_zero_is_direct_and_monopole_close():
    ps = clustered_cloud(2500, 11, seed=12, dtype=np.float64)
    rng = np.random.default_rng(13)
    v = rng.standard_normal((ps.n, 3))
    Tr, Jr = direct.direct_tidal(ps.x, ps.m, ps.h, v)
    lists = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=0.0, leaf_cap=8, group_cap=32)
    Tt, Jt = T.tree_tidal(ps.x, ps.m, ps.h, v, ps.n_gas, lists)
    assert np.allclose(Tt, Tr, rtol=1e-10, atol=1e-11 * np.abs(Tr).max())
    assert np.allclose(Jt, Jr, rtol=1e-10, atol=1e-11 * np.abs(Jr).max())
    lists = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=0.5, leaf_cap=8, group_cap=32)
    Tt, Jt = T.tree_tidal(ps.x, ps.m, ps.h, v, ps.n_gas, lists)
    eT = np.linalg.norm(Tt - Tr, axis=1) / np.linalg.norm(Tr, axis=1)
    eJ = np.linalg.norm(Jt - Jr, axis=1) / np.linalg.norm(Jr, axis=1)
    assert np.median(eT) < 2e-2 and np.median(eJ) < 2e-2, (np.median(eT), np.median(eJ))
