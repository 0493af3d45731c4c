"""Pins of the oracle's symmetrised adaptive gas softening (Sec. 2.2.1: the
symmetrisation and extra terms conserve momentum and energy).

* energy: with every kernel radius re-solved from the neighbour-number
  constraint at each perturbed position, central differences of the total
  potential energy equal -m_i a_i (the defining property of the extra terms);
  dropping the extra terms breaks it;
* momentum: sum_i m_i a_i = 0 with unequal masses;
* the radii solve (4 pi / 3) h^3 n = N_NGB (N_NGB from Table 1);
* beyond both radii the pair law is Newtonian; for equal radii everywhere
  and no correction the pair law reduces to the larger-radius rule;
* sinks keep the larger-radius rule.
"""
import json
import os

import numpy as np

from oracle import direct
from oracle import pm

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _cloud(n, seed):
    rng = np.random.default_rng(seed)
    x = np.vstack([rng.standard_normal((n // 2, 3)) * 0.1,
                   rng.standard_normal((n - n // 2, 3)) * 0.3 + 0.5])
    m = rng.uniform(0.5, 1.5, n) / n
    return x, m


def test_radii_solve_the_neighbour_constraint():
    assert GOLD["n_ngb"]["value"] == pm.N_NGB
    x, _ = _cloud(300, 1)
    h = pm.solve_h(x)
    assert np.allclose(pm.neighbour_number(x, h), pm.N_NGB, rtol=1e-12)


def test_force_is_minus_energy_gradient():
    x, m = _cloud(160, 2)
    h = pm.solve_h(x)
    a, _ = pm.pm_accel(x, m, h, G=1.3)
    eps = 1e-6
    for i in (0, 7, 100, 159):
        for c in range(3):
            xp, xm = x.copy(), x.copy()
            xp[i, c] += eps
            xm[i, c] -= eps
            fd = (pm.pm_energy(xp, m, pm.solve_h(xp), G=1.3) -
                  pm.pm_energy(xm, m, pm.solve_h(xm), G=1.3)) / (2 * eps)
            assert abs(-m[i] * a[i, c] - fd) <= 1e-6 * abs(fd) + 1e-9 * np.abs(m[:, None] * a).max(), \
                (i, c, -m[i] * a[i, c], fd)


def test_extra_terms_are_needed_for_energy():
    # planted mistake: without the correction the force is not the gradient
    x, m = _cloud(160, 3)
    h = pm.solve_h(x)
    a, _ = pm.pm_accel(x, m, h)
    om, ze = pm.omega_zeta(x, m, h)
    assert np.abs(ze).max() > 0
    d = x[None] - x[:, None]
    r = np.sqrt((d ** 2).sum(-1))
    F = np.zeros_like(r)
    for i in range(len(m)):
        Fi, *_ = direct.kernel(r[i], np.full(len(m), h[i]))
        Fj, *_ = direct.kernel(r[i], h)
        F[i] = 0.5 * (Fi + Fj)
    np.fill_diagonal(F, 0.0)
    a0 = ((m[None, :] * F)[..., None] * d).sum(1)
    i, c, eps = 5, 0, 1e-6
    xp, xm = x.copy(), x.copy()
    xp[i, c] += eps
    xm[i, c] -= eps
    fd = (pm.pm_energy(xp, m, pm.solve_h(xp)) - pm.pm_energy(xm, m, pm.solve_h(xm))) / (2 * eps)
    assert abs(-m[i] * a[i, c] - fd) < 1e-3 * abs(-m[i] * a0[i, c] - fd)


def test_momentum_is_conserved():
    x, m = _cloud(200, 4)
    h = pm.solve_h(x)
    a, _ = pm.pm_accel(x, m, h)
    net = (m[:, None] * a).sum(0)
    assert np.all(np.abs(net) <= 1e-13 * (m * np.linalg.norm(a, axis=1)).sum())


def test_newtonian_beyond_radii_and_sinks_keep_max_rule():
    # two far-apart clusters: pairs across are Newtonian in both laws
    x, m = _cloud(120, 5)
    h = pm.solve_h(x)
    a, p = pm.pm_accel(x, m, h)
    far = np.array([50.0, 0.0, 0.0])
    xs = np.vstack([x, far[None]])
    ms = np.concatenate([m, [0.3]])
    hs = np.concatenate([h, [1e-3]])
    a2, p2 = pm.pm_accel(xs, ms, hs, n_gas=120)
    # the sink's field is the plain direct sum (larger-radius rule)
    ad, pd = direct.direct(xs, ms, hs, targets=[120])
    assert np.allclose(a2[120], ad[0], rtol=1e-12) and np.isclose(p2[120], pd[0], rtol=1e-12)
    # the gas feels the far sink as a point mass on top of its own field
    dd = far - x
    rr = np.linalg.norm(dd, axis=1)
    assert np.allclose(a2[:120], a + 0.3 * dd / rr[:, None] ** 3, rtol=1e-12, atol=1e-15)


def test_neighbour_search_form_equals_dense_sums():
    # the sampled form used at full size (k-d tree neighbours of chosen
    # targets) against the dense O(N^2) sums it restates: Omega, zeta, and
    # pm_accel minus the larger-radius law, with sinks and unequal radii
    n, n_gas = 500, 470
    x, m = _cloud(n, 21)
    h = np.empty(n)
    h[:n_gas] = pm.solve_h(x[:n_gas])
    h[n_gas:] = 0.02
    om, ze = pm.omega_zeta(x[:n_gas], m[:n_gas], h[:n_gas])
    idx = [0, 7, 100, 250, 469]
    om2, ze2 = pm.omega_zeta_at(x[:n_gas], m[:n_gas], h[:n_gas], idx)
    assert np.allclose(om2, om[idx], rtol=1e-13, atol=0)
    assert np.allclose(ze2, ze[idx], rtol=1e-12, atol=1e-14 * np.abs(ze).max())
    ap, pp = pm.pm_accel(x, m, h, n_gas=n_gas)
    ad, pd = direct.direct(x, m, h)
    da, dp = pm.pm_change_at(x, m, h, n_gas, idx)
    scale = np.linalg.norm(ap[idx], axis=1)
    assert np.max(np.linalg.norm(da - (ap - ad)[idx], axis=1) / scale) < 1e-12
    assert np.max(np.abs(dp - (pp - pd)[idx]) / np.abs(pp[idx])) < 1e-12
    # the change is not trivially zero here
    assert np.min(np.linalg.norm((ap - ad)[idx], axis=1) / scale) > 1e-6
