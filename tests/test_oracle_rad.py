"""Pins of the oracle's tree-pass radiation sums (6-bin FUV columns,
IR energy density from stars).

* the centre of a uniform sphere sees the column rho R in every bin (the
  bin-averaged column of a uniform medium), within its sampling error;
* a single far mass lands in the bin of its direction with m/(Omega r^2);
* the bins are the six cube faces: each direction goes to the face of its
  largest component;
* a point source gives L/(4 pi c r^2);
* the tree at theta = 0 reproduces the direct sums; at theta 0.5 it stays
  close to them.
"""
import numpy as np

from oracle import rad
from oracle import tree as T
from synth import clustered_cloud, uniform_sphere


def test_bins_are_cube_faces():
    d = np.array([[1.0, 0.2, -0.3], [-2, 1, 1.5], [0.1, 0.5, -0.2], [0.1, -0.5, 0.2],
                  [0, 0.1, 3.0], [0.3, 0.2, -0.4]])
    assert list(rad.bin_of(d)) == [0, 1, 2, 3, 4, 5]


def test_bins_on_face_boundaries():
    # a direction on a boundary between faces goes to the lower axis, and a
    # zero component along the chosen axis counts as positive (the reading
    # the GPU walk uses too)
    d = np.array([[1.0, 1.0, 0.0], [-1.0, 1.0, 0.0], [0.0, 1.0, 1.0], [0.0, -1.0, 1.0],
                  [1.0, -1.0, -1.0], [-1.0, -1.0, -1.0], [0.0, 0.0, -2.0], [0.0, 0.0, 0.0]])
    assert list(rad.bin_of(d)) == [0, 1, 2, 3, 0, 1, 5, 0]


def test_uniform_sphere_centre_column():
    n = 200000
    rng = np.random.default_rng(3)
    u = rng.random(n) ** (1 / 3)
    v = rng.standard_normal((n, 3))
    x = u[:, None] * v / np.linalg.norm(v, axis=1)[:, None]
    x[0] = 0.0                                   # the target at the centre
    m = np.full(n, 1.0 / n)
    h = np.full(n, 1e-4)
    d = x[1:]
    w = m[1:] / (rad.OMEGA_BIN * ((d * d).sum(1) + (h[1:] / 2.8) ** 2))
    col = np.bincount(rad.bin_of(d), weights=w, minlength=6)
    rho_R = 1.0 / (4.0 / 3.0 * np.pi)            # mass 1, radius 1
    # sampling error of a 1/r^2-weighted sum is dominated by the nearest
    # points; compare the six-bin mean to rho R within 3%
    assert abs(col.mean() / rho_R - 1) < 0.03, col / rho_R
    assert np.all(np.abs(col / rho_R - 1) < 0.15)


def test_single_mass_and_point_source():
    x = np.array([[0.0, 0.0, 0.0], [0.0, -2.0, 0.5], [0.3, 0.0, 4.0]])
    m = np.array([1.0, 3.0, 0.0])
    h = np.array([1e-9, 1e-9, 2.8e-3])
    lum = np.array([0.0, 0.0, 5.0])
    col = rad.columns_direct(x, m, h, n_gas=2)
    ref = 3.0 / (rad.OMEGA_BIN * 4.25)
    assert np.isclose(col[0, 3], ref, rtol=1e-12) and np.count_nonzero(col[0]) == 1
    e = rad.e_ir_direct(x, h, lum, n_gas=2, c_light=7.0)
    assert np.isclose(e[0], 5.0 / (4 * np.pi * 7.0 * (0.09 + 16.0 + 1e-6)), rtol=1e-12)
    assert e[2] == 0.0


def test_tree_theta_zero_is_direct_and_half_close():
    ps = clustered_cloud(1500, 12, seed=14, dtype=np.float64)
    lum = np.where(np.arange(ps.n) >= ps.n_gas, np.exp(np.random.default_rng(1).normal(0, 1, ps.n)), 0.0)
    colr = rad.columns_direct(ps.x, ps.m, ps.h, ps.n_gas)
    er = rad.e_ir_direct(ps.x, ps.h, lum, ps.n_gas, 3.0)
    lists = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=0.0, leaf_cap=8, group_cap=32)
    col, e = rad.tree_rad(ps.x, ps.m, ps.h, lum, ps.n_gas, lists, 3.0)
    assert np.allclose(col, colr, rtol=1e-12, atol=1e-14 * colr.max())
    assert np.allclose(e, er, rtol=1e-12)
    lists = T.tree_lists(ps.x, ps.m, ps.h, ps.n_gas, theta=0.5, leaf_cap=8, group_cap=32)
    col, e = rad.tree_rad(ps.x, ps.m, ps.h, lum, ps.n_gas, lists, 3.0)
    g = slice(0, ps.n_gas)
    ec = np.abs(col[g] - colr[g]).sum(1) / colr[g].sum(1)
    ee = np.abs(e[g] - er[g]) / er[g]
    assert np.median(ec) < 2e-2 and np.median(ee) < 2e-2, (np.median(ec), np.median(ee))
