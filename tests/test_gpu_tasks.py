"""Every group task is walked, and walked once, under the per-XCD task
placement (chunks of 1024 Morton-consecutive groups dealt to the eight XCDs),
at sizes whose groups run through every XCD's sequence (more than 8 x 1024
groups) and past the point where waves start helping other XCDs.

theta = 0 opens every node, so each group holding gas must list no nodes and
all n particles (a closed form: a group walked twice or not at all breaks
it).  At theta = 0.5 the walks that reuse the force walk's lists (tidal
tensor and jerk, radiation sums) and the adaptive-softening walks must give
every gas target a result: the tidal walk's acceleration equals the force
walk's target by target.
"""
import numpy as np
import pytest
import torch

from synth import clustered_cloud

pytestmark = pytest.mark.gpu


def _lib():
    from paper_2010_11254_amd import _lib
    return _lib


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a)).cuda() for a in arrs]


def _groups_with_gas(L, t, n_gas):
    first = L.sf_grav_tree_export(t, "group_first").numpy().astype(np.int64)
    count = L.sf_grav_tree_export(t, "group_count").numpy().astype(np.int64)
    gas_sorted = L.sf_grav_tree_export(t, "order").numpy() < n_gas
    csum = np.concatenate([[0], np.cumsum(gas_sorted)])
    return (csum[first + count] - csum[first]) > 0


def test_every_group_walked_once_theta_zero():
    L = _lib()
    ps = clustered_cloud(300000, 64, seed=21)
    _say("theta 0 walk, clustered", ps.n)
    x, m, h = _dev(ps.x, ps.m, ps.h)
    o = L.make_opts(form="fp32c", theta=0.0, n_gas=ps.n_gas, collect_stats=True)
    t = L.sf_grav_build_tree(x, m, h, o)
    a, p = L.sf_grav_accel(t, None, None, None, o)
    torch.cuda.synchronize()
    npc = L.sf_grav_tree_export(t, "group_npc").numpy()
    npp = L.sf_grav_tree_export(t, "group_npp").numpy()
    has_gas = _groups_with_gas(L, t, ps.n_gas)
    L.sf_grav_tree_free(t)
    assert has_gas.size > 8 * 1024 + 1024, has_gas.size
    assert np.all(npc[has_gas] == 0)
    assert np.all(npp[has_gas] == ps.n), (npp[has_gas].min(), npp[has_gas].max())
    assert np.all(npc[~has_gas] == 0) and np.all(npp[~has_gas] == 0)   # sink-only groups
    a = a.cpu().numpy()
    assert np.all(np.isfinite(a)) and np.all(np.linalg.norm(a, axis=1) > 0)


def test_every_group_walked_by_each_tree_pass():
    L = _lib()
    ps = clustered_cloud(1 << 20, 256, seed=1)
    _say("theta 0.5 passes, clustered", ps.n)
    x, m, h = _dev(ps.x, ps.m, ps.h)
    o = L.make_opts(form="fp32c", n_gas=ps.n_gas, collect_stats=True)
    t = L.sf_grav_build_tree(x, m, h, o)
    a, p = L.sf_grav_accel(t, None, None, None, o)
    torch.cuda.synchronize()
    npp = L.sf_grav_tree_export(t, "group_npp").numpy()
    has_gas = _groups_with_gas(L, t, ps.n_gas)
    assert has_gas.size > 8 * 1024 + 1024, has_gas.size
    assert np.all(npp[has_gas] >= 1)   # its own leaf at least
    gas = slice(0, ps.n_gas)
    _say("tidal pass")
    a2, p2, tid, jerk = L.sf_grav_accel_tidal(t, o)
    torch.cuda.synchronize()
    ref = a.double().cpu().numpy()[gas]
    e = np.linalg.norm(a2.double().cpu().numpy()[gas] - ref, axis=1) / np.linalg.norm(ref, axis=1)
    assert e.max() < 1e-4, e.max()
    assert np.all(np.isfinite(tid.cpu().numpy()[gas]))
    _say("radiation sums")
    lum = torch.zeros(ps.n, dtype=x.dtype, device=x.device)
    lum[ps.n_gas:] = 1.0
    col, eir = L.sf_grav_rad_sums(t, o, lum=lum, c_light=1.0)
    torch.cuda.synchronize()
    assert np.all(col.cpu().numpy()[gas].sum(axis=1) > 0)
    assert np.all(eir.cpu().numpy()[gas] > 0)
    _say("adaptive softening")
    a3, p3, aux = L.sf_grav_accel_adaptive(t, o, want_aux=True)
    torch.cuda.synchronize()
    aux = aux.cpu().numpy()
    assert np.all(np.isfinite(a3.cpu().numpy())) and np.all(p3.cpu().numpy()[gas] < 0)
    assert np.all(aux[gas, 0] != 0)   # Omega of every gas cell was written
    L.sf_grav_tree_free(t)
