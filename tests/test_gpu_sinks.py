"""GPU parity of the sink dynamics (sinks-only FP64 pass, two-body time
scales and timesteps, modified Hermite step) against the oracle, and the
paper's energy-error figure for an e = 0.9 binary integrated on the GPU."""
import json
import os

import numpy as np
import pytest
import torch

from oracle import direct as odirect
from oracle import sinks as osinks

pytestmark = pytest.mark.gpu
GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _lib():
    from paper_2010_11254_amd import _lib
    return _lib


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(*arrs):
    return [torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).cuda() for a in arrs]


def _sinks(n, seed):
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((n, 3)) * 0.01
    v = rng.standard_normal((n, 3))
    m = np.exp(rng.normal(np.log(1e-3), 1.0, n))
    h = np.full(n, 1e-3)
    if n > 3:
        x[3] = x[2]                      # a coincident pair (r = 0)
    return x, v, m, h


@pytest.mark.parametrize("n", [1, 2, 65, 700])
def test_sinks_pass_matches_oracle(n):
    _say("sinks pass n =", n)
    L = _lib()
    x, v, m, h = _sinks(n, 900 + n)
    X, V, M, H = _dev(x, v, m, h)
    out = L.sf_grav_sinks(X, V, M, H, G=1.3, eta=0.01)
    torch.cuda.synchronize()
    got = {k: t.cpu().numpy() for k, t in out.items()}
    ar, pr = odirect.direct(x, m, h, G=1.3)
    Tr, Jr = odirect.direct_tidal(x, m, h, v, G=1.3)
    for k, ref in (("acc", ar), ("pot", pr), ("tidal", Tr), ("jerk", Jr)):
        scale = np.abs(ref).max() + 1e-300
        assert np.max(np.abs(got[k] - ref)) <= 1e-12 * scale, k
    tc, td = osinks.two_body_times(x, v, m, h, G=1.3)
    dt2, dtt = osinks.timesteps(x, v, m, h, eta=0.01, G=1.3)
    t = got["times"]
    if n == 1:
        assert np.all(np.isinf(t[:, :2]))
        return
    assert np.allclose(t[:, 0], tc, rtol=1e-13) and np.allclose(t[:, 1], td, rtol=1e-13)
    assert np.allclose(t[:, 2], dt2, rtol=1e-13) and np.allclose(t[:, 3], dtt, rtol=1e-12)


def test_sinks_pass_precision4m_sinks():
    # the benchmark workload's 4096 sinks (2048 close binaries, separations
    # log-uniform in [1e-5, 1e-3] around the sink softening), FP64
    from synth import precision_cloud, velocities
    _say("sinks pass, the 4096 sinks of precision4m")
    ps = precision_cloud(1 << 22, 2048, seed=2)
    sl = slice(ps.n_gas, ps.n)
    x, m, h = (np.asarray(v[sl], dtype=np.float64) for v in (ps.x, ps.m, ps.h))
    v = velocities(ps.n, seed=2, dtype=np.float64)[sl]
    L = _lib()
    X, V, M, H = _dev(x, v, m, h)
    out = L.sf_grav_sinks(X, V, M, H, G=1.0, eta=0.01)
    torch.cuda.synchronize()
    got = {k: t.cpu().numpy() for k, t in out.items()}
    ar, pr = odirect.direct(x, m, h)
    Tr, Jr = odirect.direct_tidal(x, m, h, v)
    for k, ref in (("acc", ar), ("pot", pr), ("tidal", Tr), ("jerk", Jr)):
        scale = np.abs(ref).max()
        assert np.max(np.abs(got[k] - ref)) <= 1e-12 * scale, k
    tc, td = osinks.two_body_times(x, v, m, h)
    dt2, dtt = osinks.timesteps(x, v, m, h, eta=0.01)
    t = got["times"]
    assert np.allclose(t[:, 0], tc, rtol=1e-13) and np.allclose(t[:, 1], td, rtol=1e-13)
    assert np.allclose(t[:, 2], dt2, rtol=1e-13) and np.allclose(t[:, 3], dtt, rtol=1e-12)


def test_hermite_step_matches_oracle():
    _say("hermite step")
    L = _lib()
    x, v, m, h = _sinks(300, 950)
    X, V, M, H = _dev(x, v, m, h)
    dt = 1e-4
    L.sf_grav_sink_hermite(X, V, M, H, dt)
    torch.cuda.synchronize()
    xr, vr = osinks.hermite_step(x, v, m, h, dt)
    assert np.max(np.abs(X.cpu().numpy() - xr)) <= 1e-13 * np.abs(xr).max()
    assert np.max(np.abs(V.cpu().numpy() - vr)) <= 1e-12 * np.abs(vr).max()


def test_binary_energy_error_per_orbit_on_gpu():
    # the paper's figure, integrated with the GPU's pass (timesteps) and
    # Hermite step; the energy is measured with the oracle
    g = GOLD["hermite_energy_error_per_orbit"]
    _say("binary e =", g["eccentricity"], "eta =", g["eta"])
    L = _lib()
    e, m1, m2 = g["eccentricity"], 0.6, 0.4
    Mt = m1 + m2
    rp = 1.0 - e
    vp = np.sqrt(Mt * (1 + e) / rp)
    x = np.array([[-m2 / Mt * rp, 0, 0], [m1 / Mt * rp, 0, 0]])
    v = np.array([[0, -m2 / Mt * vp, 0], [0, m1 / Mt * vp, 0]])
    m, h = np.array([m1, m2]), np.array([1e-4, 1e-4])
    P = 2 * np.pi / np.sqrt(Mt)
    X, V, M, H = _dev(x, v, m, h)
    E0 = osinks.energy(x, v, m, h)
    t, steps, orbits = 0.0, 0, 3
    while t < orbits * P:
        tm = L.sf_grav_sinks(X, V, M, H, eta=g["eta"], want=("times",))["times"].cpu().numpy()
        dt = 2.0 ** np.floor(np.log2(min(tm[:, 2].min(), tm[:, 3].min())))
        L.sf_grav_sink_hermite(X, V, M, H, dt)
        t += dt
        steps += 1
    err = abs((osinks.energy(X.cpu().numpy(), V.cpu().numpy(), m, h) - E0) / E0) / orbits
    print(f"GPU Hermite e=0.9: {steps / orbits:.0f} steps/orbit, |dE/E| per orbit {err:.2e}",
          flush=True)
    assert err < g["value"]
