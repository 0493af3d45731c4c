"""Pins of the oracle's sink dynamics (Sec. 2.3): the two-body time scales,
the timestep criteria, and the modified Hermite step.

* the paper's printed figure: with eta = 0.01 an e = 0.9 binary keeps its
  relative energy error below 1e-6 per orbit (tests/golden/paper_constants.json),
  with the timestep taken from the tidal and 2-body criteria and rounded
  down to a power of two;
* fourth order: at a fixed step the energy error of one orbit falls by at
  least 2^4 when the step is halved;
* a circular orbit returns to its start after one period;
* the 2-body times and timesteps of a hand-computed three-sink set;
* the tidal timestep of a point-mass companion equals sqrt(eta r^3 / (G M)).
"""
import json
import os

import numpy as np

from oracle import sinks as S

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))


def _binary(e, m1=0.6, m2=0.4, a=1.0, h=1e-4):
    M = m1 + m2
    rp = a * (1 - e)
    vp = np.sqrt(M * (1 + e) / rp)
    x = np.array([[-m2 / M * rp, 0.0, 0.0], [m1 / M * rp, 0.0, 0.0]])
    v = np.array([[0.0, -m2 / M * vp, 0.0], [0.0, m1 / M * vp, 0.0]])
    return x, v, np.array([m1, m2]), np.array([h, h]), 2 * np.pi * np.sqrt(a ** 3 / M)


def _integrate(x, v, m, h, t_end, eta=None, dt=None):
    t, steps = 0.0, 0
    while t < t_end:
        if eta is not None:
            dt2, dtt = S.timesteps(x, v, m, h, eta)
            dt = 2.0 ** np.floor(np.log2(min(dt2.min(), dtt.min())))
        x, v = S.hermite_step(x, v, m, h, dt)
        t += dt
        steps += 1
    return x, v, steps


def test_paper_energy_error_per_orbit():
    g = GOLD["hermite_energy_error_per_orbit"]
    x, v, m, h, P = _binary(g["eccentricity"])
    E0 = S.energy(x, v, m, h)
    orbits = 3
    x1, v1, steps = _integrate(x, v, m, h, orbits * P, eta=g["eta"])
    err = abs((S.energy(x1, v1, m, h) - E0) / E0) / orbits
    print(f"e=0.9, eta=0.01: {steps / orbits:.0f} steps/orbit, |dE/E| per orbit {err:.2e}")
    assert err < g["value"]


def test_fourth_order_convergence():
    x, v, m, h, P = _binary(0.5)
    E0 = S.energy(x, v, m, h)
    errs = []
    for k in (200, 400):
        x1, v1, _ = _integrate(x, v, m, h, P, dt=P / k)
        errs.append(abs(S.energy(x1, v1, m, h) - E0))
    assert errs[0] / errs[1] > 16.0, errs


def test_circular_orbit_closes():
    x, v, m, h, P = _binary(0.0)
    x1, v1, _ = _integrate(x, v, m, h, P - 1e-12, dt=P / 512)
    assert np.max(np.abs(x1 - x)) < 1e-7 and np.max(np.abs(v1 - v)) < 1e-7


def test_two_body_times_three_sinks():
    x = np.array([[0.0, 0.0, 0.0], [3.0, 4.0, 0.0], [0.0, 0.0, 12.0]])
    v = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 1.0], [2.0, 0.0, 0.0]])
    m = np.array([1.0, 2.0, 3.0])
    h = np.array([2.8, 0.0, 0.0])          # eps = 1 for sink 0, 0 for the others
    tc, td = S.two_body_times(x, v, m, h, G=2.0)
    # sink 0: to sink 1 r^2 + eps^2 = 26, |v| = 1; to sink 2 r^2 + 1 = 145, |v| = 2
    assert np.isclose(tc[0], min(np.sqrt(26.0) / 1.0, np.sqrt(145.0) / 2.0))
    assert np.isclose(td[0], min(np.sqrt(26.0 ** 1.5 / (2.0 * 3.0)), np.sqrt(145.0 ** 1.5 / (2.0 * 4.0))))
    # sink 1 (eps 0): to 0 r = 5, |v| = 1; to 2 r^2 = 9 + 16 + 144 = 169, |v| = sqrt(5)
    assert np.isclose(tc[1], min(5.0, 13.0 / np.sqrt(5.0)))
    assert np.isclose(td[1], min(np.sqrt(125.0 / 6.0), np.sqrt(13.0 ** 3 / 10.0)))
    dt2, _ = S.timesteps(x, v, m, h, eta=0.04, G=2.0)
    assert np.isclose(dt2[0], 0.2 / (1 / tc[0] + 1 / td[0]))


def test_tidal_timestep_point_mass():
    # a light sink beside a heavy one far outside the softening: |T|_F^2 =
    # 6 (G M / r^3)^2, so dt_tidal = sqrt(eta r^3 / (G M))
    x = np.array([[0.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    v = np.zeros((2, 3))
    m = np.array([5.0, 1e-9])
    h = np.array([1e-3, 1e-3])
    _, dtt = S.timesteps(x, v, m, h, eta=0.01)
    assert np.isclose(dtt[1], np.sqrt(0.01 * 8.0 / 5.0), rtol=1e-12)
