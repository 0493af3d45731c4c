"""Pins of the oracle's softened kernel against an independent derivation.

The oracle writes F (force factor) and P (potential factor) as closed
polynomials.  Here they are re-derived symbolically from the M4 cubic-spline
density alone (Sec. 2.1 footnote: the kernel; Sec. 2.2.1: compact support =
softening radius, Newtonian beyond it): the enclosed mass by integrating the
density, the potential by integrating the force inward from the support
radius.  A dropped term, wrong coefficient or wrong branch fails here.
"""
import json
import os

import numpy as np
import pytest
import sympy as sp

from oracle import direct

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_constants.json")))

from kernel_ref import D, NORM, W_in, W_out, s, u



def _ref(uu, hh):
    """F, P, (dF/dr)/r, dF/dh, dP/dh from the symbolic derivation."""
    r = sp.Symbol("r", positive=True)
    hs = sp.Symbol("hs", positive=True)
    if uu >= 1:
        F = 1 / r ** 3
        P = 1 / r
    elif uu < 0.5:
        F = D["F_in"].subs(u, r / hs) / hs ** 3
        P = D["psi_in"].subs(u, r / hs) / hs
    else:
        F = D["F_out"].subs(u, r / hs) / hs ** 3
        P = D["psi_out"].subs(u, r / hs) / hs
    # exact rationals: the float inputs' binary values, no 15-digit rounding
    hq = sp.Rational(hh)
    vals = {r: sp.Rational(uu * hh), hs: hq}
    if uu == 0:
        vals[r] = sp.Rational(1, 10 ** 30)   # r -> 0 limit, well inside double precision
    out = [F, P, sp.diff(F, r) / r, sp.diff(F, hs), sp.diff(P, hs)]
    # 80 digits: the outer branch cancels ~20 digits just below u = 1
    return [float(sp.N(e.subs(vals), 80)) for e in out]


def test_total_mass_is_one():
    assert sp.simplify(D["q_out"].subs(u, 1) - 1) == 0


def test_normalisation_and_second_moment():
    # int W dV = 1 and <|y|^2>_W = 9/40 h^2 (used by the uniform-sphere pin)
    m2 = sp.integrate(4 * sp.pi * NORM * W_in * s ** 4, (s, 0, sp.Rational(1, 2))) + \
        sp.integrate(4 * sp.pi * NORM * W_out * s ** 4, (s, sp.Rational(1, 2), 1))
    assert sp.nsimplify(m2) == sp.Rational(9, 40)


def test_central_potential_matches_plummer_equivalent():
    # P(0, h) = 2.8/h  <=>  Plummer-equivalent softening h/2.8 (Sec. 2.3.1)
    ratio = GOLD["plummer_equivalent_ratio"]["value"]
    assert float(D["psi_in"].subs(u, 0)) == pytest.approx(ratio, rel=1e-15)
    for hh in (1e-4, 0.2, 3.0):
        F, P, *_ = direct.kernel([0.0], [hh])
        assert P[0] == pytest.approx(ratio / hh, rel=1e-14)


@pytest.mark.parametrize("uu", [0.0, 1e-6, 0.1, 0.25, 0.4999999, 0.5, 0.5000001, 0.6,
                                0.75, 0.9, 0.9999999, 1.0, 1.0000001, 1.5, 7.0])
@pytest.mark.parametrize("hh", [1e-4, 0.3, 2.0])
def test_closed_forms_vs_derivation(uu, hh):
    got = [v[0] for v in direct.kernel([uu * hh], [hh])]
    ref = _ref(uu, hh)
    names = ["F", "P", "FrOverR", "dFdh", "dPdh"]
    # Within 1e-6 of u = 1 the factors (1-u)^3 amplify the rounding of u = r/h
    # in the double input (condition number ~ 3/(1-u)); elsewhere 1e-11.
    tol = 1e-11 if abs(uu - 1.0) > 1e-3 else 1e-7
    for name, g, r in zip(names, got, ref):
        scale = max(abs(r), 1e-300)
        assert abs(g - r) <= tol * scale + 1e-300, (name, uu, hh, g, r)


def test_continuity_at_branch_points():
    for hh in (0.01, 1.0):
        for ub in (0.5, 1.0):
            lo = direct.kernel([ub * hh * (1 - 1e-12)], [hh])
            hi = direct.kernel([ub * hh * (1 + 1e-12)], [hh])
            for a, b in zip(lo[:2], hi[:2]):
                assert a[0] == pytest.approx(b[0], rel=1e-9)


def test_newtonian_beyond_support():
    r = np.array([1.0, 1.5, 10.0, 1e3]) * 0.37
    F, P, FrR, dFh, dPh = direct.kernel(r, np.full(4, 0.37))
    assert np.allclose(F, 1 / r ** 3, rtol=1e-15, atol=0)
    assert np.allclose(P, 1 / r, rtol=1e-15, atol=0)
    assert np.all(dFh == 0) and np.all(dPh == 0)


def test_potential_derivative_is_minus_r_F():
    # dP/dr = -r F everywhere (P is the potential of the force F d)
    hh = 0.7
    r = np.linspace(0.01, 1.3, 257) * hh
    eps = 1e-7 * hh
    _, Pp, *_ = direct.kernel(r + eps, np.full_like(r, hh))
    _, Pm, *_ = direct.kernel(r - eps, np.full_like(r, hh))
    F, *_ = direct.kernel(r, np.full_like(r, hh))
    dPdr = (Pp - Pm) / (2 * eps)
    assert np.allclose(dPdr, -r * F, rtol=1e-6, atol=1e-9)
