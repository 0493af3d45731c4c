"""Independent derivation of the softened kernel, for the tests only.

Derives, with sympy, the force factor F and potential factor P of a unit mass
smoothed by the M4 cubic spline of compact support h (Sec. 2.1 footnote and
Sec. 2.2.1), starting from the density alone.  Nothing here is shared with the
oracle or the GPU library; both are checked against it.
"""
import mpmath
import sympy as sp

u, s, h = sp.symbols("u s h", positive=True)
W_in = 1 - 6 * s ** 2 + 6 * s ** 3          # density bracket, u < 1/2
W_out = 2 * (1 - s) ** 3                     # 1/2 <= u < 1
NORM = sp.Rational(8) / sp.pi                # W = 8/(pi h^3) * bracket


def _derived():
    # mass fraction enclosed within u: 4 pi int_0^u W s^2 ds (h cancels)
    q_in = sp.integrate(4 * sp.pi * NORM * W_in * s ** 2, (s, 0, u))
    q_half = q_in.subs(u, sp.Rational(1, 2))
    q_out = q_half + sp.integrate(4 * sp.pi * NORM * W_out * s ** 2, (s, sp.Rational(1, 2), u))
    # F(u) h^3 = q/u^3 ; potential: psi(u) = h P, psi(1) = 1, dpsi/du = -u F h^3
    F_in, F_out = sp.simplify(q_in / u ** 3), sp.simplify(q_out / u ** 3)
    psi_out = 1 + sp.integrate((s * F_out.subs(u, s)), (s, u, 1))
    psi_half = psi_out.subs(u, sp.Rational(1, 2))
    psi_in = psi_half + sp.integrate((s * F_in.subs(u, s)), (s, u, sp.Rational(1, 2)))
    return dict(q_in=q_in, q_out=q_out, F_in=F_in, F_out=F_out,
                psi_in=sp.expand(psi_in), psi_out=sp.expand(psi_out))


D = _derived()


_F_in_l = sp.lambdify(u, D["F_in"], "mpmath")
_F_out_l = sp.lambdify(u, D["F_out"], "mpmath")
_P_in_l = sp.lambdify(u, D["psi_in"], "mpmath")
_P_out_l = sp.lambdify(u, D["psi_out"], "mpmath")


def mp_FP(r, hh):
    """F(r,h), P(r,h) in mpmath at the current working precision."""
    r = mpmath.mpf(r)
    hh = mpmath.mpf(hh)
    uu = r / hh
    if uu >= 1:
        return 1 / r ** 3, 1 / r
    if uu < mpmath.mpf(1) / 2:
        return _F_in_l(uu) / hh ** 3, _P_in_l(uu) / hh
    return _F_out_l(uu) / hh ** 3, _P_out_l(uu) / hh


def mp_direct(x, m, h, G=1.0, dps=50):
    """Brute-force softened direct sum in mpmath (tiny N only)."""
    with mpmath.workdps(dps):
        n = len(m)
        acc = [[mpmath.mpf(0)] * 3 for _ in range(n)]
        pot = [mpmath.mpf(0)] * n
        X = [[mpmath.mpf(float(v)) for v in row] for row in x]
        for i in range(n):
            for j in range(n):
                if i == j:
                    continue
                d = [X[j][k] - X[i][k] for k in range(3)]
                r = mpmath.sqrt(d[0] ** 2 + d[1] ** 2 + d[2] ** 2)
                hij = max(mpmath.mpf(float(h[i])), mpmath.mpf(float(h[j])))
                F, P = mp_FP(r, hij)
                mj = mpmath.mpf(float(m[j]))
                for k in range(3):
                    acc[i][k] += G * mj * F * d[k]
                pot[i] -= G * mj * P
        return [[float(v) for v in row] for row in acc], [float(v) for v in pot]
