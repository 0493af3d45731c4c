"""oracle/sinks.py -- TEST INFRASTRUCTURE ONLY (never imported by the library).

Sink dynamics of Sec. 2.3, in plain FP64 numpy on top of the oracle's direct
sum:

* the sinks-only gravity pass: acceleration, jerk and tidal tensor of every
  sink from all other sinks (the exact direct sum; Sec. 2.3.2 evaluates a_s0
  and j_s0 in a special sinks-only pass);
* the two-body time scales of Sec. 2.3.1 (Eqs. tcross, tdyn) with the
  Plummer-equivalent sink softening eps = h / 2.8, the 2-body timestep
  (Eq. dt_2body) and the tidal timestep (Eq. tidaltimestep);
* one step of the modified 4th-order Hermite scheme (Sec. 2.3.2, Eqs.
  predictor and corrector): a force/jerk evaluation at the start, the
  prediction, a second evaluation at the predicted state, then the
  correction of v and, with the corrected v, of x.
"""
import numpy as np

from . import direct


def sinks_pass(x, v, m, h, G=1.0):
    """(a, j, T) of every sink from the other sinks (T as xx yy zz xy xz yz)."""
    a, _ = direct.direct(x, m, h, G=G)
    T, j = direct.direct_tidal(x, m, h, v, G=G)
    return a, j, T


def two_body_times(x, v, m, h, G=1.0):
    """t_c,min and t_dyn,min of every sink (min over the other sinks s'):
    sqrt(r^2 + eps^2) / |v_ss'| and sqrt((r^2 + eps^2)^(3/2) / (G (m_s + m_s'))),
    eps = h_s / 2.8 (the sink's own Plummer-equivalent softening)."""
    x, v, m, h = (np.asarray(u, np.float64) for u in (x, v, m, h))
    n = m.size
    tc = np.full(n, np.inf)
    td = np.full(n, np.inf)
    for s in range(n):
        o = np.arange(n) != s
        eps = h[s] / 2.8
        r2 = ((x[o] - x[s]) ** 2).sum(1) + eps * eps
        vr = np.sqrt(((v[o] - v[s]) ** 2).sum(1))
        with np.errstate(divide="ignore"):
            tc[s] = np.min(np.sqrt(r2) / vr) if o.any() else np.inf
        td[s] = np.min(np.sqrt(r2 ** 1.5 / (G * (m[s] + m[o])))) if o.any() else np.inf
    return tc, td


def timesteps(x, v, m, h, eta, G=1.0):
    """(dt_2body, dt_tidal) of every sink: sqrt(eta) / (1/t_c + 1/t_dyn) and
    sqrt(eta) (|T|_F^2 / 6)^(-1/4), T from the sinks-only pass."""
    tc, td = two_body_times(x, v, m, h, G)
    with np.errstate(divide="ignore"):   # a lone sink: infinite time scales
        dt2 = np.sqrt(eta) / (1.0 / tc + 1.0 / td)
    _, _, T = sinks_pass(x, v, m, h, G)
    fro2 = (T[:, :3] ** 2).sum(1) + 2.0 * (T[:, 3:] ** 2).sum(1)
    with np.errstate(divide="ignore"):
        dtt = np.sqrt(eta) * (fro2 / 6.0) ** -0.25
    return dt2, dtt


def hermite_step(x, v, m, h, dt, G=1.0):
    """One modified Hermite step of all sinks with a common dt."""
    x, v = np.asarray(x, np.float64), np.asarray(v, np.float64)
    a0, j0, _ = sinks_pass(x, v, m, h, G)
    xp = x + dt * v + 0.5 * dt * dt * a0 + dt ** 3 / 6.0 * j0
    vp = v + dt * a0 + 0.5 * dt * dt * j0
    a1, j1, _ = sinks_pass(xp, vp, m, h, G)
    v1 = v + 0.5 * dt * (a1 + a0) + dt * dt / 12.0 * (j0 - j1)
    x1 = x + 0.5 * dt * (v1 + v) + dt * dt / 12.0 * (a0 - a1)
    return x1, v1


def energy(x, v, m, h, G=1.0):
    """Kinetic plus softened pair potential energy of the sinks."""
    _, pot = direct.direct(x, m, h, G=G)
    return 0.5 * np.sum(m * (np.asarray(v) ** 2).sum(1)) + 0.5 * np.sum(m * pot)
