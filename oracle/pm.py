"""oracle/pm.py -- TEST INFRASTRUCTURE ONLY (never imported by the library).

Adaptive gas-gas softening with symmetrised kernels and correction terms
(Sec. 2.2.1: gas softening follows the cell's kernel radius H_i, set by the
effective neighbour number N_NGB = 32 of Table 1, with the symmetrisation and
extra terms that make the interaction conserve momentum and energy), in
plain FP64 numpy: O(N^2) dense sums, and the same sums at chosen targets
over neighbours found with scipy's k-d tree (for checks at full size).
Readings (the cited force-law equations are not in the paper):

* the kernel radius of a gas cell solves (4 pi / 3) h_i^3 n_i = N_NGB with the
  number density n_i = sum_j W(r_ij, h_i) over gas cells, self included, and
  W the M4 cubic spline of compact support h normalised to 1;
* the pair potential of two gas cells is the average P_ij = (P(r, h_i) +
  P(r, h_j)) / 2 of the softened kernel, the total potential energy
  E = -(G/2) sum_i sum_{j != i} m_i m_j P_ij, and the acceleration is exactly
  -(1/m_i) dE/dx_i with every h_j a function of the positions through its
  constraint:
      a_i = G sum_j m_j (F(r, h_i) + F(r, h_j))/2 d
            - (G/2) sum_j [z_i W_r(r, h_i) + (m_j / m_i) z_j W_r(r, h_j)] d / r,
  d = x_j - x_i, W_r = dW/dr, z_i = zeta_i / Omega_i,
      zeta_i = (dh_i/dn_i) sum_{j != i} m_j dP(r_ij, h_i)/dh,
      Omega_i = 1 - (dh_i/dn_i) sum_j dW(r_ij, h_i)/dh,   dh/dn = -h/(3 n);
* the potential reported is phi_i = -G sum_j m_j P_ij (so E = sum m_i phi_i/2).
Gas-sink and sink-sink pairs keep the larger-radius rule of Sec. 2.2.1.
"""
import numpy as np

from . import direct

N_NGB = 32.0


def kernel_W(r, h):
    """W, dW/dr and dW/dh of the normalised M4 cubic spline."""
    u = r / h
    k = np.where(u < 0.5, 1 - 6 * u ** 2 + 6 * u ** 3, np.where(u < 1, 2 * (1 - u) ** 3, 0.0))
    dk = np.where(u < 0.5, -12 * u + 18 * u ** 2, np.where(u < 1, -6 * (1 - u) ** 2, 0.0))
    c = 8.0 / np.pi
    W = c * k / h ** 3
    Wr = c * dk / h ** 4
    Wh = -c * (3 * k + u * dk) / h ** 4
    return W, Wr, Wh


def neighbour_number(x, h):
    """(4 pi / 3) h_i^3 n_i for every gas cell (self included)."""
    x = np.asarray(x, np.float64)
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    W, _, _ = kernel_W(d, np.asarray(h, np.float64)[:, None])
    return 4.0 * np.pi / 3.0 * np.asarray(h) ** 3 * W.sum(1)


def solve_h(x, n_ngb=N_NGB, iters=200):
    """Kernel radii solving the neighbour-number constraint, by bisection
    (the neighbour number grows monotonically with h)."""
    x = np.asarray(x, np.float64)
    n = x.shape[0]
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    lo = np.zeros(n)
    hi = np.sort(d, axis=1)[:, min(n - 1, int(n_ngb) + 8)] * 4 + 1e-300
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        W, _, _ = kernel_W(d, mid[:, None])
        f = 4.0 * np.pi / 3.0 * mid ** 3 * W.sum(1) - n_ngb
        lo = np.where(f < 0, mid, lo)
        hi = np.where(f < 0, hi, mid)
    return 0.5 * (lo + hi)


def omega_zeta(x, m, h):
    """Omega_i and zeta_i of every gas cell (all cells gas)."""
    x, m, h = (np.asarray(v, np.float64) for v in (x, m, h))
    n = x.shape[0]
    d = np.sqrt(((x[:, None, :] - x[None, :, :]) ** 2).sum(-1))
    hh = np.broadcast_to(h[:, None], d.shape)
    W, _, Wh = kernel_W(d, hh)
    nd = W.sum(1)
    dhdn = -h / (3.0 * nd)
    omega = 1.0 - dhdn * Wh.sum(1)
    _, _, _, _, dPdh = direct.kernel(d.ravel(), hh.ravel())
    dPdh = dPdh.reshape(d.shape)
    np.fill_diagonal(dPdh, 0.0)
    zeta = dhdn * (dPdh * m[None, :]).sum(1)
    return omega, zeta


def pm_accel(x, m, h, n_gas=None, G=1.0):
    """Accelerations and potentials with the symmetrised gas-gas law (gas
    cells [0, n_gas), sinks after them with the larger-radius rule)."""
    x, m, h = (np.asarray(v, np.float64) for v in (x, m, h))
    n = x.shape[0]
    ng = n if n_gas is None else n_gas
    d = x[None, :, :] - x[:, None, :]            # d[i, j] = x_j - x_i
    r = np.sqrt((d * d).sum(-1))
    hi = np.broadcast_to(h[:, None], r.shape)
    hj = np.broadcast_to(h[None, :], r.shape)
    Fi, Pi, _, _, _ = (v.reshape(r.shape) for v in direct.kernel(r.ravel(), hi.ravel()))
    Fj, Pj, _, _, _ = (v.reshape(r.shape) for v in direct.kernel(r.ravel(), hj.ravel()))
    Fm, Pm, _, _, _ = (v.reshape(r.shape) for v in direct.kernel(r.ravel(), np.maximum(hi, hj).ravel()))
    gas = np.arange(n) < ng
    gg = gas[:, None] & gas[None, :]
    F = np.where(gg, 0.5 * (Fi + Fj), Fm)
    P = np.where(gg, 0.5 * (Pi + Pj), Pm)
    np.fill_diagonal(F, 0.0)
    np.fill_diagonal(P, 0.0)
    acc = G * ((m[None, :] * F)[..., None] * d).sum(1)
    pot = -G * (m[None, :] * P).sum(1)
    if ng > 0:
        om, ze = omega_zeta(x[:ng], m[:ng], h[:ng])
        z = ze / om
        _, Wri, _ = kernel_W(r[:ng, :ng], hi[:ng, :ng])
        _, Wrj, _ = kernel_W(r[:ng, :ng], hj[:ng, :ng])
        rs = np.where(r[:ng, :ng] > 0, r[:ng, :ng], 1.0)
        c = z[:, None] * Wri + (m[None, :ng] / m[:ng, None]) * z[None, :] * Wrj
        np.fill_diagonal(c, 0.0)
        acc[:ng] -= 0.5 * G * ((c / rs)[..., None] * d[:ng, :ng]).sum(1)
    return acc, pot


def pm_energy(x, m, h, G=1.0):
    """Total potential energy -(G/2) sum m_i m_j (P(r,h_i) + P(r,h_j))/2 (all gas)."""
    _, pot = pm_accel(x, m, h, G=G)
    return 0.5 * np.sum(np.asarray(m) * pot)


def omega_zeta_at(x, m, h, idx, kd=None):
    """Omega_i and zeta_i of the gas cells idx (x, m, h over gas cells only),
    from their neighbours within h_i found by a k-d tree: W, dW/dh and dP/dh
    vanish at and beyond h, so these are the sums of `omega_zeta`."""
    from scipy.spatial import cKDTree
    x, m, h = (np.asarray(v, np.float64) for v in (x, m, h))
    kd = cKDTree(x) if kd is None else kd
    om = np.empty(len(idx))
    ze = np.empty(len(idx))
    for k, i in enumerate(idx):
        nb = np.asarray(kd.query_ball_point(x[i], h[i]), dtype=np.int64)
        r = np.sqrt(((x[nb] - x[i]) ** 2).sum(1))
        W, _, Wh = kernel_W(r, h[i])
        dhdn = -h[i] / (3.0 * W.sum())
        om[k] = 1.0 - dhdn * Wh.sum()
        dPdh = direct.kernel(r, np.full(r.shape, h[i]))[4]
        dPdh[nb == i] = 0.0
        ze[k] = dhdn * (dPdh * m[nb]).sum()
    return om, ze


def pm_change_at(x, m, h, n_gas, targets, G=1.0):
    """For gas targets, pm_accel minus the larger-radius law of every pair
    (direct.direct): the acceleration and potential changes, from neighbour
    searches.  Only gas pairs closer than the larger of their two radii
    differ (beyond it every kernel is Newtonian and W_r vanishes), so each
    target looks at the gas cells within max(h_i, largest h); z_j = zeta_j /
    Omega_j comes from `omega_zeta_at`."""
    from scipy.spatial import cKDTree
    x, m, h = (np.asarray(v, np.float64) for v in (x, m, h))
    xg, mg, hg = x[:n_gas], m[:n_gas], h[:n_gas]
    kd = cKDTree(xg)
    hmax = hg.max()
    zc = {}

    def z_of(js):
        need = [j for j in js if j not in zc]
        if need:
            om, ze = omega_zeta_at(xg, mg, hg, need, kd)
            zc.update(zip(need, ze / om))
        return np.array([zc[j] for j in js])

    da = np.zeros((len(targets), 3))
    dp = np.zeros(len(targets))
    for k, i in enumerate(targets):
        nb = np.asarray(kd.query_ball_point(xg[i], max(hg[i], hmax)), dtype=np.int64)
        nb = nb[nb != i]
        d = xg[nb] - xg[i]
        r = np.sqrt((d * d).sum(1))
        near = r < np.maximum(hg[i], hg[nb])
        nb, d, r = nb[near], d[near], r[near]
        hi, hj = np.full(r.shape, hg[i]), hg[nb]
        Fi, Pi = direct.kernel(r, hi)[:2]
        Fj, Pj = direct.kernel(r, hj)[:2]
        Fm, Pm = direct.kernel(r, np.maximum(hi, hj))[:2]
        da[k] = G * ((mg[nb] * (0.5 * (Fi + Fj) - Fm))[:, None] * d).sum(0)
        dp[k] = -G * (mg[nb] * (0.5 * (Pi + Pj) - Pm)).sum()
        _, Wri, _ = kernel_W(r, hi)
        _, Wrj, _ = kernel_W(r, hj)
        c = z_of([int(i)])[0] * Wri + (mg[nb] / mg[i]) * z_of(nb.tolist()) * Wrj
        rs = np.where(r > 0, r, 1.0)
        da[k] -= 0.5 * G * ((c / rs)[:, None] * d).sum(0)
    return da, dp
