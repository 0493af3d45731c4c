"""oracle/rad.py -- TEST INFRASTRUCTURE ONLY (never imported by the library).

Tree-pass radiation sums of Sec. 3 that ride on the gravity walk, in plain
FP64 numpy:

* FUV column densities in 6 angular bins (Sec. 3.1: the optical depths of
  tree nodes summed into angular bins during the gravity pass, 6 bins by
  default).  Reading: the bins are the six faces of a cube around the
  target (direction d = x_j - x_i falls in the bin of its largest |d_k| with
  that component's sign; each bin spans 4 pi / 6 sr), and a bin's value is
  the column density averaged over its solid angle, which for point masses
  is exactly sum_j m_j / (Omega_bin r_j^2); a particle's r^2 is softened to
  r^2 + (h_j / 2.8)^2 (its Plummer-equivalent radius); only gas contributes;
  an accepted tree node enters as its gas mass at its gas centre of mass.
  The optical depth of a bin is kappa times its column.
* The IR energy density from stars (Sec. 3.3, the LEBRON estimate summed in
  the gravity pass): e_IR = sum_s L_s / (4 pi c r^2) over sinks, with r^2
  softened to r^2 + (h_s / 2.8)^2; an accepted node enters with its total
  sink luminosity at the luminosity-weighted centre.
Both are computed for gas cells; sinks get zeros.
"""
import numpy as np

OMEGA_BIN = 4.0 * np.pi / 6.0


def bin_of(d):
    """Cube-face bin of directions d (.., 3): 0 +x, 1 -x, 2 +y, 3 -y, 4 +z, 5 -z."""
    ax = np.argmax(np.abs(d), axis=-1)
    s = np.take_along_axis(d, ax[..., None], axis=-1)[..., 0]
    return 2 * ax + (s < 0)


def columns_direct(x, m, h, n_gas):
    """(n, 6) bin-averaged gas column densities at every gas cell."""
    x, m, h = (np.asarray(v, np.float64) for v in (x, m, h))
    n = x.shape[0]
    out = np.zeros((n, 6))
    for i in range(n_gas):
        d = x[:n_gas] - x[i]
        w = m[:n_gas] / (OMEGA_BIN * ((d * d).sum(1) + (h[:n_gas] / 2.8) ** 2))
        w[i] = 0.0
        out[i] = np.bincount(bin_of(d), weights=w, minlength=6)
    return out


def e_ir_direct(x, h, lum, n_gas, c_light):
    """(n,) IR energy density from the sinks' luminosities at every gas cell."""
    x, h, lum = (np.asarray(v, np.float64) for v in (x, h, lum))
    n = x.shape[0]
    out = np.zeros(n)
    if n_gas == n:
        return out
    d = x[None, n_gas:, :] - x[:n_gas, None, :]
    r2 = (d * d).sum(-1) + (h[None, n_gas:] / 2.8) ** 2
    out[:n_gas] = (lum[None, n_gas:] / (4.0 * np.pi * c_light * r2)).sum(1)
    return out


def tree_rad(x, m, h, lum, n_gas, lists, c_light):
    """Columns and e_IR of gas cells from the frozen group lists: accepted
    nodes by their gas mass at the gas centre of mass and their sink
    luminosity at the luminosity centre, opened particles one by one."""
    tree = lists.tree
    x, m, h, lum = (np.asarray(v, np.float64) for v in (x, m, h, lum))
    n = x.shape[0]
    xs, ms, hs, ls = x[tree.order], m[tree.order], h[tree.order], lum[tree.order]
    sink = lists.is_sink_sorted
    col = np.zeros((n, 6))
    eir = np.zeros(n)
    for g, (pc, pp) in lists.gas_lists.items():
        f, c = lists.groups[g]
        tg = np.arange(f, f + c)
        tg = tg[~sink[tg]]
        for t in tg:
            cb = np.zeros(6)
            e = 0.0
            for k in pc:
                a, b = tree.first[k], tree.first[k] + tree.count[k]
                gm = ms[a:b] * ~sink[a:b]
                if gm.sum() > 0:
                    cg = (gm[:, None] * xs[a:b]).sum(0) / gm.sum()
                    d = cg - xs[t]
                    cb[bin_of(d)] += gm.sum() / (OMEGA_BIN * (d * d).sum())
                lk = ls[a:b] * sink[a:b]
                if lk.sum() > 0:
                    cl = (lk[:, None] * xs[a:b]).sum(0) / lk.sum()
                    d = cl - xs[t]
                    e += lk.sum() / (4.0 * np.pi * c_light * (d * d).sum())
            src = pp[pp != t]
            d = xs[src] - xs[t]
            r2 = (d * d).sum(1) + (hs[src] / 2.8) ** 2
            gsrc = ~sink[src]
            cb += np.bincount(bin_of(d[gsrc]), weights=ms[src][gsrc] / (OMEGA_BIN * r2[gsrc]),
                              minlength=6)
            e += np.sum(ls[src][~gsrc] / (4.0 * np.pi * c_light * r2[~gsrc]))
            col[tree.order[t]] = cb
            eir[tree.order[t]] = e
    return col, eir
