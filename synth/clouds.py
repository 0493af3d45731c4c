"""Synthetic gas + sink particle sets shaped like the paper's star-forming clouds.

The paper runs on giant-molecular-cloud initial conditions that are not public,
so these seeded generators stand in for them: clustered, strongly inhomogeneous
gas (Plummer clumps on a uniform background, or a Plummer-in-Plummer fractal),
adaptive gas softening equal to the radius enclosing the 32 nearest neighbours
(the kernel support with an effective neighbour number of 32, Table 1 and
Sec. 2.1), and sink particles with a fixed small softening (Sec. 2.2.1) placed
on gas positions or in close binaries.

Every array is drawn in float64 from ``numpy.random.default_rng(seed)`` in a
fixed order and only then cast to the workload dtype; softening lengths are
computed from the cast positions.  Particles ``[0, n_gas)`` are gas and
``[n_gas, n)`` are sinks.
"""
from __future__ import annotations

import dataclasses

import numpy as np
from scipy.spatial import cKDTree

N_NGB = 32          # effective neighbour number (Table 1)
SINK_SOFT = 1e-4    # fixed sink softening radius used by the clustered workloads


@dataclasses.dataclass
class ParticleSet:
    """Positions (n,3), masses (n,), softening radii (n,) and the gas/sink split."""
    x: np.ndarray
    m: np.ndarray
    h: np.ndarray
    n_gas: int
    name: str = ""
    seed: int = 0

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    @property
    def n_sink(self) -> int:
        return self.n - self.n_gas

    @property
    def dtype(self):
        return self.x.dtype


# ---------------------------------------------------------------- primitives

def _unit_ball(rng, k):
    """k points uniform in the unit ball: normals for direction, then radii."""
    v = rng.standard_normal((k, 3))
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    r = rng.random(k) ** (1.0 / 3.0)
    return v * r[:, None]


def _iso_dirs(rng, k):
    v = rng.standard_normal((k, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def _plummer(rng, n, a, rmax_factor=10.0):
    """n offsets from a Plummer sphere of scale radius a, truncated at 10a.

    Radii invert the enclosed-mass fraction X = r^3/(r^2+a^2)^(3/2); samples
    beyond rmax_factor*a are redrawn so no outlier inflates the root cell.
    """
    out = np.empty((n, 3))
    done = 0
    while done < n:
        k = n - done
        xq = rng.random(k)
        xq = np.clip(xq, 1e-300, None)
        r = a / np.sqrt(xq ** (-2.0 / 3.0) - 1.0)
        d = _iso_dirs(rng, k)
        keep = r <= rmax_factor * a
        kk = int(keep.sum())
        out[done:done + kk] = d[keep] * r[keep, None]
        done += kk
    return out


def _apportion(total, weights):
    """Largest-remainder split of `total` items in proportion to `weights`."""
    w = np.asarray(weights, dtype=np.float64)
    quota = total * w / w.sum()
    base = np.floor(quota).astype(np.int64)
    rem = total - int(base.sum())
    frac = quota - base
    order = np.lexsort((np.arange(len(w)), -frac))  # largest fraction, then index
    base[order[:rem]] += 1
    return base


def knn_radius(x, k=N_NGB, chunk=1 << 18):
    """Distance from each point to its k-th nearest *other* point (float64).

    The query asks for k+1 neighbours because each point finds itself first.
    """
    xd = np.asarray(x, dtype=np.float64)
    tree = cKDTree(xd, leafsize=32, balanced_tree=False, compact_nodes=False)
    out = np.empty(xd.shape[0])
    for s in range(0, xd.shape[0], chunk):
        d, _ = tree.query(xd[s:s + chunk], k=k + 1, workers=-1)
        out[s:s + chunk] = d[:, -1]
    return out


def _finish(name, seed, xg, mg, xs, ms, hs, dtype, h_gas=None):
    """Cast to dtype, then derive gas softening from the cast positions."""
    x = np.concatenate([xg, xs]).astype(dtype)
    m = np.concatenate([mg, ms]).astype(dtype)
    n_gas = xg.shape[0]
    if h_gas is None:
        h_gas = knn_radius(x[:n_gas])
    h = np.concatenate([np.broadcast_to(h_gas, (n_gas,)).astype(np.float64),
                        np.broadcast_to(hs, (xs.shape[0],)).astype(np.float64)])
    return ParticleSet(x=np.ascontiguousarray(x), m=np.ascontiguousarray(m),
                       h=np.ascontiguousarray(h.astype(dtype)), n_gas=n_gas,
                       name=name, seed=seed)


# ---------------------------------------------------------------- workloads

def uniform_sphere(n=4096, seed=0, dtype=np.float64, h=None):
    """Equal masses (total 1) uniform in the unit sphere, one softening for all.

    The default softening (32/n)^(1/3) makes a kernel hold about 32 neighbours.
    """
    rng = np.random.default_rng(seed)
    x = _unit_ball(rng, n)
    m = np.full(n, 1.0 / n)
    hh = (N_NGB / n) ** (1.0 / 3.0) if h is None else float(h)
    return _finish("uniform_sphere", seed, x, m, np.zeros((0, 3)), np.zeros(0),
                   np.zeros(0), dtype, h_gas=np.full(n, hh))


def _cluster_gas(rng, n_gas, n_clusters, a_lo, a_hi, frac_clustered=0.7):
    """Gas positions: Plummer clumps (70%) plus a uniform background (30%)."""
    centres = _unit_ball(rng, n_clusters)                    # normals, uniforms
    radii = np.exp(rng.uniform(np.log(a_lo), np.log(a_hi), n_clusters))
    weights = rng.lognormal(0.0, 1.0, n_clusters)
    n_cl = int(round(frac_clustered * n_gas))
    counts = _apportion(n_cl, weights)
    parts = [centres[k] + _plummer(rng, int(counts[k]), radii[k])
             for k in range(n_clusters)]
    parts.append(_unit_ball(rng, n_gas - n_cl))               # background
    return np.concatenate(parts)


def clustered_cloud(n_gas=1 << 20, n_sink=256, seed=1, dtype=np.float32,
                    n_clusters=512, a_lo=0.01, a_hi=0.05):
    """Clustered cloud: 512 Plummer clumps + background gas, sinks on gas cells.

    Sinks sit exactly on randomly chosen gas positions (so coincident distinct
    particles occur), with log-normal masses around 1e-3 and softening 1e-4.
    """
    rng = np.random.default_rng(seed)
    xg = _cluster_gas(rng, n_gas, n_clusters, a_lo, a_hi)
    mg = np.full(n_gas, 1.0 / n_gas)
    idx = rng.choice(n_gas, size=n_sink, replace=False)
    ms = rng.lognormal(np.log(1e-3), 1.0, n_sink)
    xs = xg[idx].astype(dtype).astype(np.float64)
    return _finish("clustered_cloud", seed, xg, mg, xs, ms, SINK_SOFT, dtype)


def _binaries(rng, xg, n_bin, mu, sigma):
    """n_bin binaries centred on distinct gas positions (float64 layout)."""
    idx = rng.choice(xg.shape[0], size=n_bin, replace=False)
    c = xg[idx]
    m1 = rng.lognormal(mu, sigma, n_bin)
    q = rng.uniform(0.1, 1.0, n_bin)
    m2 = q * m1
    sep = 10.0 ** rng.uniform(-5.0, -3.0, n_bin)
    axis = _iso_dirs(rng, n_bin)
    mt = m1 + m2
    x1 = c - (m2 / mt * sep)[:, None] * axis
    x2 = c + (m1 / mt * sep)[:, None] * axis
    xs = np.empty((2 * n_bin, 3))
    xs[0::2], xs[1::2] = x1, x2
    ms = np.empty(2 * n_bin)
    ms[0::2], ms[1::2] = m1, m2
    return xs, ms


def precision_cloud(n_gas=1 << 22, n_binaries=2048, seed=2, dtype=np.float32,
                    n_clusters=512, a_lo=1e-4, a_hi=0.05):
    """Precision workload: clumps down to 1e-4 scale radius + close binaries.

    Binary separations are log-uniform in [1e-5, 1e-3], below and above the
    sink softening, with mass ratios uniform in [0.1, 1].
    """
    rng = np.random.default_rng(seed)
    xg = _cluster_gas(rng, n_gas, n_clusters, a_lo, a_hi)
    mg = np.full(n_gas, 1.0 / n_gas)
    xs, ms = _binaries(rng, xg, n_binaries, np.log(1e-3), 1.0)
    return _finish("precision_cloud", seed, xg, mg, xs, ms, SINK_SOFT, dtype)


def differentiation_cloud(n_gas=1 << 18, seed=7, dtype=np.float32):
    """Gas-only clustered cloud for the gradient checks (clustered generator)."""
    rng = np.random.default_rng(seed)
    xg = _cluster_gas(rng, n_gas, 512, 0.01, 0.05)
    mg = np.full(n_gas, 1.0 / n_gas)
    return _finish("differentiation_cloud", seed, xg, mg, np.zeros((0, 3)),
                   np.zeros(0), np.zeros(0), dtype)


def fractal_cloud(n_gas=1 << 24, n_single=5000, n_binaries=2500, seed=4,
                  dtype=np.float32, levels=3, children=8, a1=0.1, shrink=0.2,
                  background=0.1):
    """Hierarchical fractal: Plummer-in-Plummer, 8 children per level.

    Level-1 centres are uniform in the unit sphere with scale radius a1; each
    child centre is drawn from its parent's (truncated) Plummer profile with a
    scale radius shrink times the parent's.  The leaves share 90% of the gas;
    10% is a uniform background.  Sinks: singles on gas positions and close
    binaries, log-normal masses with sigma 1.5.
    """
    rng = np.random.default_rng(seed)
    centres = _unit_ball(rng, children)
    a = a1
    for _ in range(levels - 1):
        kids = [c + _plummer(rng, children, a) for c in centres]
        centres = np.concatenate(kids)
        a *= shrink
    n_cl = int(round((1.0 - background) * n_gas))
    counts = _apportion(n_cl, np.ones(centres.shape[0]))
    parts = [centres[k] + _plummer(rng, int(counts[k]), a)
             for k in range(centres.shape[0])]
    parts.append(_unit_ball(rng, n_gas - n_cl))
    xg = np.concatenate(parts)
    mg = np.full(n_gas, 1.0 / n_gas)
    idx = rng.choice(n_gas, size=n_single, replace=False)
    x1 = xg[idx].astype(dtype).astype(np.float64)
    m1 = rng.lognormal(np.log(1e-3), 1.5, n_single)
    xb, mb = _binaries(rng, xg, n_binaries, np.log(1e-3), 1.5)
    return _finish("fractal_cloud", seed, xg, mg, np.concatenate([x1, xb]),
                   np.concatenate([m1, mb]), SINK_SOFT, dtype)


def cotangents(n, seed, dtype=np.float64):
    """Upstream gradients on (a, phi): i.i.d. standard normal."""
    rng = np.random.default_rng([seed, 1])
    ga = rng.standard_normal((n, 3))
    gp = rng.standard_normal(n)
    return ga.astype(dtype), gp.astype(dtype)


def velocities(n, seed, dtype=np.float32):
    """Particle velocities for the jerk: i.i.d. standard normal components."""
    rng = np.random.default_rng([seed, 5])
    return rng.standard_normal((n, 3)).astype(dtype)


def subsample(n, k, seed):
    """k distinct target indices drawn uniformly from [0, n), sorted."""
    rng = np.random.default_rng([seed, 3])
    return np.sort(rng.choice(n, size=min(k, n), replace=False)).astype(np.int64)


CONFIG_NAMES = ("uniform4k", "clustered1m", "precision4m", "diff256k", "fractal16m")


def make_config(name, scale=1.0):
    """Build one named workload; `scale` < 1 shrinks particle counts for tests."""
    def s(v):
        return max(64, int(round(v * scale)))
    if name == "uniform4k":
        return uniform_sphere(s(4096), seed=0, dtype=np.float64)
    if name == "clustered1m":
        return clustered_cloud(s(1 << 20), max(1, int(round(256 * scale))), seed=1)
    if name == "precision4m":
        return precision_cloud(s(1 << 22), max(1, int(round(2048 * scale))), seed=2)
    if name == "diff256k":
        return differentiation_cloud(s(1 << 18), seed=7)
    if name == "fractal16m":
        return fractal_cloud(s(1 << 24), max(1, int(round(5000 * scale))),
                             max(1, int(round(2500 * scale))), seed=4)
    raise ValueError(f"unknown workload {name!r}")
