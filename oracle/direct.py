"""ctypes access to the oracle's FP64 direct sum -- TEST INFRASTRUCTURE ONLY."""
import ctypes
import os

import numpy as np

from . import build as _build

_lib = None
_D = ctypes.POINTER(ctypes.c_double)
_L = ctypes.POINTER(ctypes.c_int64)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = ctypes.CDLL(_build.LIB)
        L.or_kernel.argtypes = [ctypes.c_int64, _D, _D, _D, _D, _D, _D, _D]
        L.or_direct.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                ctypes.c_int64, _L, _D, _D]
        L.or_direct_vjp.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                    _D, _D, _D, _D, _D]
        L.or_direct_vjp_sparse.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                           _D, _D, ctypes.c_int64, _L,
                                           ctypes.POINTER(ctypes.c_ubyte), _D, _D, _D]
        L.or_pair_loss.argtypes = [ctypes.c_int64, _D, _D, _D, ctypes.c_double,
                                   _D, _D, ctypes.c_int64, _D, ctypes.c_double,
                                   ctypes.c_double]
        L.or_pair_loss.restype = ctypes.c_double
        L.or_direct_tidal.argtypes = [ctypes.c_int64, _D, _D, _D, _D, ctypes.c_double,
                                      ctypes.c_int64, _L, _D, _D]
        _lib = L
    return _lib


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _p(a):
    return a.ctypes.data_as(_D)


def kernel(r, h):
    """F, P, (dF/dr)/r, dF/dh, dP/dh of the softened kernel at (r, h)."""
    r, h = np.broadcast_arrays(_d(r), _d(h))
    r, h = _d(r).ravel(), _d(h).ravel()
    outs = [np.empty_like(r) for _ in range(5)]
    lib().or_kernel(r.size, _p(r), _p(h), *[_p(o) for o in outs])
    return tuple(outs)


def direct(x, m, h, G=1.0, targets=None):
    """FP64 accelerations (n_t,3) and potentials (n_t,) by direct summation."""
    x, m, h = _d(x), _d(m), _d(h)
    n = x.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        t = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp = t.size, t.ctypes.data_as(_L)
    acc = np.empty((nt, 3))
    pot = np.empty(nt)
    lib().or_direct(n, _p(x), _p(m), _p(h), float(G), nt, tp, _p(acc), _p(pot))
    return acc, pot


def direct_tidal(x, m, h, v=None, G=1.0, targets=None):
    """FP64 tidal tensor (n_t, 6: xx yy zz xy xz yz) and, with velocities v,
    jerk (n_t, 3) by direct summation (None without v)."""
    x, m, h = _d(x), _d(m), _d(h)
    n = x.shape[0]
    if targets is None:
        nt, tp = n, None
    else:
        t = np.ascontiguousarray(targets, dtype=np.int64)
        nt, tp = t.size, t.ctypes.data_as(_L)
    T = np.empty((nt, 6))
    J = np.empty((nt, 3)) if v is not None else None
    vp = _p(_d(v)) if v is not None else None
    if v is not None:
        v = _d(v)
        vp = _p(v)
    lib().or_direct_tidal(n, _p(x), _p(m), _p(h), vp, float(G), nt, tp, _p(T),
                          _p(J) if J is not None else None)
    return T, J


def direct_vjp(x, m, h, ga, gp, G=1.0):
    """Exact gradients (dL/dx, dL/dm, dL/dh) of L = sum ga.a + gp.phi."""
    x, m, h, ga, gp = _d(x), _d(m), _d(h), _d(ga), _d(gp)
    n = x.shape[0]
    gx, gm, gh = np.empty((n, 3)), np.empty(n), np.empty(n)
    lib().or_direct_vjp(n, _p(x), _p(m), _p(h), float(G), _p(ga), _p(gp),
                        _p(gx), _p(gm), _p(gh))
    return gx, gm, gh


def direct_vjp_sparse(x, m, h, ga, gp, G=1.0):
    """direct_vjp when few particles carry nonzero cotangents: the same
    gradients, skipping the pairs whose terms are exact zeros (O(k n) for k
    particles with cotangents)."""
    x, m, h, ga, gp = _d(x), _d(m), _d(h), _d(ga), _d(gp)
    n = x.shape[0]
    flag = np.ascontiguousarray((np.abs(ga).sum(1) + np.abs(gp)) > 0, dtype=np.uint8)
    act = np.ascontiguousarray(np.nonzero(flag)[0], dtype=np.int64)
    gx, gm, gh = np.empty((n, 3)), np.empty(n), np.empty(n)
    lib().or_direct_vjp_sparse(n, _p(x), _p(m), _p(h), float(G), _p(ga), _p(gp), act.size,
                               act.ctypes.data_as(_L),
                               flag.ctypes.data_as(ctypes.POINTER(ctypes.c_ubyte)),
                               _p(gx), _p(gm), _p(gh))
    return gx, gm, gh


def pair_loss(x, m, h, ga, gp, k, xk=None, mk=None, hk=None, G=1.0):
    """Part of L that involves particle k, with k's values optionally replaced."""
    x, m, h, ga, gp = _d(x), _d(m), _d(h), _d(ga), _d(gp)
    xk3 = _d(x[k] if xk is None else xk)
    return lib().or_pair_loss(x.shape[0], _p(x), _p(m), _p(h), float(G), _p(ga), _p(gp),
                              int(k), _p(xk3), float(m[k] if mk is None else mk),
                              float(h[k] if hk is None else hk))


def fd_gradient(x, m, h, ga, gp, k, eps=1e-6, G=1.0):
    """Central differences of L in x_k (3), m_k and h_k, pair-local."""
    x = _d(x)
    out = np.empty(5)
    for d in range(3):
        xp, xm = x[k].copy(), x[k].copy()
        xp[d] += eps
        xm[d] -= eps
        out[d] = (pair_loss(x, m, h, ga, gp, k, xk=xp, G=G)
                  - pair_loss(x, m, h, ga, gp, k, xk=xm, G=G)) / (2 * eps)
    out[3] = (pair_loss(x, m, h, ga, gp, k, mk=m[k] + eps, G=G)
              - pair_loss(x, m, h, ga, gp, k, mk=m[k] - eps, G=G)) / (2 * eps)
    out[4] = (pair_loss(x, m, h, ga, gp, k, hk=h[k] + eps, G=G)
              - pair_loss(x, m, h, ga, gp, k, hk=h[k] - eps, G=G)) / (2 * eps)
    return out
