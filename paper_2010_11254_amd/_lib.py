"""ctypes binding of libsfgrav.so: the C entry points under the same names.

Argument marshalling only.  Every array is a torch tensor on the GPU (its
``data_ptr()`` is passed as a device pointer) and work is enqueued on torch's
current stream.  There is no CPU path: if the library is missing this module
raises on import of the library, and every call returns the library's status
as an exception.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsfgrav.so")

SF_OK, SF_E_INVALID, SF_E_NOMEM, SF_E_DEVICE, SF_E_STATE, SF_E_UNSUPPORTED, SF_E_INTERNAL = range(7)
SF_F32, SF_F64 = 0, 1
SF_FP32C, SF_FP32, SF_FP64 = 0, 1, 2
FORMS = {"fp32c": SF_FP32C, "fp32": SF_FP32, "fp64": SF_FP64}

EXPORTS = {
    "keys": (0, torch.int64, 1), "order": (1, torch.int32, 1),
    "node_level": (2, torch.int32, 0), "node_first": (3, torch.int32, 0),
    "node_count": (4, torch.int32, 0), "node_parent": (5, torch.int32, 0),
    "node_child": (6, torch.int32, 0), "node_nchild": (7, torch.int32, 0),
    "group_first": (8, torch.int32, 2), "group_count": (9, torch.int32, 2),
    "node_mass": (10, torch.float64, 0), "node_com": (11, torch.float64, 0),
    "node_quad": (12, torch.float64, 0), "group_npc": (13, torch.int32, 2),
    "group_npp": (14, torch.int32, 2), "group_cks": (15, torch.int64, 2),
}


class SfGravError(RuntimeError):
    def __init__(self, status, where, msg):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


class sf_grav_opts(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("form", ctypes.c_int32), ("G", ctypes.c_double),
        ("theta", ctypes.c_double), ("order", ctypes.c_int32), ("leaf_cap", ctypes.c_int32),
        ("group_cap", ctypes.c_int32), ("validate", ctypes.c_int32), ("n_gas", ctypes.c_int64),
        ("collect_stats", ctypes.c_int32), ("timing", ctypes.c_int32),
        ("alpha", ctypes.c_double),
    ]


class sf_grav_timings(ctypes.Structure):
    _fields_ = [("struct_size", ctypes.c_uint32), ("n_phases", ctypes.c_int32),
                ("ms", ctypes.c_double * 16)]


PHASES = ("sort", "topology", "moments", "groups", "sinksink", "walk", "sinkwalk",
          "b_sinksink", "b_walk", "b_sinkwalk", "b_pushdown")


class sf_grav_tree_info(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("max_level", ctypes.c_int32), ("n", ctypes.c_int64),
        ("n_gas", ctypes.c_int64), ("n_nodes", ctypes.c_int64), ("n_groups", ctypes.c_int64),
        ("n_leaves", ctypes.c_int64),
    ]


class sf_grav_stats(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32), ("max_level", ctypes.c_int32),
        ("n_nodes", ctypes.c_int64), ("n_leaves", ctypes.c_int64), ("n_groups", ctypes.c_int64),
        ("n_pc", ctypes.c_int64), ("n_pp", ctypes.c_int64), ("hist", ctypes.c_int64 * 32),
        ("checksum", ctypes.c_uint64),
    ]


_lib = None
EXPORTED = ("sf_grav_opts_default", "sf_grav_build_tree", "sf_grav_accel",
            "sf_grav_accel_backward", "sf_grav_tree_free", "sf_grav_get_tree_info",
            "sf_grav_tree_export", "sf_grav_get_timings", "sf_grav_strerror",
            "sf_grav_last_error", "sf_grav_tree_set_field", "sf_grav_tree_refit",
            "sf_grav_get_stats", "sf_grav_release_cache", "sf_grav_accel_direct_noalloc",
            "sf_grav_accel_tidal", "sf_grav_sinks", "sf_grav_sink_hermite",
            "sf_grav_accel_adaptive", "sf_grav_rad_sums")


def lib():
    """Load libsfgrav.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} not found: build it with "
                          "`python -m paper_2010_11254_amd.build` (hipcc, gfx950)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    L.sf_grav_opts_default.argtypes = [ctypes.POINTER(sf_grav_opts)]
    L.sf_grav_opts_default.restype = None
    L.sf_grav_build_tree.argtypes = [vp, vp, vp, i64, i32, ctypes.POINTER(sf_grav_opts), vp,
                                     ctypes.POINTER(vp)]
    L.sf_grav_accel.argtypes = [vp, vp, vp, vp, i64, i32, ctypes.POINTER(sf_grav_opts), vp, vp, vp]
    L.sf_grav_accel_backward.argtypes = [vp, vp, vp, vp, i64, i32, ctypes.POINTER(sf_grav_opts),
                                         vp, vp, vp, vp, vp, vp]
    L.sf_grav_tree_free.argtypes = [vp]
    L.sf_grav_get_tree_info.argtypes = [vp, ctypes.POINTER(sf_grav_tree_info)]
    L.sf_grav_tree_export.argtypes = [vp, i32, vp, ctypes.c_size_t]
    L.sf_grav_get_timings.argtypes = [vp, ctypes.POINTER(sf_grav_timings)]
    L.sf_grav_strerror.argtypes = [i32]
    L.sf_grav_strerror.restype = ctypes.c_char_p
    L.sf_grav_last_error.argtypes = []
    L.sf_grav_last_error.restype = ctypes.c_char_p
    L.sf_grav_tree_set_field.argtypes = [vp, vp, vp]
    L.sf_grav_tree_refit.argtypes = [vp, vp, vp, vp, vp]
    L.sf_grav_get_stats.argtypes = [vp, ctypes.POINTER(sf_grav_stats)]
    L.sf_grav_release_cache.argtypes = [ctypes.POINTER(ctypes.c_size_t)]
    L.sf_grav_accel_tidal.argtypes = [vp, vp, ctypes.POINTER(sf_grav_opts), vp, vp, vp, vp, vp]
    f64 = ctypes.c_double
    L.sf_grav_sinks.argtypes = [vp, vp, vp, vp, i64, f64, f64, vp, vp, vp, vp, vp, vp]
    L.sf_grav_sink_hermite.argtypes = [vp, vp, vp, vp, i64, f64, f64, vp]
    L.sf_grav_accel_adaptive.argtypes = [vp, ctypes.POINTER(sf_grav_opts), vp, vp, vp, vp]
    L.sf_grav_rad_sums.argtypes = [vp, vp, f64, ctypes.POINTER(sf_grav_opts), vp, vp, vp]
    L.sf_grav_accel_direct_noalloc.argtypes = [vp, vp, vp, i64, i32, ctypes.POINTER(sf_grav_opts),
                                               vp, vp, vp]
    for name in ("sf_grav_build_tree", "sf_grav_accel", "sf_grav_accel_backward",
                 "sf_grav_tree_free", "sf_grav_get_tree_info", "sf_grav_tree_export",
                 "sf_grav_get_timings", "sf_grav_tree_set_field", "sf_grav_tree_refit",
                 "sf_grav_get_stats", "sf_grav_release_cache", "sf_grav_accel_direct_noalloc",
                 "sf_grav_accel_tidal", "sf_grav_sinks", "sf_grav_sink_hermite",
                 "sf_grav_accel_adaptive", "sf_grav_rad_sums"):
        getattr(L, name).restype = i32
    _lib = L
    return L


def _check(status, where):
    if status != SF_OK:
        L = lib()
        msg = L.sf_grav_last_error().decode() or L.sf_grav_strerror(status).decode()
        raise SfGravError(status, where, msg)


def make_opts(form="fp32c", G=1.0, theta=0.5, order=2, leaf_cap=32, group_cap=32,
              validate=False, n_gas=-1, collect_stats=False, timing=False, alpha=None):
    """sf_grav_opts; alpha=None leaves the relative criterion off (-1)."""
    o = sf_grav_opts()
    lib().sf_grav_opts_default(ctypes.byref(o))
    o.form = FORMS[form] if isinstance(form, str) else int(form)
    o.G, o.theta, o.order = float(G), float(theta), int(order)
    o.leaf_cap, o.group_cap = int(leaf_cap), int(group_cap)
    o.validate, o.n_gas, o.collect_stats = int(bool(validate)), int(n_gas), int(bool(collect_stats))
    o.timing = int(bool(timing))
    if alpha is not None:
        o.alpha = float(alpha)
    return o


def _dt(t):
    if t.dtype == torch.float32:
        return SF_F32
    if t.dtype == torch.float64:
        return SF_F64
    raise TypeError(f"unsupported dtype {t.dtype}")


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_inputs(pos, mass, soft):
    for name, t in (("pos", pos), ("mass", mass), ("soft", soft)):
        if not t.is_cuda:
            raise ValueError(f"{name} must be a GPU tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")
    if pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("pos must have shape (n, 3)")
    n = pos.shape[0]
    if mass.shape != (n,) or soft.shape != (n,):
        raise ValueError("mass and soft must have shape (n,)")
    if not (pos.dtype == mass.dtype == soft.dtype):
        raise ValueError("pos, mass and soft must share one dtype")


class Tree:
    """Owns an sf_grav_tree handle; freed by sf_grav_tree_free or on GC."""

    def __init__(self, handle, n, dtype):
        self.handle = handle
        self.n = n
        self.dtype = dtype

    def __del__(self):
        try:
            if self.handle:
                lib().sf_grav_tree_free(self.handle)
                self.handle = None
        except Exception:
            pass


def sf_grav_build_tree(pos, mass, soft, opts):
    _check_inputs(pos, mass, soft)
    h = ctypes.c_void_p()
    st = lib().sf_grav_build_tree(_ptr(pos), _ptr(mass), _ptr(soft), pos.shape[0], _dt(pos),
                                  ctypes.byref(opts), _stream(), ctypes.byref(h))
    _check(st, "sf_grav_build_tree")
    return Tree(h, pos.shape[0], pos.dtype)


def sf_grav_accel(tree, pos, mass, soft, opts, acc=None, pot=None, want_pot=True):
    """Write accelerations (n,3) and potentials (n,) into new or given tensors."""
    if tree is not None:
        n, dtype, dev = tree.n, tree.dtype, torch.device("cuda", torch.cuda.current_device())
    else:
        _check_inputs(pos, mass, soft)
        n, dtype, dev = pos.shape[0], pos.dtype, pos.device
    if acc is None:
        acc = torch.empty((n, 3), dtype=dtype, device=dev)
    if pot is None and want_pot:
        pot = torch.empty((n,), dtype=dtype, device=dev)
    st = lib().sf_grav_accel(tree.handle if tree is not None else None, _ptr(pos), _ptr(mass),
                             _ptr(soft), n, SF_F32 if dtype == torch.float32 else SF_F64,
                             ctypes.byref(opts), _ptr(acc), _ptr(pot), _stream())
    _check(st, "sf_grav_accel")
    return acc, pot


def sf_grav_accel_backward(tree, pos, mass, soft, opts, g_acc, g_pot=None, g_pos=None,
                           g_mass=None, g_soft=None, want=(True, True, True)):
    if tree is not None:
        n, dtype = tree.n, tree.dtype
        dev = torch.device("cuda", torch.cuda.current_device())
    else:
        _check_inputs(pos, mass, soft)
        n, dtype, dev = pos.shape[0], pos.dtype, pos.device
    g_acc = g_acc.contiguous()
    if g_pot is not None:
        g_pot = g_pot.contiguous()
    if g_pos is None and want[0]:
        g_pos = torch.empty((n, 3), dtype=dtype, device=dev)
    if g_mass is None and want[1]:
        g_mass = torch.empty((n,), dtype=dtype, device=dev)
    if g_soft is None and want[2]:
        g_soft = torch.empty((n,), dtype=dtype, device=dev)
    st = lib().sf_grav_accel_backward(tree.handle if tree is not None else None, _ptr(pos),
                                      _ptr(mass), _ptr(soft), n,
                                      SF_F32 if dtype == torch.float32 else SF_F64,
                                      ctypes.byref(opts), _ptr(g_acc), _ptr(g_pot), _ptr(g_pos),
                                      _ptr(g_mass), _ptr(g_soft), _stream())
    _check(st, "sf_grav_accel_backward")
    return g_pos, g_mass, g_soft


def sf_grav_tree_free(tree):
    if tree is not None and tree.handle:
        _check(lib().sf_grav_tree_free(tree.handle), "sf_grav_tree_free")
        tree.handle = None


def sf_grav_get_tree_info(tree):
    info = sf_grav_tree_info()
    info.struct_size = ctypes.sizeof(sf_grav_tree_info)
    _check(lib().sf_grav_get_tree_info(tree.handle, ctypes.byref(info)), "sf_grav_get_tree_info")
    return {k: getattr(info, k) for k, _ in sf_grav_tree_info._fields_ if k != "struct_size"}


def sf_grav_get_timings(tree):
    """Phase times (ms) of the handle's last build/accel/backward; None if not run."""
    t = sf_grav_timings()
    t.struct_size = ctypes.sizeof(sf_grav_timings)
    _check(lib().sf_grav_get_timings(tree.handle, ctypes.byref(t)), "sf_grav_get_timings")
    return {name: (t.ms[i] if t.ms[i] >= 0 else None) for i, name in enumerate(PHASES)}


def sf_grav_tree_export(tree, what):
    """Copy one of the handle's arrays to a new host tensor."""
    wid, dtype, size_kind = EXPORTS[what]
    info = sf_grav_get_tree_info(tree)
    count = {1: info["n"], 0: info["n_nodes"], 2: info["n_groups"]}[size_kind]
    width = {"node_com": 3, "node_quad": 6}.get(what, 1)
    out = torch.empty((count * width,), dtype=dtype)
    if out.numel() == 0:
        return out.view(count, width) if width > 1 else out
    nbytes = out.numel() * out.element_size()
    _check(lib().sf_grav_tree_export(tree.handle, wid, ctypes.c_void_p(out.data_ptr()), nbytes),
           "sf_grav_tree_export")
    return out.view(count, width) if width > 1 else out


def sf_grav_tree_set_field(tree, acc_prev):
    """Previous field (n, 3) in caller order for the relative criterion."""
    if not acc_prev.is_cuda or not acc_prev.is_contiguous():
        raise ValueError("acc_prev must be a contiguous GPU tensor")
    if acc_prev.shape != (tree.n, 3) or acc_prev.dtype != tree.dtype:
        raise ValueError("acc_prev must be (n, 3) in the handle's dtype")
    _check(lib().sf_grav_tree_set_field(tree.handle, _ptr(acc_prev), _stream()),
           "sf_grav_tree_set_field")


def sf_grav_tree_refit(tree, pos, mass, soft):
    """New particle values on the handle's frozen tree."""
    _check_inputs(pos, mass, soft)
    if pos.shape[0] != tree.n or pos.dtype != tree.dtype:
        raise ValueError("refit needs the handle's n and dtype")
    _check(lib().sf_grav_tree_refit(tree.handle, _ptr(pos), _ptr(mass), _ptr(soft), _stream()),
           "sf_grav_tree_refit")


def sf_grav_get_stats(tree):
    st = sf_grav_stats()
    st.struct_size = ctypes.sizeof(sf_grav_stats)
    _check(lib().sf_grav_get_stats(tree.handle, ctypes.byref(st)), "sf_grav_get_stats")
    out = {k: getattr(st, k) for k, _ in sf_grav_stats._fields_ if k not in ("struct_size", "hist")}
    out["hist"] = list(st.hist)
    return out


def sf_grav_release_cache():
    """Return the library's cached device blocks to HIP; bytes still in use."""
    live = ctypes.c_size_t(0)
    _check(lib().sf_grav_release_cache(ctypes.byref(live)), "sf_grav_release_cache")
    return int(live.value)


def sf_grav_accel_direct_noalloc(pos, mass, soft, opts, acc=None, pot=None, want_pot=True):
    """Direct path without device allocation inside the library (n <= 2^19);
    acc/pot: caller-allocated outputs (allocated here if not given)."""
    _check_inputs(pos, mass, soft)
    n, dtype = pos.shape[0], pos.dtype
    if acc is None:
        acc = torch.empty((n, 3), dtype=dtype, device=pos.device)
    if pot is None and want_pot:
        pot = torch.empty((n,), dtype=dtype, device=pos.device)
    st = lib().sf_grav_accel_direct_noalloc(_ptr(pos), _ptr(mass), _ptr(soft), n, _dt(pos),
                                            ctypes.byref(opts), _ptr(acc), _ptr(pot), _stream())
    _check(st, "sf_grav_accel_direct_noalloc")
    return acc, pot


def sf_grav_accel_tidal(tree, opts, vel=None, want_pot=True, want_tidal=True):
    """(acc, pot, tidal (n, 6: xx yy zz xy xz yz), jerk) of every particle from
    one tree walk; jerk only with velocities vel (n, 3)."""
    n, dtype = tree.n, tree.dtype
    dev = torch.device("cuda", torch.cuda.current_device())
    if vel is not None and (vel.shape != (n, 3) or vel.dtype != dtype or not vel.is_cuda
                            or not vel.is_contiguous()):
        raise ValueError("vel must be a contiguous (n, 3) GPU tensor in the handle's dtype")
    acc = torch.empty((n, 3), dtype=dtype, device=dev)
    pot = torch.empty((n,), dtype=dtype, device=dev) if want_pot else None
    tid = torch.empty((n, 6), dtype=dtype, device=dev) if want_tidal else None
    jerk = torch.empty((n, 3), dtype=dtype, device=dev) if vel is not None else None
    st = lib().sf_grav_accel_tidal(tree.handle, _ptr(vel), ctypes.byref(opts), _ptr(acc),
                                   _ptr(pot), _ptr(tid), _ptr(jerk), _stream())
    _check(st, "sf_grav_accel_tidal")
    return acc, pot, tid, jerk


def _sink_arrays(*ts):
    for t in ts:
        if t is not None and (not t.is_cuda or t.dtype != torch.float64 or not t.is_contiguous()):
            raise ValueError("sink arrays must be contiguous FP64 GPU tensors")


def sf_grav_sinks(pos, vel, mass, soft, G=1.0, eta=0.0, want=("acc", "pot", "jerk", "tidal", "times")):
    """Sinks-only FP64 pass: dict of the requested outputs (acc n x 3, pot n,
    jerk n x 3, tidal n x 6, times n x 4: t_c, t_dyn, dt_2body, dt_tidal)."""
    _sink_arrays(pos, vel, mass, soft)
    n = pos.shape[0]
    shapes = {"acc": (n, 3), "pot": (n,), "jerk": (n, 3), "tidal": (n, 6), "times": (n, 4)}
    out = {k: torch.empty(shapes[k], dtype=torch.float64, device=pos.device) for k in want}
    out.setdefault("acc", torch.empty((n, 3), dtype=torch.float64, device=pos.device))
    st = lib().sf_grav_sinks(_ptr(pos), _ptr(vel), _ptr(mass), _ptr(soft), n, float(G), float(eta),
                             _ptr(out["acc"]), _ptr(out.get("pot")), _ptr(out.get("jerk")),
                             _ptr(out.get("tidal")), _ptr(out.get("times")), _stream())
    _check(st, "sf_grav_sinks")
    return out


def sf_grav_sink_hermite(pos, vel, mass, soft, dt, G=1.0):
    """One modified Hermite step; pos and vel (FP64, n x 3) updated in place."""
    _sink_arrays(pos, vel, mass, soft)
    st = lib().sf_grav_sink_hermite(_ptr(pos), _ptr(vel), _ptr(mass), _ptr(soft), pos.shape[0],
                                    float(G), float(dt), _stream())
    _check(st, "sf_grav_sink_hermite")


def sf_grav_accel_adaptive(tree, opts, want_pot=True, want_aux=False):
    """(acc, pot, aux) with the symmetrised adaptive gas-gas softening; aux =
    (Omega, zeta) per particle (n, 2) when asked for."""
    n, dtype = tree.n, tree.dtype
    dev = torch.device("cuda", torch.cuda.current_device())
    acc = torch.empty((n, 3), dtype=dtype, device=dev)
    pot = torch.empty((n,), dtype=dtype, device=dev) if want_pot else None
    aux = torch.zeros((n, 2), dtype=dtype, device=dev) if want_aux else None
    st = lib().sf_grav_accel_adaptive(tree.handle, ctypes.byref(opts), _ptr(acc), _ptr(pot),
                                      _ptr(aux), _stream())
    _check(st, "sf_grav_accel_adaptive")
    return acc, pot, aux


def sf_grav_rad_sums(tree, opts, lum=None, c_light=1.0, want_column=True, want_e_ir=True):
    """(column (n, 6), e_ir (n,)) of the gas cells from one tree walk."""
    n, dtype = tree.n, tree.dtype
    dev = torch.device("cuda", torch.cuda.current_device())
    if lum is not None and (lum.shape != (n,) or lum.dtype != dtype or not lum.is_cuda):
        raise ValueError("lum must be an (n,) GPU tensor in the handle's dtype")
    col = torch.zeros((n, 6), dtype=dtype, device=dev) if want_column else None
    eir = torch.zeros((n,), dtype=dtype, device=dev) if want_e_ir else None
    st = lib().sf_grav_rad_sums(tree.handle, _ptr(lum), float(c_light), ctypes.byref(opts),
                                _ptr(col), _ptr(eir), _stream())
    _check(st, "sf_grav_rad_sums")
    return col, eir
