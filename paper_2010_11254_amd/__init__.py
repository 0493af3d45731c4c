"""MI355X-native softened self-gravity (STARFORGE/GIZMO method, arXiv 2010.11254).

The compute path is libsfgrav.so (hand-written HIP for gfx950) behind a C ABI
(include/sf_grav.h).  This package is a thin binding: ``_lib`` exposes the C
entry points under their own names, ``gravity`` wraps them in a
torch.autograd.Function.
"""
from ._lib import (  # noqa: F401
    SfGravError,
    Tree,
    make_opts,
    sf_grav_accel,
    sf_grav_accel_adaptive,
    sf_grav_accel_tidal,
    sf_grav_accel_backward,
    sf_grav_build_tree,
    sf_grav_get_stats,
    sf_grav_get_timings,
    sf_grav_get_tree_info,
    sf_grav_rad_sums,
    sf_grav_release_cache,
    sf_grav_sink_hermite,
    sf_grav_sinks,
    sf_grav_tree_export,
    sf_grav_tree_free,
    sf_grav_tree_refit,
    sf_grav_tree_set_field,
)
from .gravity import SFGravity, gravity  # noqa: F401
