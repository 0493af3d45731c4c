"""Seeded synthetic particle sets for the softened self-gravity path.

This package only draws inputs (positions, masses, softening lengths,
cotangents, subsample indices).  It holds none of the force arithmetic, so the
CPU oracle and the GPU library can both be fed from it without sharing code.
"""
from .clouds import (  # noqa: F401
    ParticleSet,
    uniform_sphere,
    clustered_cloud,
    precision_cloud,
    differentiation_cloud,
    fractal_cloud,
    knn_radius,
    cotangents,
    velocities,
    subsample,
    make_config,
    CONFIG_NAMES,
)
