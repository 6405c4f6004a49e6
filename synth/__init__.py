"""Seeded synthetic RHEED/TRHEPD workloads.

This package only draws and lays out inputs: beam sets (integer rod
indices), atom positions, Gaussian scattering parameters, slab geometry,
beam energy and glancing angles.  It contains none of the simulation's
arithmetic (no wavenumbers, no potentials, no propagation), so that the
CPU oracle and the GPU library can both consume it without sharing any
computation.
"""
from .workloads import (  # noqa: F401
    Structure,
    Workload,
    beams_nearest,
    beams_row,
    bulk_layer,
    config1,
    config2,
    config3,
    config4,
    config5,
    single_angle_n521,
    small_2d,
    small_row,
    WORKLOADS,
)
