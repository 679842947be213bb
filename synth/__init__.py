"""Seeded synthetic workloads shared by the oracle tests and the GPU path.

This package only draws random numbers and lays out particles, sources and
receivers.  It holds none of the scattering method's arithmetic, so both the
CPU oracle and the HIP path can take their inputs from it without sharing any
part of the computation.
"""

from .layouts import (  # noqa: F401
    CONFIGS,
    Workload,
    make_workload,
    rejection_layout,
    receivers,
    perturbed_layout,
)
