"""Seeded synthetic inputs for the real-time Kohn-Sham step.

This package only builds input arrays (orbitals, local potential, projectors,
coupling constants, occupations, the laser vector potential, the
position-weighted projectors of the nonlocal current).  It performs none
of the propagation arithmetic, so both the FP64 CPU oracle and the HIP library
can consume the same inputs without sharing any of the method's code.
"""
from .workloads import (  # noqa: F401
    Domain,
    Workload,
    make_domain,
    pulse_midpoints,
    projector_moments,
    config,
    batched_domain_shapes,
    batched_domain,
    batched_subset,
)
