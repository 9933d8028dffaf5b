"""Seeded synthetic inputs for the direct-summation N-body workloads.

This package only *draws* inputs: Plummer-sphere positions, velocities and
masses, target positions and random adjoint seeds. It contains no force law,
no integrator and no diagnostic, so both the FP64 CPU oracle (``oracle/``) and
the HIP path (``paper_2411_18889_amd``) can consume its output without sharing
any of the method's arithmetic.
"""

from .plummer import plummer_positions_device, plummer_sphere, plummer_with_subcluster
from .configs import WORKLOADS, Workload, make_state, perturb_state, random_unit_vectors

__all__ = [
    "plummer_positions_device",
    "plummer_sphere",
    "plummer_with_subcluster",
    "WORKLOADS",
    "Workload",
    "make_state",
    "perturb_state",
    "random_unit_vectors",
]
