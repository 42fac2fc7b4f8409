"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package builds the *inputs* of the particle step and nothing else: the
frozen carrier-gas velocity field on a node grid, the initial particle
positions, diameters and base charges, the per-sample parameters of a Monte
Carlo batch, and the physical parameter set of each workload.  It holds none
of the particle step's arithmetic (no drag, no pair forces, no integration,
no wall test, no tally), so the oracle and the HIP path can both consume it
without sharing any of the method.

All random draws use NumPy's PCG64 ``default_rng(seed)``.
"""

from .workloads import WORKLOADS, Workload, make_workload, physical_params  # noqa: F401
from .field import make_field, reichardt_uplus  # noqa: F401
