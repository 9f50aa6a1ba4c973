"""Seeded synthetic workloads shared by the oracle-side tests and the GPU path.

This package only draws random numbers and lays out geometry (grid sizes,
optode cells, RBF lattices).  It contains none of the method's arithmetic:
no PDE coefficients, no absorption model, no solves, no scaling of the
Rademacher signs.  Both the CPU oracle and the HIP path consume exactly the
arrays produced here.
"""

from .configs import CONFIGS, INVERSION_CONFIGS, TEST_CONFIGS, WorkloadConfig, get_config
from .inputs import Workload, make_workload, sketch_draws

__all__ = [
    "CONFIGS",
    "TEST_CONFIGS",
    "INVERSION_CONFIGS",
    "WorkloadConfig",
    "get_config",
    "Workload",
    "make_workload",
    "sketch_draws",
]
