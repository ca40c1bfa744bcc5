"""Seeded synthetic sparse matrices shaped like the paper's workloads.

This package only draws inputs.  It holds none of the solver's arithmetic, so
that the CPU oracle and the HIP path can both take their inputs from it without
sharing any code of the method itself.
"""
from .matrices import (  # noqa: F401
    to_csr,
    random_uniform_rows,
    uniform_workload,
    banded_scaled,
    banded_workload,
    powerlaw_rows,
    powerlaw_workload,
    batched_problem,
    convection_diffusion,
    convdiff_workload,
    prescribed_dense,
    prescribed_givens,
    one_per_row,
    block_diagonal,
)
