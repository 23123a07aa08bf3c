"""FP64 CPU reference of the pore-scale CDI model (test infrastructure only).

Only the tests, the smoke check and the CPU-baseline leg of the benchmark
import this package. The GPU library never loads it. See ``cdi_oracle.h`` for
what each function computes and which passage of the paper it follows.
"""
from .oracle import (  # noqa: F401
    OracleCfg,
    OracleSolver,
    build,
    compact,
    disks,
    fibres,
    voxelize_fibres,
    library,
    spheres,
    sphere_count,
    voxelize,
    NPX_INLET_OUTLET,
    NPX_PERIODIC,
    NPX_CLOSED,
    NPX_DIRICHLET,
    DRIVE_INLET_OUTLET,
    DRIVE_BODY_FORCE,
    EQ_QUADRATIC,
    EQ_LINEAR,
    PSIX_DIRICHLET,
    PSIX_NEUMANN,
    PSIX_PERIODIC,
)
