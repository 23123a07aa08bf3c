"""MI355X (gfx950) pore-scale capacitive-deionisation solver.

Lattice Boltzmann Stokes flow on a voxelised porous electrode, coupled to an
explicit finite-volume Nernst-Planck update for Na+ and Cl- with the linear
adsorption law as a face flux (Liu, Waugh, Komini Babu, Spendelow, Kang,
2021). The numerics run in hand-written HIP kernels behind the C ABI of
``include/cdi.h``; this package is the thin Python binding.
"""
from . import _lib  # noqa: F401
from ._lib import (  # noqa: F401
    BODY_FORCE, DISKS, FIBRES, EQ_LINEAR, EQ_QUADRATIC, FP16, FP16_DEV, FP32, INLET_OUTLET, MOMENTS, NPX_CLOSED,
    NPX_DIRICHLET, NPX_INLET_OUTLET, NPX_PERIODIC, SPHERES, USER_LABELS, CdiError,
    MODE_FLOW, MODE_FUSED, MODE_IDLE, MODE_IONS, STREAM_AA, STREAM_PULL, PSIX_DIRICHLET, PSIX_NEUMANN,
    PSIX_PERIODIC, PROBE_COPY, PROBE_READ, PROBE_FILL,
)
from .solver import Batch, Geometry, Params, Potential, Solver, bandwidth_probe, flow_check, plan  # noqa: F401
from .presets import PRESETS, batch_instances, fibre_case, fibre_sweep, preset, serving_requests  # noqa: F401
