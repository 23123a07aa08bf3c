"""Shared test plumbing: run the same seeded workload through the oracle and
through the GPU library's C ABI. No model arithmetic lives here."""
from __future__ import annotations

import numpy as np

import oracle
from oracle import OracleCfg, OracleSolver


def oracle_labels(geom):
    """Labels of a Geometry, voxelised by the oracle from the shared seeded
    primitives (the oracle's own copy of the generator)."""
    from paper_2110_13055_amd import _lib as L
    if geom.kind == L.USER_LABELS:
        return np.ascontiguousarray(geom.user_labels, dtype=np.uint8).reshape(-1)
    if geom.kind == L.FIBRES:
        fib = oracle.fibres(geom.nx, geom.ny, geom.nz, geom.buffer_x, geom.seed, geom.porosity, geom.r_min,
                            geom.r_max)
        return oracle.voxelize_fibres(geom.nx, geom.ny, geom.nz, geom.buffer_x, fib)
    if geom.kind == L.DISKS:
        prims, _ = oracle.disks(geom.nx, geom.ny, geom.buffer_x, geom.walls_y, geom.seed, geom.porosity,
                                geom.r_min, geom.r_max, geom.min_gap)
        return oracle.voxelize(2, geom.nx, geom.ny, 1, geom.walls_y, geom.buffer_x, prims)
    prims = oracle.spheres(geom.nx, geom.ny, geom.nz, geom.buffer_x, geom.seed, geom.porosity,
                           geom.r_min, geom.r_max)
    return oracle.voxelize(3, geom.nx, geom.ny, geom.nz, 0, geom.buffer_x, prims)


def oracle_cfg(geom, params) -> OracleCfg:
    return OracleCfg(dim=geom.dim, nx=geom.nx, ny=geom.ny, nz=geom.nz if geom.dim == 3 else 1,
                     drive=params.drive, equilibrium=params.equilibrium, tau=params.tau,
                     u_in=params.u_in, rho_out=params.rho_out, force=tuple(params.body_force),
                     D=tuple(params.D), z=tuple(params.z), c0=params.c0, c_out=params.c_out,
                     Ka=params.Ka, dpsi=params.dpsi_vt, np_x_bc=params.np_x_bc,
                     np_substeps=params.np_substeps, no_adsorption=params.no_adsorption)


def oracle_solver(geom, params, psi=None) -> OracleSolver:
    return OracleSolver(oracle_cfg(geom, params), oracle_labels(geom), psi=psi)


def rel_l2(a, b) -> float:
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))
