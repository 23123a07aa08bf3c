"""Named synthetic workloads (seeded), shaped like the paper's electrodes.

The paper's own geometries (a digitised SEM image, Sec. 4; random fibres,
Sec. 5) are not available, so each workload is a seeded synthetic electrode
with the porosity range and grain sizes of the paper's cases, in lattice
units. Diffusivities keep the paper's equal-D statement only as a ratio
(D_Cl / D_Na = 1.52); the default adsorption constant follows the paper's
Da / Pe ratio at its base case (Sec. 4.1).
"""
from __future__ import annotations

import numpy as np

from . import _lib as L
from .solver import Geometry, Params

BASE_SEED = 2110
D_NA = 0.05
D_CL = 1.52 * D_NA

PRESETS = {
    # 2D plain method: 128x64 D2Q9, walls top/bottom, non-overlapping disks
    "channel2d_128x64": dict(
        geom=dict(dim=2, nx=128, ny=64, kind=L.DISKS, porosity=0.7, r_min=4.0, r_max=8.0,
                  min_gap=2.0, walls_y=1, buffer_x=2, seed=BASE_SEED),
        params=dict(u_in=1e-3, dpsi_vt=10.0, D=(D_NA, D_CL)),
        flow_tol=1e-8, np_steps=5000),
    # 3D plain method: 128^3 D3Q19 overlapping spheres, periodic y/z
    "spheres3d_128": dict(
        geom=dict(dim=3, nx=128, ny=128, nz=128, kind=L.SPHERES, porosity=0.5, r_min=3.0,
                  r_max=6.0, buffer_x=2, seed=BASE_SEED),
        params=dict(u_in=5e-4, dpsi_vt=20.0, D=(D_NA, D_CL)),
        flow_tol=1e-8, np_steps=20000),
    # 3D large: 512^3, porosity 0.4 (about 54M fluid nodes)
    "spheres3d_512": dict(
        geom=dict(dim=3, nx=512, ny=512, nz=512, kind=L.SPHERES, porosity=0.4, r_min=3.0,
                  r_max=6.0, buffer_x=2, seed=BASE_SEED),
        params=dict(u_in=5e-4, dpsi_vt=20.0, D=(D_NA, D_CL)),
        flow_tol=1e-8, np_steps=20000),
    # seeded 64^3 sub-case of the large electrode (same statistics)
    "spheres3d_64": dict(
        geom=dict(dim=3, nx=64, ny=64, nz=64, kind=L.SPHERES, porosity=0.4, r_min=3.0,
                  r_max=6.0, buffer_x=2, seed=BASE_SEED),
        params=dict(u_in=5e-4, dpsi_vt=20.0, D=(D_NA, D_CL)),
        flow_tol=1e-8, np_steps=20000),
}


# Sec. 5 fibrous electrodes in lattice units: voxel 100 nm, D = 1e-9 m^2/s for
# both ions (Sec. 4) mapped to D = 0.15 (the largest round value inside the
# explicit update's positivity bound, 6 D < 1, so the slow diffusive and
# adsorptive approach to steady state takes the fewest steps), so one step
# is 1.5e-6 s; the mean pore velocity 1e-6 m/s becomes 1.5e-5 and K_a =
# 1e-6 m/s becomes 1.5e-5 (same scale); the fibre surface at -1.2 V is -46.7
# thermal voltages (298.15 K).
FIBRE_DX_M = 100e-9
FIBRE_D_LU = 0.15
FIBRE_DT_S = FIBRE_D_LU * FIBRE_DX_M ** 2 / 1e-9
FIBRE_U_PORE = 1e-6 * FIBRE_DT_S / FIBRE_DX_M
FIBRE_KA = 1e-6 * FIBRE_DT_S / FIBRE_DX_M
FIBRE_PSI_SURFACE = -1.2 / (1.380649e-23 * 298.15 / 1.602176634e-19)


def fibre_case(diameter_vox: int, porosity: float, n: int = 150, seed: int = BASE_SEED,
               precision: int = L.FP32, streaming: int = L.STREAM_PULL):
    """One electrode of the Sec. 5 sweep: n^3 voxels of straight overlapping
    fibres of the given diameter (4, 6, 8 voxels = 400, 600, 800 nm), the given
    porosity, inlet/outlet flow along x with the mean pore velocity of Sec. 5
    (the inlet plug is the superficial velocity phi * U), K_a of Sec. 4.
    -> (Geometry, Params)."""
    r = diameter_vox / 2.0
    g = Geometry(dim=3, nx=n, ny=n, nz=n, kind=L.FIBRES, porosity=porosity, r_min=r, r_max=r,
                 buffer_x=2, seed=seed)
    p = Params(u_in=porosity * FIBRE_U_PORE, dpsi_vt=0.0, D=(FIBRE_D_LU, FIBRE_D_LU), Ka=FIBRE_KA,
               precision=precision, streaming=streaming)
    return g, p


def fibre_sweep(n: int = 150, **kw):
    """The 12 electrodes of Sec. 5: diameters 4/6/8 voxels x porosity 0.5-0.8.
    -> list of ((diameter, porosity), Geometry, Params)."""
    return [((d, phi),) + fibre_case(d, phi, n=n, **kw) for d in (4, 6, 8) for phi in (0.5, 0.6, 0.7, 0.8)]


def preset(name: str, precision: int = L.FP32, **overrides):
    """-> (Geometry, Params, extra) for a named workload."""
    spec = PRESETS[name]
    g = Geometry(**spec["geom"])
    pk = dict(spec["params"])
    pk.update({k: v for k, v in overrides.items() if k in Params.__dataclass_fields__})
    p = Params(precision=precision, **pk)
    for k, v in overrides.items():
        if k in Geometry.__dataclass_fields__:
            setattr(g, k, v)
    extra = {k: v for k, v in spec.items() if k not in ("geom", "params")}
    return g, p, extra


def batch_instances(n: int = 64, base_seed: int = BASE_SEED, precision: int = L.FP32,
                    edge_range=(48, 160), streaming: int = L.STREAM_AA):
    """Independent 3D electrodes of uneven size for batched stepping: cubes
    with integer edge uniform on edge_range, overlapping spheres r in [3, 6],
    porosity U[0.35, 0.75], applied potential U[4, 40] thermal voltages,
    inlet velocity U[1e-4, 5e-3]; instance k has geometry seed base_seed + k.
    -> list of (Geometry, Params)."""
    rng = np.random.default_rng(base_seed)
    out = []
    for k in range(n):
        edge = int(rng.integers(edge_range[0], edge_range[1] + 1))
        phi = float(rng.uniform(0.35, 0.75))
        dpsi = float(rng.uniform(4.0, 40.0))
        u_in = float(rng.uniform(1e-4, 5e-3))
        g = Geometry(dim=3, nx=edge, ny=edge, nz=edge, kind=L.SPHERES, porosity=phi, r_min=3.0,
                     r_max=6.0, buffer_x=2, seed=base_seed + k)
        out.append((g, Params(u_in=u_in, dpsi_vt=dpsi, D=(D_NA, D_CL), precision=precision,
                              streaming=streaming)))
    return out


def serving_requests(n: int, rate_hz: float = 2.0, base_seed: int = BASE_SEED,
                     precision: int = L.FP32, np_steps_2d: int = 5000, np_steps_3d: int = 20000,
                     flow_tol: float = 1e-6, flow_max_steps: int = 20000,
                     streaming: int = L.STREAM_AA):
    """A fixed trace of mixed solve requests with Poisson arrivals: half are
    2D 256x256 D2Q9 channels (disks r in [4, 8], walls top/bottom, porosity
    U[0.55, 0.75], the range random sequential addition reaches), half 3D
    D3Q19 cubes with integer edge U{64..192} (spheres r in [3, 6], porosity
    U[0.35, 0.75]); potential U[4, 40] thermal voltages and inlet velocity
    U[1e-4, 5e-3] for both. Request k has geometry seed base_seed + k."""
    from .serving import Request, poisson_arrivals
    arrivals = poisson_arrivals(n, rate_hz, base_seed)
    rng = np.random.default_rng(base_seed + 1)
    out = []
    for k in range(n):
        is3d = bool(rng.integers(0, 2))
        dpsi = float(rng.uniform(4.0, 40.0))
        u_in = float(rng.uniform(1e-4, 5e-3))
        if is3d:
            edge = int(rng.integers(64, 193))
            phi = float(rng.uniform(0.35, 0.75))
            g = Geometry(dim=3, nx=edge, ny=edge, nz=edge, kind=L.SPHERES, porosity=phi, r_min=3.0,
                         r_max=6.0, buffer_x=2, seed=base_seed + k)
            nps = np_steps_3d
        else:
            phi = float(rng.uniform(0.55, 0.75))
            g = Geometry(dim=2, nx=256, ny=256, kind=L.DISKS, porosity=phi, r_min=4.0, r_max=8.0,
                         min_gap=2.0, walls_y=1, buffer_x=2, seed=base_seed + k)
            nps = np_steps_2d
        p = Params(u_in=u_in, dpsi_vt=dpsi, D=(D_NA, D_CL), precision=precision, streaming=streaming)
        out.append(Request(k, arrivals[k], g, p, flow_tol=flow_tol, flow_max_steps=flow_max_steps,
                           np_steps=nps))
    return out
