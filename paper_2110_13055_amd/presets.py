"""Named synthetic workloads (seeded), shaped like the paper's electrodes.

The paper's own geometries (a digitised SEM image, Sec. 4; random fibres,
Sec. 5) are not available, so each workload is a seeded synthetic electrode
with the porosity range and grain sizes of the paper's cases, in lattice
units. Diffusivities keep the paper's equal-D statement only as a ratio
(D_Cl / D_Na = 1.52); the default adsorption constant follows the paper's
Da / Pe ratio at its base case (Sec. 4.1).
"""
from __future__ import annotations

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
