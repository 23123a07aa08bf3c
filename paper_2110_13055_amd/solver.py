"""Python binding of the C ABI: torch supplies device memory and the stream,
libcdi does all of the work.

    geom = Geometry(dim=3, nx=128, ny=128, nz=128, kind=SPHERES, porosity=0.5,
                    r_min=3, r_max=6, seed=2110)
    s = Solver(geom, Params(u_in=5e-4, dpsi_vt=20.0))
    s.flow_to_steady(1e-8)
    s.np_step(20000)
    print(s.adsorbed_total())
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

from . import _lib as L


@dataclass
class Geometry:
    dim: int
    nx: int
    ny: int
    nz: int = 1
    seed: int = 2110
    kind: int = L.DISKS
    porosity: float = 0.7
    r_min: float = 4.0
    r_max: float = 8.0
    min_gap: float = 2.0
    walls_y: int = 1
    buffer_x: int = 2
    user_labels: Optional[np.ndarray] = None

    @property
    def n_vox(self) -> int:
        return self.nx * self.ny * (1 if self.dim == 2 else self.nz)

    def to_c(self):
        g = L.CGeometry()
        g.dim, g.nx, g.ny, g.nz = self.dim, self.nx, self.ny, (1 if self.dim == 2 else self.nz)
        g.seed, g.kind = self.seed, self.kind
        g.porosity, g.r_min, g.r_max, g.min_gap = self.porosity, self.r_min, self.r_max, self.min_gap
        g.walls_y, g.buffer_x = self.walls_y, self.buffer_x
        keep = None
        if self.user_labels is not None:
            keep = np.ascontiguousarray(self.user_labels, dtype=np.uint8).reshape(-1)
            if keep.size != self.n_vox:
                raise ValueError("user_labels must hold nx*ny*nz labels")
            g.user_labels = keep.ctypes.data
        return g, keep


@dataclass
class Params:
    tau: float = 1.0
    drive: int = L.INLET_OUTLET
    equilibrium: int = L.EQ_QUADRATIC
    u_in: float = 1e-3
    rho_out: float = 1.0
    body_force: tuple = (0.0, 0.0, 0.0)
    D: tuple = (0.05, 0.076)
    z: tuple = (1, -1)
    c0: float = 1.0
    c_out: float = 0.0
    Ka: float = 0.0
    dpsi_vt: float = 0.0
    psi_field: object = None     # torch float32 CUDA tensor of N_f values, or None
    np_x_bc: int = L.NPX_INLET_OUTLET
    np_substeps: int = 1
    precision: int = L.FP32
    streaming: int = L.STREAM_AA
    no_adsorption: int = 0       # 1: K_a = 0 (a blocking electrode)

    def to_c(self):
        p = L.CParams()
        p.tau, p.drive, p.equilibrium = self.tau, self.drive, self.equilibrium
        p.u_in, p.rho_out = self.u_in, self.rho_out
        for a in range(3):
            p.body_force[a] = self.body_force[a]
        for s in range(2):
            p.D[s] = self.D[s]
            p.z[s] = self.z[s]
        p.c0, p.c_out, p.Ka, p.dpsi_vt = self.c0, self.c_out, self.Ka, self.dpsi_vt
        p.psi_field = None if self.psi_field is None else self.psi_field.data_ptr()
        p.np_x_bc, p.np_substeps, p.precision = self.np_x_bc, self.np_substeps, self.precision
        p.streaming = self.streaming
        p.no_adsorption = self.no_adsorption
        return p


def plan(geom: Geometry, params: Optional[Params] = None) -> L.CPlanInfo:
    lib = L.load()
    g, keep = geom.to_c()
    info = L.CPlanInfo()
    p = params.to_c() if params is not None else None
    L.check(lib.cdi_plan(C.byref(g), None if p is None else C.byref(p), C.byref(info)), "cdi_plan")
    return info


def bandwidth_probe(mode: int, dst, src=None, value: int = 0, stream=None) -> None:
    """One streaming kernel of known traffic (cdi_bandwidth_probe): PROBE_COPY
    dst <- src, PROBE_READ 16-byte word k of dst <- XOR of the 16-byte words of
    src's k-th 8 KiB block, PROBE_FILL dst <- value repeated. dst / src: CUDA tensors (the byte size
    of src for COPY and READ, of dst for FILL); stream: a torch stream or None
    (the current one). Asynchronous."""
    import torch
    lib = L.load()
    nbytes = (src if mode != L.PROBE_FILL else dst).numel() * (src if mode != L.PROBE_FILL else dst).element_size()
    st = stream if stream is not None else torch.cuda.current_stream()
    L.check(lib.cdi_bandwidth_probe(mode, dst.data_ptr(), None if src is None else src.data_ptr(), nbytes,
                                    value & 0xFFFFFFFF, st.cuda_stream), "cdi_bandwidth_probe")


def flow_check(geom: Geometry, params: Params, max_drho: float = 0.0):
    """Host-only admission check (cdi_flow_check): (ok, estimated steady
    density drop across the electrode, message)."""
    lib = L.load()
    g, keep = geom.to_c()
    p = params.to_c()
    est = C.c_double()
    rc = lib.cdi_flow_check(C.byref(g), C.byref(p), max_drho, C.byref(est))
    if rc not in (L.OK, L.E_UNSTABLE):
        L.check(rc, "cdi_flow_check")
    msg = lib.cdi_last_error().decode(errors="replace") if rc != L.OK else ""
    return rc == L.OK, est.value, msg


@dataclass
class Potential:
    """Settings of the potential solve (Poisson, Eq. 4-5; see cdi_potential in
    include/cdi.h). Values in thermal voltages, lattice units."""
    psi_electrode: float = 0.0
    x_bc: tuple = (L.PSIX_NEUMANN, L.PSIX_NEUMANN)
    psi_x: tuple = (0.0, 0.0)
    kappa2: float = 0.0
    tol: float = 1e-10
    max_iter: int = 100000
    check_every: int = 0
    warm_start: bool = True
    fp64: bool = False  # CG on FP64 vectors throughout instead of FP32 refinement rounds

    def to_c(self) -> L.CPotential:
        c = L.CPotential()
        c.psi_electrode = self.psi_electrode
        c.x_bc[0], c.x_bc[1] = self.x_bc
        c.psi_x[0], c.psi_x[1] = self.psi_x
        c.kappa2, c.tol, c.max_iter = self.kappa2, self.tol, self.max_iter
        c.check_every, c.warm_start = self.check_every, 1 if self.warm_start else 0
        c.fp64 = 1 if self.fp64 else 0
        return c


def _torch():
    import torch
    return torch


class Solver:
    """One electrode instance resident on a GPU. Device buffers are torch
    tensors owned by this object; the library only borrows them."""

    def __init__(self, geom: Geometry, params: Params, device: str = "cuda", stream=None):
        torch = _torch()
        self.lib = L.load()
        self.geom, self.params = geom, params
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self._sptr = C.c_void_p(self.stream.cuda_stream)
        self._g, self._keep = geom.to_c()
        self._p = params.to_c()
        self.info_plan = plan(geom, params)
        self.vox_ws = torch.empty(int(self.info_plan.vox_bytes), dtype=torch.uint8, device=self.device)
        nf = C.c_int64()
        with torch.cuda.device(self.device):
            L.check(self.lib.cdi_build_geometry(C.byref(self._g), C.c_void_p(self.vox_ws.data_ptr()),
                                                self.vox_ws.numel(), self._sptr, C.byref(nf)),
                    "cdi_build_geometry")
        self.n_fluid = nf.value
        nb = C.c_uint64()
        L.check(self.lib.cdi_node_bytes(C.byref(self._g), C.byref(self._p), self.n_fluid, C.byref(nb)),
                "cdi_node_bytes")
        self.node_ws = torch.empty(int(nb.value), dtype=torch.uint8, device=self.device)
        h = C.c_void_p()
        with torch.cuda.device(self.device):
            L.check(self.lib.cdi_flow_init(C.byref(self._g), C.byref(self._p),
                                           C.c_void_p(self.vox_ws.data_ptr()), self.vox_ws.numel(),
                                           C.c_void_p(self.node_ws.data_ptr()), self.node_ws.numel(),
                                           self.n_fluid, self._sptr, C.byref(h)), "cdi_flow_init")
        self.h = h
        self.dim = geom.dim

    # -------------------------------------------------------------- lifecycle
    def close(self):
        if getattr(self, "h", None):
            self.lib.cdi_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def footprint_bytes(self) -> int:
        return self.vox_ws.numel() + self.node_ws.numel()

    def info(self) -> L.CSolverInfo:
        out = L.CSolverInfo()
        L.check(self.lib.cdi_get_info(self.h, C.byref(out)), "cdi_get_info")
        return out

    # -------------------------------------------------------------- stepping
    def flow_steps(self, n: int):
        L.check(self.lib.cdi_flow_steps(self.h, n), "cdi_flow_steps")

    def flow_to_steady(self, tol: float = 1e-8, max_steps: int = 10 ** 6, check_every: int = 100,
                       raise_on_failure: bool = False):
        steps, res = C.c_int64(), C.c_double()
        rc = self.lib.cdi_flow_step_to_steady(self.h, tol, max_steps, check_every, C.byref(steps),
                                              C.byref(res))
        allow = (L.OK,) if raise_on_failure else (L.OK, L.STAGNATED, L.E_NOT_CONVERGED)
        L.check(rc, "cdi_flow_step_to_steady", allow)
        return rc, steps.value, res.value

    def np_step(self, n: int, fused: bool = False):
        L.check(self.lib.cdi_np_step(self.h, n, 1 if fused else 0), "cdi_np_step")

    # -------------------------------------------------------------- results
    def adsorbed_total(self) -> np.ndarray:
        out = (C.c_double * 2)()
        L.check(self.lib.cdi_adsorbed_total(self.h, out), "cdi_adsorbed_total")
        return np.array(out[:])

    def mass_balance(self) -> np.ndarray:
        out = (C.c_double * 8)()
        L.check(self.lib.cdi_mass_balance(self.h, out), "cdi_mass_balance")
        return np.array(out[:]).reshape(2, 4)

    def _get(self, fn, shape, dtype):
        a = np.empty(shape, dtype=dtype)
        L.check(getattr(self.lib, fn)(self.h, C.c_void_p(a.ctypes.data)), fn)
        return a

    def labels(self) -> np.ndarray:
        return self._get("cdi_copy_labels", (self.geom.n_vox,), np.uint8)

    def fluid_index(self):
        m = np.empty(self.geom.n_vox, dtype=np.int32)
        f = np.empty(self.n_fluid, dtype=np.int32)
        L.check(self.lib.cdi_copy_fluid_index(self.h, C.c_void_p(m.ctypes.data), C.c_void_p(f.ctypes.data)),
                "cdi_copy_fluid_index")
        return m, f

    def velocity(self) -> np.ndarray:
        return self._get("cdi_copy_velocity", (self.dim, self.n_fluid), np.float32)

    def density(self) -> np.ndarray:
        return self._get("cdi_copy_density", (self.n_fluid,), np.float32)

    def np_velocity(self) -> np.ndarray:
        return self._get("cdi_copy_np_velocity", (self.dim, self.n_fluid), np.float32)

    def concentration(self) -> np.ndarray:
        return self._get("cdi_copy_concentration", (2, self.n_fluid), np.float32)

    def set_np_velocity(self, j: np.ndarray):
        a = np.ascontiguousarray(j, dtype=np.float32).reshape(self.dim, self.n_fluid)
        L.check(self.lib.cdi_set_np_velocity(self.h, C.c_void_p(a.ctypes.data)), "cdi_set_np_velocity")

    def set_concentration(self, c: np.ndarray):
        a = np.ascontiguousarray(c, dtype=np.float32).reshape(2, self.n_fluid)
        L.check(self.lib.cdi_set_concentration(self.h, C.c_void_p(a.ctypes.data)), "cdi_set_concentration")

    # -------------------------------------------------------------- potential
    def _pot_ws(self):
        nb = C.c_uint64()
        L.check(self.lib.cdi_potential_bytes(self.h, C.byref(nb)), "cdi_potential_bytes")
        ws = getattr(self, "_pot_buf", None)
        if ws is None or ws.numel() < nb.value:
            self._pot_buf = ws = _torch().empty(int(nb.value), dtype=_torch().uint8, device=self.device)
        return ws

    def solve_potential(self, pot: "Potential", allow_not_converged: bool = False):
        """Solve Eq. (4)-(5) for the current concentrations; the result is the
        potential of later ion steps. Returns (iterations, relative residual);
        potential_stats holds those and the refinement counts."""
        ws = self._pot_ws()
        c, out = pot.to_c(), L.CPotentialResult()
        rc = self.lib.cdi_solve_potential(self.h, C.byref(c), C.c_void_p(ws.data_ptr()), ws.numel(),
                                          C.byref(out))
        self.potential_stats = dict(iterations=out.iterations, residual=out.residual,
                                    fp32_rounds=out.fp32_rounds, fp64_iterations=out.fp64_iterations)
        L.check(rc, "cdi_solve_potential", (L.OK, L.E_NOT_CONVERGED) if allow_not_converged else (L.OK,))
        return out.iterations, out.residual

    def solve_potential_noalloc(self, pot: "Potential", allow_not_converged: bool = False):
        """solve_potential without a workspace: the library's own scratch
        (cdi_solve_potential_noalloc; lattices up to its 64 MiB)."""
        c, out = pot.to_c(), L.CPotentialResult()
        rc = self.lib.cdi_solve_potential_noalloc(self.h, C.byref(c), C.byref(out))
        self.potential_stats = dict(iterations=out.iterations, residual=out.residual,
                                    fp32_rounds=out.fp32_rounds, fp64_iterations=out.fp64_iterations)
        L.check(rc, "cdi_solve_potential_noalloc", (L.OK, L.E_NOT_CONVERGED) if allow_not_converged else (L.OK,))
        return out.iterations, out.residual

    def np_step_coupled(self, n: int, pot: "Potential", every: int = 1, fused: bool = False):
        """n ion steps with the potential re-solved every `every` steps."""
        ws = self._pot_ws()
        c = pot.to_c()
        L.check(self.lib.cdi_np_step_coupled(self.h, n, 1 if fused else 0, C.byref(c), every,
                                             C.c_void_p(ws.data_ptr()), ws.numel()), "cdi_np_step_coupled")

    def potential(self) -> np.ndarray:
        return self._get("cdi_copy_potential", (self.n_fluid,), np.float32)

    # -------------------------------------------------------------- implicit ion transport
    def _nps_ws(self):
        nb = C.c_uint64()
        L.check(self.lib.cdi_np_solve_bytes(self.h, C.byref(nb)), "cdi_np_solve_bytes")
        ws = getattr(self, "_nps_buf", None)
        if ws is None or ws.numel() < nb.value:
            self._nps_buf = ws = _torch().empty(int(nb.value), dtype=_torch().uint8, device=self.device)
        return ws

    def np_steady(self, tol: float = 1e-10, max_iter: int = 100000, allow_not_converged: bool = False) -> int:
        """Steady concentrations on the frozen flow; returns the iterations."""
        ws = self._nps_ws()
        it = C.c_int32()
        rc = self.lib.cdi_np_steady(self.h, tol, max_iter, C.c_void_p(ws.data_ptr()), ws.numel(), C.byref(it))
        L.check(rc, "cdi_np_steady", (L.OK, L.E_NOT_CONVERGED) if allow_not_converged else (L.OK,))
        return it.value

    def np_implicit(self, dt: float, n: int, tol: float = 1e-10, max_iter: int = 100000) -> int:
        """n backward-Euler ion steps of length dt; returns the total iterations."""
        ws = self._nps_ws()
        it = C.c_int32()
        L.check(self.lib.cdi_np_implicit(self.h, dt, n, tol, max_iter, C.c_void_p(ws.data_ptr()), ws.numel(),
                                         C.byref(it)), "cdi_np_implicit")
        return it.value

    def np_rates(self) -> np.ndarray:
        """(2, 3): adsorption, inflow, outflow rate per species."""
        out = np.empty(6)
        L.check(self.lib.cdi_np_rates(self.h, C.c_void_p(out.ctypes.data)), "cdi_np_rates")
        return out.reshape(2, 3)

    # -------------------------------------------------------------- diagnostics (Sec. 4)
    def diagnostics(self) -> dict:
        d = L.CDiag()
        L.check(self.lib.cdi_diagnostics(self.h, C.byref(d)), "cdi_diagnostics")
        return {"n_surface": d.n_surface, "n_inlet": d.n_inlet, "specific_surface": d.specific_surface,
                "l_c": d.l_c, "U": d.U, "Pe": tuple(d.Pe), "Da": tuple(d.Da)}

    def profile_x(self) -> np.ndarray:
        """(3, nx): mean Na, mean Cl and fluid count of every x plane."""
        out = np.empty((3, self.geom.nx))
        L.check(self.lib.cdi_profile_x(self.h, C.c_void_p(out.ctypes.data)), "cdi_profile_x")
        return out

    def salt_removal(self, bal0, bal1, nsteps: int, n_inlet: int, U: float) -> np.ndarray:
        """[P_rm Na, P_rm Cl, P_rm salt, removed amount] over a window between
        two mass_balance() read-backs nsteps ion steps apart."""
        b0 = np.ascontiguousarray(bal0, dtype=np.float64).reshape(-1)
        b1 = np.ascontiguousarray(bal1, dtype=np.float64).reshape(-1)
        out = np.empty(4)
        L.check(self.lib.cdi_salt_removal(self.h, C.c_void_p(b0.ctypes.data), C.c_void_p(b1.ctypes.data),
                                          nsteps, n_inlet, U, C.c_void_p(out.ctypes.data)), "cdi_salt_removal")
        return out

    # -------------------------------------------------------------- tuning
    def tuning(self):
        t = L.CTuning()
        L.check(self.lib.cdi_get_tuning(self.h, C.byref(t)), "cdi_get_tuning")
        return (t.blocks_per_cu, t.band_rows, t.columns, t.nbr_list, t.stage_odd)

    def set_tuning(self, blocks_per_cu: int = 0, band_rows: int = 0, columns: int = 0, nbr_list: int = 0,
                   stage_odd: int = 0):
        t = L.CTuning(blocks_per_cu, band_rows, columns, nbr_list, stage_odd)
        L.check(self.lib.cdi_set_tuning(self.h, C.byref(t)), "cdi_set_tuning")

    def autotune(self, steps: int = 4, fused: bool = True):
        t, ms = L.CTuning(), C.c_double()
        L.check(self.lib.cdi_autotune(self.h, steps, 1 if fused else 0, C.byref(t), C.byref(ms)),
                "cdi_autotune")
        return (t.blocks_per_cu, t.band_rows, t.columns, t.nbr_list, t.stage_odd), ms.value

    def snapshot(self) -> bytes:
        nb = C.c_uint64()
        L.check(self.lib.cdi_snapshot_bytes(self.h, C.byref(nb)), "cdi_snapshot_bytes")
        buf = (C.c_uint8 * nb.value)()
        L.check(self.lib.cdi_snapshot(self.h, buf, nb.value), "cdi_snapshot")
        return bytes(buf)

    def restore(self, blob: bytes):
        buf = (C.c_uint8 * len(blob)).from_buffer_copy(blob)
        L.check(self.lib.cdi_restore(self.h, buf, len(blob)), "cdi_restore")

    def synchronize(self):
        self.stream.synchronize()


class Batch:
    """Independent solvers advanced together: one persistent launch per step
    for all members, step pairs replayed from a captured HIP graph. Each
    member's results equal those of advancing it alone."""

    def __init__(self, members=(), stream=None, capacity=None, device="cuda"):
        """members: the initial solvers. capacity (max_members, max_fluid):
        room to admit and retire members later without a new workspace
        (cdi_batch_create_empty + cdi_batch_admit); None: exactly the
        initial members (cdi_batch_create)."""
        torch = _torch()
        self.lib = L.load()
        self.members = list(members)
        n = len(self.members)
        if n == 0 and capacity is None:
            raise ValueError("empty batch without a capacity")
        dev = self.members[0].device if n else torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=dev)
        nb = C.c_uint64()
        h = C.c_void_p()
        if capacity is None:
            self._arr = (C.c_void_p * n)(*[s.h.value for s in self.members])
            L.check(self.lib.cdi_batch_bytes(self._arr, n, C.byref(nb)), "cdi_batch_bytes")
            self.ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=dev)
            L.check(self.lib.cdi_batch_create(self._arr, n, C.c_void_p(self.ws.data_ptr()), self.ws.numel(),
                                              C.c_void_p(self.stream.cuda_stream), C.byref(h)),
                    "cdi_batch_create")
            self.h = h
        else:
            cap_n, cap_fluid = int(capacity[0]), int(capacity[1])
            L.check(self.lib.cdi_batch_capacity_bytes(cap_n, cap_fluid, C.byref(nb)), "cdi_batch_capacity_bytes")
            self.ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=dev)
            L.check(self.lib.cdi_batch_create_empty(cap_n, cap_fluid, C.c_void_p(self.ws.data_ptr()),
                                                    self.ws.numel(), C.c_void_p(self.stream.cuda_stream),
                                                    C.byref(h)), "cdi_batch_create_empty")
            self.h = h
            members, self.members = self.members, []
            for s in members:
                self.admit(s)
        self.n = len(self.members)

    def admit(self, solver):
        """Add a member at the end (cdi_batch_admit); raises CdiError(BUFFER) when full."""
        L.check(self.lib.cdi_batch_admit(self.h, solver.h), "cdi_batch_admit")
        self.members.append(solver)
        self.n = len(self.members)

    def retire(self, solver):
        """Remove a member (cdi_batch_retire); later members move up one index."""
        L.check(self.lib.cdi_batch_retire(self.h, solver.h), "cdi_batch_retire")
        self.members = [m for m in self.members if m is not solver]
        self.n = len(self.members)

    def _modes(self, modes):
        if isinstance(modes, int):
            modes = [modes] * self.n
        a = (C.c_int32 * self.n)(*[int(m) for m in modes])
        return a

    def advance(self, nsteps: int, modes):
        L.check(self.lib.cdi_batch_advance(self.h, nsteps, self._modes(modes)), "cdi_batch_advance")

    def residuals(self) -> np.ndarray:
        r = np.empty(self.n)
        L.check(self.lib.cdi_batch_residuals(self.h, C.c_void_p(r.ctypes.data)), "cdi_batch_residuals")
        return r

    def set_launch(self, workgroups: int = 0, blocks_per_cu: int = 0):
        L.check(self.lib.cdi_batch_set_launch(self.h, workgroups, blocks_per_cu), "cdi_batch_set_launch")

    def launch(self):
        wg, occ = C.c_int32(), C.c_int32()
        L.check(self.lib.cdi_batch_get_launch(self.h, C.byref(wg), C.byref(occ)), "cdi_batch_get_launch")
        return wg.value, occ.value

    def autotune(self, steps: int, modes):
        wg, ms = C.c_int32(), C.c_double()
        L.check(self.lib.cdi_batch_autotune(self.h, steps, self._modes(modes), C.byref(wg), C.byref(ms)),
                "cdi_batch_autotune")
        return wg.value, ms.value

    def synchronize(self):
        self.stream.synchronize()

    def close(self):
        if getattr(self, "h", None):
            self.lib.cdi_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
