"""ctypes binding of liboracle.so (FP64 CPU reference; test infrastructure only).

The binding marshals arguments and nothing else: every number comes from the
C code in ``cdi_oracle.c``.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
# ORACLE_LIB names another build of the same source (the sanitizer build)
_LIB_PATH = os.environ.get("ORACLE_LIB") or os.path.join(_HERE, "liboracle.so")

DRIVE_INLET_OUTLET, DRIVE_BODY_FORCE = 0, 1
EQ_QUADRATIC, EQ_LINEAR = 0, 1
NPX_INLET_OUTLET, NPX_PERIODIC, NPX_CLOSED, NPX_DIRICHLET = 0, 1, 2, 3

OK, E_INVALID, E_UNSTABLE, E_NOT_CONVERGED, E_DIVERGED = 0, -1, -3, -4, -5
PSIX_DIRICHLET, PSIX_NEUMANN, PSIX_PERIODIC = 0, 1, 2


def build() -> str:
    """Compile liboracle.so (gcc, FP64, OpenMP)."""
    subprocess.run(["sh", os.path.join(_HERE, "build.sh")], check=True)
    return _LIB_PATH


class _Cfg(C.Structure):
    _fields_ = [
        ("dim", C.c_int), ("nx", C.c_int), ("ny", C.c_int), ("nz", C.c_int),
        ("drive", C.c_int), ("equilibrium", C.c_int),
        ("tau", C.c_double), ("u_in", C.c_double), ("rho_out", C.c_double),
        ("force", C.c_double * 3),
        ("D", C.c_double * 2), ("z", C.c_int * 2),
        ("c0", C.c_double), ("c_out", C.c_double), ("Ka", C.c_double), ("dpsi", C.c_double),
        ("np_x_bc", C.c_int), ("np_substeps", C.c_int), ("no_adsorption", C.c_int),
    ]


class _Potential(C.Structure):
    _fields_ = [("psi_electrode", C.c_double), ("x_bc", C.c_int * 2), ("psi_x", C.c_double * 2),
                ("kappa2", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int)]


class _Diag(C.Structure):
    _fields_ = [("n_surface", C.c_int64), ("n_inlet", C.c_int64), ("specific_surface", C.c_double),
                ("l_c", C.c_double), ("U", C.c_double), ("Pe", C.c_double * 2), ("Da", C.c_double * 2)]


class _Prim(C.Structure):
    _fields_ = [("r", C.c_int64), ("cx", C.c_int64), ("cy", C.c_int64), ("cz", C.c_int64)]


_lib = None


def library():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = C.CDLL(_LIB_PATH)
        P, I64, D, I = C.c_void_p, C.c_int64, C.c_double, C.c_int
        sig = {
            "oracle_voxelize": (I, [I, I, I, I, I, I, P, I64, P]),
            "oracle_compact": (I64, [P, I64, P, P]),
            "oracle_create": (P, [P, P, P]),
            "oracle_destroy": (None, [P]),
            "oracle_num_fluid": (I64, [P]),
            "oracle_ka": (D, [P]),
            "oracle_flow_steps": (None, [P, I64]),
            "oracle_flow_to_steady": (I, [P, D, I64, I, P, P]),
            "oracle_get_velocity": (None, [P, P]),
            "oracle_get_density": (None, [P, P]),
            "oracle_get_populations": (None, [P, P]),
            "oracle_freeze_velocity": (None, [P]),
            "oracle_init_equilibrium": (None, [P, P, P]),
            "oracle_set_velocity": (None, [P, P]),
            "oracle_get_np_velocity": (None, [P, P]),
            "oracle_np_steps": (I, [P, I64, I]),
            "oracle_np_stability": (D, [P]),
            "oracle_get_conc": (None, [P, P]),
            "oracle_set_conc": (None, [P, P]),
            "oracle_balance": (None, [P, P]),
            "oracle_adsorbed_total": (None, [P, P]),
            "oracle_flow_step_count": (I64, [P]),
            "oracle_np_step_count": (I64, [P]),
            "oracle_threads": (I, []),
            "oracle_set_threads": (None, [I]),
            "oracle_solve_potential": (I, [P, P, P, P]),
            "oracle_get_potential": (None, [P, P]),
            "oracle_np_steps_coupled": (I, [P, I64, I, P, I]),
            "oracle_diagnostics": (None, [P, P]),
            "oracle_profile_x": (None, [P, P]),
            "oracle_salt_removal": (None, [P, P, P, I64, I64, D, P]),
            "oracle_np_steady": (I, [P, D, I, P]),
            "oracle_np_implicit": (I, [P, D, I64, D, I, P]),
            "oracle_np_rates": (None, [P, P]),
            "geomgen_disks": (I, [I, I, I, I, C.c_uint64, D, D, D, D, P, P, P]),
            "geomgen_spheres": (I, [I, I, I, I, C.c_uint64, D, D, D, P, P]),
            "geomgen_sphere_count": (I64, [I, I, I, I, D, D, D]),
            "geomgen_free": (None, [P]),
            "geomgen_fibres": (I, [I, I, I, I, C.c_uint64, D, D, D, P, P]),
            "oracle_voxelize_fibres": (I, [I, I, I, I, P, I64, P]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


# ---------------------------------------------------------------- geometry

def _prims_to_array(pp, n) -> np.ndarray:
    if n == 0:
        return np.zeros((0, 4), dtype=np.int64)
    buf = (C.c_int64 * (4 * n)).from_address(pp.value)
    return np.frombuffer(buf, dtype=np.int64).reshape(n, 4).copy()


def disks(nx, ny, buffer_x, walls_y, seed, porosity, r_min, r_max, min_gap):
    """Seeded RSA disks -> (prims int64[n,4], n_fluid)."""
    lib = library()
    pp, n, nf = C.c_void_p(), C.c_int64(), C.c_int64()
    rc = lib.geomgen_disks(nx, ny, buffer_x, walls_y, seed, porosity, r_min, r_max, min_gap,
                           C.byref(pp), C.byref(n), C.byref(nf))
    if rc != 0:
        raise RuntimeError(f"geomgen_disks failed rc={rc}")
    arr = _prims_to_array(pp, n.value)
    lib.geomgen_free(pp)
    return arr, nf.value


def spheres(nx, ny, nz, buffer_x, seed, porosity, r_min, r_max):
    """Seeded Boolean-model spheres -> prims int64[n,4]."""
    lib = library()
    pp, n = C.c_void_p(), C.c_int64()
    rc = lib.geomgen_spheres(nx, ny, nz, buffer_x, seed, porosity, r_min, r_max,
                             C.byref(pp), C.byref(n))
    if rc != 0:
        raise RuntimeError(f"geomgen_spheres failed rc={rc}")
    arr = _prims_to_array(pp, n.value)
    lib.geomgen_free(pp)
    return arr


def sphere_count(nx, ny, nz, buffer_x, porosity, r_min, r_max) -> int:
    return int(library().geomgen_sphere_count(nx, ny, nz, buffer_x, porosity, r_min, r_max))


def fibres(nx, ny, nz, buffer_x, seed, porosity, r_min, r_max):
    """Seeded straight fibres -> int64[n, 8] (r, ox, oy, oz, dx, dy, dz, 0)."""
    lib = library()
    pp, n = C.c_void_p(), C.c_int64()
    rc = lib.geomgen_fibres(nx, ny, nz, buffer_x, seed, porosity, r_min, r_max, C.byref(pp), C.byref(n))
    if rc != 0:
        raise RuntimeError(f"geomgen_fibres failed rc={rc}")
    buf = (C.c_int64 * (8 * n.value)).from_address(pp.value)
    arr = np.frombuffer(buf, dtype=np.int64).reshape(n.value, 8).copy()
    lib.geomgen_free(pp)
    return arr


def voxelize_fibres(nx, ny, nz, buffer_x, fib) -> np.ndarray:
    fib = np.ascontiguousarray(fib, dtype=np.int64).reshape(-1, 8)
    labels = np.zeros(nx * ny * nz, dtype=np.uint8)
    rc = library().oracle_voxelize_fibres(nx, ny, nz, buffer_x, _ptr(fib), fib.shape[0], _ptr(labels))
    if rc != 0:
        raise RuntimeError("oracle_voxelize_fibres failed")
    return labels


def voxelize(dim, nx, ny, nz, walls_y, buffer_x, prims) -> np.ndarray:
    prims = np.ascontiguousarray(prims, dtype=np.int64).reshape(-1, 4)
    nz_ = 1 if dim == 2 else nz
    labels = np.zeros(nx * ny * nz_, dtype=np.uint8)
    rc = library().oracle_voxelize(dim, nx, ny, nz_, walls_y, buffer_x, _ptr(prims),
                                   prims.shape[0], _ptr(labels))
    if rc != 0:
        raise RuntimeError("oracle_voxelize failed")
    return labels


def compact(labels: np.ndarray):
    labels = np.ascontiguousarray(labels, dtype=np.uint8)
    m = np.empty(labels.size, dtype=np.int32)
    f = np.empty(labels.size, dtype=np.int32)
    n = library().oracle_compact(_ptr(labels), labels.size, _ptr(m), _ptr(f))
    return m, f[:n].copy()


# ---------------------------------------------------------------- solver

@dataclass
class OracleCfg:
    dim: int
    nx: int
    ny: int
    nz: int = 1
    drive: int = DRIVE_INLET_OUTLET
    equilibrium: int = EQ_QUADRATIC
    tau: float = 1.0
    u_in: float = 1e-3
    rho_out: float = 1.0
    force: tuple = (0.0, 0.0, 0.0)
    D: tuple = (0.05, 0.076)
    z: tuple = (1, -1)
    c0: float = 1.0
    c_out: float = 0.0
    Ka: float = 0.0
    dpsi: float = 0.0
    np_x_bc: int = NPX_INLET_OUTLET
    np_substeps: int = 1
    no_adsorption: int = 0

    def to_c(self) -> _Cfg:
        c = _Cfg()
        c.dim, c.nx, c.ny, c.nz = self.dim, self.nx, self.ny, (1 if self.dim == 2 else self.nz)
        c.drive, c.equilibrium = self.drive, self.equilibrium
        c.tau, c.u_in, c.rho_out = self.tau, self.u_in, self.rho_out
        for a in range(3):
            c.force[a] = self.force[a]
        for s in range(2):
            c.D[s] = self.D[s]
            c.z[s] = self.z[s]
        c.c0, c.c_out, c.Ka, c.dpsi = self.c0, self.c_out, self.Ka, self.dpsi
        c.np_x_bc, c.np_substeps = self.np_x_bc, self.np_substeps
        c.no_adsorption = self.no_adsorption
        return c


class OracleSolver:
    """FP64 reference solver on one labelled voxel grid."""

    def __init__(self, cfg: OracleCfg, labels: np.ndarray, psi=None):
        self.lib = library()
        self.cfg = cfg
        self._c = cfg.to_c()
        self.labels = np.ascontiguousarray(labels, dtype=np.uint8)
        self._psi = None if psi is None else np.ascontiguousarray(psi, dtype=np.float64)
        self.h = self.lib.oracle_create(C.byref(self._c), _ptr(self.labels),
                                        None if self._psi is None else _ptr(self._psi))
        if not self.h:
            raise RuntimeError("oracle_create failed (invalid configuration)")
        self.nf = int(self.lib.oracle_num_fluid(self.h))
        self.Q = 9 if cfg.dim == 2 else 19

    def __del__(self):
        h = getattr(self, "h", None)
        if h:
            self.lib.oracle_destroy(h)
            self.h = None

    @property
    def ka(self) -> float:
        return float(self.lib.oracle_ka(self.h))

    def flow_steps(self, n: int):
        self.lib.oracle_flow_steps(self.h, n)

    def flow_to_steady(self, tol=1e-8, max_steps=10**6, check_every=100):
        steps, res = C.c_int64(), C.c_double()
        rc = self.lib.oracle_flow_to_steady(self.h, tol, max_steps, check_every,
                                            C.byref(steps), C.byref(res))
        return rc, steps.value, res.value

    def velocity(self) -> np.ndarray:
        u = np.empty((self.cfg.dim, self.nf))
        self.lib.oracle_get_velocity(self.h, _ptr(u))
        return u

    def density(self) -> np.ndarray:
        r = np.empty(self.nf)
        self.lib.oracle_get_density(self.h, _ptr(r))
        return r

    def populations(self) -> np.ndarray:
        f = np.empty((self.Q, self.nf))
        self.lib.oracle_get_populations(self.h, _ptr(f))
        return f

    def init_equilibrium(self, rho=None, u=None):
        r = None if rho is None else np.ascontiguousarray(rho, dtype=np.float64)
        uu = None if u is None else np.ascontiguousarray(u, dtype=np.float64).reshape(self.cfg.dim, self.nf)
        self.lib.oracle_init_equilibrium(self.h, None if r is None else _ptr(r),
                                         None if uu is None else _ptr(uu))

    def freeze_velocity(self):
        self.lib.oracle_freeze_velocity(self.h)

    def set_velocity(self, u: np.ndarray):
        u = np.ascontiguousarray(u, dtype=np.float64).reshape(self.cfg.dim, self.nf)
        self.lib.oracle_set_velocity(self.h, _ptr(u))

    def np_velocity(self) -> np.ndarray:
        u = np.empty((self.cfg.dim, self.nf))
        self.lib.oracle_get_np_velocity(self.h, _ptr(u))
        return u

    def np_steps(self, n: int, fused: bool = False) -> int:
        return int(self.lib.oracle_np_steps(self.h, n, 1 if fused else 0))

    def np_stability(self) -> float:
        return float(self.lib.oracle_np_stability(self.h))

    def conc(self) -> np.ndarray:
        c = np.empty((2, self.nf))
        self.lib.oracle_get_conc(self.h, _ptr(c))
        return c

    def set_conc(self, c: np.ndarray):
        c = np.ascontiguousarray(c, dtype=np.float64).reshape(2, self.nf)
        self.lib.oracle_set_conc(self.h, _ptr(c))

    def balance(self) -> np.ndarray:
        """[species, (M, A, In, Out)]"""
        b = np.empty(8)
        self.lib.oracle_balance(self.h, _ptr(b))
        return b.reshape(2, 4)

    def adsorbed_total(self) -> np.ndarray:
        a = np.empty(2)
        self.lib.oracle_adsorbed_total(self.h, _ptr(a))
        return a

    def solve_potential(self, psi_electrode=0.0, x_bc=(PSIX_NEUMANN, PSIX_NEUMANN), psi_x=(0.0, 0.0),
                        kappa2=0.0, tol=1e-13, max_iter=100000):
        """Poisson solve of Eq. (4)-(5) for the current concentrations; the
        result becomes the potential of later ion steps. Returns (rc, iters,
        relative residual)."""
        pc = _Potential()
        pc.psi_electrode = psi_electrode
        pc.x_bc[0], pc.x_bc[1] = x_bc
        pc.psi_x[0], pc.psi_x[1] = psi_x
        pc.kappa2, pc.tol, pc.max_iter = kappa2, tol, max_iter
        it, rel = C.c_int(), C.c_double()
        rc = self.lib.oracle_solve_potential(self.h, C.byref(pc), C.byref(it), C.byref(rel))
        return rc, it.value, rel.value

    def np_steps_coupled(self, n: int, every: int = 1, fused: bool = False, psi_electrode=0.0,
                         x_bc=(PSIX_NEUMANN, PSIX_NEUMANN), psi_x=(0.0, 0.0), kappa2=0.0, tol=1e-13,
                         max_iter=100000) -> int:
        """n ion steps with the potential re-solved every `every` steps."""
        pc = _Potential()
        pc.psi_electrode = psi_electrode
        pc.x_bc[0], pc.x_bc[1] = x_bc
        pc.psi_x[0], pc.psi_x[1] = psi_x
        pc.kappa2, pc.tol, pc.max_iter = kappa2, tol, max_iter
        return int(self.lib.oracle_np_steps_coupled(self.h, n, int(fused), C.byref(pc), every))

    def diagnostics(self) -> dict:
        d = _Diag()
        self.lib.oracle_diagnostics(self.h, C.byref(d))
        return {"n_surface": d.n_surface, "n_inlet": d.n_inlet, "specific_surface": d.specific_surface,
                "l_c": d.l_c, "U": d.U, "Pe": tuple(d.Pe), "Da": tuple(d.Da)}

    def profile_x(self) -> np.ndarray:
        out = np.empty((3, self.cfg.nx))
        self.lib.oracle_profile_x(self.h, _ptr(out))
        return out

    def salt_removal(self, bal0, bal1, nsteps: int, n_inlet: int, U: float) -> np.ndarray:
        b0 = np.ascontiguousarray(bal0, dtype=np.float64).reshape(-1)
        b1 = np.ascontiguousarray(bal1, dtype=np.float64).reshape(-1)
        out = np.empty(4)
        self.lib.oracle_salt_removal(self.h, _ptr(b0), _ptr(b1), nsteps, n_inlet, U, _ptr(out))
        return out

    def np_steady(self, tol=1e-12, max_iter=100000):
        it = C.c_int()
        rc = self.lib.oracle_np_steady(self.h, tol, max_iter, C.byref(it))
        return rc, it.value

    def np_implicit(self, dt: float, n: int, tol=1e-12, max_iter=100000):
        it = C.c_int()
        rc = self.lib.oracle_np_implicit(self.h, dt, n, tol, max_iter, C.byref(it))
        return rc, it.value

    def np_rates(self) -> np.ndarray:
        out = np.empty(6)
        self.lib.oracle_np_rates(self.h, _ptr(out))
        return out.reshape(2, 3)

    def potential(self) -> np.ndarray:
        p = np.empty(self.nf)
        self.lib.oracle_get_potential(self.h, _ptr(p))
        return p

    @property
    def flow_step_count(self) -> int:
        return int(self.lib.oracle_flow_step_count(self.h))

    @property
    def np_step_count(self) -> int:
        return int(self.lib.oracle_np_step_count(self.h))


def threads() -> int:
    return int(library().oracle_threads())


def set_threads(n: int) -> None:
    """Threads of the following OpenMP loops (results do not depend on it)."""
    library().oracle_set_threads(int(n))
