"""ctypes declarations of libcdi.so (the C ABI of include/cdi.h).

Argument marshalling only: every step of the model runs in the library's HIP
kernels. Loading fails loudly if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcdi.so")

OK, STAGNATED = 0, 1
E_INVALID, E_GEOMETRY, E_UNSTABLE, E_NOT_CONVERGED, E_DIVERGED, E_DEVICE, E_BUFFER = -1, -2, -3, -4, -5, -6, -7
DISKS, SPHERES, USER_LABELS, FIBRES = 0, 1, 2, 3
INLET_OUTLET, BODY_FORCE = 0, 1
EQ_QUADRATIC, EQ_LINEAR = 0, 1
NPX_INLET_OUTLET, NPX_PERIODIC, NPX_CLOSED, NPX_DIRICHLET = 0, 1, 2, 3
FP32, FP16_DEV, MOMENTS, FP16 = 0, 1, 2, 3
STREAM_AA, STREAM_PULL = 0, 1
MODE_IDLE, MODE_FLOW, MODE_IONS, MODE_FUSED = 0, 1, 2, 3
PSIX_DIRICHLET, PSIX_NEUMANN, PSIX_PERIODIC = 0, 1, 2
PROBE_COPY, PROBE_READ, PROBE_FILL = 0, 1, 2

STATUS_NAMES = {
    0: "OK", 1: "STAGNATED", -1: "INVALID", -2: "GEOMETRY", -3: "UNSTABLE", -4: "NOT_CONVERGED",
    -5: "DIVERGED", -6: "DEVICE", -7: "BUFFER",
}


class CGeometry(C.Structure):
    _fields_ = [
        ("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("seed", C.c_uint64), ("kind", C.c_int32),
        ("porosity", C.c_double), ("r_min", C.c_double), ("r_max", C.c_double), ("min_gap", C.c_double),
        ("walls_y", C.c_int32), ("buffer_x", C.c_int32),
        ("user_labels", C.c_void_p),
    ]


class CParams(C.Structure):
    _fields_ = [
        ("tau", C.c_double), ("drive", C.c_int32), ("equilibrium", C.c_int32),
        ("u_in", C.c_double), ("rho_out", C.c_double), ("body_force", C.c_double * 3),
        ("D", C.c_double * 2), ("z", C.c_int32 * 2),
        ("c0", C.c_double), ("c_out", C.c_double), ("Ka", C.c_double), ("dpsi_vt", C.c_double),
        ("psi_field", C.c_void_p),
        ("np_x_bc", C.c_int32), ("np_substeps", C.c_int32), ("precision", C.c_int32),
        ("streaming", C.c_int32), ("no_adsorption", C.c_int32),
    ]


class CPlanInfo(C.Structure):
    _fields_ = [
        ("n_vox", C.c_int64), ("n_prims", C.c_int64), ("n_fluid_est", C.c_int64),
        ("vox_bytes", C.c_uint64), ("node_bytes_per_fluid", C.c_uint64),
    ]


class CSolverInfo(C.Structure):
    _fields_ = [
        ("n_vox", C.c_int64), ("n_fluid", C.c_int64),
        ("dim", C.c_int32), ("q", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("precision", C.c_int32),
        ("flow_steps", C.c_int64), ("np_steps", C.c_int64),
        ("ka", C.c_double), ("keff", C.c_double * 2), ("porosity", C.c_double),
    ]


class CTuning(C.Structure):
    _fields_ = [("blocks_per_cu", C.c_int32), ("band_rows", C.c_int32), ("columns", C.c_int32),
                ("nbr_list", C.c_int32), ("stage_odd", C.c_int32)]


class CPotential(C.Structure):
    _fields_ = [("psi_electrode", C.c_double), ("x_bc", C.c_int32 * 2), ("psi_x", C.c_double * 2),
                ("kappa2", C.c_double), ("tol", C.c_double), ("max_iter", C.c_int32),
                ("check_every", C.c_int32), ("warm_start", C.c_int32),
                ("fp64", C.c_int32)]


class CPotentialResult(C.Structure):
    _fields_ = [("iterations", C.c_int32), ("residual", C.c_double), ("fp32_rounds", C.c_int32),
                ("fp64_iterations", C.c_int32)]


class CDiag(C.Structure):
    _fields_ = [("n_surface", C.c_int64), ("n_inlet", C.c_int64), ("specific_surface", C.c_double),
                ("l_c", C.c_double), ("U", C.c_double), ("Pe", C.c_double * 2), ("Da", C.c_double * 2)]


P, I32, I64, U64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint64, C.c_double

# name -> (restype, argtypes); the list of symbols include/cdi.h declares
SIGNATURES = {
    "cdi_plan": (C.c_int, [P, P, P]),
    "cdi_flow_check": (C.c_int, [P, P, D, P]),
    "cdi_build_geometry": (C.c_int, [P, P, U64, P, P]),
    "cdi_node_bytes": (C.c_int, [P, P, I64, P]),
    "cdi_flow_init": (C.c_int, [P, P, P, U64, P, U64, I64, P, P]),
    "cdi_destroy": (C.c_int, [P]),
    "cdi_get_info": (C.c_int, [P, P]),
    "cdi_flow_steps": (C.c_int, [P, I64]),
    "cdi_flow_step_to_steady": (C.c_int, [P, D, I64, I32, P, P]),
    "cdi_np_step": (C.c_int, [P, I64, I32]),
    "cdi_adsorbed_total": (C.c_int, [P, P]),
    "cdi_mass_balance": (C.c_int, [P, P]),
    "cdi_copy_labels": (C.c_int, [P, P]),
    "cdi_copy_fluid_index": (C.c_int, [P, P, P]),
    "cdi_copy_velocity": (C.c_int, [P, P]),
    "cdi_copy_density": (C.c_int, [P, P]),
    "cdi_copy_np_velocity": (C.c_int, [P, P]),
    "cdi_set_np_velocity": (C.c_int, [P, P]),
    "cdi_copy_concentration": (C.c_int, [P, P]),
    "cdi_set_concentration": (C.c_int, [P, P]),
    "cdi_set_tuning": (C.c_int, [P, P]),
    "cdi_get_tuning": (C.c_int, [P, P]),
    "cdi_autotune": (C.c_int, [P, I32, I32, P, P]),
    "cdi_batch_bytes": (C.c_int, [P, I32, P]),
    "cdi_batch_create": (C.c_int, [P, I32, P, U64, P, P]),
    "cdi_batch_destroy": (C.c_int, [P]),
    "cdi_batch_capacity_bytes": (C.c_int, [I32, I64, P]),
    "cdi_batch_create_empty": (C.c_int, [I32, I64, P, U64, P, P]),
    "cdi_batch_admit": (C.c_int, [P, P]),
    "cdi_batch_retire": (C.c_int, [P, P]),
    "cdi_batch_members": (C.c_int, [P, P]),
    "cdi_batch_advance": (C.c_int, [P, I64, P]),
    "cdi_batch_residuals": (C.c_int, [P, P]),
    "cdi_batch_set_launch": (C.c_int, [P, I32, I32]),
    "cdi_batch_get_launch": (C.c_int, [P, P, P]),
    "cdi_batch_autotune": (C.c_int, [P, I32, P, P, P]),
    "cdi_potential_bytes": (C.c_int, [P, P]),
    "cdi_solve_potential": (C.c_int, [P, P, P, U64, P]),
    "cdi_solve_potential_noalloc": (C.c_int, [P, P, P]),
    "cdi_np_step_coupled": (C.c_int, [P, I64, I32, P, I32, P, U64]),
    "cdi_copy_potential": (C.c_int, [P, P]),
    "cdi_np_solve_bytes": (C.c_int, [P, P]),
    "cdi_np_steady": (C.c_int, [P, D, I32, P, U64, P]),
    "cdi_np_implicit": (C.c_int, [P, D, I64, D, I32, P, U64, P]),
    "cdi_np_rates": (C.c_int, [P, P]),
    "cdi_diagnostics": (C.c_int, [P, P]),
    "cdi_profile_x": (C.c_int, [P, P]),
    "cdi_salt_removal": (C.c_int, [P, P, P, I64, I64, D, P]),
    "cdi_snapshot_bytes": (C.c_int, [P, P]),
    "cdi_snapshot": (C.c_int, [P, P, U64]),
    "cdi_restore": (C.c_int, [P, P, U64]),
    "cdi_bandwidth_probe": (C.c_int, [I32, P, P, U64, C.c_uint32, P]),
    "cdi_last_error": (C.c_char_p, []),
    "cdi_struct_size": (C.c_int, [C.c_char_p, P]),
}

# the public structs and their ctypes mirrors (layouts checked at load)
STRUCTS = {"cdi_geometry": CGeometry, "cdi_params": CParams, "cdi_plan_info": CPlanInfo,
           "cdi_solver_info": CSolverInfo, "cdi_tuning": CTuning, "cdi_potential": CPotential,
           "cdi_potential_result": CPotentialResult, "cdi_diag": CDiag}

_lib = None


class CdiError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        self.code = code
        super().__init__(f"{where}: {STATUS_NAMES.get(code, code)} ({msg})")


def load():
    """Load libcdi.so; raises if it has not been built (no fallback path)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -m paper_2110_13055_amd.build`")
        # torch first: its HIP runtime must be the one the library binds to
        # (loaded before torch, the library would bind the system runtime and
        # share no device state, pointers or streams with torch's)
        import torch  # noqa: F401
        lib = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        for cname, cls in STRUCTS.items():  # a stale build with another layout fails here, not in a kernel
            n = C.c_uint64()
            if lib.cdi_struct_size(cname.encode(), C.byref(n)) != OK or n.value != C.sizeof(cls):
                raise RuntimeError(f"{LIB_PATH}: {cname} is {n.value} bytes in the library, {C.sizeof(cls)} in "
                                   "the binding: rebuild with `python -m paper_2110_13055_amd.build`")
        _lib = lib
    return _lib


def check(rc: int, where: str, allow=(OK,)) -> int:
    if rc in allow:
        return rc
    msg = load().cdi_last_error().decode(errors="replace")
    raise CdiError(rc, where, msg)
