"""Pins of the CPU reference's diagnostics (Sec. 4): specific surface and
l_c = pi / s, the mean velocity U = sum u_i / (N phi), Pe = U l_c / D,
Da = K_a l_c / D, vertically averaged concentrations and the salt removal
P_rm = (C_in - C_out) / C_in.

Closed forms: face counts of plates and boxes (2(ab + bc + ca) for an a x b x
c block), l_c of a plate channel (pi ny / 2), U of a prescribed equilibrium
state, plane means of fields that depend on x only. Cross-check: at a steady
state with a uniform prescribed velocity and no migration the flux-weighted
outlet concentration behind P_rm equals the mean over the outlet plane.
"""
import math

import numpy as np
import pytest

from oracle import (OracleCfg, OracleSolver, DRIVE_BODY_FORCE, NPX_INLET_OUTLET)


def solver(lab, dim, nx, ny, nz=1, **kw):
    cfg = OracleCfg(dim=dim, nx=nx, ny=ny, nz=nz, **kw)
    return OracleSolver(cfg, np.ascontiguousarray(lab, np.uint8).reshape(-1))


def test_plate_channel_surface_and_lc():
    nx, ny = 30, 12
    lab = np.zeros((ny, nx), np.uint8)
    lab[0, :] = lab[-1, :] = 1
    d = solver(lab, 2, nx, ny).diagnostics()
    assert d["n_surface"] == 2 * nx
    assert d["n_inlet"] == ny - 2
    assert d["specific_surface"] == 2 * nx / (nx * ny)
    assert abs(d["l_c"] - math.pi * ny / 2) < 1e-12


@pytest.mark.parametrize("a,b,c", [(1, 1, 1), (3, 2, 4), (5, 5, 2)])
def test_block_surface_is_box_area(a, b, c):
    nx, ny, nz = 14, 12, 11
    lab = np.zeros((nz, ny, nx), np.uint8)
    lab[3:3 + c, 4:4 + b, 5:5 + a] = 1
    assert solver(lab, 3, nx, ny, nz).diagnostics()["n_surface"] == 2 * (a * b + b * c + c * a)


def test_surface_wraps_in_x_only_with_the_body_force_drive():
    nx, ny, nz = 10, 8, 8
    lab = np.zeros((nz, ny, nx), np.uint8)
    lab[2:4, 2:5, 0:2] = 1  # touches the x = 0 end
    a, b, c = 2, 3, 2
    closed = solver(lab, 3, nx, ny, nz).diagnostics()["n_surface"]
    periodic = solver(lab, 3, nx, ny, nz, drive=DRIVE_BODY_FORCE).diagnostics()["n_surface"]
    assert periodic == 2 * (a * b + b * c + c * a)
    assert closed == periodic - b * c  # the face towards x = -1 is not in the domain


def test_mean_velocity_pe_da_of_a_prescribed_state():
    nx, ny = 20, 10
    lab = np.zeros((ny, nx), np.uint8)
    lab[0, :] = lab[-1, :] = 1
    s = solver(lab, 2, nx, ny, D=(0.05, 0.08), Ka=0.01, u_in=1e-3)
    rng = np.random.default_rng(1)
    u = rng.uniform(-1e-3, 3e-3, size=(2, s.nf))
    s.init_equilibrium(None, u)
    d = s.diagnostics()
    U = u[0].mean()
    assert abs(d["U"] - U) < 1e-15
    lc = math.pi * ny / 2
    assert abs(d["Pe"][0] - U * lc / 0.05) < 1e-12 and abs(d["Pe"][1] - U * lc / 0.08) < 1e-12
    assert abs(d["Da"][0] - 0.01 * lc / 0.05) < 1e-12 and abs(d["Da"][1] - 0.01 * lc / 0.08) < 1e-12


def test_profile_of_fields_that_depend_on_x_only():
    nx, ny, nz = 16, 9, 7
    rng = np.random.default_rng(2)
    lab = (rng.random((nz, ny, nx)) < 0.3).astype(np.uint8)
    s = solver(lab, 3, nx, ny, nz)
    fl = np.flatnonzero(lab.reshape(-1) == 0)
    x = fl % nx
    s.set_conc(np.vstack([1.0 + 0.1 * x, 2.0 - 0.05 * x * x]))
    pr = s.profile_x()
    counts = (lab == 0).sum(axis=(0, 1))
    assert np.array_equal(pr[2], counts.astype(float))
    has = counts > 0
    xs = np.arange(nx)
    assert np.abs(pr[0][has] - (1.0 + 0.1 * xs[has])).max() < 1e-14
    assert np.abs(pr[1][has] - (2.0 - 0.05 * xs[has] ** 2)).max() < 1e-13


def test_salt_removal_is_the_outlet_plane_mean_at_steady_state():
    # plug flow along a plate channel with adsorbing plates, no potential:
    # at steady state the outflow per step is u * sum of C over the outlet plane
    nx, ny = 40, 6
    lab = np.zeros((ny, nx), np.uint8)
    lab[0, :] = lab[-1, :] = 1
    u = 2e-3
    s = solver(lab, 2, nx, ny, D=(0.05, 0.05), Ka=5e-4, u_in=u, np_x_bc=NPX_INLET_OUTLET)
    s.set_velocity(np.vstack([np.full(s.nf, u), np.zeros(s.nf)]))
    assert s.np_steps(60000) == 0
    b0 = s.balance().copy()
    n = 2000
    assert s.np_steps(n) == 0
    b1 = s.balance()
    d = s.diagnostics()
    prm = s.salt_removal(b0, b1, n, d["n_inlet"], u)
    outlet = s.profile_x()[:2, nx - 1]
    assert np.abs(prm[:2] - (1.0 - outlet)).max() < 1e-9
    assert 0.05 < prm[2] < 0.95
    assert abs(prm[3] - u * ny * prm[2] * n / s.nf) < 1e-15


def test_no_adsorption_removes_nothing():
    nx, ny = 30, 6
    lab = np.zeros((ny, nx), np.uint8)
    lab[0, :] = lab[-1, :] = 1
    u = 2e-3
    s = solver(lab, 2, nx, ny, D=(0.05, 0.05), no_adsorption=1, u_in=u)
    s.set_velocity(np.vstack([np.full(s.nf, u), np.zeros(s.nf)]))
    b0 = s.balance().copy()
    assert s.np_steps(500) == 0
    prm = s.salt_removal(b0, s.balance(), 500, s.diagnostics()["n_inlet"], u)
    assert np.abs(prm[:3]).max() < 1e-12  # saturated channel: everything that enters leaves
