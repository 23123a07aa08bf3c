"""Pins of the CPU reference's Nernst-Planck update (Eq. 3) with adsorption (Eq. 6).

Closed forms: 1D advection-diffusion between two Dirichlet ghosts, the
Boltzmann distribution of Eq. (9) in a closed box and on the Gouy-Chapman
potential of Eq. (10) with the constants of the paper's half-channel
validation (Sec. 3), the 1D diffusion-adsorption flux. Invariants: exact
conservation of solute plus adsorbed plus outflow minus inflow, positivity,
steady state of the explicit march = direct sparse solve (the implicit
scheme's steady state), and the exact discrete transient of the periodic
scheme from its Fourier amplification factor.
"""
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
from oracle import (OracleCfg, OracleSolver, NPX_CLOSED, NPX_DIRICHLET, NPX_INLET_OUTLET,
                    NPX_PERIODIC, DRIVE_INLET_OUTLET)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def bern(x):
    x = np.asarray(x, dtype=np.float64)
    out = np.ones_like(x)
    nz = x != 0
    out[nz] = x[nz] / np.expm1(x[nz])
    return out


def _line(n):
    return np.zeros(n, np.uint8)


def test_advection_diffusion_between_dirichlet_ghosts():
    # Ghost centres at xi = 0 (C = 1) and xi = L+1 (C = 0), uniform drift w:
    # C(xi) = (exp(Pe xi / Lt) - exp(Pe)) / (1 - exp(Pe)), Pe = w Lt / D.
    L, D, w = 20, 0.1, 0.05
    cfg = OracleCfg(dim=2, nx=L, ny=1, D=(D, D), u_in=w, c0=1.0, c_out=0.0, np_x_bc=NPX_DIRICHLET)
    s = OracleSolver(cfg, _line(L))
    s.set_velocity(np.vstack([np.full(L, w), np.zeros(L)]))
    assert s.np_steps(20000) == 0
    Lt = L + 1
    Pe = w * Lt / D
    xi = np.arange(L) + 1.0
    exact = (np.exp(Pe * xi / Lt) - np.exp(Pe)) / (1 - np.exp(Pe))
    c = s.conc()
    assert np.abs(c[0] - exact).max() < 1e-12
    assert np.abs(c[1] - exact).max() < 1e-12


def test_boltzmann_equilibrium_in_closed_box():
    # Zero-flux box, no flow, linear potential: steady C ~ exp(-z psi) (Eq. 9).
    L = 16
    cfg = OracleCfg(dim=2, nx=L, ny=1, D=(0.05, 0.076), u_in=0.0, dpsi=3.0, np_x_bc=NPX_CLOSED)
    s = OracleSolver(cfg, _line(L))
    s.set_velocity(np.zeros((2, L)))
    assert s.np_steps(40000) == 0
    psi = 3.0 * (1 - (np.arange(L) + 0.5) / L)
    c = s.conc()
    for sp_, z in ((0, 1), (1, -1)):
        ref = np.exp(-z * psi)
        ref *= L / ref.sum()                  # mass is conserved in a closed box
        assert np.abs(c[sp_] - ref).max() < 1e-12
    bal = s.balance()
    assert np.allclose(bal[:, 0], L, rtol=0, atol=1e-12)


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    return vals


def test_half_channel_electromigration_paper_case():
    g = _golden("e2_half_channel.txt")
    VT = g["kB_J_K"] * g["T_K"] / g["e_C"]                     # thermal voltage
    lam = math.sqrt(g["eps_r"] * g["eps0_F_m"] * g["kB_J_K"] * g["T_K"]
                    / (2 * g["c_inf_mol_m3"] * g["e_C"] * g["faraday_C_mol"]))
    # Eq. (10); y measured from the charged wall
    def psi_gc(y):
        return 4 * VT * np.arctanh(np.tanh(g["psi_wall_V"] / (4 * VT)) * np.exp(-y / lam))
    assert abs(lam - 96.3e-9) < 0.5e-9
    # one cell holding the wall potential next to a Dirichlet ghost at psi = 0:
    # the steady value is C_inf * exp(-z psi_0 / V_T) -> 1.4753 (Na), 0.6778 (Cl)
    n = 40
    dx = g["width_m"] / n
    # cells from the centreline (x = 0, Dirichlet ghost at C_inf) to the wall
    y = g["width_m"] - (np.arange(n) + 0.5) * dx
    psi = psi_gc(y) / VT
    cfg = OracleCfg(dim=2, nx=n, ny=1, D=(0.2, 0.2), u_in=0.0, c0=1.0, np_x_bc=NPX_INLET_OUTLET)
    s = OracleSolver(cfg, _line(n), psi=psi)
    s.set_velocity(np.zeros((2, n)))
    assert s.np_steps(120000) == 0
    c = s.conc()
    for sp_, z in ((0, 1), (1, -1)):
        exact_discrete = np.exp(-z * (psi - psi[0]))       # ghost psi continues cell 0
        assert np.abs(c[sp_] - exact_discrete).max() < 1e-11
        eq9 = np.exp(-z * psi)                             # Eq. (9) with C_inf at psi = 0
        assert np.abs(c[sp_] / eq9 - 1).max() < 3e-3
    assert abs(math.exp(-g["psi_wall_V"] / VT) - 1.4753) < 1e-4
    assert abs(math.exp(g["psi_wall_V"] / VT) - 0.6778) < 1e-4


def test_one_dimensional_adsorption_flux():
    # Dirichlet c0 at the inlet ghost, L cells, adsorbing electrode at the far
    # face: J = k_eff c0 / (1 + k_eff L / D), linear profile.
    L, D, Ka = 12, 0.1, 0.05
    lab = _line(L + 1)
    lab[-1] = 1
    cfg = OracleCfg(dim=2, nx=L + 1, ny=1, D=(D, D), u_in=0.0, Ka=Ka, c0=1.0, np_x_bc=NPX_INLET_OUTLET)
    s = OracleSolver(cfg, lab)
    s.set_velocity(np.zeros((2, L)))
    assert s.np_steps(30000) == 0
    keff = Ka * D / (D + Ka / 2)
    J = keff / (1 + keff * L / D)
    c = s.conc()
    ref = 1.0 - (np.arange(L) + 1) * J / D
    assert np.abs(c[0] - ref).max() < 1e-12
    a0 = s.adsorbed_total()
    s.np_steps(10)
    a1 = s.adsorbed_total()
    assert np.allclose((a1 - a0) / 10, J, rtol=1e-11)


def test_periodic_transient_matches_fourier_amplification():
    N, D, w, n = 32, 0.08, 0.03, 50
    cfg = OracleCfg(dim=2, nx=N, ny=1, D=(D, D), u_in=0.0, np_x_bc=NPX_PERIODIC)
    s = OracleSolver(cfg, _line(N))
    s.set_velocity(np.vstack([np.full(N, w), np.zeros(N)]))
    rng = np.random.default_rng(0)
    c0 = 1.0 + 0.5 * rng.random((2, N))
    s.set_conc(c0)
    assert s.np_steps(n) == 0
    pe = w / D
    k = 2 * np.pi * np.fft.fftfreq(N)
    G = 1 - D * (bern(-pe) + bern(pe)) + D * bern(pe) * np.exp(1j * k) + D * bern(-pe) * np.exp(-1j * k)
    ref = np.real(np.fft.ifft(G ** n * np.fft.fft(c0[0])))
    assert np.abs(s.conc()[0] - ref).max() < 1e-12


def _porous_2d(nx=32, ny=20, seed=5, phi=0.75):
    prims, _ = oracle.disks(nx, ny, 2, 1, seed, phi, 2.5, 4.0, 2.0)
    return oracle.voxelize(2, nx, ny, 1, 1, 2, prims)


def test_conservation_and_positivity_frozen_and_fused():
    nx, ny = 32, 20
    lab = _porous_2d(nx, ny)
    for fused in (False, True):
        cfg = OracleCfg(dim=2, nx=nx, ny=ny, drive=DRIVE_INLET_OUTLET, u_in=2e-3, dpsi=20.0,
                        D=(0.05, 0.076), np_x_bc=NPX_INLET_OUTLET)
        s = OracleSolver(cfg, lab)
        s.flow_steps(300)
        m0 = s.balance()[:, 0].copy()
        assert s.np_stability() <= 1.0
        assert s.np_steps(1500, fused=fused) == 0
        b = s.balance()
        M, A, In, Out = b[:, 0], b[:, 1], b[:, 2], b[:, 3]
        assert np.all(np.abs(M + A + Out - In - m0) <= 1e-12 * m0)
        assert np.all(A > 0)
        assert s.conc().min() >= 0.0


def test_unstable_time_step_is_rejected():
    nx, ny = 16, 8
    lab = np.zeros(nx * ny, np.uint8)
    cfg = OracleCfg(dim=2, nx=nx, ny=ny, D=(0.3, 0.3), u_in=0.0)
    s = OracleSolver(cfg, lab)
    s.set_velocity(np.zeros((2, s.nf)))
    assert s.np_stability() > 1.0
    assert s.np_steps(1) == oracle.oracle.E_UNSTABLE
    cfg.np_substeps = 2                       # dt = 1/2 restores positivity
    s2 = OracleSolver(cfg, lab)
    s2.set_velocity(np.zeros((2, s2.nf)))
    assert s2.np_stability() <= 1.0 and s2.np_steps(5) == 0


def _assemble(lab, nx, ny, u, psi_cells, ramp, D, z, c0, keff, u_in):
    """Steady operator of the face-flux scheme as a sparse system A C = b
    (outflow sum of each cell = 0), written from the flux definitions."""
    m, fl = oracle.compact(lab)
    nf = fl.size
    rows, cols, vals = [], [], []
    b = np.zeros(nf)
    g = lab.reshape(ny, nx)
    for p, v in enumerate(fl):
        x, y = v % nx, v // nx
        for ax, sg in ((0, -1), (0, 1), (1, -1), (1, 1)):
            xn, yn = x + (sg if ax == 0 else 0), y + (sg if ax == 1 else 0)
            if ax == 0 and xn < 0:                    # inlet ghost held at c0
                wv = -u_in - z * D * (ramp(-1) - psi_cells[p])
                rows.append(p); cols.append(p); vals.append(float(D * bern(-wv / D)))
                b[p] += D * bern(wv / D) * c0
                continue
            if ax == 0 and xn >= nx:                  # open outlet: upwind drift only
                wv = u[0][p] - z * D * (ramp(nx) - psi_cells[p])
                rows.append(p); cols.append(p); vals.append(max(wv, 0.0))
                b[p] -= min(wv, 0.0) * c0
                continue
            yn %= ny
            L = g[yn, xn]
            if L == 1:
                rows.append(p); cols.append(p); vals.append(keff)
            elif L == 0:
                q = m[yn * nx + xn]
                wv = 0.5 * (u[ax][p] + u[ax][q]) * sg - z * D * (psi_cells[q] - psi_cells[p])
                rows.append(p); cols.append(p); vals.append(float(D * bern(-wv / D)))
                rows.append(p); cols.append(q); vals.append(float(-D * bern(wv / D)))
    return sp.csr_matrix((np.array(vals), (rows, cols)), shape=(nf, nf)), b


def test_explicit_steady_state_equals_sparse_direct_solve():
    nx, ny = 32, 20
    lab = _porous_2d(nx, ny)
    dpsi, u_in = 8.0, 3e-3
    cfg = OracleCfg(dim=2, nx=nx, ny=ny, drive=DRIVE_INLET_OUTLET, u_in=u_in, dpsi=dpsi,
                    D=(0.05, 0.076), np_x_bc=NPX_INLET_OUTLET)
    s = OracleSolver(cfg, lab)
    s.flow_to_steady(tol=1e-9, max_steps=200000, check_every=100)
    s.freeze_velocity()
    u = s.np_velocity()
    m, fl = oracle.compact(lab)
    def ramp(x):
        return dpsi * (1 - (x + 0.5) / nx)
    psi_cells = ramp(fl % nx)
    cstar = []
    for sp_, (D, z) in enumerate(((0.05, 1), (0.076, -1))):
        keff = s.ka * D / (D + s.ka / 2)
        A, b = _assemble(lab, nx, ny, u, psi_cells, ramp, D, z, 1.0, keff, u_in)
        cstar.append(spla.spsolve(A.tocsc(), b))
    cstar = np.array(cstar)
    # C* is a fixed point of the explicit step, and the adsorbed rate equals
    # inflow minus outflow there (mass balance at steady state).
    s.set_conc(cstar)
    b0 = s.balance()
    assert s.np_steps(1) == 0
    b1 = s.balance()
    assert np.abs(s.conc() - cstar).max() < 1e-13
    dA, dIn, dOut = b1[:, 1] - b0[:, 1], b1[:, 2] - b0[:, 2], b1[:, 3] - b0[:, 3]
    assert np.allclose(dIn - dOut, dA, rtol=1e-10)
    # and the explicit march from C = c0 approaches it
    s2 = OracleSolver(cfg, lab)
    s2.flow_to_steady(tol=1e-9, max_steps=200000, check_every=100)
    s2.np_steps(2000)
    e1 = np.abs(s2.conc() - cstar).max()
    s2.np_steps(6000)
    e2 = np.abs(s2.conc() - cstar).max()
    assert e2 < 0.5 * e1


def test_periodic_ions_in_the_applied_ramp_see_a_uniform_field():
    # The applied ramp is a uniform field. On a periodic line without flow it
    # drives each species with the uniform drift w = z D dpsi / N, across the
    # periodic seam too, so the transient is the Fourier closed form of a
    # uniform drift (opposite for the two species).
    N, D, dpsi, n = 32, 0.08, 4.0, 60
    cfg = OracleCfg(dim=2, nx=N, ny=1, D=(D, D), u_in=0.0, dpsi=dpsi, np_x_bc=NPX_PERIODIC)
    s = OracleSolver(cfg, _line(N))
    s.set_velocity(np.zeros((2, N)))
    rng = np.random.default_rng(3)
    c0 = 1.0 + 0.5 * rng.random((2, N))
    s.set_conc(c0)
    assert s.np_steps(n) == 0
    k = 2 * np.pi * np.fft.fftfreq(N)
    for sp, z in ((0, 1), (1, -1)):
        pe = z * D * dpsi / N / D
        G = 1 - D * (bern(-pe) + bern(pe)) + D * bern(pe) * np.exp(1j * k) + D * bern(-pe) * np.exp(-1j * k)
        ref = np.real(np.fft.ifft(G ** n * np.fft.fft(c0[sp])))
        assert np.abs(s.conc()[sp] - ref).max() < 1e-12
