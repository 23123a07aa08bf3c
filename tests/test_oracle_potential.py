"""Pins of the CPU reference's potential solve (Poisson, Eq. 4, with the charge
of Eq. 5 and Dirichlet values on the electrode surface, Sec. 2).

Closed forms of the discrete problem: the linear profile between two
Dirichlet x faces (exact for the two-point face flux and the half-cell
Dirichlet face), and the parabola of a uniform charge between two electrode
planes, whose discrete solution is the continuous one shifted by s h^2 / 8
(worked out by hand from the boundary cell's balance). Invariants: the
discrete Gauss law (Dirichlet-face fluxes balance the total charge), the
maximum principle of the Laplace problem, mirror symmetry, linearity in the
data, and the singular all-Neumann case.
"""
import numpy as np
import pytest

import oracle
from oracle import (OracleCfg, OracleSolver, PSIX_DIRICHLET, PSIX_NEUMANN, PSIX_PERIODIC, NPX_CLOSED)


def solver(labels, dim, nx, ny, nz=1, **kw):
    cfg = OracleCfg(dim=dim, nx=nx, ny=ny, nz=nz, u_in=0.0, np_x_bc=NPX_CLOSED, **kw)
    return OracleSolver(cfg, np.ascontiguousarray(labels, np.uint8).reshape(-1))


def coords(labels, nx, ny):
    _, fluid = oracle.compact(np.ascontiguousarray(labels, np.uint8).reshape(-1))
    return fluid % nx, (fluid // nx) % ny, fluid // (nx * ny)


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_profile_between_dirichlet_x_faces(dim):
    nx, ny, nz = 24, 6, (5 if dim == 3 else 1)
    lab = np.zeros((nz, ny, nx), np.uint8)
    if dim == 2:
        lab[:, 0, :] = lab[:, -1, :] = 2  # inert walls carry no field
    s = solver(lab, dim, nx, ny, nz)
    rc, it, rel = s.solve_potential(x_bc=(PSIX_DIRICHLET, PSIX_DIRICHLET), psi_x=(7.5, -2.0))
    assert rc == 0 and rel <= 1e-13
    x, _, _ = coords(lab, nx, ny)
    exact = 7.5 + (-2.0 - 7.5) * (x + 0.5) / nx
    assert np.abs(s.potential() - exact).max() <= 1e-11


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("charge", [(1.5, 1.0), (0.25, 2.0)])
def test_uniform_charge_between_electrode_planes(dim, charge):
    # electrode planes y = 0 and y = ny - 1; faces at a = 1/2, b = ny - 3/2
    nx, ny, nz = 8, 14, (4 if dim == 3 else 1)
    lab = np.zeros((nz, ny, nx), np.uint8)
    lab[:, 0, :] = lab[:, -1, :] = 1
    kappa2, c0, psi_e = 0.3, 1.0, -1.25
    s = solver(lab, dim, nx, ny, nz, c0=c0)
    nf = s.nf
    s.set_conc(np.vstack([np.full(nf, charge[0]), np.full(nf, charge[1])]))
    rc, _, rel = s.solve_potential(psi_electrode=psi_e, x_bc=(PSIX_NEUMANN, PSIX_NEUMANN), kappa2=kappa2)
    assert rc == 0 and rel <= 1e-13
    src = kappa2 / (2 * c0) * (charge[0] - charge[1])  # z = (+1, -1)
    _, y, _ = coords(lab, nx, ny)
    a, b = 0.5, ny - 1.5
    exact = psi_e + 0.5 * src * (y - a) * (b - y) + src / 8.0
    assert np.abs(s.potential() - exact).max() <= 1e-11


def test_periodic_x_equals_neumann_on_x_invariant_data():
    nx, ny = 10, 12
    lab = np.zeros((1, ny, nx), np.uint8)
    lab[:, 0, :] = lab[:, -1, :] = 1
    out = []
    for bc in ((PSIX_PERIODIC, PSIX_PERIODIC), (PSIX_NEUMANN, PSIX_NEUMANN)):
        s = solver(lab, 2, nx, ny)
        s.set_conc(np.vstack([np.full(s.nf, 2.0), np.full(s.nf, 1.0)]))
        assert s.solve_potential(psi_electrode=0.5, x_bc=bc, kappa2=0.2)[0] == 0
        out.append(s.potential())
    assert np.abs(out[0] - out[1]).max() <= 1e-12


def _porous(seed, nx=32, ny=20, nz=18):
    prims = oracle.spheres(nx, ny, nz, 2, seed, 0.6, 2.0, 3.5)
    return oracle.voxelize(3, nx, ny, nz, 0, 2, prims), (nx, ny, nz)


def _face_flux_sum(s, lab, shape, psi, psi_e, x_bc, psi_x):
    """Total flux of grad psi into the domain through the Dirichlet faces."""
    nx, ny, nz = shape
    L = lab.reshape(nz, ny, nx)
    m, fluid = oracle.compact(lab)
    tot = 0.0
    for n, v in enumerate(fluid):
        x, y, z = v % nx, (v // nx) % ny, v // (nx * ny)
        for d in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
            xn = x + d[0]
            if xn < 0 or xn >= nx:
                end = 0 if xn < 0 else 1
                if x_bc[end] == PSIX_DIRICHLET:
                    tot += 2 * (psi_x[end] - psi[n])
                continue
            if L[(z + d[2]) % nz, (y + d[1]) % ny, xn] == 1:
                tot += 2 * (psi_e - psi[n])
    return tot


def test_gauss_law_and_maximum_principle_on_porous_electrode():
    lab, shape = _porous(11)
    nx, ny, nz = shape
    x_bc, psi_x, psi_e = (PSIX_DIRICHLET, PSIX_NEUMANN), (0.0, 0.0), -2.0
    # Laplace: potential between the boundary values, Dirichlet fluxes sum to 0
    s = solver(lab, 3, nx, ny, nz)
    rc, it, rel = s.solve_potential(psi_electrode=psi_e, x_bc=x_bc, psi_x=psi_x)
    assert rc == 0 and it > 5
    psi = s.potential()
    assert psi.min() >= psi_e - 1e-12 and psi.max() <= 1e-12
    assert psi.max() < 0.0 and np.median(psi) > psi_e  # pores enclosed by the electrode sit at psi_e
    assert abs(_face_flux_sum(s, lab, shape, psi, psi_e, x_bc, psi_x)) <= 1e-9
    # Poisson: the Dirichlet fluxes carry away exactly the total charge
    rng = np.random.default_rng(5)
    c = rng.uniform(0.5, 1.5, size=(2, s.nf))
    s.set_conc(c)
    kappa2 = 0.4
    assert s.solve_potential(psi_electrode=psi_e, x_bc=x_bc, psi_x=psi_x, kappa2=kappa2)[0] == 0
    q = kappa2 / 2.0 * (c[0] - c[1]).sum()
    assert abs(_face_flux_sum(s, lab, shape, s.potential(), psi_e, x_bc, psi_x) + q) <= 1e-8 * (1 + abs(q))


def test_mirror_symmetry():
    lab, (nx, ny, nz) = _porous(12)
    L = lab.reshape(nz, ny, nx)
    sym = np.concatenate([L, L[:, ::-1, :]], axis=1)  # mirror image in y
    ny2 = 2 * ny
    s = solver(sym, 3, nx, ny2, nz)
    assert s.solve_potential(psi_electrode=1.0, x_bc=(PSIX_DIRICHLET, PSIX_DIRICHLET),
                             psi_x=(0.0, 3.0))[0] == 0
    full = np.full(sym.size, np.nan)
    _, fluid = oracle.compact(sym.reshape(-1))
    full[fluid] = s.potential()
    F = full.reshape(nz, ny2, nx)
    # y -> 2 ny - 1 - y maps the domain onto itself
    assert np.nanmax(np.abs(F - F[:, ::-1, :])) <= 1e-11


def test_linearity_in_boundary_values_and_charge():
    lab, (nx, ny, nz) = _porous(13)
    rng = np.random.default_rng(3)
    c = rng.uniform(0.0, 2.0, size=(2, int((lab == 0).sum())))

    def run(pe, px, k2):
        s = solver(lab, 3, nx, ny, nz)
        s.set_conc(c)
        assert s.solve_potential(psi_electrode=pe, x_bc=(PSIX_DIRICHLET, PSIX_DIRICHLET), psi_x=px,
                                 kappa2=k2)[0] == 0
        return s.potential()

    a = run(1.0, (0.0, 0.0), 0.0)
    b = run(0.0, (2.0, -1.0), 0.0)
    q = run(0.0, (0.0, 0.0), 0.5)
    both = run(3.0, (-4.0, 2.0), 1.5)
    assert np.abs(both - (3 * a - 2 * b + 3 * q)).max() <= 1e-10


def test_singular_problem_is_rejected():
    # periodic in every direction and no electrode: defined up to a constant
    s = solver(np.zeros((4, 6, 8), np.uint8), 3, 8, 6, 4)
    rc, _, _ = s.solve_potential(x_bc=(PSIX_PERIODIC, PSIX_PERIODIC))
    assert rc == oracle.oracle.E_INVALID
    # one periodic end alone is not a valid choice
    s = solver(np.zeros((1, 6, 8), np.uint8), 2, 8, 6)
    assert s.solve_potential(x_bc=(PSIX_PERIODIC, PSIX_DIRICHLET))[0] == oracle.oracle.E_INVALID


def test_no_adsorption_flag():
    lab = np.zeros((1, 8, 12), np.uint8)
    lab[:, 0, :] = lab[:, -1, :] = 1
    derived = OracleSolver(OracleCfg(dim=2, nx=12, ny=8, u_in=1e-3, Ka=-1.0), lab.reshape(-1)).ka
    assert derived > 0  # <= 0 still means the derived default
    s = solver(lab, 2, 12, 8, Ka=0.3, no_adsorption=1)
    assert s.ka == 0.0
    assert s.np_steps(50) == 0
    assert np.all(s.adsorbed_total() == 0.0)


def test_coupled_pnp_half_channel_converges_to_gouy_chapman():
    """The paper's electromigration check (Sec. 3, Fig. 3) with the potential
    solved from the charge instead of prescribed: a blocking wall at -10 mV,
    zero potential and C_inf at the centreline 1 um away. The steady state
    must satisfy the discrete Boltzmann law exactly and approach Eq. (10) for
    psi and Eq. (9) for C at second order in the cell size."""
    import math
    import os
    vals = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", "e2_half_channel.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, v = line.split()
                vals[k] = float(v)
    VT = vals["kB_J_K"] * vals["T_K"] / vals["e_C"]
    lam = math.sqrt(vals["eps_r"] * vals["eps0_F_m"] * vals["kB_J_K"] * vals["T_K"]
                    / (2 * vals["c_inf_mol_m3"] * vals["e_C"] * vals["faraday_C_mol"]))
    W, psi0 = vals["width_m"], vals["psi_wall_V"]

    def gc(y):  # Eq. (10), y from the wall
        return 4 * VT * np.arctanh(np.tanh(psi0 / (4 * VT)) * np.exp(-y / lam))

    errs = []
    for n in (20, 40):
        dx = W / n
        lab = np.zeros(n + 1, np.uint8)
        lab[-1] = 1  # the charged wall; x = 0 is the centreline
        cfg = OracleCfg(dim=2, nx=n + 1, ny=1, D=(0.2, 0.2), u_in=0.0, c0=1.0, no_adsorption=1)
        s = OracleSolver(cfg, lab)
        s.set_velocity(np.zeros((2, n)))
        rc = s.np_steps_coupled(int(10 * n * n / 0.2), every=20, psi_electrode=psi0 / VT,
                                x_bc=(PSIX_DIRICHLET, PSIX_NEUMANN), kappa2=(dx / lam) ** 2, tol=1e-12)
        assert rc == 0
        psi, c = s.potential(), s.conc()
        # discrete Boltzmann law relative to the centreline cell (zero net flux everywhere)
        assert np.abs(c[0] - np.exp(-(psi - psi[0]))).max() <= 1e-10
        assert np.abs(c[1] - np.exp(psi - psi[0])).max() <= 1e-10
        y = W - (np.arange(n) + 0.5) * dx
        errs.append(np.abs(psi - gc(y) / VT).max() / abs(psi0 / VT))
        assert np.abs(c[0] * np.exp(gc(y) / VT) - 1).max() <= 2 * errs[-1]  # Eq. (9)
    assert errs[0] < 0.025 and errs[1] < 0.008 and errs[0] / errs[1] > 3.0
