"""Implicit ion transport on the GPU (the paper's time scheme, Sec. 2):
steady states and backward-Euler steps against the FP64 oracle.

Bar: the GPU evaluates the face coefficients in FP32 (as its explicit step)
and solves in FP64 to 1e-10; the oracle is FP64 throughout, to 1e-13. The
coefficient rounding (relative 1e-7) moves the solution by far less than
the concentration bar of the explicit parity tests, which is kept:
|C_gpu - C_oracle| <= 1e-4 c0; rates within 1e-4 relative."""
import numpy as np
import pytest

from helpers import oracle_solver

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2110_13055_amd")
from paper_2110_13055_amd import _lib as L  # noqa: E402
from paper_2110_13055_amd import Geometry, Params, Potential, Solver, preset  # noqa: E402


def pair(g, p, flow=1500):
    s, o = Solver(g, p), oracle_solver(g, p)
    s.flow_steps(flow)
    o.flow_steps(flow)
    o.freeze_velocity()
    return s, o


def spheres(**pk):
    g = Geometry(dim=3, nx=40, ny=31, nz=27, kind=L.SPHERES, porosity=0.55, r_min=2.5, r_max=5.0, buffer_x=2,
                 seed=3)
    return g, Params(u_in=1e-3, dpsi_vt=6.0, D=(0.05, 0.076), **pk)


@pytest.mark.parametrize("case", ["2d", "3d", "3d_dirichlet"])
def test_steady_state_matches_oracle(case):
    if case == "2d":
        g, p, _ = preset("channel2d_128x64")
    else:
        g, p = spheres(**({"np_x_bc": L.NPX_DIRICHLET, "c_out": 0.3} if case == "3d_dirichlet" else {}))
    s, o = pair(g, p, 1500 if case == "2d" else 400)
    it = s.np_steady(tol=1e-10)
    rc, _ = o.np_steady(tol=1e-13)
    assert rc == 0 and it > 5
    assert np.abs(s.concentration() - o.conc()).max() <= 1e-4
    r, ro = s.np_rates(), o.np_rates()
    assert np.all(np.abs(r - ro) <= 1e-4 * np.abs(ro).max())
    # a steady state: adsorption = inflow - outflow
    assert np.allclose(r[:, 1] - r[:, 2], r[:, 0], rtol=1e-4)


def test_steady_state_is_what_the_explicit_march_approaches():
    g, p, _ = preset("channel2d_128x64")
    s, _ = pair(g, p)
    t = Solver(g, p)
    t.flow_steps(1500)
    t.np_steady(tol=1e-10)
    cstar = t.concentration()
    errs = []
    for _ in range(3):
        s.np_step(20000)
        errs.append(np.abs(s.concentration() - cstar).max())
    assert errs[0] > errs[1] > errs[2]  # the march closes in on the steady state


@pytest.mark.parametrize("dt", [1.0, 40.0])
def test_backward_euler_matches_oracle_and_conserves(dt):
    g, p = spheres()
    s, o = pair(g, p, 400)
    m0 = s.mass_balance()[:, 0].copy()
    s.np_implicit(dt, 12, tol=1e-11)
    assert o.np_implicit(dt, 12, tol=1e-13)[0] == 0
    assert np.abs(s.concentration() - o.conc()).max() <= 1e-4
    b, bo = s.mass_balance(), o.balance()
    assert np.all(np.abs(b[:, 1:] - bo[:, 1:]) <= 1e-4 * np.abs(bo[:, 1:]).max())
    M, A, In, Out = b[:, 0], b[:, 1], b[:, 2], b[:, 3]
    assert np.all(np.abs(M + A + Out - In - m0) <= 1e-5 * m0)
    assert s.info().np_steps == 12


def test_steady_on_a_solved_potential_and_repeatable():
    g, p, _ = preset("channel2d_128x64")
    s, o = pair(g, p)
    pot = Potential(psi_electrode=-3.0, x_bc=(L.PSIX_DIRICHLET, L.PSIX_NEUMANN), tol=1e-12)
    s.solve_potential(pot)
    o.solve_potential(pot.psi_electrode, pot.x_bc, pot.psi_x, 0.0, 1e-13)
    c0 = s.concentration()
    it = s.np_steady(tol=1e-10)
    assert o.np_steady(tol=1e-13)[0] == 0
    assert np.abs(s.concentration() - o.conc()).max() <= 1e-4
    first = s.concentration()
    s.set_concentration(c0)
    assert s.np_steady(tol=1e-10) == it
    assert np.array_equal(s.concentration(), first)


def test_iteration_cap_and_workspace_errors():
    g, p, _ = preset("channel2d_128x64")
    s, _ = pair(g, p, 200)
    it = s.np_steady(tol=1e-14, max_iter=5, allow_not_converged=True)
    assert it <= 5
    import ctypes as C
    import torch
    ws = torch.empty(4096, dtype=torch.uint8, device="cuda")
    rc = s.lib.cdi_np_steady(s.h, 1e-8, 10, C.c_void_p(ws.data_ptr()), ws.numel(), None)
    assert rc == L.E_BUFFER
    with pytest.raises(L.CdiError):
        s.np_implicit(0.0, 1)


def _bern(x):
    """B(x) = x / (e^x - 1), B(0) = 1."""
    small = np.abs(x) < 1e-12
    return np.where(small, 1.0 - 0.5 * x, x / np.where(small, 1.0, np.expm1(x)))


def _cell_balance(lab3, conc, flux, psi, D, z, keff, u_in, c0, dpsi_dx):
    """Per fluid cell and species, the net outflow of the explicit update's
    face fluxes (inlet/outlet x ends, y and z periodic), restated on the dense
    grid: fluid face D B(w/D) (C_P - C_N) + w C_P with the drift
    w = (j_P + j_N).n / 2 - z D (psi_N - psi_P); electrode face k_eff C_P;
    inlet face the same exponential-fitting flux to a c0 ghost with w =
    -u_in - z D dpsi; outlet face upwind max(w, 0) C_P + min(w, 0) c0 with
    w = j_P.n - z D dpsi (dpsi: the ramp's step, none at the x ends when psi
    is a field); inert faces none. Returns the net outflow and the sum of the
    face fluxes' magnitudes, (2, N_f) each, in fluid order."""
    fluid = lab3 == 0
    nx = lab3.shape[2]
    out = np.zeros((2,) + lab3.shape)
    gross = np.zeros((2,) + lab3.shape)
    comp = {2: 0, 1: 1, 0: 2}  # array axis (z, y, x order) -> flux component
    for axis in (2, 1, 0):
        j_p = flux[comp[axis]]
        for sg in (1, -1):
            nlab = np.roll(lab3, -sg, axis=axis)
            jn = np.roll(j_p, -sg, axis=axis)
            if axis == 2:
                end = nx - 1 if sg == 1 else 0
                nlab = nlab.copy()
                nlab[:, :, end] = 255
            if psi is not None:
                dpsi = np.roll(psi, -sg, axis=axis) - psi
            else:
                dpsi = -sg * dpsi_dx if axis == 2 else 0.0
            for s in range(2):
                cp = conc[s]
                cn = np.roll(cp, -sg, axis=axis)
                w = 0.5 * (j_p + jn) * sg - z[s] * D[s] * dpsi
                f = np.where(nlab == 0, D[s] * _bern(w / D[s]) * (cp - cn) + w * cp, 0.0)
                f = f + np.where(nlab == 1, keff[s] * cp, 0.0)
                if axis == 2:
                    sl = (slice(None), slice(None), end)
                    de = 0.0 if psi is not None else -sg * dpsi_dx
                    if sg == -1:
                        we = -u_in - z[s] * D[s] * de
                        f[sl] = D[s] * _bern(we / D[s]) * (cp[sl] - c0) + we * cp[sl]
                    else:
                        we = j_p[sl] - z[s] * D[s] * de
                        f[sl] = np.maximum(we, 0.0) * cp[sl] + np.minimum(we, 0.0) * c0
                out[s] += f
                gross[s] += np.abs(f)
    return out[:, fluid], gross[:, fluid]


def _dense(lab, fl, v):
    a = np.zeros((v.shape[0], lab.size))
    a[:, fl] = v
    return a


def test_full_size_steady_state_balances_every_cell():
    # the bench's ion steady state at the full 512^3 size: flow, a solved
    # potential (electrode -4, inlet face 0, field-free outlet), BiCGSTAB
    g, p, _ = preset("spheres3d_512")
    s = Solver(g, p)
    s.flow_steps(200)
    s.solve_potential(Potential(psi_electrode=-4.0, x_bc=(L.PSIX_DIRICHLET, L.PSIX_NEUMANN), tol=1e-10))
    it = s.np_steady(tol=1e-10, max_iter=4000)
    lab = s.labels()
    _, fl = s.fluid_index()
    c = s.concentration().astype(np.float64)
    j = s.np_velocity().astype(np.float64)
    psi = s.potential().astype(np.float64)
    del s
    # non-negative in exact arithmetic (an M-matrix); the iterative stop leaves
    # errors of the solver's size where C is close to 0
    assert c.min() >= -1e-6
    sh = (g.nz, g.ny, g.nx)
    nf_vox = fl.size / lab.size
    ka = (4.28e-3 / 1.03e-2) * p.u_in / nf_vox  # the default K_a (Sec. 4.1's Da/Pe at the mean pore velocity)
    keff = [ka * D / (D + ka / 2) for D in p.D]
    out, gross = _cell_balance(lab.reshape(sh), _dense(lab, fl, c).reshape((2,) + sh),
                               _dense(lab, fl, j).reshape((3,) + sh), _dense(lab, fl, psi[None])[0].reshape(sh),
                               p.D, p.z, keff, p.u_in, p.c0, 0.0)
    # FP32 storage of C (relative 6e-8, of values well above c0 next to the
    # attracting electrode) times the face coefficients, FP32 coefficients and
    # the 1e-10 stop: measured 1.3e-6 of the largest face flux; a 1 % error in
    # k_eff alone leaves 1e-3 of it
    print(f"512^3 ion steady state: {it} iterations, max net outflow {np.abs(out).max():.2e}, "
          f"max gross face flux {gross.max():.2e}, max C {c.max():.3g}")
    assert np.abs(out).max() <= 1e-5 * gross.max()
    assert np.abs(c - p.c0).max() > 1e-2  # the ions have moved


@pytest.mark.parametrize("npx", [L.NPX_PERIODIC, L.NPX_CLOSED], ids=["periodic", "closed"])
def test_backward_euler_with_periodic_or_closed_ion_ends(npx):
    # the implicit operator with the ions' x ends periodic (the ramp's
    # uniform field across the seam) or closed, under the open flow
    g, p = spheres(np_x_bc=npx)
    s, o = pair(g, p, 400)
    m0 = s.mass_balance()[:, 0].copy()
    s.np_implicit(5.0, 8, tol=1e-11)
    assert o.np_implicit(5.0, 8, tol=1e-13)[0] == 0
    assert np.abs(s.concentration() - o.conc()).max() <= 1e-4
    b = s.mass_balance()
    M, A, In, Out = b[:, 0], b[:, 1], b[:, 2], b[:, 3]
    assert np.all(np.abs(In) == 0) and np.all(np.abs(Out) == 0)  # nothing crosses the x ends
    assert np.all(np.abs(M + A - m0) <= 1e-5 * m0)
