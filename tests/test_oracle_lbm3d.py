"""Pins of the CPU reference's D3Q19 lattice Boltzmann solver and of the BGK
equilibrium of Eq. (8) on both lattices (Sec. 2, the LBM paragraph).

The equilibrium is pinned by its moment identities: for any (rho, u) the
populations it sets carry the mass rho, the momentum rho u and the momentum
flux rho u u + (rho/3) I (the linear Stokes form: (rho/3) I). A wrong weight,
a wrong velocity vector, or a wrong 3, 4.5 or -1.5 coefficient breaks one of
them. The D3Q19 stream, half-way bounce-back and periodic wrap are pinned by
Poiseuille's parabola between walls normal to each axis (second order in the
width, exact at Ginzburg's magic relaxation time), by the viscous decay of
shear waves along y and z, and by mass conservation with a body force.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import OracleCfg, OracleSolver, DRIVE_BODY_FORCE, DRIVE_INLET_OUTLET, EQ_LINEAR, EQ_QUADRATIC


def _velocity_set(dim):
    """Lattice vectors of the reference, recovered from its own populations:
    unit momentum along one axis at a time shows each direction's component
    sign through f_i(u) - f_i(0) = 3 w_i rho e_i.u (linear equilibrium). The
    set must then be the textbook D2Q9 / D3Q19 set: the zero vector, the 2d
    axis vectors and (D3Q19) the 12 face diagonals, or (D2Q9) the 4
    diagonals."""
    nx = 4
    cfg = OracleCfg(dim=dim, nx=nx, ny=1, nz=1, drive=DRIVE_INLET_OUTLET, equilibrium=EQ_LINEAR, u_in=0.0)
    s = OracleSolver(cfg, np.zeros(nx, np.uint8))
    s.init_equilibrium(None, None)
    w = s.populations()[:, 0].copy()
    e = np.zeros((w.size, 3))
    for a in range(dim):
        u = np.zeros((dim, s.nf))
        u[a] = 1e-3
        s.init_equilibrium(None, u)
        e[:, a] = (s.populations()[:, 0] - w) / (3e-3 * w)
    return w, e


@pytest.mark.parametrize("dim", [2, 3])
def test_lattice_is_the_textbook_velocity_set(dim):
    w, e = _velocity_set(dim)
    ei = np.rint(e).astype(int)
    assert np.abs(e - ei).max() < 1e-9
    rows = sorted(map(tuple, ei))
    if dim == 2:
        ref = [(0, 0, 0)] + [(a, b, 0) for a in (-1, 0, 1) for b in (-1, 0, 1) if (a, b) != (0, 0)]
        weights = {0: 4 / 9, 1: 1 / 9, 2: 1 / 36}
    else:
        ref = [(0, 0, 0)]
        ref += [tuple(s * (np.arange(3) == a)) for a in range(3) for s in (-1, 1)]
        ref += [tuple(v) for v in ([a, b, 0] for a in (-1, 1) for b in (-1, 1))]
        ref += [tuple(v) for v in ([a, 0, b] for a in (-1, 1) for b in (-1, 1))]
        ref += [tuple(v) for v in ([0, a, b] for a in (-1, 1) for b in (-1, 1))]
        weights = {0: 1 / 3, 1: 1 / 18, 2: 1 / 36}
    assert rows == sorted(tuple(int(c) for c in r) for r in ref)
    for i in range(w.size):
        assert abs(w[i] - weights[int(np.abs(ei[i]).sum())]) < 1e-15
    # isotropy of the set: sum w = 1, sum w e e = I/3
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs((w[:, None, None] * ei[:, :, None] * ei[:, None, :]).sum(0)[:dim, :dim]
                  - np.eye(dim) / 3).max() < 1e-15


@pytest.mark.parametrize("dim", [2, 3])
@pytest.mark.parametrize("eq", [EQ_QUADRATIC, EQ_LINEAR])
def test_equilibrium_moment_identities(dim, eq):
    # rho and u drawn at random per node; the populations the reference sets
    # must carry mass rho, momentum rho u and momentum flux
    # rho u u + (rho / 3) I (linear form: (rho / 3) I).
    w, e = _velocity_set(dim)
    e = np.rint(e)
    nx = 64
    cfg = OracleCfg(dim=dim, nx=nx, ny=1, nz=1, drive=DRIVE_INLET_OUTLET, equilibrium=eq, u_in=0.0)
    s = OracleSolver(cfg, np.zeros(nx, np.uint8))
    rng = np.random.default_rng(7 + dim + 10 * eq)
    rho = 1.0 + 0.2 * (rng.random(s.nf) - 0.5)
    u = 0.1 * (rng.random((dim, s.nf)) - 0.5)
    s.init_equilibrium(rho, u)
    f = s.populations()
    ed = e[:, :dim]
    assert np.abs(f.sum(0) - rho).max() < 1e-14
    mom = ed.T @ f
    assert np.abs(mom - rho * u).max() < 1e-14
    flux = np.einsum("ia,ib,in->abn", ed, ed, f)
    ref = np.eye(dim)[:, :, None] * (rho / 3)[None, None, :]
    if eq == EQ_QUADRATIC:
        ref = ref + rho[None, None, :] * u[:, None, :] * u[None, :, :]
    assert np.abs(flux - ref).max() < 1e-14
    # and the velocity the reference reports back is u itself
    assert np.abs(s.velocity() - u).max() < 1e-14
    assert np.abs(s.density() - rho).max() < 1e-14


AX = {"x": 0, "y": 1, "z": 2}


def _channel3d(flow, wall, H, other=2, along=2):
    """Box with inert walls at both ends of axis `wall` (width H fluid cells
    between them), periodic along the others; dims as (nx, ny, nz)."""
    n = [0, 0, 0]
    n[AX[wall]] = H + 2
    n[AX[flow]] = along
    rest = 3 - AX[wall] - AX[flow]
    n[rest] = other
    nx, ny, nz = n
    lab = np.zeros((nz, ny, nx), np.uint8)
    idx = [slice(None)] * 3
    idx[2 - AX[wall]] = 0
    lab[tuple(idx)] = 2
    idx[2 - AX[wall]] = H + 1
    lab[tuple(idx)] = 2
    return nx, ny, nz, lab.reshape(-1)


def _poiseuille3d_error(flow, wall, H, tau, eq=EQ_QUADRATIC, relax_times=None):
    """Relative L2 error of the flow against the parabola. From the parabola
    itself, either run to the steady state (residual 1e-10: FP64 round-off
    of the D3Q19 sums floors the residual near 1e-12 .. 1e-11 here), or take
    relax_times slowest viscous decay times (the start lacks the parabola's
    non-equilibrium part, a perturbation of about 3e-3 that decays by e per
    decay time), after which a scheme with another steady state would be
    visibly off it."""
    nx, ny, nz, lab = _channel3d(flow, wall, H, along=4 if flow == "x" else 2)
    nu = (tau - 0.5) / 3
    g = 8 * nu * 1e-3 / H ** 2         # peak velocity 1e-3: FP64 round-off far below the stop
    if nx < 4:                      # the reference needs nx >= 4
        nx_pad = 4
        lab = np.tile(lab.reshape(nz, ny, nx), (1, 1, nx_pad // nx)).reshape(-1)
        nx = nx_pad
    force = [0.0, 0.0, 0.0]
    force[AX[flow]] = g
    cfg = OracleCfg(dim=3, nx=nx, ny=ny, nz=nz, drive=DRIVE_BODY_FORCE, tau=tau, force=tuple(force),
                    u_in=0.0, equilibrium=eq)
    s = OracleSolver(cfg, lab)
    m, fl = oracle.compact(lab)
    coord = [fl % nx, (fl // nx) % ny, fl // (nx * ny)]
    # walls at the half-links of the wall axis: node c lies at c + 1/2, the
    # walls at 1 and H + 1
    yw = coord[AX[wall]] + 0.5
    ua = g / (2 * nu) * (yw - 1) * (H + 1 - yw)
    u0 = np.zeros((3, s.nf))
    u0[AX[flow]] = ua
    s.init_equilibrium(None, u0)
    if relax_times is None:
        rc, steps, r = s.flow_to_steady(tol=1e-10, max_steps=400000, check_every=100)
        assert rc == 0
    else:
        s.flow_steps(int(relax_times * H * H / (nu * math.pi ** 2)))
    u = s.velocity()
    for a in range(3):
        if a != AX[flow]:
            assert np.abs(u[a]).max() <= 1e-10 * ua.max()
    return np.linalg.norm(u[AX[flow]] - ua) / np.linalg.norm(ua)


@pytest.mark.parametrize("flow,wall", [("x", "y"), ("x", "z"), ("z", "x"), ("y", "z")])
def test_d3q19_poiseuille_second_order(flow, wall):
    errs = [_poiseuille3d_error(flow, wall, H, 1.0) for H in (8, 16, 32)]
    assert errs[2] <= 1e-3
    orders = [math.log2(errs[k] / errs[k + 1]) for k in range(2)]
    assert all(1.9 < o < 2.1 for o in orders), (errs, orders)


@pytest.mark.parametrize("flow,wall", [("x", "y"), ("x", "z"), ("y", "x")])
@pytest.mark.parametrize("eq", [EQ_QUADRATIC, EQ_LINEAR])
def test_d3q19_poiseuille_exact_at_magic_tau(flow, wall, eq):
    tau = 0.5 + math.sqrt(3.0 / 16.0)
    assert _poiseuille3d_error(flow, wall, 12, tau, eq=eq, relax_times=25) < 1e-9


@pytest.mark.parametrize("wave,comp", [("z", "x"), ("y", "z"), ("x", "y")])
def test_d3q19_shear_wave_viscous_decay(wave, comp):
    # u_comp(wave) = u0 sin(k wave) decays as exp(-nu k^2 t); the error of the
    # decay rate is O(k^2).
    tau = 0.8
    nu = (tau - 0.5) / 3
    rates = []
    for L in (16, 32):
        n = [4, 2, 2]
        n[AX[wave]] = L
        nx, ny, nz = n
        cfg = OracleCfg(dim=3, nx=nx, ny=ny, nz=nz, drive=DRIVE_BODY_FORCE, tau=tau, u_in=0.0)
        s = OracleSolver(cfg, np.zeros(nx * ny * nz, np.uint8))
        m, fl = oracle.compact(np.zeros(nx * ny * nz, np.uint8))
        coord = [fl % nx, (fl // nx) % ny, fl // (nx * ny)]
        k = 2 * math.pi / L
        u0 = np.zeros((3, s.nf))
        u0[AX[comp]] = 1e-4 * np.sin(k * (coord[AX[wave]] + 0.5))
        s.init_equilibrium(None, u0)
        s.flow_steps(10)
        a0 = np.abs(s.velocity()[AX[comp]]).max()
        T = 200
        s.flow_steps(T)
        u1 = s.velocity()
        a1 = np.abs(u1[AX[comp]]).max()
        for a in range(3):
            if a != AX[comp]:
                assert np.abs(u1[a]).max() < 1e-10 * 1e-4
        rates.append((-math.log(a1 / a0) / T) / (nu * k * k) - 1.0)
    assert abs(rates[1]) < 5e-3
    assert abs(rates[0] / rates[1]) > 3.0


def test_d3q19_mass_conserved_with_body_force():
    nx = ny = nz = 24
    prims = oracle.spheres(nx, ny, nz, 2, 2110, 0.6, 2.0, 4.0)
    lab = oracle.voxelize(3, nx, ny, nz, 0, 2, prims)
    cfg = OracleCfg(dim=3, nx=nx, ny=ny, nz=nz, drive=DRIVE_BODY_FORCE, tau=1.0, force=(1e-5, 2e-6, -3e-6),
                    u_in=0.0)
    s = OracleSolver(cfg, lab)
    m0 = s.density().sum()
    s.flow_steps(200)
    m1 = s.density().sum()
    assert abs(m1 - m0) / m0 < 1e-13
    u = s.velocity()
    assert u[0].mean() > 0 and u[1].mean() > 0 and u[2].mean() < 0


@pytest.mark.parametrize("dim,wave,comp", [(3, "z", "x"), (3, "y", "z"), (3, "x", "y"), (2, "y", "x"),
                                           (2, "x", "y")])
def test_shear_wave_is_carried_by_a_mean_flow(dim, wave, comp):
    # With the quadratic equilibrium the scheme is Galilean invariant to
    # second order: a shear wave u_comp = A sin(k wave) on a uniform mean flow
    # U along `wave` travels with it, so its phase turns by k U t. This fixes
    # the direction in which populations stream along every axis (a stream
    # along -e_i, mirrored consistently, passes the symmetric tests above).
    tau, L, U, T = 0.8, 32, 0.05, 100
    n = [4, 2, 2] if dim == 3 else [4, 2, 1]
    n[AX[wave]] = L
    nx, ny, nz = n
    cfg = OracleCfg(dim=dim, nx=nx, ny=ny, nz=nz, drive=DRIVE_BODY_FORCE, tau=tau, u_in=0.0)
    lab = np.zeros(nx * ny * nz, np.uint8)
    s = OracleSolver(cfg, lab)
    m, fl = oracle.compact(lab)
    coord = [fl % nx, (fl // nx) % ny, fl // (nx * ny)]
    k = 2 * math.pi / L
    u0 = np.zeros((dim, s.nf))
    u0[AX[comp]] = 1e-4 * np.sin(k * coord[AX[wave]])
    u0[AX[wave]] = U
    s.init_equilibrium(None, u0)

    def phase():
        u = s.velocity()[AX[comp]]
        line = np.array([u[coord[AX[wave]] == c].mean() for c in range(L)])
        return np.angle(np.fft.fft(line)[1])

    p0 = phase()
    s.flow_steps(T)
    turn = (phase() - p0 + math.pi) % (2 * math.pi) - math.pi
    assert abs(turn / (-k * U * T) - 1) < 0.02, turn
