"""Pins of the CPU reference's Nernst-Planck update (Eq. 3) with adsorption
(Eq. 6) on its y and z faces and in 3D, and of its open outlet.

* Uniform drift along y or z on a periodic line: the exact discrete transient
  from the scheme's Fourier amplification factor (advection, diffusion and
  the sign convention of each axis's faces).
* A closed porous box in a random potential field, no flow: at the steady
  state every fluid-fluid face carries the Boltzmann ratio of Eq. (9),
  C_N / C_P = exp(-z (psi_N - psi_P)), on x, y and z faces alike.
* A line of cells along x between two adsorbing electrode faces normal to y
  or to z, fed at the inlet, with a uniform drift that leaves through the
  open outlet or enters through it: the steady profile is the closed-form
  solution of the face-balance recurrence (two characteristic roots fixed
  by the inlet ghost and the outlet face). Inflow through the outlet carries
  the feed concentration (the outlet reading), so the inflowing case fixes
  that reading.
* Mirror symmetry of the ions (the electrode mirrored in y or z).
"""
import math

import numpy as np
import pytest

import oracle
from oracle import OracleCfg, OracleSolver, DRIVE_INLET_OUTLET, NPX_CLOSED, NPX_INLET_OUTLET, NPX_PERIODIC

AX = {"x": 0, "y": 1, "z": 2}


def bern(x):
    x = float(x)
    return 1.0 if x == 0 else x / math.expm1(x)


def _coords(fl, nx, ny):
    return [fl % nx, (fl // nx) % ny, fl // (nx * ny)]


@pytest.mark.parametrize("dim,axis", [(3, "y"), (3, "z"), (2, "y")])
@pytest.mark.parametrize("w", [0.03, -0.02])
def test_uniform_drift_transient_along_an_axis(dim, axis, w):
    N, D, n = 32, 0.08, 50
    dims = [4, 2, 2] if dim == 3 else [4, 2, 1]
    dims[AX[axis]] = N
    nx, ny, nz = dims
    lab = np.zeros(nx * ny * nz, np.uint8)
    cfg = OracleCfg(dim=dim, nx=nx, ny=ny, nz=nz, D=(D, D), u_in=0.0, np_x_bc=NPX_PERIODIC)
    s = OracleSolver(cfg, lab)
    m, fl = oracle.compact(lab)
    c = _coords(fl, nx, ny)
    u = np.zeros((dim, s.nf))
    u[AX[axis]] = w
    s.set_velocity(u)
    rng = np.random.default_rng(11)
    line = 1.0 + 0.5 * rng.random((2, N))
    s.set_conc(line[:, c[AX[axis]]])
    assert s.np_steps(n) == 0
    pe = w / D
    k = 2 * np.pi * np.fft.fftfreq(N)
    # one step: C_j -= D[B(-pe) C_j - B(pe) C_{j+1}] + D[B(pe) C_j - B(-pe) C_{j-1}]
    G = 1 - D * (bern(-pe) + bern(pe)) + D * bern(pe) * np.exp(1j * k) + D * bern(-pe) * np.exp(-1j * k)
    for sp in range(2):
        ref = np.real(np.fft.ifft(G ** n * np.fft.fft(line[sp])))
        assert np.abs(s.conc()[sp] - ref[c[AX[axis]]]).max() < 1e-12


def test_boltzmann_ratio_on_every_face_in_a_random_potential():
    # Closed box (closed x ends, blocking electrode voxels, periodic y and z),
    # no flow, an arbitrary potential field: the steady state satisfies the
    # Boltzmann law face by face, whatever the connectivity of the pores.
    nx, ny, nz = 8, 6, 6
    rng = np.random.default_rng(5)
    lab = (rng.random(nx * ny * nz) < 0.2).astype(np.uint8)       # electrode voxels
    m, fl = oracle.compact(lab)
    nf = fl.size
    psi = rng.uniform(-0.75, 0.75, nf)
    cfg = OracleCfg(dim=3, nx=nx, ny=ny, nz=nz, D=(0.05, 0.05), u_in=0.0, np_x_bc=NPX_CLOSED,
                    no_adsorption=1)
    s = OracleSolver(cfg, lab, psi=psi)
    s.set_velocity(np.zeros((3, nf)))
    m0 = s.balance()[:, 0].copy()
    assert s.np_stability() <= 1.0
    assert s.np_steps(30000) == 0
    C = s.conc()
    c = _coords(fl, nx, ny)
    checked = 0
    for a, n_a in ((0, nx), (1, ny), (2, nz)):
        for p in range(nf):
            q = [c[0][p], c[1][p], c[2][p]]
            q[a] += 1
            if a == 0 and q[0] >= nx:
                continue                                          # closed x end
            q[a] %= n_a
            v = (q[2] * ny + q[1]) * nx + q[0]
            if lab[v] != 0:
                continue
            j = m[v]
            for sp, z in ((0, 1), (1, -1)):
                assert abs(C[sp, j] / C[sp, p] - math.exp(-z * (psi[j] - psi[p]))) < 1e-11
                checked += 1
    assert checked > 3 * nf
    b = s.balance()
    assert np.allclose(b[:, 0], m0, rtol=1e-13) and np.all(b[:, 1] == 0)


def _side_channel(side, L, nother=2):
    """Cells (x, 1) for x < L between electrode voxels at side = 0 and 2;
    the third axis (nother cells) is all fluid and periodic."""
    dims = [L, nother, nother]
    dims[AX[side]] = 3
    nx, ny, nz = dims
    lab = np.zeros((nz, ny, nx), np.uint8)
    idx = [slice(None)] * 3
    for v in (0, 2):
        idx[2 - AX[side]] = v
        lab[tuple(idx)] = 1
    return nx, ny, nz, lab.reshape(-1)


def _closed_form_profile(L, D, k, w, c0):
    """Steady face balance of the line: interior Scharfetter-Gummel fluxes
    with drift w, inlet ghost at c0, two adsorbing side faces (k C each) per
    cell, open outlet max(w,0) C + min(w,0) c0."""
    pe = w / D
    bm, bp = bern(-pe), bern(pe)
    # C_i = a l1^i + b l2^i solves D bm C_i - D bp C_{i+1} - D bm C_{i-1} + D bp C_i + 2 k C_i = 0
    A2, A1, A0 = -D * bp, D * (bm + bp) + 2 * k, -D * bm
    disc = math.sqrt(A1 * A1 - 4 * A2 * A0)
    l1, l2 = (-A1 + disc) / (2 * A2), (-A1 - disc) / (2 * A2)
    i = np.arange(L, dtype=float)
    # rows: ghost C_{-1} = c0; last cell's balance
    #   max(w,0) C_{L-1} + min(w,0) c0 - D(bm C_{L-2} - bp C_{L-1}) + 2 k C_{L-1} = 0
    def last(l):
        return max(w, 0.0) * l ** (L - 1) - D * (bm * l ** (L - 2) - bp * l ** (L - 1)) + 2 * k * l ** (L - 1)
    M = np.array([[1 / l1, 1 / l2], [last(l1), last(l2)]])
    rhs = np.array([c0, -min(w, 0.0) * c0])
    a, b = np.linalg.solve(M, rhs)
    return a * l1 ** i + b * l2 ** i


@pytest.mark.parametrize("side", ["y", "z"])
@pytest.mark.parametrize("w", [0.0, 0.02, -0.02])
def test_side_adsorption_and_open_outlet_closed_form(side, w):
    L, D, Ka, c0 = 16, 0.1, 0.01, 1.0
    nx, ny, nz, lab = _side_channel(side, L)
    cfg = OracleCfg(dim=3, nx=nx, ny=ny, nz=nz, D=(D, D), u_in=w, Ka=Ka, c0=c0, np_x_bc=NPX_INLET_OUTLET)
    s = OracleSolver(cfg, lab)
    m, fl = oracle.compact(lab)
    u = np.zeros((3, s.nf))
    u[0] = w
    s.set_velocity(u)
    assert s.np_steps(60000) == 0
    keff = Ka * D / (D + Ka / 2)
    ref = _closed_form_profile(L, D, keff, w, c0)
    C = s.conc()
    x = fl % nx
    for sp in range(2):
        assert np.abs(C[sp] - ref[x]).max() < 1e-12
    # rates at the steady state: inflow - outflow = adsorption, each as the
    # closed form gives it (per line of cells, times the lines)
    lines = s.nf // L
    b0 = s.balance()
    s.np_steps(10)
    r = (s.balance() - b0) / 10 / lines
    pe = w / D
    fin = D * (bern(-pe) * c0 - bern(pe) * ref[0])
    fout = max(w, 0.0) * ref[-1] + min(w, 0.0) * c0
    for sp in range(2):
        assert abs(r[sp, 1] - 2 * keff * ref.sum()) < 1e-12
        assert abs(r[sp, 2] - fin) < 1e-12
        assert abs(r[sp, 3] - fout) < 1e-12


def test_outlet_inflow_differs_from_a_zero_gradient_ghost():
    # the two outlet readings differ for inflow: the pin above distinguishes
    # them by more than its tolerance
    L, D, k = 16, 0.1, 0.01 * 0.1 / (0.1 + 0.005)
    feed = _closed_form_profile(L, D, k, -0.02, 1.0)
    pe = -0.02 / D
    # zero-gradient ghost: inflow carries C_{L-1}; same recurrence, last row
    # max(w,0) C + min(w,0) C
    bm, bp = bern(-pe), bern(pe)
    A = np.zeros((L, L))
    rhs = np.zeros(L)
    for i in range(L):
        A[i, i] += D * bp + 2 * k
        if i > 0:
            A[i, i - 1] -= D * bm
        else:
            rhs[i] += D * bm * 1.0
        if i < L - 1:
            A[i, i] += D * bm
            A[i, i + 1] -= D * bp
        else:
            A[i, i] += -0.02
    zg = np.linalg.solve(A, rhs)
    assert np.abs(feed - zg).max() > 1e-3


@pytest.mark.parametrize("axis", ["y", "z"])
def test_ions_mirror_with_the_electrode(axis):
    nx, ny, nz = 24, 20, 16
    prims = oracle.spheres(nx, ny, nz, 2, 2110, 0.55, 2.0, 4.0)
    lab = oracle.voxelize(3, nx, ny, nz, 0, 2, prims).reshape(nz, ny, nx)
    lab_m = (lab[:, ::-1, :] if axis == "y" else lab[::-1, :, :]).copy()
    cfg = OracleCfg(dim=3, nx=nx, ny=ny, nz=nz, drive=DRIVE_INLET_OUTLET, u_in=2e-3, dpsi=20.0,
                    D=(0.05, 0.076))
    out = []
    for L_ in (lab, lab_m):
        s = OracleSolver(cfg, L_.reshape(-1))
        s.flow_steps(150)
        assert s.np_steps(150, fused=True) == 0
        C = np.zeros((2, nz, ny, nx))
        C[:, L_ == 0] = s.conc()
        out.append((C, s.adsorbed_total(), s.balance()))
    (Ca, Aa, ba), (Cb, Ab, bb) = out
    Cb = Cb[:, :, ::-1, :] if axis == "y" else Cb[:, ::-1, :, :]
    assert np.abs(Ca - Cb).max() <= 1e-12
    assert np.allclose(Aa, Ab, rtol=1e-12, atol=0)
    assert np.allclose(ba, bb, rtol=1e-12, atol=1e-300)
    assert Aa.min() > 0
