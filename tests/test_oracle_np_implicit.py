"""Pins of the CPU reference's implicit ion transport (the paper's time scheme,
Sec. 2: an implicit finite-volume method) and its steady state.

The steady solve equals a direct sparse solve of the face-flux system written
out independently (``_assemble`` of test_oracle_np.py) and is a fixed point of
the explicit step. Backward-Euler steps follow the exact discrete transient
of the periodic scheme (Fourier amplification 1/(1 + dt lambda_k)), conserve
solute + adsorbed + outflow - inflow exactly, stay within [0, c0] far beyond
the explicit step limit, and march to the steady state.
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
from oracle import OracleCfg, OracleSolver, NPX_INLET_OUTLET, NPX_PERIODIC, DRIVE_INLET_OUTLET
from test_oracle_np import _assemble, _line, _porous_2d, bern


def _flowing(nx=32, ny=20, dpsi=8.0, u_in=3e-3):
    lab = _porous_2d(nx, ny)
    cfg = OracleCfg(dim=2, nx=nx, ny=ny, drive=DRIVE_INLET_OUTLET, u_in=u_in, dpsi=dpsi, D=(0.05, 0.076),
                    np_x_bc=NPX_INLET_OUTLET)
    s = OracleSolver(cfg, lab)
    s.flow_to_steady(tol=1e-9, max_steps=200000, check_every=100)
    s.freeze_velocity()
    return s, lab, cfg


def test_steady_solve_equals_sparse_direct_solve_and_is_a_fixed_point():
    nx, ny, dpsi, u_in = 32, 20, 8.0, 3e-3
    s, lab, _ = _flowing(nx, ny, dpsi, u_in)
    u = s.np_velocity()
    _, fl = oracle.compact(lab)

    def ramp(x):
        return dpsi * (1 - (x + 0.5) / nx)
    psi_cells = ramp(fl % nx)
    direct = []
    for D, z in ((0.05, 1), (0.076, -1)):
        keff = s.ka * D / (D + s.ka / 2)
        A, b = _assemble(lab, nx, ny, u, psi_cells, ramp, D, z, 1.0, keff, u_in)
        direct.append(spla.spsolve(A.tocsc(), b))
    direct = np.array(direct)
    rc, it = s.np_steady(tol=1e-13)
    assert rc == 0 and it > 5
    assert np.abs(s.conc() - direct).max() < 1e-10
    # a fixed point of the explicit step; its rates balance
    c = s.conc().copy()
    assert s.np_steps(1) == 0
    assert np.abs(s.conc() - c).max() < 1e-12
    r = s.np_rates()
    assert np.allclose(r[:, 1] - r[:, 2], r[:, 0], rtol=1e-9)


def test_backward_euler_fourier_amplification():
    N, D, w, n, dt = 32, 0.08, 0.03, 20, 7.5  # dt far beyond the explicit limit 1 / (2 D)
    cfg = OracleCfg(dim=2, nx=N, ny=1, D=(D, D), u_in=0.0, np_x_bc=NPX_PERIODIC)
    s = OracleSolver(cfg, _line(N))
    s.set_velocity(np.vstack([np.full(N, w), np.zeros(N)]))
    rng = np.random.default_rng(0)
    c0 = 1.0 + 0.5 * rng.random((2, N))
    s.set_conc(c0)
    rc, _ = s.np_implicit(dt, n, tol=1e-14)
    assert rc == 0
    pe = w / D
    k = 2 * np.pi * np.fft.fftfreq(N)
    # outflow operator symbol: D (B(-pe) + B(pe)) - D B(pe) e^{ik} - D B(-pe) e^{-ik}
    lam = D * (bern(-pe) + bern(pe)) - D * bern(pe) * np.exp(1j * k) - D * bern(-pe) * np.exp(-1j * k)
    ref = np.real(np.fft.ifft((1.0 / (1.0 + dt * lam)) ** n * np.fft.fft(c0[0])))
    assert np.abs(s.conc()[0] - ref).max() < 1e-11


def test_backward_euler_conserves_and_stays_positive_at_large_steps():
    s, _, _ = _flowing(dpsi=20.0, u_in=2e-3)
    m0 = s.balance()[:, 0].copy()
    rc, _ = s.np_implicit(25.0, 40, tol=1e-13)
    assert rc == 0
    b = s.balance()
    M, A, In, Out = b[:, 0], b[:, 1], b[:, 2], b[:, 3]
    assert np.all(np.abs(M + A + Out - In - m0) <= 1e-10 * m0)
    c = s.conc()
    assert c.min() >= -1e-12 and np.all(A > 0)


def test_backward_euler_marches_to_the_steady_state():
    s, _, _ = _flowing()
    t = _flowing()[0]
    assert t.np_steady(tol=1e-13)[0] == 0
    cstar = t.conc()
    errs = []
    for _ in range(3):
        assert s.np_implicit(200.0, 10, tol=1e-13)[0] == 0
        errs.append(np.abs(s.conc() - cstar).max())
    assert errs[0] > errs[1] > errs[2] and errs[2] < 0.05 * errs[0]


def test_backward_euler_is_first_order_in_time():
    # against the explicit march with 32 sub-steps per unit time (its own
    # error is first order in 1/32): halving the implicit step halves the error
    T = 100
    ref, _, cfg = _flowing()
    ref32 = OracleSolver(OracleCfg(**{**cfg.__dict__, "np_substeps": 32}), ref.labels)
    ref32.flow_to_steady(tol=1e-9, max_steps=200000, check_every=100)
    ref32.freeze_velocity()
    assert ref32.np_steps(T) == 0
    errs = []
    for dt in (1.0, 0.5):
        s = _flowing()[0]
        assert s.np_implicit(dt, int(T / dt), tol=1e-13)[0] == 0
        errs.append(np.abs(s.conc() - ref32.conc()).max())
    assert 1.6 < errs[0] / errs[1] < 2.4
