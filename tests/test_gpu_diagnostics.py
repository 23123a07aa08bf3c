"""Diagnostics of Sec. 4 on the GPU against the FP64 oracle: electrode face
count and inlet count (exact integers), l_c, U, Pe, Da (U from FP32 state:
relative 1e-5, the velocity bar), vertical concentration profiles (the
concentration bar 1e-4 c0, counts exact) and salt removal over a window
(relative 1e-4, the accumulator bar). At the full 512^3 size the counts are
checked against an independent numpy count on the labels."""
import numpy as np
import pytest

from helpers import oracle_solver

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2110_13055_amd")
from paper_2110_13055_amd import _lib as L  # noqa: E402
from paper_2110_13055_amd import Geometry, Params, Solver, fibre_case, preset  # noqa: E402


def cases():
    g2, p2, _ = preset("channel2d_128x64")
    g3 = Geometry(dim=3, nx=40, ny=33, nz=29, kind=L.SPHERES, porosity=0.55, r_min=2.5, r_max=5.0, buffer_x=2,
                  seed=4)
    p3 = Params(u_in=5e-4, dpsi_vt=8.0, D=(0.05, 0.076))
    gf = Geometry(dim=3, nx=44, ny=36, nz=31, kind=L.FIBRES, porosity=0.7, r_min=2.0, r_max=2.0, buffer_x=2,
                  seed=6)
    gb = Geometry(dim=3, nx=32, ny=24, nz=24, kind=L.SPHERES, porosity=0.6, r_min=2.0, r_max=4.0, buffer_x=0,
                  seed=8)
    pb = Params(drive=L.BODY_FORCE, body_force=(1e-6, 0.0, 0.0), np_x_bc=L.NPX_PERIODIC, D=(0.05, 0.076))
    return [("2d", g2, p2), ("3d", g3, p3), ("fibres", gf, p3), ("periodic", gb, pb)]


@pytest.mark.parametrize("name,g,p", cases(), ids=lambda v: v if isinstance(v, str) else "")
def test_diagnostics_match_oracle(name, g, p):
    s = Solver(g, p)
    o = oracle_solver(g, p)
    s.flow_steps(300)
    o.flow_steps(300)
    d, do = s.diagnostics(), o.diagnostics()
    assert d["n_surface"] == do["n_surface"] and d["n_inlet"] == do["n_inlet"]
    assert d["l_c"] == pytest.approx(do["l_c"], rel=1e-14)
    assert d["U"] == pytest.approx(do["U"], rel=1e-5)
    for k in range(2):
        assert d["Pe"][k] == pytest.approx(do["Pe"][k], rel=1e-5)
        assert d["Da"][k] == pytest.approx(do["Da"][k], rel=1e-6)
    assert s.diagnostics() == d  # fixed-order sums: repeatable


@pytest.mark.parametrize("name,g,p", cases()[:3], ids=lambda v: v if isinstance(v, str) else "")
def test_profile_and_salt_removal_match_oracle(name, g, p):
    s = Solver(g, p)
    o = oracle_solver(g, p)
    s.flow_steps(400)
    o.flow_steps(400)
    o.freeze_velocity()
    s.np_step(300)
    assert o.np_steps(300) == 0
    b0, ob0 = s.mass_balance(), o.balance()
    s.np_step(200)
    assert o.np_steps(200) == 0
    pr, po = s.profile_x(), o.profile_x()
    assert np.array_equal(pr[2], po[2])
    assert np.abs(pr[:2] - po[:2]).max() <= 1e-4
    d = s.diagnostics()
    prm = s.salt_removal(b0, s.mass_balance(), 200, d["n_inlet"], d["U"])
    prm_o = o.salt_removal(ob0, o.balance(), 200, d["n_inlet"], d["U"])
    assert np.abs(prm - prm_o).max() <= 1e-4 * max(1.0, np.abs(prm_o).max())


def _numpy_counts(lab, nx, ny, nz):
    L3 = lab.reshape(nz, ny, nx)
    fluid = L3 == 0
    elec = L3 == 1
    faces = 0
    for ax in (1, 0):  # y and z wrap
        for sh in (1, -1):
            faces += int((fluid & np.roll(elec, sh, axis=ax)).sum())
    faces += int((fluid[:, :, 1:] & elec[:, :, :-1]).sum()) + int((fluid[:, :, :-1] & elec[:, :, 1:]).sum())
    return faces, fluid.sum(axis=(0, 1))


@pytest.mark.parametrize("which", ["spheres3d_512", "fibres150_d6_phi06"])
def test_full_size_counts_against_numpy(which):
    if which == "spheres3d_512":
        g, p, _ = preset("spheres3d_512")
    else:
        g, p = fibre_case(6, 0.6)
    s = Solver(g, p)
    lab = s.labels()
    faces, per_x = _numpy_counts(lab, g.nx, g.ny, g.nz)
    d = s.diagnostics()
    assert d["n_surface"] == faces
    assert d["n_inlet"] == per_x[0]
    pr = s.profile_x()
    assert np.array_equal(pr[2], per_x.astype(float))
    assert np.all(pr[:2][:, per_x > 0] == 1.0)  # the initial state is C = c0 everywhere
