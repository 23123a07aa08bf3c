"""Straight-fibre electrodes (Sec. 5) on the GPU: labels, fluid numbering and
a short coupled run against the FP64 oracle. Labels and numbering are exact
integer work: bitwise."""
import numpy as np
import pytest

import oracle
from helpers import oracle_labels, oracle_solver, rel_l2

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2110_13055_amd")
from paper_2110_13055_amd import _lib as L  # noqa: E402
from paper_2110_13055_amd import Geometry, Params, Solver, fibre_case  # noqa: E402


@pytest.mark.parametrize("shape,seed,phi,r", [((48, 40, 36), 1, 0.7, (1.5, 3.0)), ((37, 29, 41), 2, 0.5, (2.0, 2.0)),
                                              ((64, 64, 64), 3, 0.8, (4.0, 4.0))])
def test_fibre_labels_bitwise(shape, seed, phi, r):
    nx, ny, nz = shape
    g = Geometry(dim=3, nx=nx, ny=ny, nz=nz, kind=L.FIBRES, porosity=phi, r_min=r[0], r_max=r[1], buffer_x=2,
                 seed=seed)
    s = Solver(g, Params())
    ref = oracle_labels(g)
    assert np.array_equal(s.labels(), ref)
    m, f = s.fluid_index()
    om, of = oracle.compact(ref)
    assert np.array_equal(m, om) and np.array_equal(f, of)


@pytest.mark.parametrize("diameter,phi", [(4, 0.5), (8, 0.8)])
def test_sweep_size_fibre_labels_bitwise(diameter, phi):
    g, p = fibre_case(diameter, phi)
    s = Solver(g, p)
    ref = oracle_labels(g)
    assert np.array_equal(s.labels(), ref)
    assert abs((ref == 0).mean() - phi) < 0.02


def test_fibre_electrode_flow_and_ions_match_oracle():
    g = Geometry(dim=3, nx=40, ny=32, nz=30, kind=L.FIBRES, porosity=0.65, r_min=2.0, r_max=2.0, buffer_x=2,
                 seed=11)
    p = Params(u_in=5e-4, dpsi_vt=10.0, D=(0.05, 0.076))
    s = Solver(g, p)
    o = oracle_solver(g, p)
    s.flow_steps(200)
    o.flow_steps(200)
    assert rel_l2(s.velocity(), o.velocity()) <= 1e-5
    s.np_step(150, fused=True)
    assert o.np_steps(150, fused=True) == 0
    assert np.abs(s.concentration() - o.conc()).max() <= 1e-4
    ao = o.adsorbed_total()
    assert np.all(np.abs(s.adsorbed_total() - ao) <= 1e-4 * np.abs(ao))
