"""cdi_solve_potential_noalloc (the library's own scratch, no workspace)
against cdi_solve_potential (a caller workspace) through the C ABI: the same
potential, bit for bit, on two calls in a row, the second on a smaller
lattice; a lattice whose workspace exceeds the scratch is refused."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2110_13055_amd")
from paper_2110_13055_amd import _lib as L  # noqa: E402
from paper_2110_13055_amd import Geometry, Params, Potential, Solver  # noqa: E402


def _solver(n, seed):
    g = Geometry(dim=3, nx=n, ny=n - 4, nz=n - 6, kind=L.SPHERES, porosity=0.5, r_min=3.0, r_max=6.0,
                 buffer_x=2, seed=seed)
    s = Solver(g, Params(u_in=5e-4, dpsi_vt=20.0))
    s.flow_steps(20)
    s.np_step(30, fused=True)   # a nonuniform charge for the Poisson term
    return s


@pytest.mark.parametrize("kappa2", [0.0, 0.3])
def test_noalloc_solve_equals_the_workspace_solve(kappa2):
    pot = Potential(psi_electrode=-3.0, x_bc=(L.PSIX_DIRICHLET, L.PSIX_NEUMANN), kappa2=kappa2, tol=1e-10,
                    warm_start=False)
    for n, seed in ((56, 3), (36, 4)):       # the second call on a smaller lattice
        print(f"noalloc potential n={n} kappa2={kappa2}", flush=True)
        s = _solver(n, seed)
        it_ws, r_ws = s.solve_potential(pot)
        psi_ws = s.potential()
        it_na, r_na = s.solve_potential_noalloc(pot)
        psi_na = s.potential()
        assert it_na == it_ws and r_na == r_ws
        assert np.array_equal(psi_na, psi_ws)
        assert np.abs(psi_ws).max() > 0.5


def test_noalloc_refuses_a_lattice_beyond_its_scratch():
    g = Geometry(dim=3, nx=160, ny=160, nz=160, kind=L.SPHERES, porosity=0.6, r_min=3.0, r_max=6.0, buffer_x=2,
                 seed=5)
    s = Solver(g, Params(u_in=5e-4))
    with pytest.raises(L.CdiError) as e:
        s.solve_potential_noalloc(Potential(psi_electrode=-1.0, x_bc=(L.PSIX_DIRICHLET, L.PSIX_NEUMANN)))
    assert e.value.code == L.E_BUFFER
