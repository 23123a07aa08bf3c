"""FP32 populations stored relative to per-plane reference densities (renewed
at every residual check of a flow-to-steady call): the renewal is exact up to
rounding, so the flow and the ions stay on the FP64 oracle (which stores f
itself) through many renewals, for both streaming patterns (AA writes into
its neighbours' slots on odd steps, relative to their planes), with the
inlet/outlet and the periodic body-force drives; a renewal pending at the end
of a call is carried by snapshots and applied by whichever step comes next,
alone or in a batch, bit for bit."""
import numpy as np
import pytest

from helpers import oracle_solver, rel_l2

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2110_13055_amd")
from paper_2110_13055_amd import _lib as L  # noqa: E402
from paper_2110_13055_amd import Batch, Geometry, Params, Solver  # noqa: E402


def case(drive, streaming, seed=7):
    g = Geometry(dim=3, nx=40, ny=32, nz=28, kind=L.SPHERES, porosity=0.5, r_min=3.0, r_max=6.0, buffer_x=2,
                 seed=seed)
    if drive == L.BODY_FORCE:
        p = Params(drive=L.BODY_FORCE, body_force=(2e-5, 0.0, 0.0), u_in=0.0, dpsi_vt=20.0, streaming=streaming,
                   np_x_bc=L.NPX_PERIODIC)
    else:
        p = Params(u_in=1e-3, dpsi_vt=20.0, streaming=streaming)
    return g, p


@pytest.mark.parametrize("streaming", [L.STREAM_AA, L.STREAM_PULL], ids=["aa", "pull"])
@pytest.mark.parametrize("drive", [L.INLET_OUTLET, L.BODY_FORCE], ids=["inout", "bodyforce"])
def test_renewed_references_stay_on_the_oracle(drive, streaming):
    g, p = case(drive, streaming)
    print(f"plane refs drive={drive} streaming={streaming}", flush=True)
    s = Solver(g, p)
    o = oracle_solver(g, p)
    # 51 renewals (every 4 steps); the call ends on the step that stores the
    # state for the next renewal, which is then applied by the fused steps
    rc, steps, r = s.flow_to_steady(tol=0.0, max_steps=204, check_every=4)
    assert steps == 204
    o.flow_steps(204)
    assert rel_l2(s.velocity(), o.velocity()) <= 1e-5
    assert np.abs(s.density() - o.density()).max() <= 1e-6
    s.np_step(31, fused=True)
    assert o.np_steps(31, fused=True) == 0
    assert rel_l2(s.velocity(), o.velocity()) <= 1e-5
    assert np.abs(s.concentration() - o.conc()).max() <= 1e-4
    a, ao = s.adsorbed_total(), o.adsorbed_total()
    assert np.all(np.abs(a - ao) <= 1e-4 * np.abs(ao))


@pytest.mark.parametrize("streaming", [L.STREAM_AA, L.STREAM_PULL], ids=["aa", "pull"])
def test_pending_renewal_through_snapshot_and_batch(streaming):
    g, p = case(L.INLET_OUTLET, streaming, seed=9)
    s = Solver(g, p)
    s.flow_to_steady(tol=0.0, max_steps=8, check_every=4)   # ends with a renewal pending
    blob = s.snapshot()
    t = Solver(g, p)
    t.restore(blob)
    s.flow_steps(5)
    t.flow_steps(5)
    assert np.array_equal(s.velocity(), t.velocity())
    # the same pending state advanced inside a batch (one member, then the pair replay)
    u = Solver(g, p)
    u.restore(blob)
    b = Batch([u])
    b.advance(5, [L.MODE_FLOW])
    b.close()
    assert np.array_equal(s.velocity(), u.velocity())
