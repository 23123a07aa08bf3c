"""Serving on the GPU: requests arriving while others run are admitted into the
running batches; every result equals that of the same request served alone,
bit for bit, and one of them is checked against the FP64 oracle."""
import numpy as np
import pytest

from helpers import oracle_solver, rel_l2

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2110_13055_amd")
from paper_2110_13055_amd import _lib as L  # noqa: E402
from paper_2110_13055_amd import Geometry, Params  # noqa: E402
from paper_2110_13055_amd.serving import GpuExecutor, Request, Server, latency_stats  # noqa: E402


def trace(precision=L.FP32):
    rng = np.random.default_rng(7)
    out = []
    for k in range(6):
        if k % 2 == 0:
            g = Geometry(dim=2, nx=64 + 16 * k, ny=48, kind=L.DISKS, porosity=0.7, r_min=3.0, r_max=6.0,
                         min_gap=2.0, walls_y=1, buffer_x=2, seed=2110 + k)
        else:
            e = 20 + 4 * k
            g = Geometry(dim=3, nx=e, ny=e, nz=e, kind=L.SPHERES, porosity=float(rng.uniform(0.45, 0.7)),
                         r_min=2.0, r_max=4.0, buffer_x=2, seed=2110 + k)
        p = Params(u_in=float(rng.uniform(2e-4, 2e-3)), dpsi_vt=float(rng.uniform(4, 30)),
                   D=(0.05, 0.076), precision=precision)
        out.append(Request(k, 0.03 * k, g, p, flow_tol=1e-5, flow_max_steps=500, np_steps=150 + 50 * k))
    return out


class RoundClock:
    """Virtual time: 10 ms per served round plus any idle wait, so arrivals
    land between rounds the same way on every run."""

    def __init__(self):
        self.srv, self.idle = None, 0.0

    def __call__(self):
        return 0.01 * self.srv.rounds + self.idle

    def sleep(self, dt):
        self.idle += dt


def serve(reqs):
    ex = GpuExecutor(keep_fields=True)
    clock = RoundClock()
    srv = Server(ex, budget_bytes=8e9, max_slots=8, round_steps=50, clock=clock, sleep=clock.sleep)
    clock.srv = srv
    res = {r.rid: r for r in srv.run(reqs)}
    ex.close()
    return srv, res


@pytest.mark.parametrize("precision", [L.FP32, L.FP16, L.FP16_DEV, L.MOMENTS])
def test_served_results_alone_equal_mix(precision):
    reqs = trace(precision)
    srv, mix = serve(reqs)
    assert srv.backlog == 0 and srv.peak_slots >= 3 and srv.used == 0
    # a flow that stopped at its step budget short of 1e-5 is delivered as unconverged
    assert all(r.status in ("ok", "ok_unconverged") for r in mix.values())
    st = latency_stats(list(mix.values()), wall_s=1.0)
    assert st["completed"] == len(reqs)
    for r in reqs:
        solo, alone = serve([r])
        a, m = alone[r.rid], mix[r.rid]
        assert (a.flow_steps, a.np_steps, a.residual) == (m.flow_steps, m.np_steps, m.residual)
        assert a.adsorbed == m.adsorbed and a.balance == m.balance
        for name in ("concentration", "velocity"):
            assert np.array_equal(solo.fields[r.rid][name], srv.fields[r.rid][name]), (r.rid, name)


def test_served_result_matches_oracle():
    reqs = trace()
    srv, mix = serve(reqs)
    for rid in (0, 3):
        r, m = reqs[rid], mix[rid]
        o = oracle_solver(r.geom, r.params)
        o.flow_steps(m.flow_steps)
        o.freeze_velocity()
        assert o.np_steps(m.np_steps) == 0
        assert rel_l2(srv.fields[rid]["velocity"], o.velocity()) <= 1e-5
        assert np.abs(srv.fields[rid]["concentration"] - o.conc()).max() <= 1e-4
        oa = o.adsorbed_total()
        assert np.all(np.abs(np.array(m.adsorbed) - oa) <= 1e-4 * np.abs(oa))
