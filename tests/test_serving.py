"""Serving scheduler on the CPU: admission by footprint and slots, FIFO order,
phase switching, latency accounting, failure isolation, backlog at a horizon,
and (with an executor backed by the FP64 oracle) that a request's result is
the same alone and in the mix."""
import math

import numpy as np
import pytest

from paper_2110_13055_amd import _lib as L
from paper_2110_13055_amd.serving import Request, Server, latency_stats, poisson_arrivals

FLOW, IONS = L.MODE_FLOW, L.MODE_IONS


class Clock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeHandle:
    def __init__(self, req):
        self.req = req
        self.flow = 0
        self.ions = 0


class FakeExecutor:
    """Cost model: a step costs nodes * ns_per_node of virtual time (groups
    overlap, so a round costs its slowest group); the residual after t flow
    steps is exp(-t / decay)."""

    def __init__(self, clock, ns_per_node=1.0, fail_start=(), fail_ions=()):
        self.clock = clock
        self.ns = ns_per_node
        self.fail_start = set(fail_start)
        self.fail_ions = set(fail_ions)
        self.started = []
        self.live = {}
        self.log = []          # (active rids, bytes in use) per round

    @staticmethod
    def nodes(req):
        return req.geom["nodes"]

    def footprint_estimate(self, req):
        return req.geom["bytes"]

    def footprint(self, h):
        return h.req.geom["bytes"]

    def work_estimate(self, req):
        return req.geom["nodes"]

    def work(self, h):
        return h.req.geom["nodes"]

    def start(self, req):
        if req.rid in self.fail_start:
            raise RuntimeError("geometry could not be generated")
        h = FakeHandle(req)
        self.started.append(req.rid)
        self.live[req.rid] = h
        return h

    def group_key(self, h):
        return h.req.geom["dim"]

    def advance(self, groups, modes, n):
        self.log.append((sorted(h.req.rid for g in groups.values() for h in g),
                         sum(h.req.geom["bytes"] for g in groups.values() for h in g)))
        res, failed, cost = {}, {}, 0.0
        for key, members in groups.items():
            bad = [k for k, (h, m) in enumerate(zip(members, modes[key]))
                   if m == IONS and h.req.rid in self.fail_ions]
            if bad:
                failed[key] = (bad[0], f"member {bad[0]}: positivity bound violated")
                continue
            r = np.full(len(members), np.nan)
            for k, (h, m) in enumerate(zip(members, modes[key])):
                if m == FLOW:
                    h.flow += n
                    r[k] = math.exp(-h.flow / h.req.geom["decay"])
                else:
                    h.ions += n
            res[key] = r
            cost = max(cost, n * sum(self.nodes(h.req) for h in members) * self.ns * 1e-9)
        self.clock.t += cost
        return res, failed

    def finish(self, h):
        return {"adsorbed": (h.flow * 1.0, h.ions * 2.0), "balance": np.zeros((2, 4))}

    def release(self, h):
        del self.live[h.req.rid]


def req(rid, t, nodes=1e6, nbytes=1e9, decay=1000.0, dim=3, np_steps=1000, tol=1e-3, fmax=10 ** 6):
    return Request(rid, t, dict(nodes=nodes, bytes=nbytes, decay=decay, dim=dim), None,
                   flow_tol=tol, flow_max_steps=fmax, np_steps=np_steps)


def serve(reqs, **kw):
    clock = Clock()
    ex = FakeExecutor(clock, **{k: kw.pop(k) for k in ("fail_start", "fail_ions") if k in kw})
    srv = Server(ex, clock=clock, sleep=clock.sleep, **kw)
    return srv, ex, clock


def test_all_served_with_phase_switch_and_step_counts():
    reqs = [req(k, 0.1 * k, decay=500.0 + 100 * k) for k in range(6)]
    srv, ex, _ = serve(reqs, round_steps=100)
    out = {r.rid: r for r in srv.run(reqs)}
    assert sorted(out) == list(range(6)) and srv.backlog == 0 and not ex.live
    for k, r in out.items():
        decay = 500.0 + 100 * k
        want_flow = 100 * math.ceil(decay * math.log(1e3) / 100)   # first round with exp(-t/decay) <= 1e-3
        assert r.status == "ok" and r.flow_steps == want_flow and r.flow_stop == "tol"
        assert r.residual <= 1e-3
        assert r.np_steps == 1000 and r.adsorbed == (want_flow, 2000.0)
        assert r.finished_s >= r.admitted_s >= r.arrival_s
        assert r.latency_s == pytest.approx(r.finished_s - r.arrival_s)
    assert srv.peak_slots > 1   # later arrivals joined while others ran


def test_flow_budget_caps_the_flow_phase():
    # the flow stops short of its tolerance: the result is delivered, marked
    # unconverged, with the residual it reached
    reqs = [req(0, 0.0, decay=1e9, fmax=300)]
    srv, _, _ = serve(reqs, round_steps=100)
    (r,) = srv.run(reqs)
    assert r.status == "ok_unconverged" and r.flow_steps == 300 and r.residual > 1e-3
    assert r.flow_stop == "step_limit"
    st = latency_stats([r], 1.0)
    assert st["completed"] == 1 and st["unconverged"] == 1 and st["failed"] == 0
    assert st["flow_stops"] == {"tol": 0, "stagnated": 0, "step_limit": 1}
    assert st["unconverged_residual_median"] == pytest.approx(r.residual)


def test_flow_that_stops_improving_is_marked_stagnated():
    class Flat(FakeExecutor):
        def advance(self, groups, modes, n):
            res, failed = super().advance(groups, modes, n)
            return {k: np.where(np.isnan(v), v, 0.5) for k, v in res.items()}, failed

    reqs = [req(0, 0.0)]
    clock = Clock()
    srv = Server(Flat(clock), clock=clock, sleep=clock.sleep, round_steps=100, stagnation_rounds=3)
    (r,) = srv.run(reqs)
    # the first round sets the best residual; three rounds without improvement end the phase
    assert r.status == "ok_unconverged" and r.flow_stop == "stagnated" and r.flow_steps == 400


def test_request_whose_electrode_cannot_be_planned_fails_alone():
    class Planning(FakeExecutor):
        def footprint_estimate(self, r):
            if r.rid == 1:
                raise RuntimeError("random sequential addition jammed before the porosity")
            return super().footprint_estimate(r)

    clock = Clock()
    ex = Planning(clock)
    reqs = [req(k, 0.0) for k in range(3)]
    out = {r.rid: r for r in Server(ex, clock=clock, sleep=clock.sleep, round_steps=100).run(reqs)}
    assert ex.started == [0, 2] and out[1].status.startswith("rejected: random sequential")
    assert out[0].status == out[2].status == "ok"


def test_unstable_flow_is_refused_before_it_takes_a_slot():
    class Checking(FakeExecutor):
        def check(self, r):
            return (r.rid != 1, "needs a density drop of 3")

    clock = Clock()
    ex = Checking(clock)
    reqs = [req(k, 0.0) for k in range(3)]
    srv = Server(ex, clock=clock, sleep=clock.sleep, round_steps=100)
    out = {r.rid: r for r in srv.run(reqs)}
    assert ex.started == [0, 2]                       # never started, never held a slot
    assert out[1].status.startswith("rejected: unstable flow") and out[1].footprint == 0
    assert out[0].status == out[2].status == "ok"
    assert latency_stats(list(out.values()), 1.0)["rejected"] == 1


def test_host_flow_check_refuses_the_divergent_request_type():
    # a low-porosity electrode fed fast: its steady flow would need the
    # density to drop by about 1.2 across it (the request that diverged when
    # admitted); the configurations of the benchmark protocols pass
    import paper_2110_13055_amd as P
    r9 = P.serving_requests(12)[9]
    ok, est, msg = P.flow_check(r9.geom, r9.params)
    assert not ok and 1.0 < est < 1.4 and "density drop" in msg
    for name in ("channel2d_128x64", "spheres3d_128", "spheres3d_64"):
        g, p, _ = P.preset(name)
        ok, est, _ = P.flow_check(g, p)
        assert ok and 0 < est < 0.1
    # the estimate is Darcy's law: linear in u_in and in the electrode's length
    g, p, _ = P.preset("spheres3d_64")
    e1 = P.flow_check(g, p)[1]
    p.u_in *= 3
    assert P.flow_check(g, p)[1] == pytest.approx(3 * e1, rel=1e-12)
    p.drive = L.BODY_FORCE
    assert P.flow_check(g, p) == (True, 0.0, "")


def test_host_flow_check_on_user_labels_counts_the_faces():
    # a plate channel along x of height h: s = 2 faces per x cell over h + 2
    # cells, phi = h / (h + 2) (walls as solid labels, periodic in y)
    import paper_2110_13055_amd as P
    nx, ny, h = 40, 10, 8
    lab = np.zeros((ny, nx), np.uint8)
    lab[0] = 1
    lab[ny - 1] = 1
    g = P.Geometry(dim=2, nx=nx, ny=ny, kind=L.USER_LABELS, walls_y=0, user_labels=lab.reshape(-1))
    p = P.Params(u_in=1e-3)
    ok, est, _ = P.flow_check(g, p)
    phi, s = h / ny, 2.0 / ny
    k = phi ** 3 / (5 * s * s)
    assert ok and est == pytest.approx(3 * (1 / 6) * 1e-3 * (nx - 4) / k, rel=1e-12)


def test_admission_respects_budget_and_slots_fifo():
    reqs = [req(k, 0.0, nbytes=3e9) for k in range(10)]
    srv, ex, _ = serve(reqs, budget_bytes=10e9, max_slots=5, round_steps=200)
    srv.run(reqs)
    assert ex.started == list(range(10))            # FIFO admission
    for rids, used in ex.log:
        assert len(rids) <= 5 and used <= 10e9
    assert max(len(r) for r, _ in ex.log) == 3      # memory, not slots, binds
    srv2, ex2, _ = serve(reqs, budget_bytes=100e9, max_slots=4, round_steps=200)
    srv2.run(reqs)
    assert max(len(r) for r, _ in ex2.log) == 4     # slots bind
    assert srv2.peak_bytes == 12e9


def test_active_node_cap_binds_fifo_and_admits_an_oversize_first():
    reqs = [req(0, 0.0, nodes=5e6), req(1, 0.0, nodes=1e6), req(2, 0.0, nodes=2e6),
            req(3, 0.0, nodes=1e6), req(4, 0.0, nodes=1e6)]
    srv, ex, _ = serve(reqs, max_slots=16, round_steps=200, max_active_nodes=3e6)
    srv.run(reqs)
    assert ex.started == [0, 1, 2, 3, 4]              # FIFO
    nodes = {r.rid: r.geom["nodes"] for r in reqs}
    for rids, _ in ex.log:
        # over the cap only when one request alone is larger than it
        assert sum(nodes[k] for k in rids) <= 3e6 or rids == [0]
    assert [0] in [r for r, _ in ex.log]               # the 5e6 one ran alone
    assert [1, 2] in [r for r, _ in ex.log]            # the cap, not the slots, binds
    assert srv.active_nodes == 0 and all(r.status == "ok" for r in srv.results)


def test_a_waiting_head_is_planned_once():
    # the head of the queue waits for memory over many rounds; its host-side
    # check and plan run once, not every round
    class Counting(FakeExecutor):
        def __init__(self, clock):
            super().__init__(clock)
            self.calls = {}

        def footprint_estimate(self, r):
            self.calls[r.rid] = self.calls.get(r.rid, 0) + 1
            return super().footprint_estimate(r)

    reqs = [req(0, 0.0, nbytes=8e9, decay=3000.0), req(1, 0.0, nbytes=8e9), req(2, 0.0, nbytes=1e9)]
    clock = Clock()
    ex = Counting(clock)
    srv = Server(ex, budget_bytes=10e9, round_steps=100, clock=clock, sleep=clock.sleep)
    srv.run(reqs)
    assert srv.rounds > 20 and ex.started == [0, 1, 2]
    assert ex.calls == {0: 1, 1: 1, 2: 1}
    assert not srv._est


def test_continuous_batching_refills_freed_slots():
    # short and long requests: a short one's slot is reused before the long one ends
    reqs = [req(0, 0.0, decay=5000.0), req(1, 0.0, decay=100.0), req(2, 0.0, decay=100.0)]
    srv, ex, _ = serve(reqs, max_slots=2, round_steps=100)
    srv.run(reqs)
    together = [set(r) for r, _ in ex.log]
    assert {0, 2} in together and ex.started == [0, 1, 2]
    out = {r.rid: r for r in srv.results}
    assert out[2].finished_s < out[0].finished_s


def test_oversize_request_rejected_others_served():
    reqs = [req(0, 0.0), req(1, 0.0, nbytes=500e9), req(2, 0.0)]
    srv, _, _ = serve(reqs, budget_bytes=200e9)
    out = {r.rid: r for r in srv.run(reqs)}
    assert out[1].status.startswith("rejected") and out[0].status == "ok" and out[2].status == "ok"


def test_failed_start_and_failed_member_retire_only_themselves():
    reqs = [req(k, 0.0, decay=300.0) for k in range(5)]
    alone = {}
    for r in reqs:
        s, _, _ = serve([r], round_steps=100, fail_start=[1], fail_ions=[3])
        (res,) = s.run([r])
        alone[r.rid] = res
    srv, ex, _ = serve(reqs, round_steps=100, fail_start=[1], fail_ions=[3])
    out = {r.rid: r for r in srv.run(reqs)}
    assert out[1].status.startswith("failed") and out[3].status.startswith("failed")
    assert "positivity" in out[3].status
    for k in (0, 2, 4):
        assert out[k].status == "ok"
        assert (out[k].flow_steps, out[k].np_steps, out[k].adsorbed) == \
            (alone[k].flow_steps, alone[k].np_steps, alone[k].adsorbed)
    assert not ex.live and srv.used == 0


def test_horizon_leaves_backlog():
    reqs = [req(k, 0.5 * k, nodes=5e7, decay=2000.0) for k in range(40)]
    srv, _, clock = serve(reqs, round_steps=200, max_slots=8)
    res = srv.run(reqs, horizon_s=5.0)
    done = sum(r.status == "ok" for r in res)
    assert srv.backlog == 40 - len(res) and srv.backlog > 0
    st = latency_stats(res, wall_s=clock.t)
    assert st["completed"] == done and (done == 0 or st["p99_s"] >= st["p50_s"])


def test_poisson_arrivals_fixed_and_rate():
    a = poisson_arrivals(20000, 2.0, 2110)
    assert a == poisson_arrivals(20000, 2.0, 2110)
    assert np.all(np.diff(a) > 0)
    assert abs(len(a) / a[-1] - 2.0) < 0.05


def test_latency_stats_percentiles():
    from paper_2110_13055_amd.serving import Result
    rs = [Result(k, 0.0, 0.0, float(k + 1), 0) for k in range(100)]
    st = latency_stats(rs, wall_s=3600.0)
    assert st["completed"] == 100 and st["solves_per_hour"] == pytest.approx(100.0)
    assert st["p50_s"] == pytest.approx(50.5) and st["p99_s"] == pytest.approx(99.01)


# --------------------------------------------------------------- oracle-backed
class OracleExecutor:
    """Executor whose members are FP64 oracle solvers (stepped one after the
    other): checks that the scheduler gives each request the same step
    sequence alone and in the mix."""

    def __init__(self):
        self.frozen = set()

    def footprint_estimate(self, r):
        return 1e6

    def footprint(self, h):
        return 1e6

    def start(self, r):
        from helpers import oracle_solver
        o = oracle_solver(r.geom, r.params)
        o.rid = r.rid
        return o

    def group_key(self, h):
        return h.cfg.dim

    def advance(self, groups, modes, n):
        res = {}
        for key, members in groups.items():
            r = np.full(len(members), np.nan)
            for k, (o, m) in enumerate(zip(members, modes[key])):
                if m == FLOW:
                    o.flow_steps(n - 1)
                    u0 = o.velocity()
                    o.flow_steps(1)
                    u1 = o.velocity()
                    r[k] = np.linalg.norm(u1 - u0) / np.linalg.norm(u1)
                else:
                    if id(o) not in self.frozen:
                        o.freeze_velocity()
                        self.frozen.add(id(o))
                    assert o.np_steps(n) == 0
            res[key] = r
        return res, {}

    def finish(self, o):
        return {"adsorbed": o.adsorbed_total(), "balance": o.balance(), "conc": o.conc()}

    def release(self, o):
        pass


def oracle_requests():
    from paper_2110_13055_amd import Geometry, Params
    out = []
    for k in range(4):
        g = Geometry(dim=2, nx=40 + 8 * k, ny=24, kind=L.DISKS, porosity=0.7, r_min=2.0, r_max=4.0,
                     min_gap=1.0, walls_y=1, buffer_x=2, seed=2110 + k)
        p = Params(u_in=1e-3 * (k + 1), dpsi_vt=5.0 * (k + 1), D=(0.05, 0.076))
        out.append(Request(k, 0.01 * k, g, p, flow_tol=1e-5, flow_max_steps=400, np_steps=60))
    return out


def test_oracle_backed_results_alone_equal_mix():
    reqs = oracle_requests()
    clock = Clock()
    mix = Server(OracleExecutor(), round_steps=20, clock=clock, sleep=clock.sleep)
    out = {r.rid: r for r in mix.run(reqs)}
    for r in reqs:
        c2 = Clock()
        solo = Server(OracleExecutor(), round_steps=20, clock=c2, sleep=c2.sleep)
        (a,) = solo.run([r])
        m = out[r.rid]
        assert m.status == a.status and m.status in ("ok", "ok_unconverged")
        assert (m.flow_steps, m.np_steps, m.residual) == (a.flow_steps, a.np_steps, a.residual)
        assert m.adsorbed == a.adsorbed and m.balance == a.balance
        assert np.array_equal(mix.fields[r.rid]["conc"], solo.fields[r.rid]["conc"])
