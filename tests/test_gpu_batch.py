"""Batched stepping: uneven instances in one persistent launch (graph-replayed
step pairs) give, member by member, exactly the results of stepping each
instance alone with the same calls; the batch is also checked against the
FP64 oracle through one member."""
import numpy as np
import pytest

from helpers import oracle_solver, rel_l2

pytestmark = pytest.mark.gpu

P = pytest.importorskip("paper_2110_13055_amd")
from paper_2110_13055_amd import _lib as L  # noqa: E402
from paper_2110_13055_amd import Batch, Geometry, Params, Solver  # noqa: E402

FLOW, IONS, FUSED, IDLE = L.MODE_FLOW, L.MODE_IONS, L.MODE_FUSED, L.MODE_IDLE


def members(precision=L.FP32, n=5):
    rng = np.random.default_rng(2110)
    out = []
    for k in range(n):
        edge = int(rng.integers(24, 41))
        g = Geometry(dim=3, nx=edge, ny=edge, nz=edge, kind=L.SPHERES,
                     porosity=float(rng.uniform(0.45, 0.75)), r_min=2.0, r_max=4.0, buffer_x=2,
                     seed=2110 + k)
        p = Params(u_in=float(rng.uniform(1e-4, 2e-3)), dpsi_vt=float(rng.uniform(4, 40)),
                   D=(0.05, 0.076), precision=precision)
        out.append((g, p))
    return out


def state(s):
    return (s.concentration(), s.velocity(), s.adsorbed_total(), s.mass_balance())


def schedule():
    # (nsteps, modes per member)
    return [
        (7, [FLOW, FLOW, FLOW, FLOW, FLOW]),
        (10, [FLOW, IDLE, FLOW, FLOW, FLOW]),
        (9, [FUSED, FLOW, IONS, FUSED, IDLE]),
        (6, [IONS, FUSED, FUSED, IDLE, FLOW]),
    ]


def run_alone(specs):
    out = []
    for k, (g, p) in enumerate(specs):
        s = Solver(g, p)
        for n, modes in schedule():
            m = modes[k]
            if m == FLOW:
                s.flow_steps(n)
            elif m == IONS:
                s.np_step(n, fused=False)
            elif m == FUSED:
                s.np_step(n, fused=True)
        out.append(state(s))
    return out


@pytest.mark.parametrize("precision", [L.FP32, L.FP16_DEV, L.MOMENTS])
def test_batch_equals_members_stepped_alone(precision):
    specs = members(precision)
    alone = run_alone(specs)
    solvers = [Solver(g, p) for g, p in specs]
    b = Batch(solvers)
    for n, modes in schedule():
        b.advance(n, modes)
    b.synchronize()
    for k, s in enumerate(solvers):
        for a, c in zip(alone[k], state(s)):
            assert np.array_equal(a, c), f"member {k}"


@pytest.mark.parametrize("precision", [L.FP32, L.MOMENTS])
def test_long_fused_advance_rechecked_in_chunks_equals_alone(precision):
    # more than 256 fused steps in one call: the batch takes the positivity
    # bound again every 256 steps (chunks of 256 and 44, then 255 and 2); the
    # steps, and so the results, are those of each member stepped alone
    specs = members(precision, n=3)
    sched = [(3, [FLOW, FLOW, FLOW]), (300, [FUSED, FLOW, FUSED]), (257, [FUSED, IONS, FLOW])]
    alone = []
    for k, (g, p) in enumerate(specs):
        s = Solver(g, p)
        for n, modes in sched:
            m = modes[k]
            if m == FLOW:
                s.flow_steps(n)
            elif m == IONS:
                s.np_step(n, fused=False)
            else:
                s.np_step(n, fused=True)
        alone.append(state(s))
    solvers = [Solver(g, p) for g, p in specs]
    b = Batch(solvers)
    for n, modes in sched:
        b.advance(n, modes)
    b.synchronize()
    for k, s in enumerate(solvers):
        for a, c in zip(alone[k], state(s)):
            assert np.array_equal(a, c), f"member {k}"
    assert np.isfinite(b.residuals()[2])   # the flow member's residual of the chunked call


@pytest.mark.parametrize("precision", [L.FP32, L.FP16_DEV])
def test_batch_mixing_aa_and_pull_members(precision):
    specs = members(precision)
    for k, (g, p) in enumerate(specs):
        p.streaming = L.STREAM_PULL if k % 2 else L.STREAM_AA
    alone = run_alone(specs)
    solvers = [Solver(g, p) for g, p in specs]
    b = Batch(solvers)
    for n, modes in schedule():
        b.advance(n, modes)
    b.synchronize()
    for k, s in enumerate(solvers):
        for a, c in zip(alone[k], state(s)):
            assert np.array_equal(a, c), f"member {k}"


def test_batch_on_default_stream_and_launch_shapes_agree():
    import torch
    specs = members()
    ref = None
    for stream, wg in ((None, 0), (torch.cuda.default_stream(), 0), (None, 7), (None, 100000)):
        solvers = [Solver(g, p) for g, p in specs]
        b = Batch(solvers, stream=stream)
        b.set_launch(wg, 0)
        for n, modes in schedule():
            b.advance(n, modes)
        b.synchronize()
        got = [state(s) for s in solvers]
        if ref is None:
            ref = got
        else:
            for r, g in zip(ref, got):
                for a, c in zip(r, g):
                    assert np.array_equal(a, c)


def test_member_alone_vs_in_the_mix():
    specs = members()
    one = Solver(*specs[2])
    b1 = Batch([one])
    b1.advance(12, [FLOW])
    b1.advance(8, [FUSED])
    solvers = [Solver(g, p) for g, p in specs]
    bm = Batch(solvers)
    bm.advance(12, [FLOW] * 5)
    bm.advance(8, [FUSED, IONS, FUSED, FLOW, FUSED])
    for a, c in zip(state(one), state(solvers[2])):
        assert np.array_equal(a, c)


def test_batch_residuals_and_oracle_parity():
    specs = members(n=3)
    solvers = [Solver(g, p) for g, p in specs]
    b = Batch(solvers)
    b.advance(30, [FLOW] * 3)
    r = b.residuals()
    assert np.all(np.isfinite(r)) and np.all(r > 0)
    b.advance(25, [FUSED] * 3)
    assert np.all(np.isnan(b.residuals()))
    g, p = specs[1]
    o = oracle_solver(g, p)
    o.flow_steps(30)
    assert o.np_steps(25, fused=True) == 0
    s = solvers[1]
    assert rel_l2(s.velocity(), o.velocity()) <= 1e-5
    assert np.abs(s.concentration() - o.conc()).max() <= 1e-4
    assert np.all(np.abs(s.adsorbed_total() - o.adsorbed_total()) <= 1e-4 * np.abs(o.adsorbed_total()))


def test_batch_autotune_restores_members():
    specs = members(n=3)
    solvers = [Solver(g, p) for g, p in specs]
    b = Batch(solvers)
    b.advance(4, [FLOW] * 3)
    before = [state(s) for s in solvers]
    wg, ms = b.autotune(4, [FUSED] * 3)
    assert wg > 0 and ms > 0
    assert b.launch()[0] == wg
    after = [state(s) for s in solvers]
    for r, g in zip(before, after):
        for a, c in zip(r, g):
            assert np.array_equal(a, c)


def test_unstable_member_is_reported():
    specs = members(n=2)
    specs[1][1].D = (0.3, 0.3)
    solvers = [Solver(g, p) for g, p in specs]
    b = Batch(solvers)
    with pytest.raises(L.CdiError) as e:
        b.advance(2, [IONS, IONS])
    assert e.value.code == L.E_UNSTABLE and "member 1" in str(e.value)


@pytest.mark.parametrize("streaming", [L.STREAM_AA, L.STREAM_PULL], ids=["aa", "pull"])
def test_full_size_batch_of_64_instances(streaming):
    # the bench's batched workload at its full size (64 cubes of edge 48-160,
    # 49.5M fluid nodes) in its launch configuration: FP32, AA streaming (the
    # bench's default; pull too), autotuned grid, graph-replayed fused step
    # pairs. Every member equals the same instance stepped alone, bit for bit;
    # the smallest one also matches the oracle.
    specs = P.batch_instances(64, precision=L.FP32, streaming=streaming)
    n = len(specs)
    solvers = [Solver(g, p) for g, p in specs]
    for s in solvers:
        s.flow_steps(2)
    b = Batch(solvers)
    b.autotune(4, [FUSED] * n)
    b.advance(12, [FUSED] * n)
    b.synchronize()
    got = [state(s) for s in solvers]
    b.close()
    del b, solvers
    for k, (g, p) in enumerate(specs):
        s = Solver(g, p)
        s.flow_steps(2)
        s.np_step(12, fused=True)
        for a, c in zip(state(s), got[k]):
            assert np.array_equal(a, c), f"member {k}"
        del s
    k = int(np.argmin([g.nx * g.ny * g.nz for g, _ in specs]))
    g, p = specs[k]
    o = oracle_solver(g, p)
    o.flow_steps(2)
    assert o.np_steps(12, fused=True) == 0
    c, u = got[k][0], got[k][1]
    assert rel_l2(u, o.velocity()) <= 1e-5
    assert np.abs(c - o.conc()).max() <= 1e-4


@pytest.mark.parametrize("precision", [L.FP32, L.MOMENTS])
def test_batch_members_in_a_solved_potential_equal_members_alone(precision):
    # members whose ions migrate in a solved potential field (the batched
    # kernels read the neighbours' potential in the face loop, the
    # single-instance kernels with their other early loads): the same numbers
    from paper_2110_13055_amd import Potential
    specs = members(precision, n=3)
    pot = Potential(psi_electrode=-1.0, x_bc=(L.PSIX_DIRICHLET, L.PSIX_NEUMANN), tol=1e-12)

    def prepared():
        out = []
        for g, p in specs:
            s = Solver(g, p)
            s.flow_steps(20)
            s.solve_potential(pot)
            out.append(s)
        return out
    alone = prepared()
    for s in alone:
        s.np_step(9, fused=True)
        s.np_step(6)
    batched = prepared()
    b = Batch(batched)
    b.advance(9, [FUSED] * 3)
    b.advance(6, [IONS] * 3)
    b.synchronize()
    for k, (a, c) in enumerate(zip(alone, batched)):
        for x, y in zip(state(a), state(c)):
            assert np.array_equal(x, y), f"member {k}"


@pytest.mark.parametrize("precision", [L.FP32, L.FP16, L.MOMENTS])
def test_members_admitted_and_retired_mid_run(precision):
    # a batch created with room to spare: members join while others run and
    # leave before the end, in place (no new workspace); every member ends
    # bitwise where the same sequence of steps takes it alone
    specs = members(precision, n=5)
    # (member, first stage, last stage) and the per-stage (steps, mode of every member)
    life = {0: (0, 3), 1: (0, 1), 2: (1, 3), 3: (2, 3), 4: (1, 2)}
    stages = [(9, FLOW), (8, FUSED), (11, FLOW), (7, FUSED)]

    def mode_at(k, q):
        a, b = life[k]
        if not (a <= q <= b):
            return None
        return stages[q][1] if (k + q) % 3 else IONS if q > a else FLOW

    alone = []
    for k, (g, p) in enumerate(specs):
        s = Solver(g, p)
        for q, (n, _) in enumerate(stages):
            m = mode_at(k, q)
            if m == FLOW:
                s.flow_steps(n)
            elif m == IONS:
                s.np_step(n, fused=False)
            elif m == FUSED:
                s.np_step(n, fused=True)
        alone.append(state(s))

    print(f"admit/retire precision={precision}", flush=True)
    sol = [Solver(g, p) for g, p in specs]
    b = Batch(capacity=(4, 10 ** 6))
    ws = b.ws.data_ptr()
    for q, (n, _) in enumerate(stages):
        for k in range(5):
            if life[k][0] == q:
                b.admit(sol[k])
        assert b.n <= 4
        b.advance(n, [mode_at(sol.index(s), q) for s in b.members])
        for k in range(5):
            if life[k][1] == q:
                b.retire(sol[k])
    assert b.n == 0 and b.ws.data_ptr() == ws
    b.close()
    for k in range(5):
        got = state(sol[k])
        for a, c in zip(alone[k], got):
            assert np.array_equal(a, c), k


def test_admit_refuses_a_full_batch_and_a_mismatch():
    specs = members(L.FP32, n=3)
    sol = [Solver(g, p) for g, p in specs]
    b = Batch(capacity=(2, 10 ** 6))
    b.admit(sol[0])
    with pytest.raises(L.CdiError) as e:
        b.admit(sol[0])
    assert e.value.code == L.E_INVALID
    b.admit(sol[1])
    with pytest.raises(L.CdiError) as e:
        b.admit(sol[2])                       # two members is the room it has
    assert e.value.code == L.E_BUFFER
    b.retire(sol[0])
    b.admit(sol[2])
    g, p = specs[0]
    p.precision = L.MOMENTS
    with pytest.raises(L.CdiError):
        b.admit(Solver(g, p))                 # another storage precision
    b.close()
