"""Benchmark of the coupled LBM + Nernst-Planck step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: the 512^3 D3Q19 overlapping-sphere electrode (porosity 0.4, radii
3-6 lattice units, seeded, about 54M fluid nodes), inlet/outlet flow, Na+/Cl-
with a 20-thermal-voltage ramp. A "step" is one fused LBM collide-stream +
Nernst-Planck update over all fluid nodes (with the inlet/outlet condition and
the FP64 adsorbed/flux accumulators). Geometry, compaction and
initialisation happen once, before the timed region; all state is resident
in HBM. MLUPS counts fluid nodes only.

Prints one JSON line. ``value`` is the FP32-storage fused MLUPS; the FP16
deviation and moment storage forms, LBM-only and NP-only rates are reported
beside it. ``roofline`` prices the fused kernel's algorithmic bytes per node
against 8 TB/s (``traffic``: the HBM bytes per launch the committed counter
record holds for the current kernel sources); ``cpu_baseline`` is the FP64
reference on this host's cores, on a bounded sample (the seeded 64^3
sub-case). Beside them: ``potential`` (the Poisson solve of Eq. 4-5, a
coupled PNP step, and the steady ion state by the implicit solver, on the
same electrode), ``batched`` (64 uneven electrodes in one launch
per step) and ``serving`` (a Poisson arrival trace through the continuous-
batching server). --potential-only runs the solver leg alone.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOAD = "spheres3d_512"
HBM_PEAK_GBS = 8000.0
# algorithmic bytes per fluid-node update (D3Q19): populations read + write,
# concentrations read + write (2 species, FP32 values and FP16 remainders:
# 2 x (8 + 4) B), ion-advecting flux read + write (FP32 and FP16 populations:
# j, 3 floats; FP16 deviations and moment storage: the moments rho-1, u as one
# float4, which also carry j)
BYTES_C = 2 * (8 + 4)
BYTES_FUSED = {"fp32": 19 * 4 * 2 + BYTES_C + 24, "fp16": 19 * 2 * 2 + BYTES_C + 24,
               "fp16_dev": 19 * 2 * 2 + BYTES_C + 32, "moments": BYTES_C + 32}
BYTES_LBM = {"fp32": 19 * 4 * 2, "fp16": 19 * 2 * 2, "fp16_dev": 19 * 2 * 2 + 32, "moments": 32}
BYTES_NP = BYTES_C + 12  # C and remainders read + write, frozen j read


_T0 = time.perf_counter()


def log(msg: str) -> None:
    """Progress on stderr (stdout carries only the JSON record)."""
    print(f"[bench {time.perf_counter() - _T0:7.1f} s] {msg}", file=sys.stderr, flush=True)


def measured_traffic(kind: str):
    """HBM bytes per fused-step launch (mean of the even and odd kernels) from
    the committed counter summary, if it was taken on the current kernel
    source; else None."""
    from paper_2110_13055_amd.profile_summary import kernel_source_hash
    path = os.path.join(ROOT, "profiles", "step_kernel_spheres3d_512_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    v = rec.get("bytes_per_launch", {}).get(kind)
    return None if v is None else round(v)


def time_region(fn, stream):
    import torch
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    fn()
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3


def gpu_rates(precision: int, steps: int, warmup: int, streaming: int):
    import torch
    import paper_2110_13055_amd as P
    g, p, _ = P.preset(WORKLOAD, precision=precision, streaming=streaming)
    s = P.Solver(g, p)
    nf = s.n_fluid
    stream = s.stream
    # develop the flow a little so the step sees a realistic state
    s.flow_steps(2)
    if warmup:
        s.np_step(warmup, fused=True)
    fused = time_region(lambda: s.np_step(steps, fused=True), stream)
    lbm = time_region(lambda: s.flow_steps(steps), stream)
    npo = time_region(lambda: s.np_step(steps, fused=False), stream)
    res = dict(n_fluid=nf, fused_s=fused, lbm_s=lbm, np_s=npo)
    del s
    torch.cuda.empty_cache()
    return res


def hbm_probe(mib: int = 2048, reps: int = 5):
    """Attainable HBM bandwidth: the library's streaming kernels (128-bit
    accesses, a flat grid) over two buffers of `mib` MiB each: a copy (reads
    and writes mib MiB), a read-only checksum pass and a fill. GB/s of
    bytes moved, best of `reps` launches timed with HIP events on the stream
    they run on."""
    import torch
    import paper_2110_13055_amd as P
    n = mib << 18
    src = torch.ones(n, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    chk = torch.empty(n // 512 + 4, dtype=torch.int32, device="cuda")  # 16 B per 8 KiB block
    st = torch.cuda.current_stream()
    out = {"buffer_mib": mib}
    for name, mode, d, sr, moved in (("copy", P.PROBE_COPY, dst, src, 2), ("read", P.PROBE_READ, chk, src, 1),
                                     ("fill", P.PROBE_FILL, dst, None, 1)):
        P.bandwidth_probe(mode, d, sr, stream=st)
        best = min(time_region(lambda: P.bandwidth_probe(mode, d, sr, stream=st), st) for _ in range(reps))
        out[f"{name}_gbs"] = round(moved * n * 4 / best / 1e9, 1)
    del src, dst
    torch.cuda.empty_cache()
    return out


def potential_rates(coupled_steps: int = 10):
    """The potential (Poisson, Eq. 4-5) on the bench electrode. Static solve:
    Laplace with the electrode at -20 thermal voltages, the inlet face at 0
    and a field-free outlet, Jacobi-PCG from zero to a relative residual of
    1e-8. Coupled: fused LBM + ion steps with the potential re-solved from the
    current charge (electrode at -4, kappa2 = 0.5, warm start, 1e-6) before
    every step.
    Algorithmic bytes of one CG iteration per fluid node (the iterations of
    the mixed-precision refinement run on FP32 vectors): the stencil kernel
    reads r, the old direction, the diagonal byte and the six face-neighbour
    indices and writes the new direction and q = A p (41 B); the update
    kernel reads x, r, p, q and the diagonal byte and writes x, r (25 B). The
    refinement rounds' FP64 residuals (two or three per solve) are inside the
    timed solve but not in this per-iteration count."""
    import torch
    import paper_2110_13055_amd as P
    g, p, _ = P.preset(WORKLOAD)
    s = P.Solver(g, p)
    nf = s.n_fluid
    per_iter = (4 + 4 + 1 + 24 + 4 + 4) + (16 + 1 + 8)
    out = {"n_fluid": nf, "algorithmic_bytes_per_node_iter": round(per_iter, 1)}
    pot = P.Potential(psi_electrode=-20.0, x_bc=(P.PSIX_DIRICHLET, P.PSIX_NEUMANN), tol=1e-8,
                      warm_start=False, check_every=16)
    s.solve_potential(pot)  # first launches
    res = {}

    def run():
        res["it"], res["r"] = s.solve_potential(pot)
    sec = time_region(run, s.stream)
    it = res["it"]
    out["laplace"] = {"iterations": it, "residual": res["r"], "solve_ms": round(sec * 1e3, 2),
                      "ms_per_iter": round(sec * 1e3 / max(it, 1), 4),
                      "gbs": round(per_iter * nf * it / sec / 1e9, 1),
                      "fp32_rounds": s.potential_stats["fp32_rounds"],
                      "fp64_iterations": s.potential_stats["fp64_iterations"]}
    # the same solve by CG on FP64 vectors alone, for comparison
    pot64 = P.Potential(psi_electrode=-20.0, x_bc=(P.PSIX_DIRICHLET, P.PSIX_NEUMANN), tol=1e-8,
                        warm_start=False, check_every=16, fp64=True)

    def run64():
        res["it"], res["r"] = s.solve_potential(pot64)
    sec = time_region(run64, s.stream)
    out["laplace_fp64"] = {"iterations": res["it"], "residual": res["r"], "solve_ms": round(sec * 1e3, 2)}
    # -4 thermal voltages (about -100 mV) keeps the explicit ion update within
    # its positivity bound on this lattice; -20 would not
    cp = P.Potential(psi_electrode=-4.0, x_bc=(P.PSIX_DIRICHLET, P.PSIX_NEUMANN), kappa2=0.5, tol=1e-6,
                     warm_start=True)
    try:
        s.flow_steps(2)
        s.np_step_coupled(2, cp, every=1, fused=True)
        sec = time_region(lambda: s.np_step_coupled(coupled_steps, cp, every=1, fused=True), s.stream)
        out["coupled_pnp"] = {"steps": coupled_steps, "ms_per_step": round(sec * 1e3 / coupled_steps, 3),
                              "mlups": round(nf * coupled_steps / sec / 1e6, 1), "psi_electrode": -4.0,
                              "kappa2": 0.5, "every": 1}
    except P.CdiError as exc:
        out["coupled_pnp"] = {"error": str(exc)}
    # the steady ion state on this flow and potential (implicit scheme),
    # BiCGSTAB to 1e-8; per iteration both species (directions stored
    # preconditioned): direction 72 B (r, v, p^, diagonal; p^ written), two
    # operator applications 78 + 70 B (own vectors, neighbour indices, flux
    # and potential; the second also the diagonal), s^ 56 B, update 120 B per
    # fluid node
    per_it_np = 72 + 78 + 56 + 70 + 120
    try:
        s.np_steady(tol=1e-8, max_iter=20, allow_not_converged=True)  # first launches
        res = {}

        def run_np():
            res["it"] = s.np_steady(tol=1e-8, max_iter=4000, allow_not_converged=True)
        sec = time_region(run_np, s.stream)
        out["ion_steady"] = {"iterations": res["it"], "solve_ms": round(sec * 1e3, 2),
                             "ms_per_iter": round(sec * 1e3 / max(res["it"], 1), 4),
                             "algorithmic_bytes_per_node_iter": per_it_np,
                             "gbs": round(per_it_np * nf * res["it"] / sec / 1e9, 1)}
    except P.CdiError as exc:
        out["ion_steady"] = {"error": str(exc)}
    del s
    torch.cuda.empty_cache()
    return out


def batched_rates(steps: int, streaming: int, n: int = 64, flow_steps: int = 1000, ion_steps: int = 500):
    """Batched stepping of n uneven instances (cubes of edge 48-160, own seed,
    porosity, potential and inlet velocity): the fused step of all instances
    in one launch per step class (graph-replayed, grid size autotuned),
    against the same steps run instance by instance with the plain solver;
    and whole solves of a fixed protocol (flow_steps flow steps, then
    ion_steps ion steps on the frozen flow), batched in FP32 and with moment
    storage, against the n plain FP32 solves one after the other."""
    import torch
    import paper_2110_13055_amd as P
    out = {"instances": n}
    for prec, name in ((P.FP32, "fp32"), (P.FP16_DEV, "fp16_dev"), (P.MOMENTS, "moments")):
        specs = P.batch_instances(n, precision=prec, streaming=streaming)
        solvers = [P.Solver(g, p) for g, p in specs]
        nf = sum(s.n_fluid for s in solvers)
        out["n_fluid_total"] = nf
        for s in solvers:
            s.flow_steps(2)
        b = P.Batch(solvers)
        wg, _ = b.autotune(4, [P.MODE_FUSED] * n)
        b.advance(2, [P.MODE_FUSED] * n)
        t = time_region(lambda: b.advance(steps, [P.MODE_FUSED] * n), b.stream)
        out[f"{name}_batched_mlups"] = round(nf * steps / t / 1e6, 1)
        out[f"{name}_workgroups"] = wg
        if prec == P.FP32:
            def seq():
                for s in solvers:
                    s.np_step(steps, fused=True)
            t = time_region(seq, solvers[0].stream)
            out["fp32_sequential_mlups"] = round(nf * steps / t / 1e6, 1)
        b.close()
        del b, solvers
        torch.cuda.empty_cache()
    for name in ("fp32", "fp16_dev", "moments"):
        out[f"{name}_batched_vs_fp32_sequential"] = round(out[f"{name}_batched_mlups"] / out["fp32_sequential_mlups"], 3)
    out["solve_protocol"] = f"{flow_steps} flow + {ion_steps} ion steps per instance, from rest"
    for prec, name in ((P.FP32, "fp32"), (P.MOMENTS, "moments")):
        solvers = [P.Solver(g, p) for g, p in P.batch_instances(n, precision=prec, streaming=streaming)]
        b = P.Batch(solvers)

        def batched_solves():
            b.advance(flow_steps, [P.MODE_FLOW] * n)
            b.advance(ion_steps, [P.MODE_IONS] * n)
        out[f"solves_{name}_batched_s"] = round(time_region(batched_solves, b.stream), 3)
        b.close()
        del b, solvers
        torch.cuda.empty_cache()
    solvers = [P.Solver(g, p) for g, p in P.batch_instances(n, precision=P.FP32, streaming=streaming)]

    def sequential_solves():
        for s in solvers:
            s.flow_steps(flow_steps)
            s.np_step(ion_steps, fused=False)
    ts = time_region(sequential_solves, solvers[0].stream)
    out["solves_fp32_sequential_s"] = round(ts, 3)
    for name in ("fp32", "moments"):
        out[f"solves_{name}_batched_vs_fp32_sequential"] = round(ts / out[f"solves_{name}_batched_s"], 3)
    del solvers
    torch.cuda.empty_cache()
    return out


def small_batch_rates(steps: int, streaming: int, n: int = 64, flow_steps: int = 2000, ion_steps: int = 1000):
    """Batching where one instance leaves the GPU idle: n small electrodes
    (cubes of edge 48-64, the cfg3 parameter ranges otherwise), FP32. Fused
    step rate batched vs each instance stepped alone; and whole solves of a
    fixed protocol (flow_steps flow steps, then ion_steps ion steps on the
    frozen flow) batched vs the n solves one after the other."""
    import torch
    import paper_2110_13055_amd as P
    specs = P.batch_instances(n, precision=P.FP32, streaming=streaming, edge_range=(48, 64))
    out = {"instances": n, "edge_range": [48, 64]}
    solvers = [P.Solver(g, p) for g, p in specs]
    nf = sum(s.n_fluid for s in solvers)
    out["n_fluid_total"] = nf
    for s in solvers:
        s.flow_steps(2)
    b = P.Batch(solvers)
    b.advance(2, [P.MODE_FUSED] * n)
    t = time_region(lambda: b.advance(steps, [P.MODE_FUSED] * n), b.stream)
    out["fused_batched_mlups"] = round(nf * steps / t / 1e6, 1)

    def seq():
        for s in solvers:
            s.np_step(steps, fused=True)
    t = time_region(seq, solvers[0].stream)
    out["fused_sequential_mlups"] = round(nf * steps / t / 1e6, 1)
    out["fused_batched_vs_sequential"] = round(out["fused_batched_mlups"] / out["fused_sequential_mlups"], 3)
    b.close()
    del solvers
    torch.cuda.empty_cache()
    # whole solves: fresh instances each way
    solvers = [P.Solver(g, p) for g, p in specs]
    b = P.Batch(solvers)

    def batched_solves():
        b.advance(flow_steps, [P.MODE_FLOW] * n)
        b.advance(ion_steps, [P.MODE_IONS] * n)
    tb = time_region(batched_solves, b.stream)
    b.close()
    del solvers
    solvers = [P.Solver(g, p) for g, p in specs]

    def sequential_solves():
        for s in solvers:
            s.flow_steps(flow_steps)
            s.np_step(ion_steps, fused=False)
    ts = time_region(sequential_solves, solvers[0].stream)
    out["solve_protocol"] = f"{flow_steps} flow + {ion_steps} ion steps per instance"
    out["solves_batched_s"] = round(tb, 3)
    out["solves_sequential_s"] = round(ts, 3)
    out["solves_batched_vs_sequential"] = round(ts / tb, 3)
    del solvers
    torch.cuda.empty_cache()
    return out


# Slots of the continuous-batching server: enough concurrent requests to fill
# the GPU with the small ones (a 2D 256^2 request or a 64^3 cube alone leaves
# most compute units idle) without sharing it among so many that none finish
# (with 64 slots every admitted request advanced at 1/64 of the rate).
SERVE_SLOTS = 16
# Fluid nodes stepped together at most. One 3D request of 2-4 million fluid
# nodes already keeps the FP32 step at its full node rate; admitting more
# beyond that only time-slices the GPU among them and delays every one.
SERVE_ACTIVE_NODES = 4_000_000


def serving_run(n_requests: int, precision: int, slots: int, streaming: int, horizon_s: float,
                max_active_nodes: float = math.inf):
    """Serve a fixed Poisson trace (2 requests/s, half 2D 256^2, half 3D
    64^3-192^3) with a 200 GB admission budget and the given slot count, up to
    horizon_s seconds; what is left then is the backlog."""
    import torch
    import paper_2110_13055_amd as P
    from paper_2110_13055_amd.serving import GpuExecutor, Server, latency_stats
    reqs = P.serving_requests(n_requests, precision=precision, streaming=streaming)
    ex = GpuExecutor()
    srv = Server(ex, budget_bytes=200e9, max_slots=slots, round_steps=250,
                 max_active_nodes=max_active_nodes)
    node_steps = [0]
    advance = ex.advance

    def counted(groups, modes, nsteps):
        node_steps[0] += nsteps * sum(h.n_fluid for hs in groups.values() for h in hs)
        return advance(groups, modes, nsteps)
    ex.advance = counted
    t0 = time.perf_counter()
    res = srv.run(reqs, horizon_s=horizon_s, progress=lambda m: log(f"serving: {m}"))
    wall = time.perf_counter() - t0
    ex.close()
    torch.cuda.empty_cache()
    st = latency_stats(res, wall)
    st = {k: (float(f"{v:.4g}") if isinstance(v, float) else v) for k, v in st.items()}  # 4 significant digits
    st.update(failures=[f"{r.rid}: {r.status[:60]}" for r in res if r.status.startswith("failed")],
              rejected_ids=[r.rid for r in res if r.status.startswith("rejected")])
    st.update(wall_s=round(wall, 2), backlog=srv.backlog, peak_slots=srv.peak_slots,
              peak_gb=round(srv.peak_bytes / 1e9, 2), rounds=srv.rounds,
              flow_steps=sum(r.flow_steps for r in res), np_steps=sum(r.np_steps for r in res),
              node_steps_g=round(node_steps[0] / 1e9, 2), mlups=round(node_steps[0] / wall / 1e6, 1))
    return st


def cpu_baseline(budget_s: float = 12.0):
    """FP64 reference on the host: fused steps of the seeded 64^3 sub-case."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    import oracle
    import paper_2110_13055_amd as P
    from helpers import oracle_solver
    g, p, _ = P.preset("spheres3d_64")
    o = oracle_solver(g, p)
    o.flow_steps(2)
    o.np_steps(2, fused=True)
    steps, t0 = 0, time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        o.np_steps(10, fused=True)
        steps += 10
    dt = time.perf_counter() - t0
    cores = oracle.oracle.threads()
    # the same steps on one thread, a shorter sample (results do not depend on the thread count)
    oracle.oracle.set_threads(1)
    try:
        steps1, t1 = 0, time.perf_counter()
        while time.perf_counter() - t1 < budget_s / 3:
            o.np_steps(2, fused=True)
            steps1 += 2
        dt1 = time.perf_counter() - t1
    finally:
        oracle.oracle.set_threads(cores)
    return {"value": o.nf * steps / dt / 1e6, "unit": "MLUPS", "cores": cores,
            "kind": "oracle",
            "sample": f"{steps} fused LBM+NP steps (FP64) of the seeded 64^3 sub-case "
                      f"({o.nf} fluid nodes), {dt:.1f} s",
            "single_thread": {"value": o.nf * steps1 / dt1 / 1e6, "unit": "MLUPS",
                              "sample": f"{steps1} more steps of the same case on 1 thread, {dt1:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=4)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU reference timing")
    ap.add_argument("--streaming", choices=("aa", "pull"), default="aa",
                    help="population streaming of the FP32 / FP16 forms: AA (one array, in place) "
                         "or pull (two arrays)")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-instances leg")
    ap.add_argument("--no-probe", action="store_true", help="skip the streaming bandwidth probe")
    ap.add_argument("--no-potential", action="store_true", help="skip the potential-solve leg")
    ap.add_argument("--potential-only", action="store_true",
                    help="run only the potential-solve leg and print its record (for profiling)")
    ap.add_argument("--serve-requests", type=int, default=120,
                    help="requests in the serving trace (0 skips the serving leg)")
    ap.add_argument("--serve-horizon", type=float, default=50.0,
                    help="seconds each serving run lasts (the rest is reported as backlog)")
    ap.add_argument("--serve-whole-limit", type=float, default=240.0,
                    help="the chosen serving form also serves the whole trace, up to this many "
                         "seconds (0 skips it)")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run the probe's copy kernel over this size (a kernel of known "
                         "traffic, to calibrate HBM byte counters under a profiler)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)
    if args.steps % 2:
        args.steps += 1  # whole AA step pairs (even + odd)

    import torch
    import paper_2110_13055_amd as P

    if args.copy_probe_mib > 0:
        a = torch.ones(args.copy_probe_mib << 18, dtype=torch.int32, device="cuda")
        b = torch.empty_like(a)
        P.bandwidth_probe(P.PROBE_COPY, b, a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()
    if args.potential_only:
        print(json.dumps({"workload": WORKLOAD, "potential": potential_rates()}), flush=True)
        return
    strm = P.STREAM_PULL if args.streaming == "pull" else P.STREAM_AA
    log("fused / flow / ion steps, FP32")
    r32 = gpu_rates(P.FP32, args.steps, args.warmup, strm)
    log("FP16 populations")
    rh16 = gpu_rates(P.FP16, args.steps, args.warmup, strm)
    log("FP16 deviations")
    r16 = gpu_rates(P.FP16_DEV, args.steps, args.warmup, strm)
    log("moments")
    rmo = gpu_rates(P.MOMENTS, args.steps, args.warmup, strm)
    nf = r32["n_fluid"]
    K = args.steps

    def mlups(sec):
        return nf * K / sec / 1e6

    def form(name, r):
        return {"fused_mlups": round(mlups(r["fused_s"]), 1),
                "lbm_mlups": round(mlups(r["lbm_s"]), 1),
                "np_mlups": round(mlups(r["np_s"]), 1),
                "algorithmic_bytes_per_node": BYTES_FUSED[name],
                "fused_gbs": round(BYTES_FUSED[name] * nf / (r["fused_s"] / K) / 1e9, 1),
                "lbm_gbs": round(BYTES_LBM[name] * nf / (r["lbm_s"] / K) / 1e9, 1),
                "np_gbs": round(BYTES_NP * nf / (r["np_s"] / K) / 1e9, 1)}

    ms_step = r32["fused_s"] / K * 1e3
    achieved = BYTES_FUSED["fp32"] * nf / (r32["fused_s"] / K) / 1e9
    traffic = measured_traffic("fp32")
    out = {
        "metric": "MLUPS coupled LBM+NP step (FP32 vs FP16-store); solves/hr + p50/p99 latency",
        "value": round(mlups(r32["fused_s"]), 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "lattice": "D3Q19 512^3", "porosity": 0.4,
                   "n_fluid": nf, "storage": "fp32", "streaming": args.streaming,
                   "step": "fused LBM+NP"},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "algorithmic_bytes_per_node": BYTES_FUSED["fp32"]},
        "fp32": form("fp32", r32),
        "fp16": form("fp16", rh16),
        "fp16_dev": form("fp16_dev", r16),
        "moments": form("moments", rmo),
        "device": torch.cuda.get_device_name(0),
    }
    if not args.no_probe:
        log("bandwidth probe")
        out["hbm_probe"] = hbm_probe()
        # the same achieved rate against what a plain copy attains on this GPU
        cp = out["hbm_probe"]["copy_gbs"]
        out["roofline"]["attainable_copy_gbs"] = cp
        out["roofline"]["frac_of_copy"] = round(achieved / cp, 4)
    if not args.no_potential:
        log("potential")
        out["potential"] = potential_rates()
    if not args.no_batch:
        log("batched, 64 cubes of edge 48-160")
        out["batched"] = batched_rates(K, strm)
        log("batched, 64 cubes of edge 48-64")
        out["batched_small"] = small_batch_rates(K, strm)
    if args.serve_requests > 0:
        H = args.serve_horizon
        sv = {"requests": args.serve_requests, "rate_hz": 2.0, "budget_gb": 200, "horizon_s": H,
              "slots": SERVE_SLOTS, "max_active_nodes": SERVE_ACTIVE_NODES}
        log("serving: continuous batching, moments")
        sv["continuous_batching_moments"] = serving_run(args.serve_requests, P.MOMENTS, SERVE_SLOTS, strm, H,
                                                         SERVE_ACTIVE_NODES)
        log("serving: continuous batching, FP32")
        sv["continuous_batching_fp32"] = serving_run(args.serve_requests, P.FP32, SERVE_SLOTS, strm, H,
                                                      SERVE_ACTIVE_NODES)
        log("serving: FP32 one at a time")
        sv["plain_fp32_one_at_a_time"] = serving_run(args.serve_requests, P.FP32, 1, strm, H)
        if args.serve_whole_limit > 0:
            log("serving: continuous batching, moments, the whole trace")
            sv["continuous_batching_moments_whole_trace"] = serving_run(
                args.serve_requests, P.MOMENTS, SERVE_SLOTS, strm, args.serve_whole_limit, SERVE_ACTIVE_NODES)
        out["serving"] = sv
    if not args.no_cpu:
        log("CPU baseline (FP64 oracle)")
        out["cpu_baseline"] = cpu_baseline()
    log("done")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
