"""Continuous-batching solve server.

Requests (a seeded electrode plus its parameters: one point of the paper's
sweeps over porosity, applied potential and inlet velocity, Sec. 4-5) arrive
over time. The server admits a request when a slot is free and its HBM
footprint fits the budget, keeps its state resident on the GPU, and advances
all admitted requests together in rounds. A round is one batched advance per
group (requests of one lattice dimension and storage precision form a group;
each group has its own stream, so the 2D and 3D groups overlap on the device).
Before a request takes a slot its flow is checked on the host: an inlet
velocity that would need a density drop beyond the weakly compressible
range of the lattice Boltzmann method (Kozeny-Carman estimate,
``cdi_flow_check``) is rejected at once. A request runs its flow phase in
rounds until its steady-state residual reaches the tolerance, stops falling
(no new minimum for ``stagnation_rounds`` rounds: the floor of
single-precision storage) or its flow budget is spent, then its ion phase on
the frozen flow for the requested number of steps; it is then retired:
results read back, slot and memory released. A request whose flow stopped
short of its tolerance retires as ``ok_unconverged`` (its reached residual is
in the result). Latency is arrival to result.

Members join and leave each group's batch in place (``cdi_batch_admit`` /
``cdi_batch_retire`` on a batch created with room to spare): no new
workspace, and the captured step graph is kept while the launch shape
allows.

A request's step sequence depends only on the request (rounds of
``round_steps`` counted from its own admission, the phase switch decided by
its own residual), and a batched step equals a solo step bit for bit, so a
result is the same alone and in any mix.

The scheduler talks to an executor: ``GpuExecutor`` drives libcdi through the
binding; the protocol is small enough for test doubles (``start``,
``footprint_estimate``, ``footprint``, ``group_key``, ``advance``, ``finish``,
``release``, and optionally ``check``).
"""
from __future__ import annotations

import math
import re
import time
from dataclasses import dataclass
from typing import Callable, Dict, List, Optional, Tuple

import numpy as np

from . import _lib as L


@dataclass
class Request:
    rid: int
    arrival_s: float
    geom: object            # solver.Geometry
    params: object          # solver.Params
    flow_tol: float = 1e-6
    flow_max_steps: int = 20000
    np_steps: int = 5000


@dataclass
class Result:
    rid: int
    arrival_s: float
    admitted_s: float
    finished_s: float
    footprint: int
    flow_steps: int = 0
    residual: float = math.nan
    np_steps: int = 0
    adsorbed: tuple = (math.nan, math.nan)
    balance: tuple = ()
    status: str = "ok"
    flow_stop: str = ""     # why the flow phase ended: tol, stagnated or step_limit

    @property
    def latency_s(self) -> float:
        return self.finished_s - self.arrival_s


@dataclass
class _Active:
    req: Request
    handle: object
    admitted_s: float
    footprint: int
    phase: int = L.MODE_FLOW
    flow_steps: int = 0
    np_done: int = 0
    residual: float = math.inf
    best: float = math.inf
    since_best: int = 0
    converged: bool = False
    stop: str = ""
    work: int = 0        # fluid nodes it adds to each step of its group


_MEMBER = re.compile(r"member (\d+):")


class GpuExecutor:
    """Solver per request, one Batch per group, one stream per group."""

    # per-request device overhead not in the plan's node bytes (batch
    # descriptors, tile lists, allocator rounding)
    OVERHEAD = 4 << 20

    def __init__(self, device: str = "cuda", keep_fields: bool = False, max_members: int = 64,
                 max_fluid: int = 1 << 26, max_drho: float = 0.0):
        import torch
        from .solver import Batch, Solver, flow_check, plan
        self.torch = torch
        self.Solver, self.Batch, self.plan, self.flow_check = Solver, Batch, plan, flow_check
        self.device = torch.device(device)
        self.keep_fields = keep_fields
        self.max_members, self.max_fluid, self.max_drho = int(max_members), int(max_fluid), float(max_drho)
        self.streams: Dict[tuple, object] = {}
        self._batches: Dict[tuple, object] = {}   # group -> Batch with room to admit
        self._planned = (None, None)               # the last request planned and its plan

    def _stream(self, key):
        if key not in self.streams:
            self.streams[key] = self.torch.cuda.Stream(device=self.device)
        return self.streams[key]

    def check(self, req: Request):
        """(admissible, message): the host-side flow check."""
        ok, est, msg = self.flow_check(req.geom, req.params, self.max_drho)
        return ok, msg

    def _plan(self, req: Request):
        if self._planned[0] != req.rid:
            self._planned = (req.rid, self.plan(req.geom, req.params))
        return self._planned[1]

    def footprint_estimate(self, req: Request) -> int:
        info = self._plan(req)
        return int(info.vox_bytes + info.node_bytes_per_fluid * max(info.n_fluid_est, 1) * 1.1
                   + self.OVERHEAD)

    def work_estimate(self, req: Request) -> int:
        """Fluid nodes the request would add to a step (the plan's estimate)."""
        return int(self._plan(req).n_fluid_est)

    def work(self, handle) -> int:
        return int(handle.n_fluid)

    def start(self, req: Request):
        key = (req.geom.dim, req.params.precision)
        return self.Solver(req.geom, req.params, device=str(self.device), stream=self._stream(key))

    def footprint(self, handle) -> int:
        return handle.footprint_bytes + self.OVERHEAD

    def group_key(self, handle):
        return (handle.dim, handle.params.precision)

    def _batch_for(self, key, members):
        """The group's batch holding exactly `members`, in that order: members
        that left are retired and new ones admitted in place; a batch that is
        full is replaced by one with twice the room."""
        b = self._batches.get(key)
        if b is None:
            b = self._batches[key] = self.Batch(stream=self._stream(key), capacity=(self.max_members, self.max_fluid),
                                                device=str(self.device))
        want = {id(m) for m in members}
        for m in list(b.members):
            if id(m) not in want:
                b.retire(m)
        have = [id(m) for m in b.members]
        if have != [id(m) for m in members[:len(have)]]:   # order differs: start over
            for m in list(b.members):
                b.retire(m)
        for m in members[len(b.members):]:
            try:
                b.admit(m)
            except L.CdiError as exc:
                if exc.code != L.E_BUFFER:
                    raise
                cap_n = max(self.max_members, 2 * len(members))
                self.max_fluid *= 2
                old = b
                b = self._batches[key] = self.Batch(list(old.members), stream=self._stream(key),
                                                    capacity=(cap_n, self.max_fluid), device=str(self.device))
                old.close()
                b.admit(m)
        return b

    def advance(self, groups: Dict[tuple, List[object]], modes: Dict[tuple, List[int]], nsteps: int):
        """Every group advances nsteps (groups overlap on their streams).
        Returns (residuals per group, failures {group: (member, message)});
        a failed group was not stepped."""
        failed = {}
        for key, members in groups.items():
            b = self._batch_for(key, members)
            try:
                b.advance(nsteps, modes[key])
            except L.CdiError as exc:
                m = _MEMBER.search(str(exc))
                if exc.code != L.E_UNSTABLE or m is None:
                    raise
                failed[key] = (int(m.group(1)), str(exc))
        res = {key: self._batches[key].residuals() for key in groups if key not in failed}
        return res, failed

    def finish(self, handle):
        out = {"adsorbed": handle.adsorbed_total(), "balance": handle.mass_balance()}
        if self.keep_fields:
            out["concentration"] = handle.concentration()
            out["velocity"] = handle.velocity()
        return out

    def release(self, handle):
        for b in self._batches.values():
            if any(m is handle for m in b.members):
                b.retire(handle)
        handle.synchronize()
        handle.close()

    def close(self):
        for b in self._batches.values():
            b.close()
        self._batches.clear()


class Server:
    """Admission, continuous batching and retirement over an executor."""

    def __init__(self, executor, budget_bytes: float = 200e9, max_slots: int = 64,
                 round_steps: int = 200, stagnation_rounds: int = 3,
                 max_active_nodes: float = math.inf,
                 clock: Optional[Callable[[], float]] = None,
                 sleep: Optional[Callable[[float], None]] = None):
        if round_steps < 2:
            raise ValueError("round_steps must be >= 2 (the residual spans two steps)")
        self.ex = executor
        self.budget = float(budget_bytes)
        self.max_slots = int(max_slots)
        self.round_steps = int(round_steps)
        self.stagnation_rounds = int(stagnation_rounds)
        # fluid nodes stepped together at most (the first request is always
        # admitted): past what fills the GPU, batching more only time-slices it
        self.max_active_nodes = float(max_active_nodes)
        self.active_nodes = 0
        self._est: Dict[int, object] = {}   # queued request -> (footprint, work) or a rejection
        self.clock = clock or time.perf_counter
        self.sleep = sleep or time.sleep
        self.queue: List[Request] = []
        self.active: List[_Active] = []
        self.results: List[Result] = []
        self.fields: Dict[int, dict] = {}
        self.used = 0
        self.rounds = 0
        self.peak_slots = 0
        self.peak_bytes = 0
        self.backlog = 0
        self.t0 = 0.0

    def _now(self) -> float:
        return self.clock() - self.t0

    # ------------------------------------------------------------ admission
    def _estimates(self, req: Request):
        """(footprint, work) of a queued request, or a rejection message. The
        host-side check and plan run once per request; a head of the queue
        that waits for room is not planned again every round."""
        if req.rid in self._est:
            return self._est[req.rid]
        check = getattr(self.ex, "check", None)
        out = None
        if check is not None:
            ok, msg = check(req)
            if not ok:  # refused before it takes a slot
                out = f"rejected: unstable flow: {msg}"
        if out is None:
            try:
                est = self.ex.footprint_estimate(req)
                work_estimate = getattr(self.ex, "work_estimate", None)
                out = (est, work_estimate(req) if work_estimate is not None else 0)
            except Exception as exc:  # e.g. its electrode cannot be generated: refused, nothing else affected
                out = f"rejected: {exc}"
        self._est[req.rid] = out
        return out

    def _admit(self):
        while self.queue and len(self.active) < self.max_slots:
            req = self.queue[0]
            now = self._now()
            est = self._estimates(req)
            if isinstance(est, str):
                self.queue.pop(0)
                self._est.pop(req.rid, None)
                self.results.append(Result(req.rid, req.arrival_s, now, now, 0, status=est))
                continue
            est, work_est = est
            if est > self.budget:
                self.queue.pop(0)
                self._est.pop(req.rid, None)
                self.results.append(Result(req.rid, req.arrival_s, now, now, est,
                                           status="rejected: footprint exceeds the budget"))
                continue
            if self.used + est > self.budget:
                break  # FIFO: wait until retirements free memory
            if self.active and self.active_nodes + work_est > self.max_active_nodes:
                break  # FIFO: wait until the active work drops
            self.queue.pop(0)
            self._est.pop(req.rid, None)
            try:
                h = self.ex.start(req)
            except Exception as exc:  # a failed request retires only itself
                self.results.append(Result(req.rid, req.arrival_s, now, self._now(), est,
                                           status=f"failed: {exc}"))
                continue
            fp = self.ex.footprint(h)
            work = self.ex.work(h) if hasattr(self.ex, "work") else 0
            self.used += fp
            self.active_nodes += work
            self.active.append(_Active(req, h, now, fp, work=work))
        self.peak_slots = max(self.peak_slots, len(self.active))
        self.peak_bytes = max(self.peak_bytes, self.used)

    def _retire(self, a: _Active, status: str):
        out = {}
        if status == "ok" and not a.converged:
            status = "ok_unconverged"
        if status in ("ok", "ok_unconverged"):
            try:
                out = self.ex.finish(a.handle)
            except Exception as exc:
                status = f"failed: {exc}"
        self.ex.release(a.handle)
        self.used -= a.footprint
        self.active_nodes -= a.work
        self.active.remove(a)
        ads = tuple(np.asarray(out["adsorbed"], dtype=float).tolist()) if "adsorbed" in out else (math.nan,) * 2
        bal = tuple(np.asarray(out["balance"], dtype=float).reshape(-1).tolist()) if "balance" in out else ()
        self.results.append(Result(a.req.rid, a.req.arrival_s, a.admitted_s, self._now(), a.footprint,
                                   a.flow_steps, a.residual, a.np_done, ads, bal, status, a.stop))
        extra = {k: v for k, v in out.items() if k not in ("adsorbed", "balance")}
        if extra:
            self.fields[a.req.rid] = extra

    # ------------------------------------------------------------ main loop
    def run(self, requests: List[Request], horizon_s: float = math.inf,
            progress: Optional[Callable[[str], None]] = None, progress_every_s: float = 10.0) -> List[Result]:
        """Serve requests (arrival_s relative to the start of the run). Ends
        when all are done, or at horizon_s; what is left then is the backlog
        (queued, not yet arrived, or still active). progress (optional)
        receives a status line every progress_every_s seconds."""
        pending = sorted(requests, key=lambda r: (r.arrival_s, r.rid))
        self.t0 = self.clock()
        i = 0
        next_report = progress_every_s
        while True:
            now = self._now()
            if progress is not None and now >= next_report:
                progress(f"t={now:.0f} s: {len(self.results)} done, {len(self.active)} active, "
                         f"{len(self.queue)} queued, {len(pending) - i} to arrive")
                next_report += progress_every_s
            while i < len(pending) and pending[i].arrival_s <= now:
                self.queue.append(pending[i])
                i += 1
            if now >= horizon_s:
                break
            self._admit()
            if self.active:
                self._round()
            elif self.queue:
                raise RuntimeError("a queued request cannot be admitted on an idle server")
            elif i < len(pending):
                self.sleep(max(0.0, min(pending[i].arrival_s, horizon_s) - now))
            else:
                break
        self.backlog = len(self.queue) + (len(pending) - i) + len(self.active)
        return self.results

    def _round(self):
        groups: Dict[tuple, List[object]] = {}
        modes: Dict[tuple, List[int]] = {}
        owners: Dict[tuple, List[_Active]] = {}
        for a in self.active:
            key = self.ex.group_key(a.handle)
            groups.setdefault(key, []).append(a.handle)
            owners.setdefault(key, []).append(a)
            modes.setdefault(key, []).append(a.phase)
        n = self.round_steps
        res, failed = self.ex.advance(groups, modes, n)
        self.rounds += 1
        retire: List[Tuple[_Active, str]] = []
        for key, lst in owners.items():
            if key in failed:
                # nothing of this group was stepped; only the named member leaves
                k, msg = failed[key]
                retire.append((lst[k], f"failed: {msg}"))
                continue
            r = res[key]
            for k, a in enumerate(lst):
                if a.phase == L.MODE_FLOW:
                    a.flow_steps += n
                    a.residual = float(r[k])
                    if a.residual < a.best:
                        a.best, a.since_best = a.residual, 0
                    else:
                        a.since_best += 1
                    if not math.isfinite(a.residual):
                        retire.append((a, "failed: flow diverged"))
                    elif (a.residual <= a.req.flow_tol or a.since_best >= self.stagnation_rounds
                          or a.flow_steps >= a.req.flow_max_steps):
                        a.converged = a.residual <= a.req.flow_tol
                        a.stop = ("tol" if a.converged else
                                  "step_limit" if a.flow_steps >= a.req.flow_max_steps else "stagnated")
                        a.phase = L.MODE_IONS
                        if a.req.np_steps <= 0:
                            retire.append((a, "ok"))
                else:
                    a.np_done += n
                    if a.np_done >= a.req.np_steps:
                        retire.append((a, "ok"))
        for a, status in retire:
            self._retire(a, status)


def poisson_arrivals(n: int, rate_hz: float, seed: int) -> List[float]:
    """Arrival times of a Poisson process (exponential gaps) with a fixed seed."""
    rng = np.random.default_rng(seed)
    return np.cumsum(rng.exponential(1.0 / rate_hz, size=n)).tolist()


def latency_stats(results: List[Result], wall_s: float) -> dict:
    """Completed = results delivered ("ok", or "ok_unconverged": flow stopped
    short of its tolerance, counted apart too); latency over those."""
    ok = [r for r in results if r.status in ("ok", "ok_unconverged")]
    lat = np.array([r.latency_s for r in ok], dtype=float)
    unc = np.array([r.residual for r in ok if r.status == "ok_unconverged"], dtype=float)
    return {
        "completed": len(ok),
        "unconverged": sum(1 for r in ok if r.status == "ok_unconverged"),
        "rejected": sum(1 for r in results if r.status.startswith("rejected")),
        "failed": sum(1 for r in results if r.status.startswith("failed")),
        "solves_per_hour": len(ok) / wall_s * 3600.0 if wall_s > 0 else math.nan,
        "p50_s": float(np.percentile(lat, 50)) if ok else math.nan,
        "p99_s": float(np.percentile(lat, 99)) if ok else math.nan,
        "mean_s": float(lat.mean()) if ok else math.nan,
        # how the delivered requests' flow phases ended, and how far the
        # unconverged ones were from their tolerance
        "flow_stops": {k: sum(1 for r in ok if r.flow_stop == k) for k in ("tol", "stagnated", "step_limit")},
        "unconverged_residual_median": float(np.median(unc)) if len(unc) else math.nan,
    }
