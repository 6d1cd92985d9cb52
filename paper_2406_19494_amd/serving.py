"""Continuous-batching request server for forward and gradient solves.

Requests (a solve of one workload family and size, forward or gradient, with a
step count) arrive over time.  The scheduler admits them FIFO into slots while
the sum of their device footprints (state + workspace, as reported by the
library) stays within an HBM budget, keeps every admitted solve's state
resident on the device, and advances all active solves in epochs of
``steps_per_epoch`` steps.  Each slot runs on its own HIP stream, so the
kernels of different solves overlap on the GPU; a forward epoch is one replay
of a hipGraph captured at admission, a gradient epoch advances the library's
incremental checkpointed gradient.  A slot is refilled as soon as its request
finishes (continuous batching), and every request's latency is recorded.

The scheduling logic (``Scheduler``) is independent of the GPU: it drives a
backend object, so the admission and batching rules are tested on the CPU with
a simulated backend.  ``GpuBackend`` is the real one.
"""
from __future__ import annotations

import dataclasses
import math
import time
from collections import deque
from typing import Dict, List, Optional

import numpy as np

from . import workloads as W

FAMILIES = ("sod", "tgv", "bl")


@dataclasses.dataclass
class RequestSpec:
    rid: int
    family: str       # "sod" | "tgv" | "bl"
    size: int         # sod: cells; tgv: cells per side; bl: scale s -> (256 s) x (64 s)
    kind: str         # "forward" | "gradient"
    nsteps: int
    arrival: float    # seconds after the start of the trace


@dataclasses.dataclass
class RequestResult:
    rid: int
    status: str = "pending"   # ok | nonphysical | rejected | error
    arrival: float = 0.0
    admitted: float = math.nan
    finished: float = math.nan
    cell_stages: float = 0.0
    message: str = ""
    output: Optional[dict] = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival


def draw_trace(M: int, rate: float, seed: int, steps=(50, 2000), sod=(200, 4096),
               tgv=(32, 48, 64, 96, 128), bl=(1, 2, 3, 4), families=FAMILIES,
               gradient_fraction=0.5) -> List[RequestSpec]:
    """Seeded request trace: Poisson arrivals (exponential gaps of mean
    1/rate), family uniform over `families`, sizes uniform over the given
    ranges/sets, step counts uniform over `steps`, forward/gradient mix."""
    u = [W.uniform01(seed, M, c) for c in range(6)]
    out = []
    t = 0.0
    for i in range(M):
        t += -math.log(1.0 - u[0][i]) / rate
        fam = families[min(int(u[1][i] * len(families)), len(families) - 1)]
        if fam == "sod":
            size = sod[0] + int(u[2][i] * (sod[1] - sod[0] + 1))
        elif fam == "tgv":
            size = tgv[min(int(u[2][i] * len(tgv)), len(tgv) - 1)]
        else:
            size = bl[min(int(u[2][i] * len(bl)), len(bl) - 1)]
        nsteps = steps[0] + int(u[3][i] * (steps[1] - steps[0] + 1))
        kind = "gradient" if u[4][i] < gradient_fraction else "forward"
        out.append(RequestSpec(i, fam, size, kind, nsteps, t))
    return out


def cells_of(spec: RequestSpec) -> int:
    if spec.family == "sod":
        return spec.size
    if spec.family == "tgv":
        return spec.size ** 3
    return (256 * spec.size) * (64 * spec.size)


_CASES: Dict[tuple, tuple] = {}


def build_case(spec: RequestSpec):
    """Case, initial primitives and porous coefficients of a request
    (cached per family and size).  Gradient requests differentiate the
    wall-pressure cost: the porous wall for the boundary layer, the cells next
    to the x- face for the other families."""
    key = (spec.family, spec.size)
    if key not in _CASES:
        if spec.family == "sod":
            case, P = W.sod(spec.size)
            K = None
            case.cost_face, case.p_inf = 1, 0.1
        elif spec.family == "tgv":
            case, P = W.tgv(spec.size)
            K = None
            case.cost_face, case.p_inf = 0, case.R
        else:
            s = spec.size
            case, P, K = W.porous_bl(nx=256 * s, ny=64 * s)
        _CASES[key] = (case, P, K)
    return _CASES[key]


def register_case(family: str, size: int, case, P, K=None):
    """Serve requests of (family, size) with this case, initial primitives
    and boundary parameters instead of the family's built-in one."""
    _CASES[(family, size)] = (case, P, K)


def seg_len_for(nsteps: int) -> int:
    """Checkpoint spacing ~ sqrt(n) (memory ~ 2 sqrt(n) states)."""
    return max(1, int(round(math.sqrt(nsteps))))


class Scheduler:
    """FIFO admission under an HBM budget and a slot limit; continuous
    batching in epochs.  `backend` provides footprint/start/step/poll/finish."""

    def __init__(self, backend, budget_bytes: float, max_slots: int = 16,
                 clock=time.perf_counter, idle_sleep: float = 2e-4, on_finish=None):
        self.b = backend
        self.on_finish = on_finish  # called as on_finish(result) as each solve retires
        self.budget = float(budget_bytes)
        self.max_slots = max_slots
        self.clock = clock
        self.idle_sleep = idle_sleep
        self.in_use = 0.0
        self.peak_in_use = 0.0
        self.peak_active = 0

    def run(self, trace: List[RequestSpec], realtime: bool = True) -> Dict[int, RequestResult]:
        pending = deque(sorted(trace, key=lambda r: (r.arrival, r.rid)))
        queue: deque = deque()
        active: list = []
        results: Dict[int, RequestResult] = {}
        t0 = self.clock()
        now = lambda: self.clock() - t0  # noqa: E731
        while pending or queue or active:
            t = now()
            while pending and (pending[0].arrival <= t or not realtime):
                r = pending.popleft()
                results[r.rid] = RequestResult(r.rid, arrival=r.arrival if realtime else 0.0)
                queue.append(r)
            # admission, FIFO: the head waits until it fits (no overtaking)
            while queue and len(active) < self.max_slots:
                r = queue[0]
                fp = self.b.footprint(r)
                if fp > self.budget:
                    queue.popleft()
                    res = results[r.rid]
                    res.status, res.message = "rejected", f"footprint {fp:.3e} B > budget"
                    res.admitted = res.finished = now()
                    continue
                if self.in_use + fp > self.budget:
                    break
                queue.popleft()
                try:
                    job = self.b.start(r)
                except Exception as e:  # isolate a request that cannot start
                    res = results[r.rid]
                    res.status, res.message = "error", str(e)
                    res.admitted = res.finished = now()
                    continue
                job.footprint = fp
                self.in_use += fp
                self.peak_in_use = max(self.peak_in_use, self.in_use)
                results[r.rid].admitted = now()
                active.append(job)
            self.peak_active = max(self.peak_active, len(active))
            # keep every active solve's stream fed; retire finished ones
            progressed = False
            for job in list(active):
                if self.b.poll(job):
                    if job.remaining == 0:
                        res = results[job.spec.rid]
                        self.b.finish(job, res)
                        res.finished = now()
                        res.cell_stages = 3.0 * cells_of(job.spec) * job.spec.nsteps
                        active.remove(job)
                        self.in_use -= job.footprint
                        progressed = True
                        if self.on_finish is not None:
                            self.on_finish(res)
                    else:
                        if not self.b.step(job) and not job.events:
                            raise RuntimeError(f"request {job.spec.rid}: no work in flight "
                                               f"but {job.remaining} remaining")
                        progressed = True
            flush = getattr(self.b, "flush", None)
            if flush is not None:
                flush()
            if not progressed:
                if not active and not queue and pending and realtime:
                    wait = pending[0].arrival - now()
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                elif self.idle_sleep:
                    time.sleep(self.idle_sleep)
        return results


def summarize(results: Dict[int, RequestResult], makespan: float) -> dict:
    ok = [r for r in results.values() if r.status == "ok"]
    lat = np.array([r.latency for r in ok]) if ok else np.array([math.nan])
    work = sum(r.cell_stages for r in ok)
    return {
        "requests": len(results), "completed": len(ok),
        "rejected": sum(r.status == "rejected" for r in results.values()),
        "failed": sum(r.status in ("error", "nonphysical") for r in results.values()),
        "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
        "mean_s": float(lat.mean()), "makespan_s": makespan,
        "cell_updates_per_s": work / makespan if makespan > 0 else math.nan,
    }


class _Entry:
    """A pooled solve: its context and workspace (Solver) and the device
    state and step arrays the requests that use it write into.  Entries are
    kept between requests of the same family, size and kind, so that
    retiring a request frees nothing (no device-wide synchronisation) and the
    next such request reuses the memory and, for forward requests, the
    captured epoch graph."""

    def __init__(self, key, solver, U, dt, nbytes):
        self.key = key
        self.solver = solver
        self.U = U
        self.dt = dt
        self.nbytes = nbytes
        self.graph = None      # forward: k-step epoch captured on first use


class GpuBackend:
    """Runs requests with the HIP library: each request on one of a few
    streams (the box has 4 hardware queues), forward epochs as replays of a
    hipGraph of k CFL steps, gradient epochs as units of the library's
    incremental checkpointed gradient.  Solves are pooled per (family, size,
    kind); gradient workspaces are sized for the longest trajectory
    (`grad_cap` steps, checkpoints every round(sqrt(grad_cap)) steps), so
    every gradient request of a family and size fits one."""

    def __init__(self, steps_per_epoch: int = 10, graphs: bool = True, keep_outputs: bool = False,
                 inflight: int = 2, fault: Optional[Dict[int, str]] = None, nstreams: int = 4,
                 grad_cap: int = 2000, budget_bytes: float = math.inf):
        import torch
        self.torch = torch
        self.k = steps_per_epoch
        self.graphs = graphs
        self.keep = keep_outputs
        self.inflight = inflight
        self.fault = fault or {}
        self.grad_cap = grad_cap
        self.grad_seg = seg_len_for(grad_cap)
        self.budget = budget_bytes
        self.streams = [torch.cuda.Stream() for _ in range(nstreams)]
        self._rr = 0
        self.pool: Dict[tuple, list] = {}   # idle entries per key
        self.idle_bytes = 0.0
        self.live_bytes = 0.0
        self._fp: Dict[tuple, float] = {}

    # -- sizes --------------------------------------------------------------
    def _key(self, spec: RequestSpec):
        return (spec.family, spec.size, spec.kind)

    def footprint(self, spec: RequestSpec) -> float:
        """Device bytes of a request: workspace (from the library's size
        formula, no context created), state, step, and for gradients the
        initial state, J, dJ/dtheta and dJ/dU0."""
        from .solver import workspace_bytes_for
        key = self._key(spec)
        if key not in self._fp:
            case, P, K = build_case(spec)
            state = 8 * case.nv * case.ncells
            if spec.kind == "gradient":
                ws = workspace_bytes_for(case, 2, self.grad_cap, self.grad_seg)
                extra = 2 * state
            else:
                ws = workspace_bytes_for(case, 0)
                extra = 0
            self._fp[key] = float(ws + state + extra + 4096)
        return self._fp[key]

    # -- pool -----------------------------------------------------------------
    def _entry(self, spec: RequestSpec) -> _Entry:
        torch = self.torch
        from .solver import Solver
        key = self._key(spec)
        free = self.pool.get(key)
        if free:
            e = free.pop()
            self.idle_bytes -= e.nbytes
            self.live_bytes += e.nbytes
            return e
        nbytes = self.footprint(spec)
        # idle entries of other keys give their memory back when a new one
        # would not fit beside them (the only place a context is destroyed
        # while serving)
        for k2 in list(self.pool):
            while self.pool[k2] and self.live_bytes + self.idle_bytes + nbytes > self.budget:
                old = self.pool[k2].pop()
                self.idle_bytes -= old.nbytes
                del old
        case, P, K = build_case(spec)
        if spec.kind == "gradient":
            solver = Solver(case, K=K, mode=2, nsteps=self.grad_cap, seg_len=self.grad_seg)
        else:
            solver = Solver(case, K=K, mode=0)
        # written (init_state, compute_dt) before anything reads them
        U = solver.empty_state()
        dt = torch.empty(1, dtype=torch.float64, device="cuda")
        e = _Entry(key, solver, U, dt, nbytes)
        self.live_bytes += nbytes
        return e

    def _release(self, e: _Entry):
        self.pool.setdefault(e.key, []).append(e)
        self.live_bytes -= e.nbytes
        self.idle_bytes += e.nbytes

    def _stream(self):
        st = self.streams[self._rr % len(self.streams)]
        self._rr += 1
        return st

    # -- lifecycle ------------------------------------------------------------
    def _init_job(self, spec: RequestSpec, stream):
        case, P, K = build_case(spec)
        if spec.rid in self.fault:
            P = P.copy()
            if self.fault[spec.rid] == "nonphysical":
                P[4].flat[len(P[4].flat) // 2] = -1.0
        job = _Job(spec)
        job.entry = self._entry(spec)
        job.solver, job.U, job.dt = job.entry.solver, job.entry.U, job.entry.dt
        job.stream = stream
        job.solver.init_state(P, stream=stream, out=job.U)
        return job

    def start(self, spec: RequestSpec):
        torch = self.torch
        job = self._init_job(spec, self._stream())
        s, case = job.solver, job.solver.case
        with torch.cuda.stream(job.stream):
            if spec.kind == "gradient":
                # the trajectory's step is fixed at the initial CFL step
                s.compute_dt(job.U, cfl=case.cfl, out=job.dt, stream=job.stream)
                job.J = torch.zeros(1, dtype=torch.float64, device="cuda")
                job.gK = torch.zeros(max(s.nk, 1), dtype=torch.float64, device="cuda")
                job.gU = torch.empty_like(job.U)
                s.gradient_begin(job.U, job.dt, job.J, job.gK, stream=job.stream,
                                 nsteps=spec.nsteps)
                job.remaining = 1
            else:
                job.remaining = spec.nsteps
                # the first CFL step; every step then returns the next one
                s.compute_dt(job.U, cfl=case.cfl, out=job.dt, stream=job.stream)
                e = job.entry
                if self.graphs and spec.nsteps >= self.k and e.graph is None:
                    # capture records without running (state unchanged so
                    # far); capture_begin/end directly, without the device
                    # synchronisation and cache release of torch.cuda.graph
                    e.graph = torch.cuda.CUDAGraph()
                    e.graph.capture_begin()
                    s.steps_cfl(job.U, job.dt, self.k, cfl=case.cfl, stream=job.stream)
                    e.graph.capture_end()
                job.graph = e.graph if self.graphs else None
        job.events = deque()
        for _ in range(self.inflight):
            if job.remaining:
                self.step(job)
        return job

    def step(self, job) -> bool:
        """Enqueue one epoch on the job's stream; False if nothing was left."""
        torch = self.torch
        spec = job.spec
        s = job.solver
        with torch.cuda.stream(job.stream):
            if spec.kind == "gradient":
                if job.enqueued_done:
                    return False
                done = s.gradient_advance(self.k * 4, stream=job.stream)
                if done:
                    s.gradient_finish(job.gU, stream=job.stream)
                    job.enqueued_done = True
                n = 0
            else:
                n = min(self.k, spec.nsteps - job.enqueued)
                if n <= 0:
                    return False
                if job.graph is not None and n == self.k:
                    job.graph.replay()
                else:
                    s.steps_cfl(job.U, job.dt, n, cfl=s.case.cfl, stream=job.stream)
                job.enqueued += n
            ev = torch.cuda.Event()
            ev.record(job.stream)
            job.events.append((ev, n))
        return True

    def poll(self, job) -> bool:
        """True when the oldest in-flight epoch has completed (or nothing is
        in flight); updates job.remaining."""
        if job.events:
            ev, n = job.events[0]
            if not ev.query():
                return False
            job.events.popleft()
            job.completed += n
        if job.spec.kind == "gradient":
            job.remaining = 0 if (job.enqueued_done and not job.events) else 1
        else:
            job.remaining = job.spec.nsteps - job.completed
        return True

    def finish(self, job, res: RequestResult):
        # every epoch of the job has completed (poll): reading its flags and
        # outputs waits on nothing else
        flags = job.solver.flags(stream=job.stream)
        res.status = "ok" if flags == 0 else "nonphysical"
        if self.keep and res.status == "ok":
            if job.spec.kind == "gradient":
                res.output = {"J": job.J.item(), "dJdK": job.gK.cpu().numpy()[: job.solver.nk],
                              "dJdU0": job.gU.cpu().numpy(), "dt": job.dt.item()}
            else:
                res.output = {"U": job.U.cpu().numpy()}
        self._release(job.entry)
        job.solver = job.U = job.graph = job.entry = None


class _Job:
    def __init__(self, spec):
        self.spec = spec
        self.solver = None
        self.entry = None
        self.graph = None
        self.U = self.dt = self.J = self.gK = self.gU = None
        self.remaining = spec.nsteps
        self.enqueued = 0
        self.completed = 0
        self.enqueued_done = False
        self.footprint = 0.0
        self.events = deque()
        self.batched = False


class _Family:
    """Forward solves of one family on one stream: the current batch plan
    and the hipGraph of k batched steps captured for it."""

    def __init__(self, stream):
        self.stream = stream
        self.members = ()
        self.plan = None
        self.graph = None
        self.retired = deque(maxlen=4)  # previous (plan, graph) pairs kept alive a while


class BatchedGpuBackend(GpuBackend):
    """Small forward solves (at most batch_max_cells cells: too few
    workgroups per launch to fill the GPU alone) of one family (grid
    dimension, viscous or not, no source) advance together: an epoch is one
    replay of a hipGraph of k batched steps (one launch per kernel and stage
    for all members, dcf_batch_rk3_step_table over a device table written
    outside the capture), on the family's stream.  The graph is captured
    again only when the members change; a member with fewer than k steps
    left runs them eagerly.  Larger forward solves and gradient solves run as
    in GpuBackend (per-solve graph epochs on the shared streams), so that
    solves which fill the GPU by themselves still overlap instead of queueing
    on one family stream."""

    def __init__(self, steps_per_epoch: int = 10, keep_outputs: bool = False, inflight: int = 2,
                 fault: Optional[Dict[int, str]] = None, budget_bytes: float = math.inf,
                 batch_max_cells: int = 1 << 17):
        super().__init__(steps_per_epoch=steps_per_epoch, graphs=True, keep_outputs=keep_outputs,
                         inflight=inflight, fault=fault, budget_bytes=budget_bytes)
        self.batch_max_cells = batch_max_cells
        self.families: Dict[tuple, _Family] = {}
        self.want: Dict[tuple, list] = {}
        self.recaptures = 0

    @staticmethod
    def _fkey(case):
        return (case.ndim, case.visc_law != "none", case.cfl)

    def start(self, spec: RequestSpec):
        case, _, _ = build_case(spec)
        if spec.kind == "gradient" or case.source != "none" or cells_of(spec) > self.batch_max_cells:
            return super().start(spec)
        torch = self.torch
        fk = self._fkey(case)
        if fk not in self.families:
            self.families[fk] = _Family(torch.cuda.Stream())
        fam = self.families[fk]
        job = self._init_job(spec, fam.stream)
        job.batched = True
        job.fkey = fk
        job.remaining = spec.nsteps
        job.events = deque()
        for _ in range(self.inflight):
            if job.remaining:
                self.step(job)
        self.flush()
        return job

    def step(self, job) -> bool:
        if not job.batched:
            return super().step(job)
        n = min(self.k, job.spec.nsteps - job.enqueued)
        if n <= 0:
            return False
        self.want.setdefault(job.fkey, []).append((job, n))
        job.enqueued += n
        return True

    def _graph_for(self, fam: _Family, jobs, cfl):
        torch = self.torch
        from .solver import BatchPlan
        members = tuple(id(j.entry) for j in jobs)
        if members == fam.members and fam.graph is not None:
            return fam.graph
        if fam.plan is not None:
            fam.retired.append((fam.plan, fam.graph))
        plan = BatchPlan([j.solver for j in jobs], [j.U for j in jobs], [j.dt for j in jobs],
                         stream=fam.stream)
        # the table copy precedes the replays on the family stream; the
        # capture itself records launches only
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.stream(fam.stream):
            graph.capture_begin()
            for _ in range(self.k):
                plan.step(cfl=cfl, stream=fam.stream)
            graph.capture_end()
        fam.members, fam.plan, fam.graph = members, plan, graph
        self.recaptures += 1
        return graph

    def flush(self):
        """Launch the requested epochs: per family, the members that asked
        for a full epoch replay the family's graph together; shorter final
        epochs run eagerly (a CFL step, then that many fused CFL steps)."""
        torch = self.torch
        for fk, reqs in self.want.items():
            fam = self.families.get(fk)
            while reqs:
                # one round: at most one pending epoch per solve
                seen, rnd, rest = set(), [], []
                for j, n in reqs:
                    (rest if id(j) in seen else rnd).append((j, n))
                    seen.add(id(j))
                reqs[:] = rest
                full = [j for j, n in rnd if n == self.k]
                part = [(j, n) for j, n in rnd if n < self.k]
                with torch.cuda.stream(fam.stream):
                    if full:
                        full.sort(key=lambda j: id(j.entry))
                        self._graph_for(fam, full, fk[2]).replay()
                    for j, n in part:
                        s = j.solver
                        s.compute_dt(j.U, cfl=s.case.cfl, out=j.dt, stream=fam.stream)
                        s.steps_cfl(j.U, j.dt, n, cfl=s.case.cfl, stream=fam.stream)
                    ev = torch.cuda.Event()
                    ev.record(fam.stream)
                for j, n in rnd:
                    j.events.append((ev, n))


def serve(trace, budget_bytes=200e9, max_slots=16, steps_per_epoch=10, graphs=True,
          keep_outputs=False, realtime=True, fault=None, batched=False, backend=None,
          on_finish=None):
    """Serve a trace; returns (results, makespan in s, scheduler).  A backend
    may be passed in to keep its pooled solves between calls."""
    if backend is None:
        if batched:
            backend = BatchedGpuBackend(steps_per_epoch=steps_per_epoch,
                                        keep_outputs=keep_outputs, fault=fault,
                                        budget_bytes=budget_bytes)
        else:
            backend = GpuBackend(steps_per_epoch=steps_per_epoch, graphs=graphs,
                                 keep_outputs=keep_outputs, fault=fault,
                                 budget_bytes=budget_bytes)
    sch = Scheduler(backend, budget_bytes, max_slots, on_finish=on_finish)
    t0 = time.perf_counter()
    res = sch.run(trace, realtime=realtime)
    backend.torch.cuda.synchronize()
    return res, time.perf_counter() - t0, sch


def serve_sequential(trace, steps_per_epoch=10, graphs=True, keep_outputs=False, realtime=True,
                     backend=None, on_finish=None):
    """Baseline: the same trace FIFO, one solve at a time on the same GPU."""
    return serve(trace, budget_bytes=float("inf"), max_slots=1, steps_per_epoch=steps_per_epoch,
                 graphs=graphs, keep_outputs=keep_outputs, realtime=realtime, backend=backend,
                 on_finish=on_finish)
