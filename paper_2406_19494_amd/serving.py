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


def seg_len_for(nsteps: int) -> int:
    """Checkpoint spacing ~ sqrt(n) (memory ~ 2 sqrt(n) states)."""
    return max(1, int(round(math.sqrt(nsteps))))


class Scheduler:
    """FIFO admission under an HBM budget and a slot limit; continuous
    batching in epochs.  `backend` provides footprint/start/step/poll/finish."""

    def __init__(self, backend, budget_bytes: float, max_slots: int = 16,
                 clock=time.perf_counter, idle_sleep: float = 2e-4):
        self.b = backend
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


class GpuBackend:
    """Runs requests with the HIP library: one stream per slot, hipGraph
    replays for forward epochs, incremental gradients for gradient epochs."""

    def __init__(self, steps_per_epoch: int = 10, graphs: bool = True, keep_outputs: bool = False,
                 inflight: int = 2, fault: Optional[Dict[int, str]] = None):
        import torch
        self.torch = torch
        self.k = steps_per_epoch
        self.graphs = graphs
        self.keep = keep_outputs
        self.inflight = inflight
        self.fault = fault or {}

    # -- sizes --------------------------------------------------------------
    def footprint(self, spec: RequestSpec) -> float:
        from . import binding as B
        import ctypes as C
        case, P, K = build_case(spec)
        from .solver import Solver
        # measure with a context (no workspace yet): state + workspace + dt/J
        mode = 2 if spec.kind == "gradient" else 0
        seg = seg_len_for(spec.nsteps) if mode == 2 else 0
        key = (spec.family, spec.size, mode, spec.nsteps if mode == 2 else 0)
        cache = getattr(self, "_fp", {})
        self._fp = cache
        if key not in cache:
            g = B.dcf_grid()
            g.ndim = case.ndim
            for d in range(3):
                g.n[d], g.lo[d], g.hi[d] = case.n[d], case.lo[d], case.hi[d]
                g.stretch[d], g.beta[d] = B.STRETCH[case.stretch[d]], case.beta[d]
            gas = B.dcf_gas(case.gamma, case.R, case.Pr, B.VISC[case.visc_law], case.mu_ref,
                            case.T_ref, case.visc_param)
            ctx = C.c_void_p()
            B.call("dcf_create", C.byref(g), C.byref(gas), C.byref(ctx))
            size = C.c_size_t()
            B.call("dcf_workspace_size", ctx, mode, spec.nsteps if mode == 2 else 0, seg,
                   C.byref(size))
            B.lib().dcf_destroy(ctx)
            state = 8 * case.nv * case.ncells
            extra = 2 * state if mode == 2 else 0   # U0 copy and dJ/dU0
            cache[key] = float(size.value + state + extra)
        return cache[key]

    # -- lifecycle ------------------------------------------------------------
    def start(self, spec: RequestSpec):
        torch = self.torch
        from .solver import Solver
        case, P, K = build_case(spec)
        if spec.rid in self.fault:
            P = P.copy()
            if self.fault[spec.rid] == "nonphysical":
                P[4].flat[len(P[4].flat) // 2] = -1.0
        job = _Job(spec)
        job.stream = torch.cuda.Stream()
        with torch.cuda.stream(job.stream):
            if spec.kind == "gradient":
                job.solver = Solver(case, K=K, mode=2, nsteps=spec.nsteps,
                                    seg_len=seg_len_for(spec.nsteps))
            else:
                job.solver = Solver(case, K=K, mode=0)
            job.U = job.solver.init_state(P, stream=job.stream)
            job.dt = torch.empty(1, dtype=torch.float64, device="cuda")
            if spec.kind == "gradient":
                # the trajectory's step is fixed at the initial CFL step
                job.solver.compute_dt(job.U, cfl=case.cfl, out=job.dt, stream=job.stream)
                job.J = torch.zeros(1, dtype=torch.float64, device="cuda")
                job.gK = torch.zeros(max(job.solver.nk, 1), dtype=torch.float64, device="cuda")
                job.gU = torch.empty_like(job.U)
                job.solver.gradient_begin(job.U, job.dt, job.J, job.gK, stream=job.stream)
                job.remaining = 1
            else:
                job.remaining = spec.nsteps
                # the first CFL step; every step then returns the next one
                job.solver.compute_dt(job.U, cfl=case.cfl, out=job.dt, stream=job.stream)
                if self.graphs and spec.nsteps >= self.k:
                    job.graph = torch.cuda.CUDAGraph()
                    job.stream.synchronize()
                    with torch.cuda.graph(job.graph, stream=job.stream):
                        job.solver.steps_cfl(job.U, job.dt, self.k, cfl=case.cfl)
                    # capture records without running: state unchanged so far
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
        flags = job.solver.flags(stream=job.stream)
        res.status = "ok" if flags == 0 else "nonphysical"
        if self.keep and res.status == "ok":
            if job.spec.kind == "gradient":
                res.output = {"J": job.J.item(), "dJdK": job.gK.cpu().numpy()[: job.solver.nk],
                              "dJdU0": job.gU.cpu().numpy()}
            else:
                res.output = {"U": job.U.cpu().numpy()}
        job.solver = job.U = job.graph = None


class _Job:
    def __init__(self, spec):
        self.spec = spec
        self.solver = None
        self.graph = None
        self.U = self.dt = self.J = self.gK = self.gU = None
        self.remaining = spec.nsteps
        self.enqueued = 0
        self.completed = 0
        self.enqueued_done = False
        self.footprint = 0.0
        self.events = deque()


class BatchedGpuBackend(GpuBackend):
    """Forward solves of one family (grid dimension, viscous or not, no
    source) advance together: each epoch is k batched steps, one launch per
    kernel and stage for all of the family's active solves
    (dcf_batch_rk3_step), on the family's stream.  Gradient solves run as in
    GpuBackend.  Solves join and leave a family between epochs."""

    def __init__(self, steps_per_epoch: int = 10, keep_outputs: bool = False, inflight: int = 2,
                 fault: Optional[Dict[int, str]] = None):
        super().__init__(steps_per_epoch=steps_per_epoch, graphs=False, keep_outputs=keep_outputs,
                         inflight=inflight, fault=fault)
        self.families = {}   # key -> [stream, BatchStepper]
        self.want = {}       # key -> jobs that asked for an epoch

    @staticmethod
    def _key(job):
        c = job.solver.case
        return (c.ndim, c.visc_law != "none", c.cfl)

    def start(self, spec: RequestSpec):
        if spec.kind == "gradient":
            return super().start(spec)
        torch = self.torch
        from .solver import BatchStepper, Solver
        case, P, K = build_case(spec)
        if case.source != "none":
            return super().start(spec)
        if spec.rid in self.fault:
            P = P.copy()
            if self.fault[spec.rid] == "nonphysical":
                P[4].flat[len(P[4].flat) // 2] = -1.0
        job = _Job(spec)
        job.solver = Solver(case, K=K, mode=0)
        key = self._key(job)
        if key not in self.families:
            self.families[key] = [torch.cuda.Stream(), BatchStepper()]
        job.stream = self.families[key][0]
        job.batched = True
        job.U = job.solver.init_state(P, stream=job.stream)
        job.dt = torch.zeros(1, dtype=torch.float64, device="cuda")
        job.remaining = spec.nsteps
        job.events = deque()
        for _ in range(self.inflight):
            if job.remaining:
                self.step(job)
        self.flush()
        return job

    def step(self, job) -> bool:
        if not getattr(job, "batched", False):
            return super().step(job)
        n = min(self.k, job.spec.nsteps - job.enqueued)
        if n <= 0:
            return False
        self.want.setdefault(self._key(job), []).append((job, n))
        job.enqueued += n
        return True

    def flush(self):
        """Launch the requested epochs: per family, step i of the epoch
        batches every solve that asked for more than i steps."""
        torch = self.torch
        for key, reqs in self.want.items():
            stream, stepper = self.families.get(key, (None, None))
            while reqs:
                # one round: at most one pending epoch per solve
                seen, rnd, rest = set(), [], []
                for j, n in reqs:
                    (rest if id(j) in seen else rnd).append((j, n))
                    seen.add(id(j))
                reqs[:] = rest
                with torch.cuda.stream(stream):
                    for i in range(max(n for _, n in rnd)):
                        members = [j for j, n in rnd if n > i]
                        stepper.step([j.solver for j in members], [j.U for j in members],
                                     [j.dt for j in members], cfl=key[2], stream=stream)
                    ev = torch.cuda.Event()
                    ev.record(stream)
                for j, n in rnd:
                    j.events.append((ev, n))


def serve(trace, budget_bytes=200e9, max_slots=16, steps_per_epoch=10, graphs=True,
          keep_outputs=False, realtime=True, fault=None, batched=False):
    if batched:
        backend = BatchedGpuBackend(steps_per_epoch=steps_per_epoch, keep_outputs=keep_outputs,
                                    fault=fault)
    else:
        backend = GpuBackend(steps_per_epoch=steps_per_epoch, graphs=graphs,
                             keep_outputs=keep_outputs, fault=fault)
    sch = Scheduler(backend, budget_bytes, max_slots)
    t0 = time.perf_counter()
    res = sch.run(trace, realtime=realtime)
    backend.torch.cuda.synchronize()
    return res, time.perf_counter() - t0, sch


def serve_sequential(trace, steps_per_epoch=10, graphs=True, keep_outputs=False, realtime=True):
    """Baseline: the same trace FIFO, one solve at a time on the same GPU."""
    return serve(trace, budget_bytes=float("inf"), max_slots=1, steps_per_epoch=steps_per_epoch,
                 graphs=graphs, keep_outputs=keep_outputs, realtime=realtime)
