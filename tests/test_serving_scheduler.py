"""Scheduler rules on the CPU with a simulated backend: admission never
exceeds the HBM budget, oversize requests are rejected, FIFO without
overtaking, continuous batching refills slots while others run, and a request
that fails to start is isolated."""
import pytest

from paper_2406_19494_amd.serving import RequestSpec, Scheduler, draw_trace, summarize


class FakeClock:
    def __init__(self):
        self.t = 0.0

    def __call__(self):
        self.t += 1e-3  # every look at the clock costs 1 ms of simulated time
        return self.t


class FakeJob:
    def __init__(self, spec, clock, epoch_s, k):
        self.spec = spec
        self.remaining = spec.nsteps
        self.clock = clock
        self.epoch_s = epoch_s
        self.k = k
        self.busy_until = clock.t + epoch_s
        self.events = 1
        self.footprint = 0.0


class FakeBackend:
    def __init__(self, clock, epoch_s=0.01, k=10, fail=()):
        self.clock = clock
        self.epoch_s = epoch_s
        self.k = k
        self.fail = set(fail)
        self.live = []
        self.max_live_bytes = 0.0
        self.log = []

    def footprint(self, spec):
        return float(spec.size)

    def start(self, spec):
        if spec.rid in self.fail:
            raise RuntimeError("cannot start")
        j = FakeJob(spec, self.clock, self.epoch_s, self.k)
        self.live.append(j)
        self.max_live_bytes = max(self.max_live_bytes, sum(x.spec.size for x in self.live))
        self.log.append(("start", spec.rid, self.clock.t))
        return j

    def poll(self, job):
        if self.clock.t < job.busy_until:
            return False
        if job.events:
            job.remaining = max(0, job.remaining - self.k)
            job.events = 0
        return True

    def step(self, job):
        job.busy_until = self.clock.t + self.epoch_s
        job.events = 1
        return True

    def finish(self, job, res):
        res.status = "ok"
        self.live.remove(job)
        self.log.append(("finish", job.spec.rid, self.clock.t))


def _trace(sizes, steps=30, gap=0.001):
    return [RequestSpec(i, "sod", s, "forward", steps, i * gap) for i, s in enumerate(sizes)]


def test_budget_never_exceeded_and_all_complete():
    clock = FakeClock()
    be = FakeBackend(clock)
    sch = Scheduler(be, budget_bytes=100.0, max_slots=8, clock=clock, idle_sleep=0)
    res = sch.run(_trace([30, 40, 20, 50, 10, 60, 25, 35]))
    assert all(r.status == "ok" for r in res.values())
    assert be.max_live_bytes <= 100.0
    assert sch.peak_in_use <= 100.0


def test_completion_callback_sees_each_retired_solve_once():
    clock = FakeClock()
    be = FakeBackend(clock)
    seen = []
    sch = Scheduler(be, budget_bytes=100.0, max_slots=3, clock=clock, idle_sleep=0,
                    on_finish=lambda r: seen.append((r.rid, r.status, r.finished is not None)))
    res = sch.run(_trace([30, 40, 20, 50, 10]))
    assert sorted(rid for rid, _, _ in seen) == sorted(res)
    assert all(st == "ok" and done for _, st, done in seen)


def test_oversize_request_rejected_others_complete():
    clock = FakeClock()
    be = FakeBackend(clock)
    sch = Scheduler(be, budget_bytes=100.0, max_slots=4, clock=clock, idle_sleep=0)
    res = sch.run(_trace([30, 500, 20]))
    assert res[1].status == "rejected"
    assert res[0].status == "ok" and res[2].status == "ok"


def test_fifo_no_overtaking():
    clock = FakeClock()
    be = FakeBackend(clock)
    sch = Scheduler(be, budget_bytes=100.0, max_slots=4, clock=clock, idle_sleep=0)
    res = sch.run(_trace([80, 90, 10]))
    # request 1 (90) must wait for 0 to finish; request 2 (10) may not start before 1
    starts = {rid: t for ev, rid, t in be.log if ev == "start"}
    assert starts[2] >= starts[1] > starts[0]


def test_continuous_batching_refills_slots():
    clock = FakeClock()
    be = FakeBackend(clock, epoch_s=0.005)
    sch = Scheduler(be, budget_bytes=1e9, max_slots=2, clock=clock, idle_sleep=0)
    tr = [RequestSpec(0, "sod", 1, "forward", 200, 0.0), RequestSpec(1, "sod", 1, "forward", 20, 0.0),
          RequestSpec(2, "sod", 1, "forward", 20, 0.0)]
    res = sch.run(tr)
    # request 2 is admitted when 1 finishes, while 0 is still running
    assert res[2].admitted >= res[1].finished - 1e-2
    assert res[2].admitted < res[0].finished
    assert sch.peak_active == 2


def test_failed_start_is_isolated():
    clock = FakeClock()
    be = FakeBackend(clock, fail={1})
    sch = Scheduler(be, budget_bytes=1e9, max_slots=4, clock=clock, idle_sleep=0)
    res = sch.run(_trace([10, 10, 10]))
    assert res[1].status == "error" and res[0].status == "ok" and res[2].status == "ok"
    s = summarize(res, makespan=1.0)
    assert s["completed"] == 2 and s["failed"] == 1


class StallingBackend(FakeBackend):
    """A backend whose solve still counts steps left but has nothing more to
    enqueue and no epoch in flight: the state in which a polling loop would
    spin for ever."""

    def step(self, job):
        if job.remaining <= 10:
            job.events = 0
            return False
        return super().step(job)


def test_stalled_solve_raises_instead_of_spinning():
    clock = FakeClock()
    be = StallingBackend(clock)
    sch = Scheduler(be, budget_bytes=1e9, max_slots=4, clock=clock, idle_sleep=0)
    with pytest.raises(RuntimeError, match="no work in flight"):
        sch.run(_trace([10], steps=30))
    assert clock.t < 10.0  # raised within the simulated seconds, not after a spin


def test_trace_is_seeded_and_in_range():
    a = draw_trace(50, 20.0, seed=3)
    b = draw_trace(50, 20.0, seed=3)
    assert a == b
    assert all(50 <= r.nsteps <= 2000 for r in a)
    assert all(a[i].arrival < a[i + 1].arrival for i in range(49))
    fams = {r.family for r in a}
    assert fams == {"sod", "tgv", "bl"}
    assert all(200 <= r.size <= 4096 for r in a if r.family == "sod")
    assert all(r.size in (32, 48, 64, 96, 128) for r in a if r.family == "tgv")
    kinds = [r.kind for r in a]
    assert 10 < kinds.count("gradient") < 40


# ---------------------------------------------------------------------------
# The GPU backend's epoch accounting, driven with stand-ins for torch and the
# solver: every forward request enqueues exactly its step count and ends; a
# gradient request ends once the library reports the sweep complete.
# ---------------------------------------------------------------------------
class _Ev:
    def __init__(self):
        self.done = False

    def record(self, stream):
        pass

    def query(self):
        self.done = True
        return True


class _Ctx:
    def __enter__(self):
        return self

    def __exit__(self, *a):
        return False


class _FakeCuda:
    Event = _Ev

    @staticmethod
    def stream(s):
        return _Ctx()


class _FakeTorch:
    cuda = _FakeCuda


class _FakeSolver:
    def __init__(self, units_needed):
        self.units = 0
        self.units_needed = units_needed
        self.steps = 0
        self.case = type("C", (), {"cfl": 0.5})()

    def compute_dt(self, *a, **k):
        pass

    def step(self, *a, **k):
        self.steps += 1

    def step_cfl(self, *a, **k):
        self.steps += 1

    def steps_cfl(self, U, dt, n, *a, **k):
        self.steps += n

    def gradient_advance(self, n, stream=None):
        self.units = min(self.units_needed, self.units + n)
        return self.units == self.units_needed

    def gradient_finish(self, *a, **k):
        pass


@pytest.mark.parametrize("nsteps,k", [(60, 10), (55, 10), (7, 10), (10, 10), (123, 16)])
def test_gpu_backend_forward_accounting_terminates(nsteps, k):
    from collections import deque
    from paper_2406_19494_amd.serving import GpuBackend, _Job
    be = GpuBackend.__new__(GpuBackend)
    be.torch, be.k, be.inflight = _FakeTorch, k, 2
    spec = RequestSpec(0, "sod", 200, "forward", nsteps, 0.0)
    job = _Job(spec)
    job.solver, job.stream, job.events = _FakeSolver(0), None, deque()
    for _ in range(be.inflight):
        be.step(job)
    for it in range(10000):
        if be.poll(job):
            if job.remaining == 0:
                break
            assert be.step(job) or job.events
    else:
        raise AssertionError("did not terminate")
    assert job.solver.steps == nsteps and job.completed == nsteps and job.enqueued == nsteps


def test_gpu_backend_gradient_accounting_terminates():
    from collections import deque
    from paper_2406_19494_amd.serving import GpuBackend, _Job
    be = GpuBackend.__new__(GpuBackend)
    be.torch, be.k, be.inflight = _FakeTorch, 10, 2
    spec = RequestSpec(0, "bl", 1, "gradient", 30, 0.0)
    job = _Job(spec)
    job.solver, job.stream, job.events = _FakeSolver(137), None, deque()
    job.remaining = 1
    for _ in range(be.inflight):
        be.step(job)
    for it in range(10000):
        if be.poll(job):
            if job.remaining == 0:
                break
            assert be.step(job) or job.events
    else:
        raise AssertionError("did not terminate")
    assert job.solver.units == 137 and job.enqueued_done


class _FakeStepper:
    def __init__(self):
        self.calls = []

    def step(self, solvers, Us, dts, cfl=None, stream=None):
        assert len(set(map(id, solvers))) == len(solvers), "a solve twice in one batch"
        self.calls.append(len(solvers))
        for s in solvers:
            s.steps += 1


def test_batched_backend_rounds_and_accounting():
    # forward solves of one family: every graph epoch holds each solve at most
    # once, a solve with two pending epochs gets two rounds, the short final
    # epoch runs eagerly, and every solve receives exactly its steps
    from collections import deque
    from paper_2406_19494_amd.serving import BatchedGpuBackend, _Family, _Job
    be = BatchedGpuBackend.__new__(BatchedGpuBackend)
    be.torch, be.k, be.inflight = _FakeTorch, 10, 2
    fk = (1, False, 0.5)
    be.families = {fk: _Family(None)}
    be.want = {}
    calls = []

    class _Graph:
        def __init__(self, jobs):
            self.jobs = jobs

        def replay(self):
            assert len(set(map(id, self.jobs))) == len(self.jobs), "a solve twice in one epoch"
            calls.append(len(self.jobs))
            for j in self.jobs:
                j.solver.steps += be.k

    be._graph_for = lambda fam, jobs, cfl: _Graph(list(jobs))
    jobs = []
    for rid, n in enumerate((25, 7, 40)):
        job = _Job(RequestSpec(rid, "sod", 200, "forward", n, 0.0))
        job.solver, job.stream, job.events, job.batched = _FakeSolver(0), None, deque(), True
        job.fkey, job.entry = fk, object()
        for _ in range(be.inflight):
            be.step(job)
        jobs.append(job)
    be.flush()
    for it in range(10000):
        active = [j for j in jobs if j.remaining or j.events]
        if not active:
            break
        for j in active:
            if be.poll(j) and j.remaining:
                be.step(j)
        be.flush()
    else:
        raise AssertionError("did not terminate")
    for j in jobs:
        assert j.solver.steps == j.spec.nsteps == j.completed
    assert max(calls) == 2  # the 25- and 40-step solves share full epochs
