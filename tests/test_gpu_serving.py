"""GPU serving: each request's result is the same alone and in the mix
(bitwise) and matches the oracle, graph replays equal eager steps, a
non-physical request is isolated, and batched serving beats sequential solves
on throughput."""
import numpy as np
import pytest
import torch

from paper_2406_19494_amd import serving as S
from paper_2406_19494_amd import workloads as W
from paper_2406_19494_amd.solver import Solver

pytestmark = pytest.mark.gpu


def _small_trace():
    return [
        S.RequestSpec(0, "sod", 300, "forward", 60, 0.0),
        S.RequestSpec(1, "tgv", 32, "forward", 40, 0.0),
        S.RequestSpec(2, "bl", 1, "gradient", 30, 0.0),
        S.RequestSpec(3, "sod", 1000, "gradient", 25, 0.0),
        S.RequestSpec(4, "tgv", 32, "gradient", 12, 0.0),
        S.RequestSpec(5, "bl", 1, "forward", 55, 0.0),
    ]


def test_alone_equals_in_mix_bitwise():
    trace = _small_trace()
    mix, _, sch = S.serve(trace, max_slots=6, keep_outputs=True, realtime=False)
    assert sch.peak_active >= 4
    for spec in trace:
        alone, _, _ = S.serve([spec], max_slots=1, keep_outputs=True, realtime=False)
        a, m = alone[spec.rid], mix[spec.rid]
        assert a.status == m.status == "ok", (spec, a.status, m.status, m.message)
        for key, va in a.output.items():
            vm = m.output[key]
            assert np.array_equal(np.asarray(va), np.asarray(vm)), (spec, key)


def test_graph_replays_match_eager_steps():
    case, P = W.tgv(16)
    s_eager = Solver(case)
    U_e = s_eager.init_state(P)
    dt_e = torch.empty(1, dtype=torch.float64, device="cuda")
    s_graph = Solver(case)
    U_g = s_graph.init_state(P)
    dt_g = torch.empty(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=stream):
        for _ in range(3):
            s_graph.compute_dt(U_g, cfl=0.5, out=dt_g)
            s_graph.step(U_g, dt_g)
    for rep in range(4):
        with torch.cuda.stream(stream):
            g.replay()
        for _ in range(3):
            s_eager.compute_dt(U_e, cfl=0.5, out=dt_e)
            s_eager.step(U_e, dt_e)
        torch.cuda.synchronize()
        # eager work of the program itself between replays
        _ = (U_e * 2.0).sum().item()
        assert torch.equal(U_g, U_e), rep


def test_nonphysical_request_is_isolated():
    trace = _small_trace()[:3]
    res, _, _ = S.serve(trace, max_slots=3, keep_outputs=True, realtime=False, fault={0: "nonphysical"})
    assert res[0].status == "nonphysical"
    assert res[1].status == "ok" and res[2].status == "ok"
    ref, _, _ = S.serve([trace[1]], max_slots=1, keep_outputs=True, realtime=False)
    assert np.array_equal(ref[1].output["U"], res[1].output["U"])


def test_oversize_request_rejected_on_gpu():
    trace = _small_trace()[:2]
    res, _, _ = S.serve(trace, budget_bytes=2e6, max_slots=2, realtime=False)
    assert res[0].status == "ok"       # Sod 300 fits in 2 MB
    assert res[1].status == "rejected"  # TGV 32^3 does not


def test_batched_beats_sequential():
    trace = S.draw_trace(24, rate=1e9, seed=7, steps=(50, 150), tgv=(32, 48), bl=(1,))
    _, t_batched, _ = S.serve(trace, max_slots=16, realtime=False)
    _, t_seq, _ = S.serve_sequential(trace, realtime=False)
    print(f"[serving] batched {t_batched:.3f} s, sequential {t_seq:.3f} s", flush=True)
    assert t_batched < t_seq


def test_batched_kernels_backend_matches_unbatched_alone():
    # forward solves of one family step together in batched launches; every
    # result equals the solve served alone by the per-request backend
    trace = [
        S.RequestSpec(0, "sod", 300, "forward", 33, 0.0),
        S.RequestSpec(1, "sod", 1000, "forward", 20, 0.0),
        S.RequestSpec(2, "sod", 513, "forward", 47, 0.0),
        S.RequestSpec(3, "tgv", 16, "forward", 25, 0.0),
        S.RequestSpec(4, "tgv", 24, "forward", 12, 0.0),
        S.RequestSpec(5, "bl", 1, "forward", 21, 0.0),
        S.RequestSpec(6, "tgv", 16, "gradient", 8, 0.0),
    ]
    mix, _, sch = S.serve(trace, max_slots=7, keep_outputs=True, realtime=False, batched=True)
    assert sch.peak_active >= 5
    for spec in trace:
        alone, _, _ = S.serve([spec], max_slots=1, keep_outputs=True, realtime=False)
        a, m = alone[spec.rid], mix[spec.rid]
        assert a.status == m.status == "ok", (spec, a.status, m.status, m.message)
        for key, va in a.output.items():
            assert np.array_equal(np.asarray(va), np.asarray(m.output[key])), (spec, key)


def test_batched_backend_serves_large_solves_per_request():
    # above the size cut-off a forward solve leaves the family batch and runs
    # per-solve graph epochs on the shared streams; every result still equals
    # the solve served alone
    trace = [
        S.RequestSpec(0, "sod", 300, "forward", 33, 0.0),
        S.RequestSpec(1, "sod", 700, "forward", 20, 0.0),
        S.RequestSpec(2, "tgv", 16, "forward", 25, 0.0),
        S.RequestSpec(3, "tgv", 24, "forward", 12, 0.0),
        S.RequestSpec(4, "bl", 1, "forward", 21, 0.0),
    ]
    be = S.BatchedGpuBackend(keep_outputs=True, batch_max_cells=1000)
    mix, _, _ = S.serve(trace, max_slots=5, keep_outputs=True, realtime=False, backend=be)
    assert {f[0] for f in be.families} == {1}  # only the Sod solves were batched
    for spec in trace:
        alone, _, _ = S.serve([spec], max_slots=1, keep_outputs=True, realtime=False)
        a, m = alone[spec.rid], mix[spec.rid]
        assert a.status == m.status == "ok", (spec, a.status, m.status, m.message)
        for key, va in a.output.items():
            assert np.array_equal(np.asarray(va), np.asarray(m.output[key])), (spec, key)


def test_batched_kernels_backend_isolates_nonphysical():
    trace = [S.RequestSpec(0, "sod", 300, "forward", 30, 0.0),
             S.RequestSpec(1, "sod", 400, "forward", 30, 0.0)]
    res, _, _ = S.serve(trace, max_slots=2, keep_outputs=True, realtime=False, batched=True,
                        fault={0: "nonphysical"})
    assert res[0].status == "nonphysical" and res[1].status == "ok"
    ref, _, _ = S.serve([trace[1]], max_slots=1, keep_outputs=True, realtime=False)
    assert np.array_equal(ref[1].output["U"], res[1].output["U"])


def test_served_results_match_oracle():
    # forward and gradient requests served together (per-request streams and
    # family-batched graph epochs), each output against the oracle: forward
    # states after their CFL steps, gradients (J, dJ/dK, dJ/dU0) over the
    # fixed-step trajectory the request ran
    from oracle.pyoracle import Oracle
    from tests.test_oracle_pins import _tiny_porous
    case, P, K = _tiny_porous()
    S.register_case("bl", 0, case, P, K)
    # a Sod tube whose cost (wall pressure at the x- end against 0.9) is
    # nonzero from the first step
    sod, Ps = W.sod(40)
    sod.cost_face, sod.p_inf = 0, 0.9
    S.register_case("sod", 41, sod, Ps, None)
    trace = [
        S.RequestSpec(0, "sod", 40, "forward", 23, 0.0),
        S.RequestSpec(1, "sod", 64, "forward", 17, 0.0),
        S.RequestSpec(2, "tgv", 8, "forward", 12, 0.0),
        S.RequestSpec(3, "bl", 0, "forward", 14, 0.0),
        S.RequestSpec(4, "sod", 41, "gradient", 6, 0.0),
        S.RequestSpec(5, "bl", 0, "gradient", 5, 0.0),
    ]
    for batched in (False, True):
        res, _, _ = S.serve(trace, max_slots=6, keep_outputs=True, realtime=False,
                            batched=batched)
        for spec in trace:
            r = res[spec.rid]
            assert r.status == "ok", (spec, r.status, r.message)
            c, Pc, Kc = S.build_case(spec)
            o = Oracle(c, K=Kc)
            U0 = o.cons(Pc)
            if spec.kind == "forward":
                U_or = U0.copy()
                for _ in range(spec.nsteps):
                    U_or = o.step(U_or, o.dt(U_or, c.cfl))
                err = np.abs(r.output["U"] - U_or).max(axis=(1, 2, 3)) / \
                    np.abs(U_or).max(axis=(1, 2, 3))
                assert np.all(err <= 1e-10), (batched, spec, err)
            else:
                dt = r.output["dt"]
                assert abs(dt - o.dt(U0, c.cfl)) <= 1e-13 * dt
                J, gk, gu = o.gradient(U0, spec.nsteps, dt)
                assert J > 0.0
                assert abs(r.output["J"] - J) <= 1e-12 * abs(J), (batched, spec)
                if o.nk:
                    assert np.abs(r.output["dJdK"] - gk).max() <= 1e-10 * np.abs(gk).max()
                # per variable, in units of the change of J under a relative
                # change of the state: max|d gu_v| max|U_v| against the
                # largest max|gu_v'| max|U_v'| (a component the cost hardly
                # feels, such as the density at rest, is held to that scale)
                um = np.abs(U0).max(axis=(1, 2, 3))
                ref = (np.abs(gu).max(axis=(1, 2, 3)) * um).max()
                err = np.abs(r.output["dJdU0"] - gu).max(axis=(1, 2, 3)) * um / ref
                assert np.all(err <= 1e-10), (batched, spec, err)
