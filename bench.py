"""Benchmark: FP64 cell-updates per second per RK stage on one MI355X.

One step = CFL time step + one TVD-RK3 step (three right-hand-side
evaluations with halo fill, face fluxes, divergence and stage update) of the
whole grid, inputs resident in HBM.  Default workload: the channel-shaped
box, 192 x 128 x 128 cells on 4 pi x 2 x 4 pi/3 (tanh stretching beta 2,
isothermal walls, periodic x/z, Ma_b 0.5, Re_b 3000, constant mass flux),
the largest single-GPU configuration; its three states (427 MB) exceed the
256 MB Infinity Cache, so HBM figures measure HBM.  Prints one JSON line.
"""
import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12     # MI355X FP64 vector FLOP/s (256 CUs x 2.4 GHz x 128 flop/clk)
PEAK_HBM = 8.0e12       # MI355X HBM3E bytes/s

# Algorithmic work of one cell through one RK stage of the 3D viscous
# right-hand side, the unit figures the roofline is quoted against: about
# 3000 FP64 instructions = 4.3 kflop (30 WENO5-JS reconstructions, 3 HLLC
# fluxes, the viscous and heat fluxes, conversion, divergence and update),
# and 106.7 B of HBM traffic (stage 1 reads U^n and writes U^(1): 80 B;
# stages 2 and 3 read U^n and U^(s-1) and write U^(s): 120 B).  A face of one
# direction carries a third of the flops.
FLOPS_PER_CELL_STAGE_3DV = 4300.0
BYTES_PER_CELL_STAGE = {1: 64.0, 2: 85.3, 3: 106.7}

# Algorithmic FP64 operations per face of the flux kernel counted from the
# kernel source (10 WENO5-JS reconstructions x 69, HLLC star branch 79, 3D
# viscous/heat flux 183), used where no unit figure above applies (1D/2D,
# inviscid), and algorithmic bytes per face: the inputs of one cell read
# once (rho, u, v, w, p, plus T and mu when viscous; the tangential velocity
# derivatives are computed from the velocities), 5 x 8 B of flux written.
FLOPS_PER_FACE = {(1, False): 6 * 69 + 79, (1, True): 6 * 69 + 79 + 40,
                  (2, False): 8 * 69 + 79, (2, True): 8 * 69 + 79 + 101,
                  (3, False): 10 * 69 + 79, (3, True): 10 * 69 + 79 + 183}
BYTES_PER_FACE = {(1, False): 5 * 8 + 40, (1, True): 7 * 8 + 40,
                  (2, False): 5 * 8 + 40, (2, True): 7 * 8 + 40,
                  (3, False): 5 * 8 + 40, (3, True): 7 * 8 + 40}


def flops_per_face(case):
    """Algorithmic flops per face: the unit figure's third for 3D viscous
    cases, the source-counted figure otherwise."""
    visc = case.visc_law != "none"
    if case.ndim == 3 and visc:
        return FLOPS_PER_CELL_STAGE_3DV / 3.0
    return float(FLOPS_PER_FACE[(case.ndim, visc)])


def flops_per_cell_stage(case):
    return flops_per_face(case) * case.ndim


def algorithmic_bytes(case, kernel):
    """Bytes one launch must move at least (each input value read once, each
    output written once) for the memory-bound kernels."""
    nd = case.ndim
    h = [3 if d < nd else 0 for d in range(3)]
    N = [case.n[d] + 2 * h[d] for d in range(3)]
    nbox = N[0] * N[1] * N[2]
    visc = case.visc_law != "none"
    if kernel == "k_prim_halo":
        nq = nd + 2 + (2 if visc else 0)
        return 8 * (case.ncells * case.nv + nbox * nq)
    if kernel == "k_prim_ghost":  # each ghost reads its source cell's values, writes its own
        nq = nd + 2 + (2 if visc else 0)
        return 8 * 2 * nq * (nbox - case.ncells)
    if kernel == "k_update":
        faces = 0
        for D in range(nd):
            f = 1
            for e in range(3):
                f *= case.n[e] + (1 if e == D else 0)
            faces += f
        return 8 * (5 * faces + 3 * case.ncells * case.nv)
    raise KeyError(kernel)


def workload(name):
    from paper_2406_19494_amd import workloads as W
    if name == "tgv64":
        case, P = W.tgv(64)
        return case, P, None, "3D Taylor-Green vortex 64^3, Re 1600, Ma 0.1, FP64, CFL 0.5"
    if name == "channel":
        case, P = W.channel()
        return case, P, None, "channel 192x128x128, tanh beta 2, Ma_b 0.5, Re_b 3000, FP64"
    if name == "porous_bl":
        case, P, K = W.porous_bl()
        return case, P, K, "Mach-6 porous boundary layer 1024x256, FP64"
    if name == "sod":
        case, P = W.sod(200)
        return case, P, None, "Sod 200 cells, FP64"
    raise SystemExit(f"unknown workload {name}")


def progress(msg):
    """A progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(case, P, K, budget_s):
    """The oracle on the host cores: RK3 steps (each with its CFL step) of
    the same workload until the time budget is spent (at least one step),
    with all threads, then with one thread for half the budget."""
    from oracle import pyoracle as O
    o = O.Oracle(case, K=K)

    def sample(threads, budget):
        used = O.set_threads(threads)
        U = o.cons(P)
        t0 = time.perf_counter()
        steps = 0
        while True:
            dt = o.dt(U, case.cfl)
            U = o.step(U, dt)
            steps += 1
            if time.perf_counter() - t0 > budget:
                break
        return case.ncells * 3 * steps / (time.perf_counter() - t0), steps, used, \
            time.perf_counter() - t0

    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    v, steps, used, el = sample(threads, budget_s)
    v1, steps1, _, el1 = sample(1, budget_s / 2)
    O.set_threads(threads)
    return {"value": v, "unit": "cell-updates/s per RK stage", "cores": used, "kind": "oracle",
            "sample": f"{steps} CFL+RK3 steps of the same {case.n[0]}x{case.n[1]}x{case.n[2]} "
                      f"workload ({el:.1f} s, OpenMP threads={used})",
            "single_thread": {"value": v1, "cores": 1,
                              "sample": f"{steps1} CFL+RK3 steps ({el1:.1f} s, 1 thread)"}}


def source_digest():
    """sha256 of the forward kernel sources (counters are tied to them)."""
    import hashlib
    h = hashlib.sha256()
    for f in ("dcf_forward.hip", "dcf_common.hpp"):
        with open(os.path.join(ROOT, "paper_2406_19494_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE in KiB per dispatch, scaled by the
    factors a plain 512 MiB copy gives), or None when no summary exists or
    the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.txt")
    if not os.path.exists(path):
        return None
    vals, kern = {}, {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) >= 2 and parts[0] in ("source_sha", "copy_factor_fetch",
                                                  "copy_factor_write"):
                vals[parts[0]] = parts[1]
            elif len(parts) == 4 and parts[0] == "kernel":
                kern[parts[1]] = (float(parts[2]), float(parts[3]))
    if vals.get("source_sha") != source_digest() or kernel not in kern:
        return None
    fk, wk = kern[kernel]
    return 1024.0 * (fk * float(vals["copy_factor_fetch"]) + wk * float(vals["copy_factor_write"]))


def step_kernel_ids(case):
    """dcf_time_kernel ids of the launches one RK3 stage of `case` runs:
    halo fill (0; 8 = ghosts only, stages 2-3 of a fused step), fluxes (7 =
    x+y of a 3D grid, 1..3 per direction; on 2D and 3D grids they compute the
    velocity derivatives they need themselves, so no derivative launch),
    then the fused last-direction flux + update (6, 2D/3D without source) or
    the separate update (4)."""
    last = 2 * (case.ndim - 1)
    fused = case.ndim >= 2 and (case.source == "none" or (
        case.bc[last] == "periodic" and case.bc[last + 1] == "periodic"))
    ids = [0] + ([8] if fused else [])
    if case.ndim == 3:
        ids += [7] + ([6] if fused else [3, 4])
    elif case.ndim == 2:
        ids += [1] + ([6] if fused else [2, 4])
    else:
        ids += [1, 4]
    return ids


def measured_valu(kernel, workload):
    """FP64 VALU work per launch of `kernel` from the committed counter
    summary: 64 lanes x (2 FMA + MUL + ADD + TRANS) FP64 instructions
    (SQ_INSTS_VALU_*_F64 per dispatch; every lane of a wave counted), or
    None when no summary exists or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.txt")
    if not os.path.exists(path):
        return None
    sha, row = None, None
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) >= 2 and parts[0] == "source_sha":
                sha = parts[1]
            elif len(parts) == 6 and parts[0] == "valu" and parts[1] == kernel:
                row = [float(x) for x in parts[2:]]
    if sha != source_digest() or row is None:
        return None
    fma, mul, add, trans = row
    return 64.0 * (2.0 * fma + mul + add + trans)


def serving_bench(M=40, rate=20.0, seed=2024, M_low=12, rate_low=2.0, seed_low=2025):
    """Continuous batching against sequential solves on a seeded trace of M
    forward and gradient requests drawn from the serving mix (Sod 200-4096
    cells, TGV 32^3-128^3, porous BL 256x64-1024x256, 50-2000 steps, half
    gradients, Poisson arrivals at `rate`/s: an overloaded GPU), and a short
    trace of small solves at `rate_low`/s whose offered load stays below
    capacity (latency near the service time)."""
    from paper_2406_19494_amd import serving as S

    def offered(trace):
        work = sum(3.0 * S.cells_of(r) * r.nsteps for r in trace)
        span = max(r.arrival for r in trace)
        return work, (work / span if span > 0 else float("nan"))

    trace = S.draw_trace(M, rate, seed)
    out = {"trace": f"{M} requests, Poisson {rate}/s (seed {seed}), steps 50-2000, sod "
                    "200-4096 / tgv 32-128^3 / porous BL 256x64-1024x256, 50% gradients, "
                    "HBM budget 200 GB",
           "offered_cell_updates": offered(trace)[0],
           "offered_load_cell_updates_per_s": offered(trace)[1]}
    runs = {}
    for name, kw in (("sequential", None), ("streams", {"batched": False}),
                     ("batched", {"batched": True})):
        progress(f"serving: {name}")
        retired = [0]

        def on_finish(res, name=name):  # a progress line per 20 retired solves
            retired[0] += 1
            if retired[0] % 20 == 0:
                progress(f"serving: {name}, {retired[0]} of {M} retired")
        if kw is None:
            res, t, sch = S.serve_sequential(trace, on_finish=on_finish)
        else:
            res, t, sch = S.serve(trace, budget_bytes=200e9, max_slots=16, on_finish=on_finish,
                                  **kw)
        runs[name] = S.summarize(res, t) | {"peak_active": sch.peak_active}
        if name == "batched":
            runs[name]["graph_captures"] = getattr(sch.b, "recaptures", None)
    out |= runs
    seq = runs["sequential"]
    for name in ("streams", "batched"):
        out[f"throughput_ratio_{name}"] = runs[name]["cell_updates_per_s"] / \
            seq["cell_updates_per_s"]
        out[f"p99_ratio_{name}"] = runs[name]["p99_s"] / seq["p99_s"]
    low = S.draw_trace(M_low, rate_low, seed_low, steps=(50, 400), tgv=(32, 48, 64), bl=(1, 2))
    res_l, t_l, _ = S.serve(low, budget_bytes=200e9, max_slots=16, batched=True)
    res_ls, t_ls, _ = S.serve_sequential(low)
    work_l, load_l = offered(low)
    out["low_rate"] = {"trace": f"{M_low} requests, Poisson {rate_low}/s (seed {seed_low}), "
                                "steps 50-400, TGV <= 64^3, BL <= 512x128",
                       "offered_cell_updates": work_l, "offered_load_cell_updates_per_s": load_l,
                       "batched": S.summarize(res_l, t_l),
                       "sequential": S.summarize(res_ls, t_ls)}
    out["note"] = ("sequential: FIFO, one solve at a time, each forward epoch a hipGraph replay; "
                   "streams: up to 16 admitted solves on 4 streams, per-solve graph epochs; "
                   "batched: forward solves of one family of at most 2^17 cells share one "
                   "hipGraph of batched step launches per epoch (captured again when the members "
                   "change), larger forward solves and gradients as in streams; solves pooled "
                   "per (family, size, kind); offered load = the "
                   "trace's cell updates over its arrival span")
    return out


def _trajectory_phases(case, K, P, dt, n, seg, mode):
    """One checkpointed trajectory gradient over n steps with checkpoints
    every seg steps, its phases timed with HIP events between the
    dcf_gradient_advance calls that run them (after one warm-up gradient)."""
    import torch
    from paper_2406_19494_amd.solver import Solver
    stream = torch.cuda.current_stream()
    sg = Solver(case, K=K, mode=mode, nsteps=n, seg_len=seg)
    U0 = sg.init_state(P)
    sg.gradient(U0, dt)  # warm-up
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    gK = torch.zeros(sg.nk, dtype=torch.float64, device="cuda")
    nseg = (n + seg - 1) // seg
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 + 2 * nseg)]
    torch.cuda.synchronize()
    sg.gradient_begin(U0, dt, J, gK)
    evs[0].record(stream)
    sg.gradient_advance(n)
    evs[1].record(stream)
    for k in range(nseg):
        units = min(seg, n - (nseg - 1 - k) * seg)
        if k > 0:  # the last segment kept its data in the forward sweep
            sg.gradient_advance(units)  # recompute of the segment
        evs[2 + 2 * k].record(stream)
        sg.gradient_advance(units)  # reverse steps of the segment
        evs[3 + 2 * k].record(stream)
    done = sg.gradient_advance(1)
    torch.cuda.synchronize()
    assert done, "gradient did not complete in the expected number of units"
    sg.gradient_finish()
    fwd = evs[0].elapsed_time(evs[1])
    rec = sum(evs[1 + 2 * k].elapsed_time(evs[2 + 2 * k]) for k in range(nseg))
    rev = sum(evs[2 + 2 * k].elapsed_time(evs[3 + 2 * k]) for k in range(nseg))
    g = evs[0].elapsed_time(evs[-1])
    ws = sg.workspace_bytes()
    del sg
    return {"steps": n, "seg_len": seg, "mode": mode, "workspace_gb": ws / 1e9,
            "gradient_ms": g, "forward_sweep_ms": fwd, "recompute_ms": rec, "reverse_ms": rev}


def adjoint_ratio(steps=20, n=2000, seg=45):
    """Adjoint/forward cost on the Mach-6 porous boundary layer (1024 x 256),
    both definitions: per step, t(vjp_step) / t(rk3_step) with the stage
    states recomputed by the VJP and with them kept by the forward step; end
    to end, (t(gradient) - t(forward sweep with checkpoints)) / t(forward
    trajectory) over the n-step checkpointed trajectory."""
    import torch
    from paper_2406_19494_amd import workloads as W
    from paper_2406_19494_amd.solver import Solver
    case, P, K = W.porous_bl()
    s = Solver(case, K=K, mode=1)
    U = s.init_state(P)
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    s.compute_dt(U, cfl=0.5, out=dt)
    lam = torch.ones_like(U)
    gK = torch.zeros(s.nk, dtype=torch.float64, device="cuda")
    stages = torch.empty((2,) + tuple(U.shape), dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()
    for _ in range(3):
        s.step(U, dt)
        s.vjp_step(U, dt, lam, dJdK=gK)
        s.step_keep(U, dt, stages)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(5)]
    Us = [U.clone() for _ in range(steps)]
    st = [torch.empty_like(stages) for _ in range(steps)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(steps):
        s.step(U, dt)
    ev[1].record(stream)
    for _ in range(steps):
        s.vjp_step(U, dt, lam, dJdK=gK)
    ev[2].record(stream)
    for i in range(steps):  # forward steps that keep their stage states
        s.step_keep(Us[i], dt, st[i])
    ev[3].record(stream)
    for i in range(steps):  # VJPs that read them instead of recomputing
        s.vjp_step(Us[i], dt, lam, dJdK=gK, stages=st[i])
    ev[4].record(stream)
    torch.cuda.synchronize()
    f = ev[0].elapsed_time(ev[1]) / steps
    a = ev[1].elapsed_time(ev[2]) / steps
    fk = ev[2].elapsed_time(ev[3]) / steps
    ac = ev[3].elapsed_time(ev[4]) / steps
    del Us, st
    U0 = s.init_state(P)
    s.compute_dt(U0, cfl=0.5, out=dt)
    traj = {}
    for name, mode, sl in (("mode2_S%d" % seg, 2, seg), ("mode3_S%d" % seg, 3, seg),
                           ("mode2_one_segment", 2, n)):
        progress(f"trajectory gradient {name}")
        r = _trajectory_phases(case, K, P, dt, n, sl, mode)
        r["end_to_end_over_forward"] = (r["gradient_ms"] - r["forward_sweep_ms"]) / (n * f)
        r["gradient_over_forward"] = r["gradient_ms"] / (n * f)
        r["reverse_step_over_forward"] = r["reverse_ms"] / (n * f)
        traj[name] = r
    # an end-to-end optimisation run on the same trajectory: projected Adam
    # on the 512 porous coefficients, one checkpointed gradient per iteration
    from paper_2406_19494_amd.autograd import optimize_porous
    so = Solver(case, K=K, mode=2, nsteps=n, seg_len=seg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    progress("optimisation run")
    hist = optimize_porous(so, U0, dt, K, iters=6, lr=0.05, k_max=1.0)
    t_opt = time.perf_counter() - t0
    Js = [h[0] for h in hist]
    del so
    opt = {"method": "projected Adam (lr 0.05, K_i in [0, 1])", "iterations": len(Js),
           "J": Js, "J_last_over_first": Js[-1] / Js[0], "seconds": t_opt,
           "trajectory": f"{n} fixed-dt steps, checkpoints every {seg}"}
    return {"workload": "Mach-6 porous boundary layer 1024x256, 512 porous K_i",
            "optimisation": opt,
            "forward_ms_per_step": f,
            "per_step": {"vjp_recompute_ms": a, "vjp_recompute_over_forward": a / f,
                         "forward_keeping_stages_ms": fk,
                         "vjp_cached_stages_ms": ac, "vjp_cached_stages_over_forward": ac / f,
                         "note": "vjp_recompute: dcf_vjp_step without stage states (it "
                                 "recomputes U(1), U(2) and every stage's boxes); "
                                 "vjp_cached_stages: with the stage states a forward step "
                                 "kept (dcf_rk3_step_keep), each stage's boxes recomputed"},
            "end_to_end": {k: v["end_to_end_over_forward"] for k, v in traj.items()},
            "trajectory": traj,
            "trajectory_note": "end_to_end_over_forward = (gradient - forward sweep with "
                               "checkpoints and cost) / forward trajectory, n = %d fixed-dt "
                               "steps; mode2 recomputes each stage's boxes in the reverse "
                               "sweep, mode3 keeps them from the segment recompute; the last "
                               "segment keeps its data from the forward sweep, so one segment "
                               "(S = n, the whole trajectory resident in HBM) has no "
                               "recompute" % n}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="channel")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--adjoint-steps", type=int, default=2000,
                    help="trajectory length of the adjoint measurement (the porous boundary "
                         "layer's is 2000)")
    ap.add_argument("--adjoint-seg", type=int, default=45,
                    help="checkpoint spacing of the adjoint measurement")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-teno", action="store_true",
                    help="skip the channel timing with the TENO6-A scheme")
    ap.add_argument("--serving-requests", type=int, default=40,
                    help="requests in the serving trace (the full serving mix is 200)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run a plain 512 MiB device copy (counter calibration) and exit")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = 512 * 1024 * 1024 // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 8 * n, "copy_bytes_written": 8 * n, "launches": 3}))
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported by this build "
              "(the multi-GPU block decomposition is designed, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2406_19494_amd.solver import Solver

    case, P, K, desc = workload(args.workload)
    s = Solver(case, K=K)
    U = s.init_state(P)
    dt = torch.empty(1, dtype=torch.float64, device="cuda")
    stream = torch.cuda.current_stream()

    # each step takes the CFL step of its input state: the last stage of the
    # previous step reduces it, the first comes from dcf_compute_dt; the K
    # steps are one dcf_rk3_steps_cfl call (bitwise K dcf_rk3_step_cfl calls)
    s.compute_dt(U, cfl=case.cfl, out=dt)
    if args.warmup:
        s.steps_cfl(U, dt, args.warmup, cfl=case.cfl)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    t0 = time.perf_counter()
    s.steps_cfl(U, dt, args.steps, cfl=case.cfl)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    assert s.flags() == 0, "non-physical state during the benchmark"
    ms_step = ms / args.steps
    value = case.ncells * 3 / (ms_step * 1e-3)

    # Kernels of a step.  A 2D/3D step without source term (or with the
    # body force and a periodic last direction) runs the last direction's
    # fluxes fused with the stage update (k_flux_update); a 3D step launches
    # the x and y fluxes as one grid (k_flux_xy).  The update of stages 1 and
    # 2 also writes the next stage's primitive interior, so later stages fill
    # only the ghosts (k_prim_ghost, 8; the first step of a call runs the
    # whole halo fill, 0).  The unfused kernels are timed too, for the record.
    names = {0: "k_prim_halo", 1: "k_flux_x", 2: "k_flux_yz<y>", 3: "k_flux_yz<z>", 4: "k_update",
             6: "k_flux_update", 7: "k_flux_xy", 8: "k_prim_ghost"}
    step_kinds = step_kernel_ids(case)
    kinds = sorted(set(step_kinds) | set(range(1, case.ndim + 1)) | {4})
    kt = {w: s.time_kernel(U, w, reps=20) for w in kinds}  # back-to-back launches

    # Every step kernel timed on its launches inside the stepping loop: HIP
    # event pairs around each of its launches on the stream of the stepping
    # call (dcf_probe_*), one replay of the timed region per kernel (the
    # timed value above runs without events).
    probed = {}
    for w in step_kinds:
        if w in (1, 6, 7, 8):
            s.probe_begin(w, 4 * args.steps + 8)
            s.steps_cfl(U, dt, args.steps, cfl=case.cfl)
            torch.cuda.synchronize()
            n_l, t_l = s.probe_end()
            if n_l > 0:
                probed[w] = (n_l, t_l)
    assert s.flags() == 0, "non-physical state during the probe replays"

    def faces_of(D):
        f = 1
        for e in range(3):
            f *= case.n[e] + (1 if e == D else 0)
        return f

    def flux_faces(w):  # faces whose fluxes kernel w computes, or None
        if 1 <= w <= 3:
            return faces_of(w - 1)
        if w == 6:
            return faces_of(case.ndim - 1)
        if w == 7:
            return faces_of(0) + faces_of(1)
        return None

    visc = case.visc_law != "none"

    def kernel_roof(w, t_ms):
        # a launch against the roof that binds it: the larger of the FP64
        # lower bound (algorithmic flops / 78.6 TFLOP/s) and the HBM lower
        # bound (algorithmic bytes of the launch / 8 TB/s)
        nf = flux_faces(w)
        t = t_ms * 1e-3
        if nf is not None:
            fpf = flops_per_face(case)
            bpf = BYTES_PER_FACE[(case.ndim, visc)]
            flops = fpf * nf
            if w == 6:
                # inputs of one cell once (primitives), the other
                # directions' face fluxes, Un and Uin; Uout written
                cells = case.ncells
                nbytes = cells * (bpf - 40) + 3 * cells * case.nv * 8
                nbytes += sum(40 * faces_of(D) for D in range(case.ndim - 1))
            else:
                nbytes = bpf * nf
            t_alu, t_hbm = flops / PEAK_FP64, nbytes / PEAK_HBM
            out = {"algorithmic_flops_per_face": fpf, "faces_per_launch": nf,
                   "algorithmic_flops": flops, "algorithmic_bytes": nbytes,
                   "alu_frac": t_alu / t, "hbm_frac": t_hbm / t}
            if t_hbm > t_alu:
                return {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": PEAK_HBM / 1e9,
                        "unit": "GB/s", "frac": t_hbm / t} | out
            return {"bound": "alu", "achieved": flops / t / 1e12, "peak": PEAK_FP64 / 1e12,
                    "unit": "TFLOP/s", "frac": t_alu / t} | out
        nbytes = algorithmic_bytes(case, names[w])
        return {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": nbytes / t / PEAK_HBM, "algorithmic_bytes": nbytes}

    # dominant kernel: the step kernel with the most in-loop time per step
    # (launches per step x mean duration)
    if probed:
        dom = max(probed, key=lambda w: probed[w][0] * probed[w][1])
        probe_n, t_dom = probed[dom]
    else:
        dom = max(step_kinds, key=lambda w: kt[w])
        probe_n, t_dom = 0, kt[dom]
    timing = ("HIP events around each launch inside the stepping loop, replay of the timed region"
              if probe_n else "HIP events over back-to-back launches")
    roof = kernel_roof(dom, t_dom)
    roof = {k: roof[k] for k in ("bound", "achieved", "peak", "unit", "frac")} | {
        "traffic": measured_traffic(names[dom], args.workload), "kernel": names[dom],
        "avg_ms": t_dom, "launches_timed": probe_n, "timing": timing,
        "avg_ms_back_to_back": kt[dom]} | {k: v for k, v in roof.items()
                                          if k not in ("bound", "achieved", "peak", "unit", "frac")}
    # the same launch against both roofs from the hardware counters: FP64
    # VALU operations issued and HBM bytes moved, per launch, over its time
    vf = measured_valu(names[dom], args.workload)
    roof["valu_fp64_tflops"] = None if vf is None else vf / (t_dom * 1e-3) / 1e12
    roof["valu_frac"] = None if vf is None else vf / (t_dom * 1e-3) / PEAK_FP64
    tr = roof["traffic"]
    roof["hbm_frac_measured"] = None if tr is None else tr / (t_dom * 1e-3) / PEAK_HBM
    # every step kernel in the loop, and every kernel back to back, against
    # its own roof
    roof["in_loop"] = {names[w]: {"launches_per_step": n_l / args.steps, "avg_ms": t_l,
                                  "ms_per_step": n_l / args.steps * t_l,
                                  "frac": kernel_roof(w, t_l)["frac"],
                                  "bound": kernel_roof(w, t_l)["bound"]}
                       for w, (n_l, t_l) in probed.items()}
    per_kernel = {}
    for w in kinds:
        r = kernel_roof(w, kt[w])
        per_kernel[names[w]] = {"bound": r["bound"], "frac": r["frac"], "avg_ms": kt[w],
                                ("achieved_tflops" if r["bound"] == "alu" else "achieved_gbs"):
                                    r["achieved"], "in_step": w in step_kinds}
        for k in ("alu_frac", "hbm_frac"):
            if k in r:
                per_kernel[names[w]][k] = r[k]
    roof["per_kernel_back_to_back"] = per_kernel

    # The whole RK stage (every launch of a stage, CFL step included) against
    # the unit figures: flops and bytes per cell-stage x cells / stage time.
    # Its binding roof is the FP64 one when flops/bytes exceeds the ridge
    # (78.6 TFLOP/s / 8 TB/s = 9.8 flop/B).
    stage_s = ms_step * 1e-3 / 3.0
    fcs = flops_per_cell_stage(case)
    bcs = BYTES_PER_CELL_STAGE[case.ndim]
    t_alu = case.ncells * fcs / PEAK_FP64
    t_hbm = case.ncells * bcs / PEAK_HBM
    stage = {"bound": "alu" if t_alu >= t_hbm else "hbm",
             "flops_per_cell_stage": fcs, "bytes_per_cell_stage": bcs,
             "achieved_tflops": case.ncells * fcs / stage_s / 1e12,
             "alu_frac": t_alu / stage_s,
             "achieved_gbs_algorithmic": case.ncells * bcs / stage_s / 1e9,
             "hbm_frac_algorithmic": t_hbm / stage_s,
             "stage_ms": stage_s * 1e3}
    stage["frac"] = max(t_alu, t_hbm) / stage_s
    # HBM bytes the stage's launches move by the counters (where the
    # committed summary matches the kernel sources)
    moved, complete = 0.0, True
    for w, (n_l, _) in probed.items():
        tw = measured_traffic(names[w], args.workload)
        if tw is None:
            complete = False
            break
        moved += tw * n_l / args.steps / 3.0
    stage["hbm_bytes_measured_per_stage"] = moved if complete and probed else None
    stage["hbm_frac_measured"] = (moved / stage_s / PEAK_HBM) if complete and probed else None
    stage["traffic_over_algorithmic"] = (moved / (case.ncells * bcs)) if complete and probed \
        else None

    out = {
        "metric": "FP64 cell-updates/s per RK stage",
        "value": value,
        "unit": "cell-updates/s per RK stage",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "pid_s_per_cell_stage": 1.0 / value,  # wall time x GPUs / (cells x RK stages)
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic (analytic initial condition, seeded where random)",
        "config": {"workload": desc, "cells": case.ncells, "rk_stages": 3,
                   "step": "CFL dt + TVD-RK3 (WENO5-JS, HLLC, 4th-order viscous)",
                   "name": args.workload},
        "roofline": roof,
        "stage_roofline": stage,
        "kernel_ms": {names[k]: v for k, v in kt.items()},
        "step_kernels": [names[k] for k in step_kinds],
        "source_sha": source_digest(),
        "wall_s": wall,
    }
    progress(f"timed {args.steps} steps: {value:.4g} cell-updates/s per stage")
    if args.workload == "channel" and not args.no_teno:
        # the same workload with the paper's channel scheme (TENO6-A with
        # the interpolation limiter, 6th-order dissipative fluxes)
        from paper_2406_19494_amd import workloads as W
        ct, Pt = W.channel(scheme="teno6a")
        st_ = Solver(ct)
        Ut = st_.init_state(Pt)
        dtt = torch.empty(1, dtype=torch.float64, device="cuda")
        st_.compute_dt(Ut, cfl=ct.cfl, out=dtt)
        if args.warmup:
            st_.steps_cfl(Ut, dtt, args.warmup, cfl=ct.cfl)
        torch.cuda.synchronize()
        e0.record(stream)
        st_.steps_cfl(Ut, dtt, args.steps, cfl=ct.cfl)
        e1.record(stream)
        torch.cuda.synchronize()
        assert st_.flags() == 0, "non-physical state during the TENO6-A benchmark"
        ms_t = e0.elapsed_time(e1) / args.steps
        out["teno6a"] = {"workload": "channel 192x128x128 with TENO6-A + 6th-order dissipative "
                                     "fluxes (the paper's channel scheme)",
                         "ms_per_step": ms_t,
                         "cell_updates_per_s_per_stage": ct.ncells * 3 / (ms_t * 1e-3),
                         "steps": args.steps}
        del st_, Ut
        progress(f"TENO6-A channel: {out['teno6a']['cell_updates_per_s_per_stage']:.4g}")
    if not args.no_adjoint:
        progress("adjoint and trajectory gradients")
        out["adjoint"] = adjoint_ratio(n=args.adjoint_steps, seg=args.adjoint_seg)
    if not args.no_serving:
        progress("serving")
        out["serving"] = serving_bench(M=args.serving_requests)
    if not args.no_cpu:
        progress("oracle on the host cores")
        out["cpu_baseline"] = cpu_baseline(case, P, K, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
