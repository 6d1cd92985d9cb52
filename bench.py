"""Benchmark: FP64 cell-updates per second per RK stage on one MI355X.

One step = CFL time step + one TVD-RK3 step (three right-hand-side
evaluations with halo fill, face fluxes, divergence and stage update) of the
whole grid, inputs resident in HBM.  Default workload: 3D Taylor-Green vortex,
64^3 cells, Re 1600, Ma 0.1, viscous (power law).  Prints one JSON line.
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

# Algorithmic FP64 operations per face of the flux kernel (counted from the
# kernel source: 10 WENO5-JS reconstructions x 69, HLLC star branch 79, 3D
# viscous/heat flux 183) and algorithmic bytes per face: the inputs of one
# cell read once (rho, u, v, w, p, plus T, mu and the 2 (2D) or 4 (3D)
# tangential derivatives a viscous face reads), 5 x 8 B of flux written.
FLOPS_PER_FACE = {(1, False): 6 * 69 + 79, (1, True): 6 * 69 + 79 + 40,
                  (2, False): 8 * 69 + 79, (2, True): 8 * 69 + 79 + 101,
                  (3, False): 10 * 69 + 79, (3, True): 10 * 69 + 79 + 183}
BYTES_PER_FACE = {(1, False): 5 * 8 + 40, (1, True): 7 * 8 + 40,
                  (2, False): 5 * 8 + 40, (2, True): 9 * 8 + 40,
                  (3, False): 5 * 8 + 40, (3, True): 11 * 8 + 40}


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
    if kernel == "k_ghost_grad_periodic":  # the ghost fill and the derivatives of one launch
        return algorithmic_bytes(case, "k_prim_ghost") + algorithmic_bytes(case, "k_grad")
    if kernel == "k_grad":
        writes = 0
        for t in range(nd):
            cnt = case.n[t]
            for e in range(nd):
                if e != t:
                    cnt *= case.n[e] + 4
            writes += nd * cnt
        return 8 * (nbox * nd + writes)
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
    halo fill (0; 8 = ghosts only, stages 2-3 of a fused step), derivatives
    (5, viscous 2D/3D; 9 = ghosts and derivatives in one launch when every
    face is periodic), fluxes (7 = x+y of a 3D grid, 1..3 per direction),
    then the fused last-direction flux + update (6, 2D/3D without source) or
    the separate update (4)."""
    visc = case.visc_law != "none"
    last = 2 * (case.ndim - 1)
    fused = case.ndim >= 2 and (case.source == "none" or (
        case.bc[last] == "periodic" and case.bc[last + 1] == "periodic"))
    periodic = all(case.bc[2 * d] == "periodic" and case.bc[2 * d + 1] == "periodic"
                   and case.n[d] >= 3 for d in range(case.ndim))
    if fused and visc and periodic:
        ids = [0, 9]
    else:
        ids = [0] + ([8] if fused else []) + ([5] if visc and case.ndim >= 2 else [])
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


def serving_bench(M=32, rate=20.0, seed=2024, M_low=12, rate_low=2.0, seed_low=2025):
    """Continuous batching vs sequential solves on a seeded trace of forward
    and gradient requests (Sod 200-4096 cells, TGV 32^3/48^3/64^3, porous BL
    256x64/512x128), 50-400 steps each, Poisson arrivals at `rate`/s (an
    overloaded GPU), and a shorter trace at `rate_low`/s whose offered load
    stays below the GPU's capacity (latency near the service time)."""
    from paper_2406_19494_amd import serving as S

    def offered(trace):
        work = sum(3.0 * S.cells_of(r) * r.nsteps for r in trace)
        span = max(r.arrival for r in trace)
        return work, (work / span if span > 0 else float("nan"))

    trace = S.draw_trace(M, rate, seed, steps=(50, 400), tgv=(32, 48, 64), bl=(1, 2))
    res, t_b, sch = S.serve(trace, budget_bytes=200e9, max_slots=16)
    sb = S.summarize(res, t_b)
    res_k, t_k, sch_k = S.serve(trace, budget_bytes=200e9, max_slots=16, batched=True)
    sk = S.summarize(res_k, t_k)
    res_s, t_s, _ = S.serve_sequential(trace)
    ss = S.summarize(res_s, t_s)
    work, load = offered(trace)
    low = S.draw_trace(M_low, rate_low, seed_low, steps=(50, 400), tgv=(32, 48, 64), bl=(1, 2))
    res_l, t_l, _ = S.serve(low, budget_bytes=200e9, max_slots=16)
    res_ls, t_ls, _ = S.serve_sequential(low)
    work_l, load_l = offered(low)
    return {"trace": f"{M} requests, Poisson {rate}/s (seed {seed}), steps 50-400, "
                     "sod 200-4096 / tgv 32-64^3 / porous BL 256x64-512x128, 50% gradients",
            "offered_cell_updates": work, "offered_load_cell_updates_per_s": load,
            "batched": sb, "batched_kernels": sk, "sequential": ss,
            "peak_active": sch.peak_active,
            "throughput_ratio": sb["cell_updates_per_s"] / ss["cell_updates_per_s"],
            "throughput_ratio_batched_kernels": sk["cell_updates_per_s"] / ss["cell_updates_per_s"],
            "low_rate": {"trace": f"{M_low} requests, Poisson {rate_low}/s (seed {seed_low}), "
                                  "same mix", "offered_cell_updates": work_l,
                         "offered_load_cell_updates_per_s": load_l,
                         "batched": S.summarize(res_l, t_l),
                         "sequential": S.summarize(res_ls, t_ls)},
            "note": "batched: one stream and hipGraph-captured epochs per request; "
                    "batched_kernels: forward requests of one family share batched step "
                    "launches (dcf_batch_rk3_step); offered load = the trace's cell updates "
                    "over its arrival span"}


def adjoint_ratio(steps=20):
    """Adjoint/forward cost on the Mach-6 porous boundary layer (1024 x 256):
    per step, t(vjp_step incl. stage recompute) / t(rk3_step), HIP events."""
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
    stream = torch.cuda.current_stream()
    for _ in range(3):
        s.step(U, dt)
        s.vjp_step(U, dt, lam, dJdK=gK)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    torch.cuda.synchronize()
    ev[0].record(stream)
    for _ in range(steps):
        s.step(U, dt)
    ev[1].record(stream)
    for _ in range(steps):
        s.vjp_step(U, dt, lam, dJdK=gK)
    ev[2].record(stream)
    torch.cuda.synchronize()
    f = ev[0].elapsed_time(ev[1]) / steps
    a = ev[1].elapsed_time(ev[2]) / steps
    # whole checkpointed trajectory gradient (forward sweep with checkpoints
    # and cost, per-segment recompute, reverse sweep), each phase timed with
    # HIP events between the dcf_gradient_advance calls that run it
    n = 100
    U0 = s.init_state(P)
    traj = {}
    for name, mode, seg in (("mode2", 2, 10), ("mode3", 3, 10), ("mode3_one_segment", 3, n)):
        sg = Solver(case, K=K, mode=mode, nsteps=n, seg_len=seg)
        sg.gradient(U0, dt)  # warm-up
        J = torch.zeros(1, dtype=torch.float64, device="cuda")
        gKt = torch.zeros(sg.nk, dtype=torch.float64, device="cuda")
        nseg = (n + seg - 1) // seg
        evs = [torch.cuda.Event(enable_timing=True) for _ in range(2 + 2 * nseg)]
        torch.cuda.synchronize()
        sg.gradient_begin(U0, dt, J, gKt)
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
        traj[name] = {"steps": n, "seg_len": seg, "mode": mode, "gradient_ms": g,
                      "forward_sweep_ms": fwd, "recompute_ms": rec, "reverse_ms": rev,
                      "gradient_over_forward": g / (n * f),
                      "end_to_end_over_forward": (g - fwd) / (n * f),
                      "reverse_step_over_forward": rev / (n * f)}
        del sg
    return {"workload": "Mach-6 porous boundary layer 1024x256", "forward_ms_per_step": f,
            "vjp_ms_per_step": a, "vjp_step_over_forward": a / f,
            "adjoint_forward_ratio": traj["mode3"]["reverse_step_over_forward"],
            "vjp_step_note": "dcf_vjp_step alone recomputes the two inner stage states and "
                             "every stage's primitive and derivative boxes of its step",
            "trajectory": traj,
            "trajectory_note": "reverse_step_over_forward: reverse sweep (one VJP of the RK3 "
                               "step per step, cost adjoint included) over the forward "
                               "rk3_step, per step; end_to_end_over_forward: (gradient - "
                               "forward sweep) / forward trajectory; mode2 recomputes each "
                               "stage's boxes in the reverse sweep, mode3 keeps them from the "
                               "segment recompute; the last segment keeps its data from the "
                               "forward sweep (one segment: no recompute); "
                               "adjoint_forward_ratio is mode3's (S = 10)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="tgv64")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-adjoint", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
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

    # per-kernel timing (HIP events on the same stream) -> dominant kernel.
    # A 2D/3D step without source term runs the last direction's fluxes
    # fused with the stage update (k_flux_update); the unfused pair is timed
    # too, for the record.
    # A 3D step launches the x and y fluxes as one grid (k_flux_xy).  In a
    # fused step the update of stages 1 and 2 also writes the next stage's
    # primitive interior, so stages 2 and 3 fill only the ghosts
    # (k_prim_ghost, 8) where stage 1 runs the whole halo fill (0).
    names = {0: "k_prim_halo", 1: "k_flux_x", 2: "k_flux_yz<y>", 3: "k_flux_yz<z>", 4: "k_update",
             5: "k_grad", 6: "k_flux_update", 7: "k_flux_xy", 8: "k_prim_ghost",
             9: "k_ghost_grad_periodic"}
    visc = case.visc_law != "none"
    step_kinds = step_kernel_ids(case)
    kinds = sorted(set(step_kinds) | set(range(1, case.ndim + 1)) | {4})
    kt = {w: s.time_kernel(U, w, reps=20) for w in kinds}

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

    def kernel_roof(w, t_ms=None):
        # every launch against the roof that binds it: the larger of the
        # FP64 lower bound (algorithmic flops / 78.6 TFLOP/s) and the HBM
        # lower bound (algorithmic bytes / 8 TB/s); the flux kernels have
        # both, the others only bytes.  t_ms: the launch duration (default:
        # the back-to-back launches of dcf_time_kernel)
        nf = flux_faces(w)
        t = (kt[w] if t_ms is None else t_ms) * 1e-3
        if nf is not None:
            fpf, bpf = FLOPS_PER_FACE[(case.ndim, visc)], BYTES_PER_FACE[(case.ndim, visc)]
            flops = fpf * nf
            if w == 6:
                # inputs of one cell once (primitives and derivatives), the
                # other directions' face fluxes, Un and Uin; Uout written
                cells = case.ncells
                nbytes = cells * (bpf - 40) + 3 * cells * case.nv * 8
                nbytes += sum(40 * faces_of(D) for D in range(case.ndim - 1))
            else:
                nbytes = bpf * nf
            t_alu, t_hbm = flops / PEAK_FP64, nbytes / PEAK_HBM
            out = {"algorithmic_flops_per_face": fpf, "faces_per_launch": nf,
                   "algorithmic_bytes": nbytes, "alu_frac": t_alu / t, "hbm_frac": t_hbm / t}
            if t_hbm >= t_alu:
                return {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": PEAK_HBM / 1e9,
                        "unit": "GB/s", "frac": t_hbm / t} | out
            return {"bound": "alu", "achieved": flops / t / 1e12, "peak": PEAK_FP64 / 1e12,
                    "unit": "TFLOP/s", "frac": t_alu / t} | out
        nbytes = algorithmic_bytes(case, names[w])
        return {"bound": "hbm", "achieved": nbytes / t / 1e9, "peak": PEAK_HBM / 1e9,
                "unit": "GB/s", "frac": nbytes / t / PEAK_HBM, "algorithmic_bytes": nbytes}

    # dominant kernel: the step's slowest launch.  Its duration is measured
    # on its launches inside the stepping loop: HIP event pairs around each
    # of them on the stream of the stepping call (dcf_probe_*), over a replay
    # of the timed region (the same call with the same step count; the timed
    # value above runs without events)
    dom = max(step_kinds, key=lambda w: kt[w])
    probe_n, t_dom = 0, kt[dom]
    if dom in (1, 5, 6, 7, 8, 9):  # launches of the fused stepping path (2D/3D)
        s.probe_begin(dom, 4 * args.steps + 8)
        s.steps_cfl(U, dt, args.steps, cfl=case.cfl)
        torch.cuda.synchronize()
        probe_n, t_probe = s.probe_end()
        assert s.flags() == 0, "non-physical state during the probe replay"
        if probe_n > 0:
            t_dom = t_probe
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
    # every kernel against its own roofline, for the record (durations of
    # back-to-back launches, dcf_time_kernel)
    per_kernel = {}
    for w in kinds:
        r = kernel_roof(w)
        per_kernel[names[w]] = {"bound": r["bound"], "frac": r["frac"],
                                ("achieved_tflops" if r["bound"] == "alu" else "achieved_gbs"):
                                    r["achieved"], "in_step": w in step_kinds}
        for k in ("alu_frac", "hbm_frac"):
            if k in r:
                per_kernel[names[w]][k] = r[k]
    roof["per_kernel"] = per_kernel

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
                   "step": "CFL dt + TVD-RK3 (WENO5-JS, HLLC, 4th-order viscous)"},
        "roofline": roof,
        "kernel_ms": {names[k]: v for k, v in kt.items()},
        "step_kernels": [names[k] for k in step_kinds],
        "source_sha": source_digest(),
        "wall_s": wall,
    }
    if not args.no_adjoint:
        out["adjoint"] = adjoint_ratio()
    if not args.no_serving:
        out["serving"] = serving_bench()
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(case, P, K, args.cpu_budget)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
