"""Error paths of the C ABI on a device context: every argument error is a
status (never a crash), reported before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2406_19494_amd import binding as B
from paper_2406_19494_amd import workloads as W
from paper_2406_19494_amd.solver import Solver

pytestmark = pytest.mark.gpu


def _ctx(case):
    g = B.dcf_grid()
    g.ndim = case.ndim
    for d in range(3):
        g.n[d], g.lo[d], g.hi[d] = case.n[d], case.lo[d], case.hi[d]
        g.stretch[d], g.beta[d] = B.STRETCH[case.stretch[d]], case.beta[d]
    gas = B.dcf_gas(case.gamma, case.R, case.Pr, B.VISC[case.visc_law], case.mu_ref, case.T_ref,
                    case.visc_param)
    ctx = C.c_void_p()
    B.call("dcf_create", C.byref(g), C.byref(gas), C.byref(ctx))
    return ctx


def test_workspace_too_small_and_unset():
    case, P = W.tgv(8)
    L = B.lib()
    ctx = _ctx(case)
    U = torch.zeros((5, 8, 8, 8), dtype=torch.float64, device="cuda")
    R = torch.empty_like(U)
    # no workspace yet
    assert L.dcf_rhs(ctx, C.c_void_p(U.data_ptr()), C.c_void_p(R.data_ptr()), None) == -2
    size = C.c_size_t()
    B.call("dcf_workspace_size", ctx, 0, 0, 0, C.byref(size))
    ws = torch.empty(size.value, dtype=torch.uint8, device="cuda")
    assert L.dcf_set_workspace(ctx, 0, 0, 0, C.c_void_p(ws.data_ptr()), size.value - 1) == -2
    # misaligned
    assert L.dcf_set_workspace(ctx, 0, 0, 0, C.c_void_p(ws.data_ptr() + 8), size.value) == -1
    B.call("dcf_set_workspace", ctx, 0, 0, 0, C.c_void_p(ws.data_ptr()), size.value)
    # mode-0 workspace cannot run the adjoint
    lam = torch.zeros_like(U)
    dt = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
    rc = L.dcf_vjp_step(ctx, C.c_void_p(U.data_ptr()), None, C.c_void_p(dt.data_ptr()),
                        C.c_void_p(lam.data_ptr()), C.c_void_p(R.data_ptr()), None, None)
    assert rc == -2
    L.dcf_destroy(ctx)


def test_unpaired_periodic_face_rejected():
    case, P = W.channel(nx=8, ny=8, nz=8)
    case = W.Case(**{**case.__dict__, "bc": ("periodic", "zerograd", "wall", "wall",
                                             "periodic", "periodic")})
    with pytest.raises(B.DcfError) as ei:
        s = Solver(case)
        s.rhs(s.init_state(P))
    assert ei.value.code == -1 and "pairs" in str(ei.value)


def test_bad_porous_strip_and_params():
    case, P, K = W.porous_bl(nx=32, ny=16, strip=(8, 24), nsteps=1)
    bad = W.Case(**{**case.__dict__, "porous_end": 40})
    with pytest.raises(B.DcfError) as ei:
        Solver(bad, K=K)
    assert ei.value.code == -1
    s = Solver(case, K=K)
    with pytest.raises(B.DcfError):
        s.set_params(torch.zeros(case.nk + 1, dtype=torch.float64, device="cuda"))


def test_gradient_sized_for_other_trajectory_rejected():
    case, P, K = W.porous_bl(nx=32, ny=16, strip=(8, 24), nsteps=1)
    s = Solver(case, K=K, mode=2, nsteps=4, seg_len=2)
    U = s.init_state(P)
    dt = torch.full((1,), 1e-6, dtype=torch.float64, device="cuda")
    s.nsteps = 5  # not what the workspace was sized for
    with pytest.raises(B.DcfError) as ei:
        s.gradient(U, dt)
    assert ei.value.code == -1


def test_time_kernel_families_and_unknown_ids():
    # every kernel family of a 3D viscous periodic case times to a positive
    # duration; ids 5 and 9 (no derivative launch exists: the flux kernels
    # compute the velocity derivatives while staging) are refused; the fused
    # flux + update (6) and the combined x + y flux launch (7) are refused
    # where the case has none (1D)
    case, P = W.tgv(16)
    L = B.lib()
    ms = C.c_double()
    for mode in (0, 1):
        s = Solver(case, mode=mode)
        U = s.init_state(P)
        for w in (0, 1, 2, 3, 4, 6, 7, 8):
            assert s.time_kernel(U, w, reps=2) > 0.0
        for bad in (-1, 5, 9, 10):
            assert L.dcf_time_kernel(s.ctx, C.c_void_p(U.data_ptr()), bad, 2, C.byref(ms),
                                     None) == -1
    case1, P1 = W.sod(64)
    s1 = Solver(case1)
    U1 = s1.init_state(P1)
    assert s1.time_kernel(U1, 1, reps=2) > 0.0
    for bad in (2, 6, 7, 9):
        assert L.dcf_time_kernel(s1.ctx, C.c_void_p(U1.data_ptr()), bad, 2, C.byref(ms), None) == -1


def test_probe_counts_in_loop_launches_and_changes_nothing():
    # event pairs around the stepping calls' launches of one kernel family:
    # one launch per stage, the same state bitwise as an unprobed run
    print("[probe] tgv 12, porous BL 24x16", flush=True)
    for case, P, K, ids in ((*W.tgv(12), None, (7, 6, 8)),
                            (*W.porous_bl(nx=24, ny=16, strip=(6, 18)), (1, 6, 8))):
        s = Solver(case, K=K)
        U0 = s.init_state(P)
        ref = U0.clone()
        dt_ref = s.compute_dt(ref, cfl=0.4)
        s.steps_cfl(ref, dt_ref, 4, cfl=0.4)
        for w in ids:
            U = U0.clone()
            dt = s.compute_dt(U, cfl=0.4)
            s.probe_begin(w, 100)
            s.steps_cfl(U, dt, 4, cfl=0.4)
            n, ms = s.probe_end()
            # ghosts alone (8) run in stages 2-3 and later first stages; the
            # first stage of the call fills the whole halo
            assert n == (4 * 3 - 1 if w == 8 else 4 * 3), (case.name, w, n)
            assert ms > 0.0
            assert torch.equal(U, ref) and torch.equal(dt, dt_ref), (case.name, w)
    # capped at max_launches
    s.probe_begin(6, 5)
    U = U0.clone()
    s.steps_cfl(U, s.compute_dt(U, cfl=0.4), 4, cfl=0.4)
    assert s.probe_end()[0] == 5


def test_probe_argument_errors():
    case, P = W.tgv(8)
    s = Solver(case)
    L = B.lib()
    n, ms = C.c_int(), C.c_double()
    for bad in (-1, 0, 2, 3, 4, 5, 9, 10):
        assert L.dcf_probe_begin(s.ctx, bad, 10) == -1
    assert L.dcf_probe_begin(s.ctx, 7, 0) == -1
    assert L.dcf_probe_end(s.ctx, C.byref(n), C.byref(ms)) == -1  # nothing armed
    assert L.dcf_probe_begin(s.ctx, 7, 10) == 0
    assert L.dcf_probe_begin(s.ctx, 7, 10) == -1  # armed twice
    assert L.dcf_probe_end(s.ctx, C.byref(n), C.byref(ms)) == 0
    assert n.value == 0 and ms.value == 0.0
