"""The step that allocates nothing (dcf_rk3_step_noalloc) against the
workspace step (dcf_rk3_step), through the C ABI: bitwise the same state on
two calls in a row, the second on a smaller grid, and the size limit of its
static scratch."""
import ctypes as C

import numpy as np
import pytest
import torch

from paper_2406_19494_amd import binding as B
from paper_2406_19494_amd import workloads as W
from paper_2406_19494_amd.solver import Solver

pytestmark = pytest.mark.gpu


def _ptr(t):
    return C.c_void_p(t.data_ptr())


def _noalloc_step(s, U, dt, flags):
    st = C.c_void_p(torch.cuda.current_stream().cuda_stream)
    B.call("dcf_rk3_step_noalloc", s.ctx, _ptr(U), _ptr(dt), _ptr(flags), st)


def _cases():
    tgv, P_tgv = W.tgv(24)
    ch, P_ch = W.channel(nx=20, ny=18, nz=11)   # walls, stretching, body force
    sod, P_sod = W.sod(300)                      # 1D path
    return [("tgv24", tgv, P_tgv), ("channel20x18x11", ch, P_ch), ("sod300", sod, P_sod)]


def test_noalloc_step_matches_workspace_step_bitwise():
    # consecutive calls share the scratch: the second and third are on
    # smaller grids than the first, so stale contents of the larger one lie
    # under and beyond every buffer they use
    for name, case, P in _cases():
        print(f"[noalloc] {name} n={case.n}", flush=True)
        ref = Solver(case)                  # workspace step
        bare = Solver(case, mode=-1)        # context without a workspace
        U_ref = ref.init_state(P)
        U_bare = U_ref.clone()
        dt = ref.compute_dt(U_ref, cfl=case.cfl)
        flags = torch.zeros(1, dtype=torch.int32, device="cuda")
        for _ in range(2):
            ref.step(U_ref, dt)
            _noalloc_step(bare, U_bare, dt, flags)
        torch.cuda.synchronize()
        assert torch.equal(U_ref, U_bare), name
        assert int(flags.item()) == 0, name
        assert ref.flags() == 0


def test_noalloc_flags_reach_the_callers_word():
    case, P = W.sod(64)
    bare = Solver(case, mode=-1)
    P = np.array(P)
    P[4, 0, 0, 20] = -1.0  # a negative pressure: the kernels flag it
    U = bare.init_state(P)
    dt = torch.full((1,), 1e-4, dtype=torch.float64, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    _noalloc_step(bare, U, dt, flags)
    torch.cuda.synchronize()
    assert int(flags.item()) & 1


def test_noalloc_rejects_a_case_beyond_the_scratch():
    case, _ = W.tgv(96)  # ~0.25 GB of forward workspace
    bare = Solver(case, mode=-1)
    U = torch.zeros(bare.shape, dtype=torch.float64, device="cuda")
    dt = torch.full((1,), 1e-4, dtype=torch.float64, device="cuda")
    flags = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(B.DcfError) as ei:
        _noalloc_step(bare, U, dt, flags)
    assert ei.value.code == -5  # DCF_EBUDGET
