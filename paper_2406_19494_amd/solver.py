"""Python front end of the HIP library: one ``Solver`` per case.

PyTorch provides device memory and the stream; every computation runs in the
library's HIP kernels behind the C ABI (include/dcf.h).  The methods here
only marshal arguments.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import binding as B
from .workloads import Case


def _ptr(t: Optional[torch.Tensor]):
    if t is None:
        return None
    assert t.is_cuda and t.is_contiguous(), "device tensors must be contiguous CUDA tensors"
    return C.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = torch.cuda.current_stream() if stream is None else stream
    return C.c_void_p(s.cuda_stream)


class Solver:
    """A solve on the GPU.

    mode: -1 no workspace (only dcf_rk3_step_noalloc runs), 0 forward, 1
    forward + single-step VJP, 2 trajectory gradient with
    ``nsteps`` steps and checkpoints every ``seg_len`` steps, 3 as 2 with the
    stage boxes of a segment kept for the reverse sweep (more memory, no
    recompute in the reverse sweep).  In modes 2 and 3 seg_len = 0 takes the
    longest spacing whose workspace fits ``seg_budget`` bytes (default 90 %
    of the device memory free now): the whole trajectory resident whenever
    it fits, which recomputes nothing (segment_length_for).
    """

    def __init__(self, case: Case, K=None, mode: int = 0, nsteps: int = 0, seg_len: int = 0,
                 device: str = "cuda", seg_budget=None):
        if not torch.cuda.is_available():
            raise RuntimeError("the dcf library needs a GPU (no CPU fallback)")
        self.case = case
        self.device = torch.device(device)
        L = B.lib()
        g = B.dcf_grid()
        g.ndim = case.ndim
        for d in range(3):
            g.n[d] = case.n[d]
            g.lo[d] = case.lo[d]
            g.hi[d] = case.hi[d]
            g.stretch[d] = B.STRETCH[case.stretch[d]]
            g.beta[d] = case.beta[d]
        gas = B.dcf_gas(case.gamma, case.R, case.Pr, B.VISC[case.visc_law], case.mu_ref,
                        case.T_ref, case.visc_param)
        ctx = C.c_void_p()
        B.call("dcf_create", C.byref(g), C.byref(gas), C.byref(ctx))
        self.ctx = ctx
        self._keep = []
        for f in range(2 * case.ndim):
            bc = B.dcf_bc()
            bc.kind = B.BC[case.bc[f]]
            bc.T_wall = case.T_wall[f]
            if f in case.dirichlet:
                prof = torch.as_tensor(np.ascontiguousarray(case.dirichlet[f]), dtype=torch.float64,
                                       device=self.device)
                self._keep.append(prof)
                bc.dirichlet = prof.data_ptr()
            if case.bc[f] == "porous":
                bc.porous_begin, bc.porous_end, bc.p_inf = (case.porous_begin, case.porous_end,
                                                            case.p_inf)
            B.call("dcf_set_bc", ctx, f, C.byref(bc))
        B.call("dcf_set_source", ctx, B.SOURCE[case.source])
        B.call("dcf_set_scheme", ctx, B.SCHEME[getattr(case, "scheme", "weno5")])
        if case.cost_face >= 0:
            B.call("dcf_set_cost", ctx, case.cost_face, case.p_inf)
        self.nk = L.dcf_num_params(ctx)
        self.K = None
        if self.nk != case.nk:
            raise ValueError(f"library reports {self.nk} boundary parameters, the case "
                             f"{case.nk}")
        if self.nk:
            # porous coefficients (or the full parameter vector), with the
            # case's disturbance amplitudes and wavenumbers appended
            th = K if torch.is_tensor(K) and K.numel() == self.nk else case.theta(
                None if K is None else (K.cpu().numpy() if torch.is_tensor(K) else K))
            self.set_params(torch.as_tensor(th, dtype=torch.float64, device=self.device))
        if mode >= 2 and seg_len == 0:
            if seg_budget is None:
                free, _ = torch.cuda.mem_get_info(self.device)
                seg_budget = int(0.9 * free)
            seg_len = segment_length_for(case, mode, nsteps, int(seg_budget))
        self.mode, self.nsteps, self.seg_len = mode, nsteps, seg_len
        self.workspace = None
        if mode >= 0:  # mode -1: no workspace (for dcf_rk3_step_noalloc)
            size = C.c_size_t()
            B.call("dcf_workspace_size", ctx, mode, nsteps, seg_len, C.byref(size))
            self.workspace = torch.empty(size.value, dtype=torch.uint8, device=self.device)
            B.call("dcf_set_workspace", ctx, mode, nsteps, seg_len, _ptr(self.workspace),
                   size.value)
        nv, ncell, nbytes = C.c_int(), C.c_long(), C.c_size_t()
        B.call("dcf_state_info", ctx, C.byref(nv), C.byref(ncell), C.byref(nbytes))
        self.nv, self.ncell = nv.value, ncell.value

    def __del__(self):
        ctx = getattr(self, "ctx", None)
        if ctx is not None and ctx.value:
            try:
                B.lib().dcf_destroy(ctx)
            except Exception:
                pass
            self.ctx = None

    # ---------------------------------------------------------------- state
    @property
    def shape(self):
        c = self.case
        return (c.nv, c.n[2], c.n[1], c.n[0])

    def empty_state(self):
        return torch.empty(self.shape, dtype=torch.float64, device=self.device)

    def set_params(self, K: torch.Tensor):
        K = K.to(device=self.device, dtype=torch.float64).contiguous()
        self.K = K
        B.call("dcf_set_params", self.ctx, _ptr(K), int(K.numel()))

    def init_state(self, P, stream=None, out=None) -> torch.Tensor:
        """Conserved state from primitives P (into `out` when given).  The
        staged copy of P is made on the stream that reads it, so that its
        memory is not handed out again while the conversion is pending."""
        st = torch.cuda.current_stream() if stream is None else stream
        with torch.cuda.stream(st):
            Pt = torch.as_tensor(np.ascontiguousarray(P), dtype=torch.float64,
                                 device=self.device)
            U = self.empty_state() if out is None else out
            B.call("dcf_init_state", self.ctx, _ptr(Pt), _ptr(U), _stream(st))
        return U

    # -------------------------------------------------------------- forward
    def rhs(self, U: torch.Tensor, stream=None) -> torch.Tensor:
        R = torch.empty_like(U)
        B.call("dcf_rhs", self.ctx, _ptr(U), _ptr(R), _stream(stream))
        return R

    def compute_dt(self, U, cfl=None, dt_max=0.0, out=None, stream=None) -> torch.Tensor:
        dt = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        B.call("dcf_compute_dt", self.ctx, _ptr(U), float(self.case.cfl if cfl is None else cfl),
               float(dt_max), _ptr(dt), _stream(stream))
        return dt

    def step(self, U: torch.Tensor, dt: torch.Tensor, stream=None):
        B.call("dcf_rk3_step", self.ctx, _ptr(U), _ptr(dt), _stream(stream))

    def step_keep(self, U: torch.Tensor, dt: torch.Tensor, stages: torch.Tensor, stream=None):
        """One RK3 step that also writes its stage states U(1), U(2) into
        `stages` (shape (2,) + U.shape)."""
        assert stages.numel() == 2 * U.numel()
        B.call("dcf_rk3_step_keep", self.ctx, _ptr(U), _ptr(dt), _ptr(stages), _stream(stream))

    def step_cfl(self, U: torch.Tensor, dt: torch.Tensor, cfl=None, dt_max=0.0, out=None,
                 stream=None) -> torch.Tensor:
        """One RK3 step with dt, returning (in `out`, default dt itself) the
        CFL step of the new state from the last stage's fused reduction."""
        out = dt if out is None else out
        B.call("dcf_rk3_step_cfl", self.ctx, _ptr(U), _ptr(dt),
               float(self.case.cfl if cfl is None else cfl), float(dt_max), _ptr(out),
               _stream(stream))
        return out

    def steps_cfl(self, U: torch.Tensor, dt: torch.Tensor, nsteps: int, cfl=None, dt_max=0.0,
                  stream=None) -> torch.Tensor:
        """nsteps of step_cfl in one call (dt updated in place after each
        step); bitwise the same, with less work per step."""
        B.call("dcf_rk3_steps_cfl", self.ctx, _ptr(U), _ptr(dt), int(nsteps),
               float(self.case.cfl if cfl is None else cfl), float(dt_max), _stream(stream))
        return dt

    def run(self, U: torch.Tensor, nsteps: int, dt_fixed: float = 0.0, t_end: float = 0.0,
            cfl=None):
        """Advance U in place.  With dt_fixed > 0 the step is fixed; otherwise
        the CFL step is computed on the device each step (t_end > 0 clips the
        last step, which reads the step size back to the host)."""
        dt = torch.empty(1, dtype=torch.float64, device=self.device)
        t = 0.0
        steps = 0
        if dt_fixed > 0.0:
            dt.fill_(dt_fixed)
            for _ in range(nsteps):
                self.step(U, dt)
            return nsteps, dt_fixed * nsteps
        while steps < nsteps:
            if t_end > 0.0 and t >= t_end:
                break
            self.compute_dt(U, cfl=cfl, dt_max=(t_end - t) if t_end > 0.0 else 0.0, out=dt)
            if t_end > 0.0:
                t += float(dt.item())
            self.step(U, dt)
            steps += 1
        return steps, t

    def diagnostics(self, U: torch.Tensor, stream=None) -> dict:
        out = torch.empty(8, dtype=torch.float64, device=self.device)
        B.call("dcf_diagnostics", self.ctx, _ptr(U), _ptr(out), _stream(stream))
        o = out.cpu().numpy()
        return dict(ek=o[0], eps=o[1], mass=o[2], mom=o[3:6].copy(), energy=o[6], vol=o[7])

    def time_kernel(self, U, which: int, reps: int = 20, stream=None) -> float:
        """Mean duration (ms) of one kernel family, timed with HIP events."""
        ms = C.c_double()
        B.call("dcf_time_kernel", self.ctx, _ptr(U), int(which), int(reps), C.byref(ms),
               _stream(stream))
        return ms.value

    def probe_begin(self, which: int, max_launches: int) -> None:
        """Arm HIP event pairs around the stepping calls' launches of one
        kernel family (dcf_probe_begin)."""
        B.call("dcf_probe_begin", self.ctx, int(which), int(max_launches))

    def probe_end(self):
        """(launches recorded, mean duration in ms) of the armed probe
        (dcf_probe_end; waits for its last event)."""
        n, ms = C.c_int(), C.c_double()
        B.call("dcf_probe_end", self.ctx, C.byref(n), C.byref(ms))
        return n.value, ms.value

    def flags(self, stream=None) -> int:
        f = C.c_uint()
        B.call("dcf_flags", self.ctx, C.byref(f), _stream(stream))
        return f.value

    # -------------------------------------------------------------- adjoint
    def cost_term(self, U, w=1.0, J=None, grad=None, stream=None):
        J = torch.zeros(1, dtype=torch.float64, device=self.device) if J is None else J
        B.call("dcf_cost_term", self.ctx, _ptr(U), float(w), _ptr(J), _ptr(grad), _stream(stream))
        return J

    def vjp_step(self, Un, dt, lam, dJdK=None, stages=None, stream=None) -> torch.Tensor:
        """lam_n of one step; `stages` (2 state arrays from step_keep) spares
        the VJP the recompute of the stage states."""
        out = torch.empty_like(lam)
        B.call("dcf_vjp_step", self.ctx, _ptr(Un), _ptr(stages), _ptr(dt), _ptr(lam), _ptr(out),
               _ptr(dJdK), _stream(stream))
        return out

    def workspace_bytes(self) -> int:
        return 0 if self.workspace is None else int(self.workspace.numel())

    def gradient_begin(self, U0, dt, J, gK, stream=None, nsteps=None):
        """Start a trajectory gradient of `nsteps` steps (default: the size
        the workspace was made for; fewer fit the same workspace)."""
        n = self.nsteps if nsteps is None else int(nsteps)
        B.call("dcf_gradient_begin", self.ctx, _ptr(U0), n, _ptr(dt),
               int(self.seg_len), _ptr(J), _ptr(gK) if self.nk else None, _stream(stream))

    def gradient_advance(self, max_units: int, stream=None) -> bool:
        done = C.c_int()
        B.call("dcf_gradient_advance", self.ctx, int(max_units), C.byref(done), _stream(stream))
        return bool(done.value)

    def gradient_finish(self, gU=None, stream=None):
        B.call("dcf_gradient_finish", self.ctx, _ptr(gU), _stream(stream))

    def gradient(self, U0, dt, stream=None):
        """J, dJ/dK, dJ/dU0 over the trajectory sized at construction."""
        J = torch.zeros(1, dtype=torch.float64, device=self.device)
        gK = torch.zeros(max(self.nk, 1), dtype=torch.float64, device=self.device)
        gU = torch.empty_like(U0)
        B.call("dcf_gradient", self.ctx, _ptr(U0), int(self.nsteps), _ptr(dt), int(self.seg_len),
               _ptr(J), _ptr(gK) if self.nk else None, _ptr(gU), _stream(stream))
        return J, gK[: self.nk], gU


def grid_gas(case: Case):
    """The C structs of a case's grid and gas."""
    g = B.dcf_grid()
    g.ndim = case.ndim
    for d in range(3):
        g.n[d] = case.n[d]
        g.lo[d] = case.lo[d]
        g.hi[d] = case.hi[d]
        g.stretch[d] = B.STRETCH[case.stretch[d]]
        g.beta[d] = case.beta[d]
    gas = B.dcf_gas(case.gamma, case.R, case.Pr, B.VISC[case.visc_law], case.mu_ref,
                    case.T_ref, case.visc_param)
    return g, gas


def workspace_bytes_for(case: Case, mode: int, nsteps: int = 0, seg_len: int = 0) -> int:
    """Workspace size of a solve without creating one (host arithmetic in the
    library, dcf_workspace_size_for)."""
    g, gas = grid_gas(case)
    size = C.c_size_t()
    B.call("dcf_workspace_size_for", C.byref(g), C.byref(gas), int(mode), int(nsteps),
           int(seg_len), C.byref(size))
    return size.value


def segment_length_for(case: Case, mode: int, nsteps: int, budget_bytes: int) -> int:
    """The checkpoint spacing of an nsteps-step trajectory gradient (mode 2 or
    3) that recomputes the fewest steps within a workspace budget: the
    largest seg_len whose workspace fits (every segment but the last is
    recomputed, so a longer segment recomputes less; seg_len = nsteps keeps
    the whole trajectory resident and recomputes nothing).  The workspace,
    about (ceil(nsteps / seg_len) + 3 seg_len) states in mode 2, is not
    monotonic in seg_len, so every spacing is tried from the longest down
    (host arithmetic, one library call each).  Raises ValueError when none
    fits."""
    if mode not in (2, 3) or nsteps < 1:
        raise ValueError("a trajectory gradient workspace (mode 2 or 3, nsteps >= 1)")
    for S in range(nsteps, 0, -1):
        if workspace_bytes_for(case, mode, nsteps, S) <= budget_bytes:
            return S
    raise ValueError(f"no checkpoint spacing fits {budget_bytes} bytes")


class BatchPlan:
    """A fixed batch of solves stepped together: the device table is written
    once (outside any graph capture); step() enqueues launches only
    (dcf_batch_rk3_step_table), so it can be captured and replayed while the
    batch stays the same."""

    def __init__(self, solvers, Us, dts, stream=None):
        n = len(solvers)
        size = C.c_size_t()
        B.call("dcf_batch_table_bytes", n, C.byref(size))
        dev = Us[0].device
        self.n = n
        self.host = torch.empty(size.value, dtype=torch.uint8, pin_memory=True)
        VP = C.c_void_p * n
        B.call("dcf_batch_table_fill", VP(*[s.ctx.value for s in solvers]),
               VP(*[U.data_ptr() for U in Us]), VP(*[d.data_ptr() for d in dts]), n,
               C.c_void_p(self.host.data_ptr()), size.value)
        s = torch.cuda.current_stream() if stream is None else stream
        with torch.cuda.stream(s):
            # allocated on the stream whose launches read it: freed memory
            # is handed out again only in that stream's order
            self.dev = torch.empty(size.value, dtype=torch.uint8, device=dev)
            self.dev.copy_(self.host, non_blocking=True)
        # keep the members alive while the plan (or a graph of it) exists
        self.members = (list(solvers), list(Us), list(dts))

    def step(self, cfl=None, stream=None):
        B.call("dcf_batch_rk3_step_table", _ptr(self.dev), C.c_void_p(self.host.data_ptr()),
               self.n, float(cfl) if cfl else 0.0, _stream(stream))


class BatchStepper:
    """One TVD-RK3 step of several solves with one launch per kernel and
    stage (dcf_batch_rk3_step); keeps the device tile table between calls."""

    def __init__(self):
        self.table = None

    def step(self, solvers, Us, dts, cfl=None, stream=None):
        n = len(solvers)
        if n == 0:
            return
        size = C.c_size_t()
        B.call("dcf_batch_table_bytes", n, C.byref(size))
        if self.table is None or self.table.numel() < size.value:
            dev = Us[0].device
            self.table = torch.empty(max(size.value, 4096), dtype=torch.uint8, device=dev)
        VP = C.c_void_p * n
        ctxs = VP(*[s.ctx.value for s in solvers])
        us = VP(*[U.data_ptr() for U in Us])
        ds = VP(*[d.data_ptr() for d in dts])
        B.call("dcf_batch_rk3_step", ctxs, us, ds, n, float(cfl) if cfl else 0.0,
               _ptr(self.table), self.table.numel(), _stream(stream))
