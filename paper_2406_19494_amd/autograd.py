"""torch.autograd bindings of the hand-written adjoint.

* ``RK3Step``: one TVD-RK3 step U^n -> U^{n+1} (fixed dt, porous
  coefficients K); backward is the library's VJP kernel sequence
  (``dcf_vjp_step``), which also returns dJ/dK.
* ``TrajectoryCost``: J = (1/N) sum_n j(U^n) over an N-step trajectory from
  U0; forward runs the forward sweep with checkpoints (the first N units of
  the library's incremental gradient), backward finishes the reverse sweep and
  returns dJ/dU0 and dJ/dK.

Both only marshal tensors to the C ABI; the computation is in the kernels.
"""
from __future__ import annotations

import torch

from .solver import Solver


class RK3Step(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U: torch.Tensor, K: torch.Tensor, solver: Solver, dt: torch.Tensor):
        if K is not None and solver.nk:
            solver.set_params(K.detach())
        out = U.detach().clone()
        solver.step(out, dt)
        ctx.save_for_backward(U.detach(), dt)
        ctx.solver = solver
        return out

    @staticmethod
    def backward(ctx, gout: torch.Tensor):
        U, dt = ctx.saved_tensors
        s = ctx.solver
        gK = torch.zeros(max(s.nk, 1), dtype=torch.float64, device=U.device)
        gU = s.vjp_step(U, dt, gout.contiguous(), dJdK=gK if s.nk else None)
        return gU, (gK[: s.nk] if s.nk else None), None, None


class TrajectoryCost(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U0: torch.Tensor, K: torch.Tensor, solver: Solver, dt: torch.Tensor):
        if K is not None and solver.nk:
            solver.set_params(K.detach())
        J = torch.zeros(1, dtype=torch.float64, device=U0.device)
        gK = torch.zeros(max(solver.nk, 1), dtype=torch.float64, device=U0.device)
        U0c = U0.detach().contiguous()
        solver.gradient_begin(U0c, dt, J, gK)
        solver.gradient_advance(solver.nsteps)  # exactly the forward sweep
        ctx.solver, ctx.gK = solver, gK
        ctx.save_for_backward(U0c, dt)
        return J.clone()

    @staticmethod
    def backward(ctx, gJ: torch.Tensor):
        s = ctx.solver
        U0, dt = ctx.saved_tensors
        while not s.gradient_advance(1 << 20):
            pass
        gU = torch.empty_like(U0)
        s.gradient_finish(gU)
        gK = ctx.gK[: s.nk] if s.nk else None
        return gU * gJ, (gK * gJ if gK is not None else None), None, None


def optimize_porous(solver: Solver, U0: torch.Tensor, dt: torch.Tensor, K0, iters: int = 10,
                    lr: float = 0.05, k_max: float = 1.0, betas=(0.9, 0.999)):
    """Projected Adam on the boundary parameters (porous coefficients K_i,
    then any disturbance-wall (A, kappa)) to reduce the wall-pressure cost J
    (the end-to-end optimisation the gradient is for).  The porous
    coefficients are kept in [0, k_max].  Returns the history of (J, theta)."""
    n_por = solver.case.n_porous
    K = torch.as_tensor(K0, dtype=torch.float64, device=U0.device).clone()
    m = torch.zeros_like(K)
    v = torch.zeros_like(K)
    hist = []
    for it in range(1, iters + 1):
        Kv = K.clone().requires_grad_(True)
        J = TrajectoryCost.apply(U0, Kv, solver, dt)
        J.backward()
        g = Kv.grad
        hist.append((J.item(), K.clone()))
        m = betas[0] * m + (1 - betas[0]) * g
        v = betas[1] * v + (1 - betas[1]) * g * g
        mh = m / (1 - betas[0] ** it)
        vh = v / (1 - betas[1] ** it)
        K = K - lr * mh / (vh.sqrt() + 1e-30)
        K[:n_por].clamp_(0.0, k_max)
    return hist
