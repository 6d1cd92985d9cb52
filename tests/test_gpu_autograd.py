"""torch.autograd bindings of the adjoint: RK3Step agrees with finite
differences (gradcheck) and with the oracle's dense adjoint; TrajectoryCost
agrees with dcf_gradient; the optimisation loop over K lowers the cost."""
import numpy as np
import pytest
import torch

from oracle.pyoracle import Oracle
from paper_2406_19494_amd import workloads as W
from paper_2406_19494_amd.autograd import RK3Step, TrajectoryCost, optimize_porous
from paper_2406_19494_amd.solver import Solver
from tests.test_oracle_pins import _tiny_porous

pytestmark = pytest.mark.gpu


def test_rk3step_gradcheck_1d():
    case, P = W.sod(24)
    s = Solver(case, mode=1)
    U = s.init_state(P).requires_grad_(True)
    dt = torch.full((1,), 2e-3, dtype=torch.float64, device="cuda")
    f = lambda u: RK3Step.apply(u, None, s, dt)  # noqa: E731
    assert torch.autograd.gradcheck(f, (U,), eps=1e-7, atol=1e-6, rtol=1e-5)


def test_rk3step_matches_oracle_adjoint_incl_K():
    case, P, K = _tiny_porous()
    o = Oracle(case, K=K)
    s = Solver(case, K=K, mode=1)
    U0 = o.cons(P)
    dt = 1e-3
    rng = np.random.default_rng(3)
    lam = rng.normal(size=U0.shape)
    lu_or, lk_or = o.vjp_step(U0, lam, dt)
    U = torch.as_tensor(U0, device="cuda").requires_grad_(True)
    Kt = torch.as_tensor(K, device="cuda").requires_grad_(True)
    out = RK3Step.apply(U, Kt, s, torch.full((1,), dt, dtype=torch.float64, device="cuda"))
    (out * torch.as_tensor(lam, device="cuda")).sum().backward()
    gu = U.grad.cpu().numpy()
    gk = Kt.grad.cpu().numpy()
    assert np.abs(gu - lu_or).max() <= 1e-10 * np.abs(lu_or).max()
    assert np.abs(gk - lk_or).max() <= 1e-10 * np.abs(lk_or).max()


def test_trajectory_cost_matches_gradient_and_optimises():
    case, P, K = W.porous_bl(nx=64, ny=32, strip=(16, 48), nsteps=40)
    s = Solver(case, K=K, mode=2, nsteps=40, seg_len=7)
    U0 = s.init_state(P)
    dt = torch.full((1,), 0.5 * s.compute_dt(U0, cfl=1.0).item(), dtype=torch.float64,
                    device="cuda")
    J_ref, gK_ref, gU_ref = s.gradient(U0, dt)
    Kt = torch.as_tensor(K, device="cuda").requires_grad_(True)
    U = U0.clone().requires_grad_(True)
    J = TrajectoryCost.apply(U, Kt, s, dt)
    J.backward()
    assert torch.equal(J, J_ref)
    assert torch.equal(Kt.grad, gK_ref) and torch.equal(U.grad, gU_ref)
    hist = optimize_porous(s, U0, dt, K, iters=6, lr=0.05)
    Js = [h[0] for h in hist]
    print("[optimise] J history", Js, flush=True)
    assert Js[-1] < Js[0]
