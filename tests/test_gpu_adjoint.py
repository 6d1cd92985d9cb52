"""GPU adjoint parity: the hand-written VJP of one RK3 step and the
checkpointed trajectory gradient against the oracle's dense-Jacobian adjoint,
its forward-mode JVP (dot-product test) and finite differences."""
import numpy as np
import pytest
import torch

from oracle.pyoracle import Oracle
from paper_2406_19494_amd import workloads as W
from paper_2406_19494_amd.solver import Solver, workspace_bytes_for
from tests.test_oracle_pins import _tiny_disturb, _tiny_porous

pytestmark = pytest.mark.gpu

VJP_TOL = 1e-10


def adjoint_cases():
    out = []
    c, P = W.sod(24)
    out.append(("sod1d", c, P, None, 2e-3))
    c = W.Case(name="p1d", ndim=1, n=(16, 1, 1), lo=(0, 0, 0), hi=(2, 1, 1), gamma=1.4, R=1.3,
               Pr=0.7, visc_law="power", mu_ref=0.01, T_ref=1.0, visc_param=0.7,
               bc=("periodic",) * 6)
    out.append(("periodic1d_visc", c, W.random_smooth(c, seed=3, amp=0.2), None, 1e-3))
    c = W.Case(name="w2d", ndim=2, n=(10, 9, 1), lo=(0, -1, 0), hi=(1.5, 1, 1),
               stretch=("uniform", "tanh2", "uniform"), beta=(0, 1.8, 0), gamma=1.4, R=1.0,
               Pr=0.72, visc_law="sutherland", mu_ref=0.02, T_ref=1.0, visc_param=0.4,
               bc=("periodic", "periodic", "wall", "wall", "periodic", "periodic"),
               T_wall=(0, 0, 1.2, 0.9, 0, 0))
    out.append(("wall2d_visc", c, W.random_smooth(c, seed=4, amp=0.2), None, 5e-4))
    case, P, K = _tiny_porous()
    out.append(("porous_bl2d", case, P, K, 1e-3))
    c, P = W.tgv(6)
    out.append(("tgv3d", c, P, None, 1e-2))
    c = W.Case(name="mix3d", ndim=3, n=(7, 6, 5), lo=(0, 0, 0), hi=(1, 1, 1),
               stretch=("tanh1", "uniform", "uniform"), beta=(1.5, 0, 0), gamma=1.4, R=1.0,
               Pr=0.7, visc_law="power", mu_ref=0.005, T_ref=1.0, visc_param=0.7,
               bc=("zerograd", "zerograd", "wall", "wall", "periodic", "periodic"),
               T_wall=(0, 0, 1.0, 1.0, 0, 0))
    out.append(("mixed3d_visc", c, W.random_smooth(c, seed=9, amp=0.2), None, 1e-3))
    c, P = W.laminar_bl(nx=12, ny=8, amp=0.01, kappa=10.0)
    out.append(("disturb_bl2d", c, P, None, 2e-4))
    # Dirichlet faces on two axes next to an isothermal and an adiabatic wall:
    # box edges whose ghost adjoints are discarded
    c = W.Case(name="dir3d", ndim=3, n=(6, 5, 5), lo=(0, 0, 0), hi=(1, 1, 1),
               stretch=("uniform", "tanh2", "uniform"), beta=(0, 1.5, 0), gamma=1.4, R=1.0,
               Pr=0.7, visc_law="power", mu_ref=0.01, T_ref=1.0, visc_param=0.7,
               bc=("dirichlet", "zerograd", "wall", "wall", "dirichlet", "zerograd"),
               T_wall=(0, 0, 1.0, 0.0, 0, 0))
    P = W.random_smooth(c, seed=21, amp=0.2)
    c.dirichlet = {0: np.ascontiguousarray(P[:, :, :, 0]) * 1.01,
                   4: np.ascontiguousarray(P[:, 0, :, :]) * 0.99}
    out.append(("dirichlet3d_visc", c, P, None, 1e-3))
    # the constant-mass-flux body force: a 3D channel (periodic last axis:
    # the fused step, force from the x and y boundary fluxes) and a 2D one
    # (walls on the last axis: the unfused step)
    out.append(("channel_force3d", *_channel3d(), None, 2e-3))
    out.append(("channel_force2d", *_channel2d(), None, 2e-3))
    return out


def _channel3d():
    """8 x 8 x 6 body-forced channel with a seeded 10 % pressure
    perturbation.  (The channel's initial state has T = T_w everywhere, so
    the isothermal wall ghost is the exact mirror image of its source and the
    HLLC contact speed at the wall faces is zero to rounding: its branch, and
    with it the linearisation, is then decided by rounding noise, differently
    in any two implementations.  With T != T_w at the walls it is not.)"""
    c, P = W.channel(nx=8, ny=8, nz=6)
    x, y, z = W._mesh(c)
    P = P.copy()
    P[4] = P[4] * (1.0 + 0.1 * np.sin(2 * np.pi * x / 6.0) * np.cos(2.0 * y + 0.3) *
                   np.cos(2 * np.pi * z / 4.0))
    return c, P


def _channel2d():
    """12 x 10 plane channel with the constant-mass-flux body force (walls
    along y, periodic along x), a seeded perturbation on the Poiseuille
    profile."""
    c = W.Case(name="channel2d", ndim=2, n=(12, 10, 1), lo=(0.0, -1.0, 0.0), hi=(3.0, 1.0, 1.0),
               stretch=("uniform", "tanh2", "uniform"), beta=(0.0, 1.5, 0.0), gamma=1.4,
               R=1.0 / 1.4 * 4.0, Pr=0.72, visc_law="power", mu_ref=1.0 / 300.0, T_ref=1.0,
               visc_param=0.7, bc=("periodic", "periodic", "wall", "wall", "periodic", "periodic"),
               T_wall=(0.0, 0.0, 1.0, 1.0, 0.0, 0.0), source="massflux")
    x, y, _ = W._mesh(c)
    P = W.random_smooth(c, seed=5, amp=0.1, p0=c.R)
    P[1] = P[1] + 1.5 * (1.0 - y * y)
    return c, P


CASES = adjoint_cases()


@pytest.mark.parametrize("name,case,P,K,dt", CASES, ids=[c[0] for c in CASES])
def test_vjp_step_matches_dense_oracle_adjoint(name, case, P, K, dt):
    print(f"[vjp parity] {name} n={case.n}", flush=True)
    o = Oracle(case, K=K)
    s = Solver(case, K=K, mode=1)
    U = o.cons(P)
    rng = np.random.default_rng(11)
    lam = rng.normal(size=U.shape)
    lu_or, lk_or = o.vjp_step(U, lam, dt)
    Ug = torch.as_tensor(U, device="cuda")
    dtg = torch.full((1,), dt, dtype=torch.float64, device="cuda")
    gK = torch.zeros(max(s.nk, 1), dtype=torch.float64, device="cuda")
    lu = s.vjp_step(Ug, dtg, torch.as_tensor(lam, device="cuda"),
                    dJdK=gK if s.nk else None).cpu().numpy()
    scale = np.abs(lu_or).max(axis=(1, 2, 3))
    err = np.abs(lu - lu_or).max(axis=(1, 2, 3)) / scale
    assert np.all(err <= VJP_TOL), (name, err)
    if s.nk:
        gk = gK.cpu().numpy()[: s.nk]
        assert np.abs(gk - lk_or).max() <= VJP_TOL * np.abs(lk_or).max(), (gk, lk_or)


@pytest.mark.parametrize("name,case,P,K,dt", CASES, ids=[c[0] for c in CASES])
def test_repeated_vjp_steps_are_bitwise_identical(name, case, P, K, dt):
    # the adjoint boxes are not cleared between stages or calls: every cell a
    # stage reads is either set afresh by it or kept at zero, so a call after
    # one with another adjoint and state gives the first call's result bit for
    # bit
    print(f"[vjp repeat] {name} n={case.n}", flush=True)
    o = Oracle(case, K=K)
    s = Solver(case, K=K, mode=1)
    U = torch.as_tensor(o.cons(P), device="cuda")
    rng = np.random.default_rng(13)
    lam1 = torch.as_tensor(rng.normal(size=tuple(U.shape)), device="cuda")
    lam2 = torch.as_tensor(rng.normal(size=tuple(U.shape)) * 1e3, device="cuda")
    dtg = torch.full((1,), dt, dtype=torch.float64, device="cuda")
    out = []
    for k, lam in enumerate((lam1, lam2, lam1)):
        gK = torch.zeros(max(s.nk, 1), dtype=torch.float64, device="cuda")
        Uk = U if k != 1 else U * (1.0 + 1e-3 * torch.cos(torch.arange(U.numel(), device="cuda")
                                                          .reshape(U.shape).double()))
        out.append((s.vjp_step(Uk, dtg, lam, dJdK=gK if s.nk else None), gK))
    assert torch.equal(out[0][0], out[2][0]), name
    assert torch.equal(out[0][1], out[2][1]), name


@pytest.mark.parametrize("name,case,P,K,dt", CASES, ids=[c[0] for c in CASES])
def test_vjp_with_kept_stage_states_equals_recompute(name, case, P, K, dt):
    # dcf_rk3_step_keep advances U exactly as dcf_rk3_step and hands its
    # stage states to dcf_vjp_step, which then skips their recompute: the
    # same lam_n and dJ/dK bit for bit
    o = Oracle(case, K=K)
    s = Solver(case, K=K, mode=1)
    U = torch.as_tensor(o.cons(P), device="cuda")
    dtg = torch.full((1,), dt, dtype=torch.float64, device="cuda")
    rng = np.random.default_rng(17)
    lam = torch.as_tensor(rng.normal(size=tuple(U.shape)), device="cuda")
    U_a, U_b = U.clone(), U.clone()
    stages = torch.empty((2,) + tuple(U.shape), dtype=torch.float64, device="cuda")
    s.step(U_a, dtg)
    s.step_keep(U_b, dtg, stages)
    assert torch.equal(U_a, U_b), name
    gk = [torch.zeros(max(s.nk, 1), dtype=torch.float64, device="cuda") for _ in range(2)]
    l0 = s.vjp_step(U, dtg, lam, dJdK=gk[0] if s.nk else None)
    l1 = s.vjp_step(U, dtg, lam, dJdK=gk[1] if s.nk else None, stages=stages)
    assert torch.equal(l0, l1), name
    assert torch.equal(gk[0], gk[1]), name


@pytest.mark.parametrize("name,case,P,K,dt", CASES[3:4], ids=[CASES[3][0]])
def test_dot_product_gpu_vjp_vs_oracle_jvp(name, case, P, K, dt):
    o = Oracle(case, K=K)
    s = Solver(case, K=K, mode=1)
    U = o.cons(P)
    rng = np.random.default_rng(12)
    v = rng.normal(size=U.shape) * np.abs(U).max(axis=(1, 2, 3), keepdims=True)
    vk = rng.normal(size=o.nk)
    lam = rng.normal(size=U.shape)
    _, jv = o.jvp_step(U, v, dt, vk)
    gK = torch.zeros(s.nk, dtype=torch.float64, device="cuda")
    lu = s.vjp_step(torch.as_tensor(U, device="cuda"),
                    torch.full((1,), dt, dtype=torch.float64, device="cuda"),
                    torch.as_tensor(lam, device="cuda"), dJdK=gK).cpu().numpy()
    lhs = np.sum(lam * jv)
    rhs = np.sum(lu * v) + np.sum(gK.cpu().numpy() * vk)
    assert abs(lhs - rhs) <= 1e-10 * max(abs(lhs), np.sum(np.abs(lam * jv))), (lhs, rhs)


@pytest.mark.parametrize("which", ["porous", "disturb"])
def test_cached_stage_boxes_give_the_same_gradient_bitwise(which):
    case, P, K = _tiny_porous() if which == "porous" else _tiny_disturb()
    o = Oracle(case, K=K)
    U0 = torch.as_tensor(o.cons(P), device="cuda")
    dt = torch.full((1,), 1e-3 if which == "porous" else 2e-4, dtype=torch.float64, device="cuda")
    out = []
    for mode in (2, 3):
        s = Solver(case, K=K, mode=mode, nsteps=7, seg_len=3)
        out.append(s.gradient(U0, dt))
    for a, b in zip(out[0], out[1]):
        assert torch.equal(a, b)


def test_gradient_shorter_than_its_workspace_is_bitwise_the_same():
    # a workspace sized for 9 steps (checkpoints every 3) serves a 7-step
    # gradient exactly as one sized for 7
    case, P, K = _tiny_porous()
    U0 = torch.as_tensor(Oracle(case, K=K).cons(P), device="cuda")
    dt = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
    exact = Solver(case, K=K, mode=2, nsteps=7, seg_len=3).gradient(U0, dt)
    big = Solver(case, K=K, mode=2, nsteps=9, seg_len=3)
    J = torch.zeros(1, dtype=torch.float64, device="cuda")
    gK = torch.zeros(big.nk, dtype=torch.float64, device="cuda")
    gU = torch.empty_like(U0)
    big.gradient_begin(U0, dt, J, gK, nsteps=7)
    while not big.gradient_advance(1 << 20):
        pass
    big.gradient_finish(gU)
    for a, b in zip(exact, (J, gK, gU)):
        assert torch.equal(a, b)


def test_budgeted_segment_length_gives_the_same_gradient():
    # seg_len = 0 picks the spacing from a workspace budget: with room for the
    # whole trajectory one segment (no recompute), with less a shorter one;
    # the gradient is the same up to summation order either way
    case, P, K = _tiny_porous()
    U0 = torch.as_tensor(Oracle(case, K=K).cons(P), device="cuda")
    dt = torch.full((1,), 1e-3, dtype=torch.float64, device="cuda")
    ref = Solver(case, K=K, mode=2, nsteps=12, seg_len=4).gradient(U0, dt)
    whole = Solver(case, K=K, mode=2, nsteps=12, seg_len=0)
    assert whole.seg_len == 12
    tight_budget = workspace_bytes_for(case, 2, 12, 6)
    tight = Solver(case, K=K, mode=2, nsteps=12, seg_len=0, seg_budget=tight_budget)
    assert tight.seg_len == 6
    for s in (whole, tight):
        out = s.gradient(U0, dt)
        for a, b in zip(ref, out):
            assert torch.allclose(a, b, rtol=1e-12, atol=1e-14 * float(b.abs().max()))


@pytest.mark.parametrize("which", ["porous", "disturb", "channel"])
def test_trajectory_gradient_matches_oracle(which):
    if which == "channel":  # wall-pressure cost through the body-forced channel
        case, P = _channel3d()
        case.cost_face = 2
        K = None
    else:
        case, P, K = _tiny_porous() if which == "porous" else _tiny_disturb()
    print(f"[trajectory gradient] {which}", flush=True)
    o = Oracle(case, K=K)
    U0 = o.cons(P)
    dt, nsteps = {"porous": (1e-3, 5), "disturb": (2e-4, 5), "channel": (2e-3, 5)}[which]
    J_or, gk_or, gu_or = o.gradient(U0, nsteps, dt)
    for seg in (2, 5):
        s = Solver(case, K=K, mode=2, nsteps=nsteps, seg_len=seg)
        J, gk, gu = s.gradient(torch.as_tensor(U0, device="cuda"),
                               torch.full((1,), dt, dtype=torch.float64, device="cuda"))
        assert abs(J.item() - J_or) <= 1e-12 * abs(J_or)
        if s.nk:
            gk = gk.cpu().numpy()
            assert np.abs(gk - gk_or).max() <= VJP_TOL * np.abs(gk_or).max(), (seg, gk, gk_or)
        gu = gu.cpu().numpy()
        err = np.abs(gu - gu_or).max(axis=(1, 2, 3)) / np.abs(gu_or).max(axis=(1, 2, 3))
        assert np.all(err <= VJP_TOL), (seg, err)


def test_gradient_matches_gpu_finite_differences_full_bl():
    """Mach-6 porous boundary layer at full size (1024 x 256), 2000-step
    checkpointed trajectory; dJ/dK_i against central differences of the GPU
    forward on 8 seeded K_i."""
    case, P, K = W.porous_bl()
    s0 = Solver(case, K=K)
    U0 = s0.init_state(P)
    dt = 0.5 * s0.compute_dt(U0, cfl=1.0).item()
    nsteps, seg = 2000, 45
    dtg = torch.full((1,), dt, dtype=torch.float64, device="cuda")
    s = Solver(case, K=K, mode=2, nsteps=nsteps, seg_len=seg)
    J, gk, _ = s.gradient(U0, dtg)
    gk = gk.cpu().numpy()
    print(f"[bl gradient] J={J.item():.6e} |g|max={np.abs(gk).max():.3e} dt={dt:.3e}", flush=True)

    def J_of(Kp):
        sf = Solver(case, K=Kp, mode=0)
        U = U0.clone()
        Jt = torch.zeros(1, dtype=torch.float64, device="cuda")
        for _ in range(nsteps):
            sf.step(U, dtg)
            sf.cost_term(U, w=1.0 / nsteps, J=Jt)
        return Jt.item()

    assert abs(J_of(K) - J.item()) <= 1e-13 * abs(J.item())
    # Per entry, fourth-order central differences
    # (-J(+2h) + 8 J(+h) - 8 J(-h) + J(-2h)) / (12 h) with h = 1e-3: the
    # truncation, O(h^4), is far below 1e-6 of every checked entry, and J's
    # round-off (~1e-22 absolute) stays below it too.  The step is kept small
    # because J(K) is only piecewise smooth: HLLC selects its star state by
    # the sign of S*, which is near zero at some wall faces, so a larger
    # perturbation can cross a branch change and leave an O(h) error (seen at
    # h = 4e-3 on one entry).  The wall-pressure pulse (2 % of p_inf) makes
    # J ~ 6e-9.  The seeded K_i are drawn among the strip faces under the
    # pulse (within one radius of its centre): over 2000 steps (t ~ 3e-3) the
    # disturbance travels little, and coefficients towards its edge change J
    # by 1e-4 .. 1e-8 of the largest entry, where the round-off of J
    # (~1e-15 relative) is no longer below 1e-6 of the entry.  Each entry is
    # held to 1e-6 relative to itself.
    xc = case.lo[0] + (case.porous_begin + np.arange(case.nk) + 0.5) * (
        (case.hi[0] - case.lo[0]) / case.n[0])
    near = np.flatnonzero(np.abs(xc - 0.5 * (case.lo[0] + case.hi[0])) < 0.02)
    rng = np.random.default_rng(5)
    idx = rng.choice(near, size=8, replace=False)
    for i in idx:
        h = 1e-3
        Jv = {}
        for mlt in (-2, -1, 1, 2):
            e = np.zeros_like(K)
            e[i] = mlt * h
            Jv[mlt] = J_of(K + e)
        fd = (-Jv[2] + 8 * Jv[1] - 8 * Jv[-1] + Jv[-2]) / (12 * h)
        rel = abs(fd - gk[i]) / max(abs(fd), abs(gk[i]))
        print(f"[bl fd] i={i} K={K[i]:.4f} fd={fd:.12e} adj={gk[i]:.12e} rel={rel:.2e}",
              flush=True)
        assert rel <= 1e-6, (i, fd, gk[i], rel)
