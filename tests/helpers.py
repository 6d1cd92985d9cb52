"""Shared test helpers: build the oracle and the GPU solver from one Case and
compare their outputs with the tolerances of the parity contract."""
import numpy as np

from paper_2406_19494_amd import workloads as W


def flux_scale(case, U):
    """Per-variable guard scale s_v = max|U_v| * max(|u| + c) / dx_min, so that
    a right-hand side that is ~0 is compared against the size of the fluxes."""
    from oracle.pyoracle import Oracle
    o = Oracle(case)
    dxmin = min(o.grid(d)[1].min() for d in range(case.ndim))
    rho = U[0]
    nd = case.ndim
    vel = [U[1 + d] / rho for d in range(nd)]
    ke = 0.5 * rho * sum(v * v for v in vel)
    p = (case.gamma - 1.0) * (U[nd + 1] - ke)
    c = np.sqrt(np.abs(case.gamma * p / rho))
    smax = (max(np.abs(v).max() for v in vel) + c.max())
    return np.abs(U).max(axis=(1, 2, 3)) * smax / dxmin


def rel_err_per_var(a, b, scale):
    """max_cells |a_v - b_v| / max(max|b_v|, scale_v) per variable."""
    diff = np.abs(a - b).max(axis=(1, 2, 3))
    ref = np.maximum(np.abs(b).max(axis=(1, 2, 3)), scale)
    return diff / ref


def small_cases():
    """Small configurations covering every axis count, boundary kind, grid
    map, viscosity law and the source term, with ragged sizes."""
    cases = []
    # 1D Sod (zero-gradient), 200 cells
    c, P = W.sod(200)
    cases.append(("sod1d", c, P, None))
    # 1D periodic viscous, rough data, odd size
    c = W.Case(name="p1d", ndim=1, n=(37, 1, 1), lo=(0, 0, 0), hi=(2, 1, 1), gamma=1.4, R=1.3,
               Pr=0.7, visc_law="power", mu_ref=0.01, T_ref=1.0, visc_param=0.7,
               bc=("periodic",) * 6)
    cases.append(("periodic1d_visc", c, W.random_rough(c, seed=3), None))
    # 2D walls + stretched, viscous Sutherland
    c = W.Case(name="w2d", ndim=2, n=(23, 19, 1), lo=(0, -1, 0), hi=(1.5, 1, 1),
               stretch=("uniform", "tanh2", "uniform"), beta=(0, 1.8, 0), gamma=1.4, R=1.0,
               Pr=0.72, visc_law="sutherland", mu_ref=0.02, T_ref=1.0, visc_param=0.4,
               bc=("periodic", "periodic", "wall", "wall", "periodic", "periodic"),
               T_wall=(0, 0, 1.2, 0.9, 0, 0))
    cases.append(("wall2d_visc", c, W.random_smooth(c, seed=4, amp=0.2), None))
    # 2D porous boundary layer (Dirichlet in, zero-gradient out/top, porous wall)
    c, P, K = W.porous_bl(nx=40, ny=24, strip=(10, 30), nsteps=1)
    cases.append(("porous_bl2d", c, P, K + 0.05))
    # 2D Mach-2.25 laminar boundary layer: adiabatic disturbance wall
    # (v = A sin(2 pi kappa x)), Dirichlet similarity inflow, zero-gradient
    c, P = W.laminar_bl(nx=36, ny=20, amp=0.01, kappa=10.0)
    cases.append(("disturb_bl2d", c, P, None))
    # 2D box closed by adiabatic walls, stretched both ways, rough data
    c = W.Case(name="adi2d", ndim=2, n=(17, 21, 1), lo=(0, 0, 0), hi=(1, 1.3, 1),
               stretch=("tanh2", "tanh1", "uniform"), beta=(1.2, 1.6, 0), gamma=1.4, R=1.0,
               Pr=0.72, visc_law="power", mu_ref=0.01, T_ref=1.0, visc_param=0.76,
               bc=("wall",) * 4 + ("periodic",) * 2, T_wall=(0.0,) * 6)
    cases.append(("adiabatic2d_rough", c, W.random_rough(c, seed=13, rho=(0.8, 1.2),
                                                         vel=(-0.3, 0.3), p=(0.8, 1.2)), None))
    # 3D TGV 16^3 viscous
    c, P = W.tgv(16)
    cases.append(("tgv3d", c, P, None))
    # 3D channel with walls, stretching and the mass-flux source, ragged sizes
    c, P = W.channel(nx=20, ny=18, nz=11)
    cases.append(("channel3d", c, P, None))
    # 3D mixed: zero-gradient x, walls y, periodic z, inviscid rough data
    c = W.Case(name="mix3d", ndim=3, n=(13, 9, 7), lo=(0, 0, 0), hi=(1, 1, 1),
               stretch=("tanh1", "uniform", "uniform"), beta=(1.5, 0, 0), gamma=1.4, R=1.0,
               visc_law="none", bc=("zerograd", "zerograd", "wall", "wall", "periodic", "periodic"),
               T_wall=(0, 0, 1.0, 1.0, 0, 0))
    # cell-wise random data with T in [0.67, 1.5]: the mirror 2 T_w - T stays
    # positive and the reconstructed states stay physical
    cases.append(("mixed3d_rough", c, W.random_rough(c, seed=9, rho=(0.8, 1.2), vel=(-0.3, 0.3),
                                                     p=(0.8, 1.2)), None))
    return cases
