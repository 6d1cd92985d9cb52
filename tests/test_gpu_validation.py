"""Physics validation on the GPU path (Section 3.2): the Mach-2.25 laminar
boundary layer over an adiabatic wall against the compressible similarity
solution, and the disturbance wall of Eq. (8) driving the same layer."""
import math

import numpy as np
import pytest

from paper_2406_19494_amd import workloads as W
from paper_2406_19494_amd.solver import Solver

pytestmark = pytest.mark.gpu


def _advance(s, U, t_end, dt, chunk=5000):
    n = int(math.ceil(t_end / dt))
    done = 0
    while done < n:
        k = min(chunk, n - done)
        s.run(U, k, dt_fixed=dt)
        done += k
        assert s.flags() == 0, f"non-physical state after {done} steps"
        print(f"  {done}/{n} steps", flush=True)
    return n


def _outlet_profiles(case, U):
    """u/u_e, T/T_e and eta = int_0^y rho dy / sqrt(2 mu_e x / (rho_e u_e))
    at the last cell column (free stream rho = u = T = 1)."""
    from oracle.pyoracle import Oracle
    o = Oracle(case)
    xf, _, _, _ = o.grid(0)
    dy = o.grid(1)[1]
    x = 0.5 * (xf[-2] + xf[-1])
    rho = U[0, 0, :, -1]
    u = U[1, 0, :, -1] / rho
    v = U[2, 0, :, -1] / rho
    p = (case.gamma - 1.0) * (U[3, 0, :, -1] - 0.5 * rho * (u * u + v * v))
    T = p / (rho * case.R)
    m = rho * dy
    eta = (np.cumsum(m) - 0.5 * m) / math.sqrt(2.0 * case.mu_ref * x)
    return eta, u, T


def test_mach225_laminar_bl_matches_similarity_solution():
    case, P = W.laminar_bl()
    print(f"[validation] laminar BL {case.n[:2]}", flush=True)
    s = Solver(case)
    U = s.init_state(P)
    dt = float(s.compute_dt(U).item())
    _advance(s, U, 1.0, dt)  # two free-stream flow-through times
    eta, u, T = _outlet_profiles(case, U.cpu().numpy())
    e, f, fp, g = W.similarity_profile(2.25, case.Pr, case.gamma, None, case.visc_param)
    inside = eta < 8.0
    du = np.abs(u - np.interp(eta, e, fp))[inside].max()
    dT = np.abs(T - np.interp(eta, e, g))[inside].max()
    print(f"  max |u/u_e - f'| = {du:.3e}, max |T/T_e - g| = {dT:.3e}, "
          f"T_wall/T_e = {T[0]:.4f} (similarity {g[0]:.4f})", flush=True)
    assert du < 0.02
    assert dT < 0.02 * g[0]


def test_disturbance_wall_drives_the_boundary_layer():
    # A = 0.01, kappa = 10 (the paper's values): the run stays physical and
    # the disturbance leaves a wall-normal velocity field periodic in x with
    # the imposed wavenumber near the wall.
    case, P = W.laminar_bl(amp=0.01, kappa=10.0)
    print(f"[validation] disturbance wall {case.n[:2]}", flush=True)
    s = Solver(case)
    U = s.init_state(P)
    dt = float(s.compute_dt(U).item())
    _advance(s, U, 0.1, 0.8 * dt)
    Uh = U.cpu().numpy()
    v = Uh[2, 0, 0, :] / Uh[0, 0, 0, :]
    from oracle.pyoracle import Oracle
    xf = Oracle(case).grid(0)[0]
    xc = 0.5 * (xf[:-1] + xf[1:])
    ref = np.sin(2 * np.pi * 10.0 * xc)
    corr = np.dot(v - v.mean(), ref) / (np.linalg.norm(v - v.mean()) * np.linalg.norm(ref))
    print(f"  corr(v_wall_row, sin(2 pi kappa x)) = {corr:.4f}", flush=True)
    assert corr > 0.9
