"""Seeded synthetic workloads: case parameters and initial primitive fields.

This module is the only code that the GPU library's tests and the CPU oracle
have in common.  It holds case *descriptions* (grid sizes, gas constants,
boundary kinds) and the initial primitive fields (rho, u, v, w, p) sampled at
cell centres; it holds none of the solver's arithmetic (no conversion to
conserved variables, no fluxes, no boundary ghost values).

The workloads are the paper's problem shapes:

* ``sod``       -- 1D shock tube, gamma = 1.4, 200 uniform cells on [0, 1];
* ``tgv``       -- 3D Taylor-Green vortex on the periodic 2*pi box, Re = 1600,
                   Ma = 0.1, Pr = 0.71, power-law viscosity;
* ``channel``   -- compressible channel (Section 3.1 of the paper gives the
                   flow: isothermal walls, Ma_b defined with the wall sound
                   speed, Re_b with the wall viscosity): 192 x 128 x 128 cells
                   on 4*pi x 2 x 4*pi/3, tanh wall-normal stretching beta = 2,
                   Ma_b = 0.5, Re_b = 3000, Poiseuille profile plus seeded 5 %
                   uniform velocity perturbations;
* ``porous_bl`` -- 2D Mach-6 laminar boundary layer over a stretched grid with
                   a porous wall strip (Section 3.2: a boundary layer over a
                   wall whose normal velocity is a differentiable function of
                   solver-level parameters); compressible similarity inflow.

Random numbers come from SplitMix64 (Steele, Lea & Flood, OOPSLA 2014) keyed
by (seed, cell, component) so that every consumer sees the same inputs.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional, Sequence, Tuple

import numpy as np

BC_KINDS = ("periodic", "wall", "porous", "zerograd", "dirichlet", "disturb")
VISC_LAWS = ("none", "power", "sutherland")
STRETCH = ("uniform", "tanh2", "tanh1")
SOURCES = ("none", "massflux")


@dataclasses.dataclass
class Case:
    """Parameters of one solve.  Faces are ordered x-, x+, y-, y+, z-, z+."""

    name: str
    ndim: int
    n: Tuple[int, int, int]
    lo: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    hi: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    stretch: Tuple[str, str, str] = ("uniform", "uniform", "uniform")
    beta: Tuple[float, float, float] = (0.0, 0.0, 0.0)
    gamma: float = 1.4
    R: float = 1.0
    Pr: float = 0.72
    visc_law: str = "none"
    mu_ref: float = 0.0
    T_ref: float = 1.0
    visc_param: float = 0.0
    bc: Tuple[str, ...] = ("periodic",) * 6
    T_wall: Tuple[float, ...] = (0.0,) * 6        # 0 on a wall face: adiabatic
    dist_amp: Tuple[float, ...] = (0.0,) * 6      # disturbance wall amplitude
    dist_kappa: Tuple[float, ...] = (0.0,) * 6    # disturbance wall wavenumber
    dirichlet: Dict[int, np.ndarray] = dataclasses.field(default_factory=dict)
    porous_face: int = -1
    porous_begin: int = 0
    porous_end: int = 0
    p_inf: float = 1.0
    source: str = "none"
    cost_face: int = -1
    # spatial scheme: "weno5" (WENO5-JS + 4th-order central dissipative
    # fluxes) or "teno6a" (TENO6-A with the interpolation limiter + 6th-order
    # central dissipative fluxes, the channel scheme of Section 3.1)
    scheme: str = "weno5"
    # run parameters
    cfl: float = 0.5
    dt_fixed: float = 0.0
    t_end: float = 0.0
    nsteps: int = 0

    @property
    def ncells(self) -> int:
        return self.n[0] * self.n[1] * self.n[2]

    @property
    def nv(self) -> int:
        return self.ndim + 2

    @property
    def n_porous(self) -> int:
        """Porous coefficients K_i (strip index fastest)."""
        if self.porous_face < 0:
            return 0
        d = self.porous_face // 2
        t2 = 1 if d == 2 else 2
        return (self.porous_end - self.porous_begin) * self.n[t2]

    @property
    def disturb_faces(self) -> Tuple[int, ...]:
        return tuple(f for f in range(2 * self.ndim) if self.bc[f] == "disturb")

    @property
    def nk(self) -> int:
        """Length of the boundary-parameter vector theta: the porous
        coefficients, then (A, kappa) of each disturbance face in face order."""
        return self.n_porous + 2 * len(self.disturb_faces)

    def theta(self, K=None) -> np.ndarray:
        """The boundary-parameter vector.  K may be the full vector (length
        nk), the porous coefficients alone (the disturbance amplitudes and
        wavenumbers are then this case's), or None (porous coefficients 0)."""
        if K is not None and np.size(K) == self.nk and self.nk:
            return np.asarray(K, dtype=np.float64).reshape(-1).copy()
        Kp = np.zeros(self.n_porous) if K is None else np.asarray(K, dtype=np.float64).reshape(-1)
        if Kp.size != self.n_porous:
            raise ValueError(f"expected {self.n_porous} porous coefficients or {self.nk} "
                             f"boundary parameters, got {Kp.size}")
        extra = [v for f in self.disturb_faces for v in (self.dist_amp[f], self.dist_kappa[f])]
        return np.concatenate([Kp, np.asarray(extra, dtype=np.float64)])


# --------------------------------------------------------------------------
# Seeded random numbers: SplitMix64 keyed by (seed, cell, component).
# --------------------------------------------------------------------------
_M64 = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output function applied to uint64 keys (vectorised)."""
    with np.errstate(over="ignore"):
        z = (x + np.uint64(0x9E3779B97F4A7C15)) & np.uint64(_M64)
        z = ((z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)) & np.uint64(_M64)
        z = ((z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)) & np.uint64(_M64)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, component: int) -> np.ndarray:
    """`count` uniform doubles in [0, 1) for one component, keyed by cell index."""
    cell = np.arange(count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        key = (np.uint64(seed) * np.uint64(0x100000001B3)) ^ (cell * np.uint64(8) + np.uint64(component))
    bits = splitmix64(key) >> np.uint64(11)
    return bits.astype(np.float64) * (1.0 / float(1 << 53))


# --------------------------------------------------------------------------
# Sampling points.  Initial fields are point values at cell centres.  The
# centre of cell i sits at computational coordinate xi = i + 1/2 of the axis
# map used by the case (uniform, two-sided tanh, one-sided tanh).
# --------------------------------------------------------------------------
def sample_points(kind: str, lo: float, hi: float, beta: float, n: int) -> np.ndarray:
    s = (np.arange(n, dtype=np.float64) + 0.5) / n
    L = hi - lo
    if kind == "tanh2":
        return lo + L * 0.5 * (1.0 - np.tanh(beta * (1.0 - 2.0 * s)) / math.tanh(beta))
    if kind == "tanh1":
        return lo + L * (1.0 + np.tanh(beta * (s - 1.0)) / math.tanh(beta))
    return lo + L * s


def _mesh(case: Case):
    ax = [sample_points(case.stretch[d], case.lo[d], case.hi[d], case.beta[d], case.n[d])
          for d in range(3)]
    z, y, x = np.meshgrid(ax[2], ax[1], ax[0], indexing="ij")
    return x, y, z


def _prim(nx, ny, nz):
    return np.zeros((5, nz, ny, nx), dtype=np.float64)


# --------------------------------------------------------------------------
# Sod shock tube (1D; optionally embedded along any axis of a 3D box).
# --------------------------------------------------------------------------
def sod(n: int = 200, axis: int = 0, ndim: int = 1, cross: int = 4) -> Tuple[Case, np.ndarray]:
    """Left (rho, u, p) = (1, 0, 1), right (0.125, 0, 0.1), interface at x = 0.5."""
    shape = [1, 1, 1]
    if ndim == 1:
        shape[0] = n
    else:
        for d in range(ndim):
            shape[d] = cross
        shape[axis] = n
    bc = ["periodic"] * 6
    bc[2 * axis] = bc[2 * axis + 1] = "zerograd"
    case = Case(name="sod", ndim=ndim, n=tuple(shape), lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                gamma=1.4, R=1.0, visc_law="none", bc=tuple(bc), cfl=0.5, t_end=0.2)
    nx, ny, nz = shape
    P = _prim(nx, ny, nz)
    xs = (np.arange(n) + 0.5) / n
    left = xs < 0.5
    rho1 = np.where(left, 1.0, 0.125)
    p1 = np.where(left, 1.0, 0.1)
    bshape = [1, 1, 1]
    bshape[2 - axis] = n
    P[0] = np.broadcast_to(rho1.reshape(bshape), (nz, ny, nx))
    P[4] = np.broadcast_to(p1.reshape(bshape), (nz, ny, nx))
    return case, P


# --------------------------------------------------------------------------
# Taylor-Green vortex.
# --------------------------------------------------------------------------
def tgv(n: int = 64, Re: float = 1600.0, Ma: float = 0.1, Pr: float = 0.71,
        omega: float = 0.7, viscous: bool = True) -> Tuple[Case, np.ndarray]:
    """u = sin x cos y cos z, v = -cos x sin y cos z, w = 0,
    p = p0 + (cos 2x + cos 2y)(cos 2z + 2)/16, T = T0 = 1, rho = p/(R T0),
    with p0 = 1/(gamma Ma^2) and R = p0 so that rho0 = 1."""
    gamma = 1.4
    p0 = 1.0 / (gamma * Ma * Ma)
    L = 2.0 * math.pi
    case = Case(name="tgv", ndim=3, n=(n, n, n), lo=(0.0, 0.0, 0.0), hi=(L, L, L), gamma=gamma,
                R=p0, Pr=Pr, visc_law="power" if viscous else "none",
                mu_ref=1.0 / Re if viscous else 0.0, T_ref=1.0, visc_param=omega,
                bc=("periodic",) * 6, cfl=0.5, nsteps=1000)
    x, y, z = _mesh(case)
    P = _prim(n, n, n)
    p = p0 + (np.cos(2 * x) + np.cos(2 * y)) * (np.cos(2 * z) + 2.0) / 16.0
    P[0] = p / (p0 * 1.0)
    P[1] = np.sin(x) * np.cos(y) * np.cos(z)
    P[2] = -np.cos(x) * np.sin(y) * np.cos(z)
    P[3] = 0.0
    P[4] = p
    return case, P


# --------------------------------------------------------------------------
# Channel: isothermal walls at y = -1, +1, periodic x and z.
# --------------------------------------------------------------------------
def channel(nx: int = 192, ny: int = 128, nz: int = 128, Ma_b: float = 0.5,
            Re_b: float = 3000.0, Pr: float = 0.72, omega: float = 0.7,
            beta: float = 2.0, amp: float = 0.05, seed: int = 2406,
            scheme: str = "weno5") -> Tuple[Case, np.ndarray]:
    """Bulk velocity, bulk density, wall temperature and half-width are 1.
    Ma_b = U_b / c_w gives R = c_w^2 / gamma with c_w = 1/Ma_b; Re_b = 3000
    gives mu_w = 1/Re_b.  u = 1.5 (1 - y^2) plus amp * U_b * (2 r - 1) on all
    three velocity components, rho = 1, T = 1."""
    gamma = 1.4
    cw = 1.0 / Ma_b
    R = cw * cw / gamma
    case = Case(name="channel", ndim=3, n=(nx, ny, nz), lo=(0.0, -1.0, 0.0),
                hi=(4.0 * math.pi, 1.0, 4.0 * math.pi / 3.0),
                stretch=("uniform", "tanh2", "uniform"), beta=(0.0, beta, 0.0), gamma=gamma,
                R=R, Pr=Pr, visc_law="power", mu_ref=1.0 / Re_b, T_ref=1.0, visc_param=omega,
                bc=("periodic", "periodic", "wall", "wall", "periodic", "periodic"),
                T_wall=(0.0, 0.0, 1.0, 1.0, 0.0, 0.0), source="massflux", cfl=0.5, nsteps=500,
                scheme=scheme)
    x, y, z = _mesh(case)
    ncell = nx * ny * nz
    P = _prim(nx, ny, nz)
    P[0] = 1.0
    P[1] = 1.5 * (1.0 - y * y)
    for comp in range(3):
        r = uniform01(seed, ncell, comp).reshape(nz, ny, nx)
        P[1 + comp] += amp * (2.0 * r - 1.0)
    P[4] = 1.0 * R * 1.0
    return case, P


# --------------------------------------------------------------------------
# Mach-6 boundary layer over a porous strip (2D).
# --------------------------------------------------------------------------
def _sutherland_ratio(t, s):
    """mu(T)/mu(T_e) for T = t * T_e with Sutherland constant s = S/T_e."""
    return t ** 1.5 * (1.0 + s) / (t + s)


def similarity_profile(Ma: float, Pr: float, gamma: float, Tw_ratio: float, S_ratio: float,
                       eta_max: float = 12.0, npts: int = 2001):
    """Compressible laminar boundary-layer similarity solution (the Blasius
    problem in the Howarth-Dorodnitsyn variable eta = u_e / sqrt(2 rho_e mu_e
    u_e x) * int_0^y rho dy, paper Section 3.2, Eq. (7)):

        (C f'')' + f f'' = 0,
        (C/Pr g')' + f g' + (gamma - 1) Ma^2 C f''^2 = 0,

    with C = rho mu / (rho_e mu_e) = mu(T)/mu_e / g, g = T/T_e,
    f(0) = f'(0) = 0, g(0) = Tw_ratio (g'(0) = 0 when Tw_ratio is None: an
    adiabatic wall), f'(inf) = 1, g(inf) = 1.
    Returns (eta, f, f', g)."""
    from scipy.integrate import solve_bvp

    def C_of(g):
        return _sutherland_ratio(g, S_ratio) / g

    def rhs(eta, Y):
        f, fp, Cfpp, g, Cgp = Y
        g = np.maximum(g, 1e-6)
        C = C_of(g)
        fpp = Cfpp / C
        gp = Cgp / (C / Pr)
        return np.vstack([fp, fpp, -f * fpp, gp, -f * gp - (gamma - 1.0) * Ma * Ma * C * fpp * fpp])

    def bc(Ya, Yb):
        wall_T = Ya[4] if Tw_ratio is None else Ya[3] - Tw_ratio
        return np.array([Ya[0], Ya[1], wall_T, Yb[1] - 1.0, Yb[3] - 1.0])

    eta = np.linspace(0.0, eta_max, npts)
    fp0 = np.tanh(eta)
    if Tw_ratio is None:  # adiabatic: recovery temperature (factor Pr^(1/2)) as first guess
        g0 = 1.0 + 0.5 * (gamma - 1.0) * Ma * Ma * math.sqrt(Pr)
        gguess = 1.0 + (g0 - 1.0) * (1 - fp0 ** 2)
    else:
        gguess = 1.0 + (Tw_ratio - 1.0) * (1 - fp0)
    Y0 = np.vstack([eta - np.tanh(eta) + np.tanh(eta) * 0.0, fp0, 0.5 * (1 - fp0 ** 2),
                    gguess, np.zeros_like(eta)])
    Y0[0] = np.cumsum(np.r_[0.0, 0.5 * (fp0[1:] + fp0[:-1]) * np.diff(eta)])
    sol = solve_bvp(rhs, bc, eta, Y0, tol=1e-9, max_nodes=200000)
    if not sol.success:
        raise RuntimeError("similarity solution did not converge: " + sol.message)
    Y = sol.sol(eta)
    return eta, Y[0], Y[1], Y[3]


def _similarity_fields(case: Case, Ma: float, Pr: float, Tw_ratio: Optional[float],
                       S_ratio: float, Re_unit: float, p_e: float) -> np.ndarray:
    """Primitive field of the similarity boundary layer at every cell of a 2D
    case (free stream rho = u = T = 1, pressure p_e), with the wall-normal
    velocity from continuity, and the matching Dirichlet inflow profile on
    face x- (stored into case.dirichlet)."""
    nx, ny = case.n[0], case.n[1]
    x0, x1 = case.lo[0], case.hi[0]
    x, y, _ = _mesh(case)
    eta, f, fp, g = similarity_profile(Ma, Pr, case.gamma, Tw_ratio, S_ratio)
    # y(eta) at station x: y = sqrt(2 mu_e x / (rho_e u_e)) * int_0^eta g d eta
    Y_eta = np.concatenate([[0.0], np.cumsum(0.5 * (g[1:] + g[:-1]) * np.diff(eta))])

    def profile(xs, ys):
        scale = np.sqrt(2.0 * (1.0 / Re_unit) * xs)
        yt = ys / scale
        u = np.interp(yt, Y_eta, fp, right=1.0)
        T = np.interp(yt, Y_eta, g, right=1.0)
        return u, T

    u, T = profile(x[0], y[0])
    # wall-normal velocity from continuity: rho v = -int_0^y d(rho u)/dx dy
    hx = 1e-4
    up, Tp = profile(x[0] + hx, y[0])
    um, Tm = profile(x[0] - hx, y[0])
    drhou = (up / Tp - um / Tm) / (2 * hx)
    yy = y[0][:, 0]
    dy = np.diff(np.concatenate([[0.0], yy]))
    rhov = -np.cumsum(drhou * dy[:, None], axis=0)
    rho = 1.0 / T
    P = _prim(nx, ny, 1)
    P[0, 0] = rho
    P[1, 0] = u
    P[2, 0] = rhov / rho
    P[4, 0] = p_e
    # Dirichlet inflow profile at x- : [5][n_t2 = 1][n_t1 = ny]
    uin, Tin = profile(np.full(ny, x0 - 0.5 * (x1 - x0) / nx), yy)
    D = np.zeros((5, 1, ny))
    D[0, 0] = 1.0 / Tin
    D[1, 0] = uin
    D[2, 0] = P[2, 0, :, 0]
    D[4, 0] = p_e
    case.dirichlet = {0: D}
    return P


def porous_bl(nx: int = 1024, ny: int = 256, Ma: float = 6.0, T_inf_K: float = 65.0,
              Tw_K: float = 300.0, Re_unit: float = 1.0e4, Pr: float = 0.72,
              x0: float = 1.0, x1: float = 1.5, H: float = 0.4, beta: float = 2.2,
              strip: Optional[Tuple[int, int]] = None, k_max: float = 0.5,
              seed: int = 1994, nsteps: int = 2000, dt_fixed: float = 0.0,
              pulse: float = 0.02, pulse_radius: float = 0.02
              ) -> Tuple[Case, np.ndarray, np.ndarray]:
    """Free stream rho = u = T = 1; p_inf = 1/(gamma Ma^2), R = p_inf; mu_inf =
    1/Re_unit (lengths in mm, Re_unit = 1e7/m * 1 mm).  Isothermal wall at
    Tw_K, Sutherland viscosity with S = 110.4 K, similarity inflow (Dirichlet)
    at x-, zero-gradient at x+ and y+, porous strip on y- over the middle half
    of the wall faces.  Returns (case, P, K) with K seeded uniform in
    [0, k_max)."""
    gamma = 1.4
    p_inf = 1.0 / (gamma * Ma * Ma)
    R = p_inf
    S_ratio = 110.4 / T_inf_K
    Tw = Tw_K / T_inf_K
    if strip is None:
        strip = (nx // 4, 3 * nx // 4)
    case = Case(name="porous_bl", ndim=2, n=(nx, ny, 1), lo=(x0, 0.0, 0.0), hi=(x1, H, 1.0),
                stretch=("uniform", "tanh1", "uniform"), beta=(0.0, beta, 0.0), gamma=gamma,
                R=R, Pr=Pr, visc_law="sutherland", mu_ref=1.0 / Re_unit, T_ref=1.0,
                visc_param=S_ratio,
                bc=("dirichlet", "zerograd", "porous", "zerograd", "periodic", "periodic"),
                T_wall=(0.0, 0.0, Tw, 0.0, 0.0, 0.0), porous_face=2, porous_begin=strip[0],
                porous_end=strip[1], p_inf=p_inf, cost_face=2, nsteps=nsteps, dt_fixed=dt_fixed)
    P = _similarity_fields(case, Ma, Pr, Tw, S_ratio, Re_unit, p_inf)
    x, y, _ = _mesh(case)
    xm = 0.5 * (x0 + x1)
    pw = p_inf * (1.0 + pulse * np.exp(-((x[0] - xm) ** 2 + y[0] ** 2) / pulse_radius ** 2))
    P[0, 0] *= pw / p_inf
    P[4, 0] = pw
    K = k_max * uniform01(seed, case.n_porous, 7)
    return case, P, K


def laminar_bl(nx: int = 300, ny: int = 200, Ma: float = 2.25, T_e_K: float = 169.44,
               Re_unit: float = 1.0e4, Pr: float = 0.72, x0: float = 1.0, x1: float = 1.5,
               H: float = 0.4, beta: float = 2.2, amp: float = 0.0, kappa: float = 10.0,
               nsteps: int = 20000) -> Tuple[Case, np.ndarray]:
    """Mach-2.25 laminar boundary layer over an adiabatic no-slip wall
    (Section 3.2): (x, y) in [1, 1.5] x [0, 0.4], uniform in x, tanh
    clustering toward the wall in y (beta = 2.2), similarity inflow at x-,
    zero-gradient at x+ and y+, unit Reynolds number 1e4, Sutherland
    viscosity, Pr = 0.72.  With amp != 0 the wall is the disturbance wall of
    Eq. (8), v = amp sin(2 pi kappa x).  Free stream rho = u = T = 1, p_e =
    1/(gamma Ma^2) = R.  T_e_K only sets the Sutherland constant ratio
    S/T_e (S = 110.4 K).  The initial field is the similarity solution
    everywhere.  Returns (case, P)."""
    gamma = 1.4
    p_e = 1.0 / (gamma * Ma * Ma)
    S_ratio = 110.4 / T_e_K
    case = Case(name="laminar_bl", ndim=2, n=(nx, ny, 1), lo=(x0, 0.0, 0.0), hi=(x1, H, 1.0),
                stretch=("uniform", "tanh1", "uniform"), beta=(0.0, beta, 0.0), gamma=gamma,
                R=p_e, Pr=Pr, visc_law="sutherland", mu_ref=1.0 / Re_unit, T_ref=1.0,
                visc_param=S_ratio,
                bc=("dirichlet", "zerograd", "disturb", "zerograd", "periodic", "periodic"),
                T_wall=(0.0,) * 6, dist_amp=(0.0, 0.0, amp, 0.0, 0.0, 0.0),
                dist_kappa=(0.0, 0.0, kappa, 0.0, 0.0, 0.0), p_inf=p_e, nsteps=nsteps)
    P = _similarity_fields(case, Ma, Pr, None, S_ratio, Re_unit, p_e)
    return case, P


# --------------------------------------------------------------------------
# Small generic fields for tests.
# --------------------------------------------------------------------------
def random_smooth(case: Case, seed: int = 0, amp: float = 0.05, rho0: float = 1.0,
                  p0: float = 1.0, u0: Sequence[float] = (0.3, -0.2, 0.1)) -> np.ndarray:
    """Smooth periodic perturbations of a uniform state with seeded phases."""
    x, y, z = _mesh(case)
    P = _prim(*case.n)
    L = [case.hi[d] - case.lo[d] for d in range(3)]
    r = uniform01(seed, 16, 0)
    k = [2 * math.pi / L[d] for d in range(3)]

    def wave(c):
        ph = 2 * math.pi * r[c:c + 3]
        s = np.sin(k[0] * x + ph[0])
        if case.ndim >= 2:
            s = s * np.cos(k[1] * y + ph[1])
        if case.ndim >= 3:
            s = s * np.cos(k[2] * z + ph[2])
        return s

    P[0] = rho0 * (1.0 + amp * wave(0))
    for d in range(case.ndim):
        P[1 + d] = u0[d] + amp * wave(3 + 3 * d)
    P[4] = p0 * (1.0 + amp * wave(12))
    return P


def random_rough(case: Case, seed: int = 0, rho=(0.5, 1.5), vel=(-0.5, 0.5), p=(0.5, 1.5)) -> np.ndarray:
    """Cell-wise independent uniform values (discontinuous data)."""
    nc = case.ncells
    P = _prim(*case.n)
    shp = (case.n[2], case.n[1], case.n[0])
    P[0] = (rho[0] + (rho[1] - rho[0]) * uniform01(seed, nc, 0)).reshape(shp)
    for d in range(case.ndim):
        P[1 + d] = (vel[0] + (vel[1] - vel[0]) * uniform01(seed, nc, 1 + d)).reshape(shp)
    P[4] = (p[0] + (p[1] - p[0]) * uniform01(seed, nc, 4)).reshape(shp)
    return P
