"""Pins of the oracle's channel scheme (TENO6-A reconstruction with the
interpolation limiter, 6th-order central dissipative fluxes) against facts
that do not come from the oracle: the Jiang-Shu integral definition of the
smoothness indicators, exactness of the linear scheme on polynomials, the ENO
property on steps, the two ends of the adaptive cut-off, exactness of the
central stencils, and the invariants and closed forms the solver must keep
with this scheme."""
import math

import numpy as np
import pytest
from numpy.polynomial import polynomial as Pn

from oracle import pyoracle
from oracle.pyoracle import Oracle
from paper_2406_19494_amd import workloads as W
from tests import exact_riemann as ER


# --------------------------------------------------------------------------
# Reconstruction polynomials from cell averages (unit cells, cell i = [-1/2,
# 1/2]), built with numpy: the definitions the indicators are pinned to.
# --------------------------------------------------------------------------
def _poly_from_averages(offsets, avgs):
    """Coefficients (ascending) of the polynomial of degree len-1 whose
    averages over the unit cells at `offsets` are `avgs`."""
    r = len(offsets)
    A = np.zeros((r, r))
    for row, j in enumerate(offsets):
        for m in range(r):
            A[row, m] = ((j + 0.5) ** (m + 1) - (j - 0.5) ** (m + 1)) / (m + 1)
    return np.linalg.solve(A, np.asarray(avgs, dtype=np.float64))


def _jiang_shu_indicator(coef):
    """sum_{l >= 1} of the integral over cell i of (d^l p / dx^l)^2."""
    total = 0.0
    c = np.array(coef)
    for _ in range(len(coef) - 1):
        c = Pn.polyder(c)
        sq = Pn.polyint(Pn.polymul(c, c))
        total += Pn.polyval(0.5, sq) - Pn.polyval(-0.5, sq)
    return total


STENCILS = [(-1, 0, 1), (0, 1, 2), (-2, -1, 0), (0, 1, 2, 3), (-2, -1, 0, 1, 2, 3)]


def test_smoothness_indicators_are_the_jiang_shu_integrals():
    rng = np.random.default_rng(61)
    for _ in range(20):
        v = rng.normal(size=6) * rng.uniform(0.1, 10.0)
        beta = pyoracle.teno6a_beta(v)
        for k, st in enumerate(STENCILS):
            ref = _jiang_shu_indicator(_poly_from_averages(st, [v[j + 2] for j in st]))
            assert abs(beta[k] - ref) <= 1e-11 * max(abs(ref), 1e-300), (k, beta[k], ref)


def _face_exact(coef):
    return Pn.polyval(0.5, coef)


@pytest.mark.parametrize("degree", [0, 1, 2, 3, 4, 5])
def test_linear_scheme_on_smooth_polynomials(degree):
    # cell averages of a slowly varying polynomial (small scale h): every
    # candidate is kept and the value is the sixth-order central
    # reconstruction, exact up to degree 5; the weights are the linear ones
    rng = np.random.default_rng(degree)
    h = 0.02
    c = rng.uniform(0.5, 1.5, size=degree + 1) * h ** np.arange(degree + 1)
    if degree >= 1:
        c[1] = 1.3 * h
    offsets = np.arange(-2, 4)
    avg = [(Pn.polyval(j + 0.5, Pn.polyint(c)) - Pn.polyval(j - 0.5, Pn.polyint(c)))
           for j in offsets]
    y, ct, w = pyoracle.teno6a(avg)
    assert ct == 1e-10
    if degree >= 1:
        # (constant data: every candidate gives the constant, and round-off
        # of the averages decides the scale separation, so only the value is
        # fixed)
        assert np.array_equal(w, [0.45, 0.3, 0.05, 0.2])
    assert abs(y - _face_exact(c)) <= 1e-13 * max(1.0, abs(_face_exact(c)))


def test_sixth_order_convergence_on_a_sine():
    errs = []
    for n in (20, 40, 80):
        h = 2 * math.pi / n
        # cell averages of sin around the face at x = 0.3
        x0 = 0.3 - 0.5 * h
        avg = [(math.cos(x0 + (j - 0.5) * h) - math.cos(x0 + (j + 0.5) * h)) / h
               for j in range(-2, 4)]
        errs.append(abs(pyoracle.teno6a(avg)[0] - math.sin(0.3)))
    assert errs[0] / errs[1] > 50 and errs[1] / errs[2] > 50, errs


@pytest.mark.parametrize("p", [1, 2, 3, 4, 5])
def test_eno_on_a_step(p):
    # a jump between cells p-1 and p of the six (the face lies between 2 and
    # 3): every candidate that straddles the jump is cut off, the value is the
    # one of the smooth side upstream, exactly, and the cut-off is the one of
    # a discontinuity
    v = np.array([0.0] * p + [1.0] * (6 - p))
    y, ct, w = pyoracle.teno6a(v)
    crosses = [st[0] + 2 < p <= st[-1] + 2 for st in STENCILS[:4]]
    assert ct == 1e-7
    for k in range(4):
        if crosses[k]:
            assert w[k] == 0.0, (p, k, w)
        else:
            assert w[k] > 0.0, (p, k, w)
    assert y == (1.0 if p <= 2 else 0.0), (p, y)
    # the mirrored data give the mirrored value
    y2, _, _ = pyoracle.teno6a(1.0 - v)
    assert y2 == 1.0 - y


def test_cutoff_runs_from_smooth_to_discontinuous():
    # Ren et al.'s measure is 1 for equal neighbouring differences and falls
    # towards 0 as one difference dwarfs the other: C_T must not rise as the
    # data get smoother, and spans 1e-7 (jump) .. 1e-10 (linear)
    cts = []
    for ratio in (1e6, 1e3, 100.0, 30.0, 12.0, 8.0, 4.0, 2.0, 1.0):
        v = np.array([0.0, 1.0, 2.0, 2.0 + ratio, 2.0 + 2 * ratio, 2.0 + 3 * ratio])
        cts.append(pyoracle.teno6a(v)[1])
    assert cts[0] == 1e-7 and cts[-1] == 1e-10
    assert all(a >= b for a, b in zip(cts, cts[1:])), cts
    assert set(cts) <= {1e-7, 1e-8, 1e-9, 1e-10}


@pytest.mark.parametrize("degree", [1, 2, 3, 4, 5, 6])
def test_central_stencils_are_exact_for_polynomials(degree):
    rng = np.random.default_rng(100 + degree)
    c = rng.normal(size=degree + 1)
    off = np.arange(-3, 4)
    v = Pn.polyval(off, c)
    out = pyoracle.central_stencils(v)
    dc = Pn.polyder(c)
    scale = np.abs(c).sum() * 4.0 ** degree
    if degree <= 5:  # 6th-order face value and face derivative
        assert abs(out[0] - Pn.polyval(0.5, c)) <= 1e-13 * scale
        assert abs(out[1] - Pn.polyval(0.5, dc)) <= 1e-13 * scale
    assert abs(out[2] - Pn.polyval(0.0, dc)) <= 1e-13 * scale  # 7-point central: degree 6
    if degree <= 3:
        assert abs(out[3] - Pn.polyval(0.5, c)) <= 1e-13 * scale
        assert abs(out[4] - Pn.polyval(0.5, dc)) <= 1e-13 * scale
    if degree <= 4:
        assert abs(out[5] - Pn.polyval(0.0, dc)) <= 1e-13 * scale
    if degree == 6:  # the face stencils are not exact one degree higher
        assert abs(out[0] - Pn.polyval(0.5, c)) > 1e-10 * scale


# --------------------------------------------------------------------------
# The solver with the channel scheme.
# --------------------------------------------------------------------------
def _teno(case):
    case.scheme = "teno6a"
    return case


@pytest.mark.parametrize("ndim", [1, 2, 3])
def test_free_stream_preservation_teno(ndim):
    st = ("tanh2", "tanh1", "tanh2")
    nn = [1, 1, 1]
    for d in range(ndim):
        nn[d] = 8
    case = _teno(W.Case(name="u", ndim=ndim, n=tuple(nn), lo=(0, -1, 0), hi=(2, 1, 1.5),
                        stretch=st, beta=(1.5, 2.0, 1.2), gamma=1.4, R=1.7, Pr=0.7,
                        visc_law="power", mu_ref=0.01, T_ref=1.0, visc_param=0.7,
                        bc=("periodic",) * 6))
    o = Oracle(case)
    P = np.zeros((5, case.n[2], case.n[1], case.n[0]))
    P[0], P[1], P[4] = 1.3, 0.4, 0.9
    if ndim >= 2:
        P[2] = -0.7
    if ndim >= 3:
        P[3] = 0.25
    assert np.all(o.rhs(o.cons(P)) == 0.0)


def test_conservation_periodic_tgv_teno():
    case, P = W.tgv(16)
    o = Oracle(_teno(case))
    U0 = o.cons(P)
    d0 = o.diag(U0)
    U, n, t = o.run(U0, 10)
    d1 = o.diag(U)
    assert abs(d1["mass"] - d0["mass"]) <= 1e-13 * d0["mass"]
    assert abs(d1["energy"] - d0["energy"]) <= 1e-13 * d0["energy"]
    absmom = np.sum(np.abs(U[1:4]), axis=(1, 2, 3)).max() * d0["vol"] / case.ncells
    assert np.max(np.abs(d1["mom"] - d0["mom"])) <= 1e-13 * absmom


def test_direction_permutation_bitwise_teno():
    case1, P1 = W.sod(64)
    o1 = Oracle(_teno(case1))
    U1, _, _ = o1.run(o1.cons(P1), 20, dt_fixed=2e-3)
    ref = U1[:, 0, 0, :]
    for axis in range(3):
        case, P = W.sod(64, axis=axis, ndim=3, cross=4)
        o = Oracle(_teno(case))
        U, _, _ = o.run(o.cons(P), 20, dt_fixed=2e-3)
        idx = [1, 1, 1]
        idx[2 - axis] = slice(None)
        assert np.array_equal(U[0][tuple(idx)], ref[0])
        assert np.array_equal(U[1 + axis][tuple(idx)], ref[1])
        assert np.array_equal(U[4][tuple(idx)], ref[2])


def test_mirror_symmetry_teno():
    case = _teno(W.Case(name="m", ndim=2, n=(12, 12, 1), lo=(0, -1, 0), hi=(2, 1, 1),
                        gamma=1.4, R=1.7, Pr=0.7, visc_law="power", mu_ref=0.01, T_ref=1.0,
                        visc_param=0.7, bc=("periodic",) * 6))
    o = Oracle(case)
    P = W.random_smooth(case, seed=3, amp=0.2)
    R = o.rhs(o.cons(P))
    Pm = P[:, :, :, ::-1].copy()
    Pm[1] = -Pm[1]
    Rm = o.rhs(o.cons(Pm))
    scale = np.abs(R).max()
    for v, sgn in ((0, 1), (1, -1), (2, 1), (3, 1)):
        assert np.max(np.abs(sgn * Rm[v][:, :, ::-1] - R[v])) < 1e-13 * scale


def test_sod_with_teno_against_exact():
    # the exact Riemann solution: L1 error of the density below 1e-2 at 200
    # cells, no new extrema (the targeted selection keeps the density within
    # the two initial states), and the plateaus within 2 % beyond 3 cells of
    # the shock and rarefaction edges and 8 cells of the contact and of the
    # initial discontinuity (the low-dissipation scheme leaves a small
    # start-up error there)
    case, P = W.sod(200)
    o = Oracle(_teno(case))
    U, steps, t = o.run(o.cons(P), 100000, t_end=0.2)
    assert abs(t - 0.2) < 1e-14
    rho = U[0, 0, 0]
    ex = ER.cell_average(200, 0.2)[0]
    assert np.mean(np.abs(rho - ex)) < 1e-2
    assert rho.min() > 0.125 * (1 - 1e-3) and rho.max() < 1.0 + 1e-3
    x = (np.arange(200) + 0.5) / 200
    waves = np.array([0.26336, 0.48595, 0.68549, 0.85043])
    plateau = (x < waves[0]) | ((x > waves[1]) & (x < waves[3])) | (x > waves[3])
    far = (np.min(np.abs(x[:, None] - waves[None, :]), axis=1) > 3.0 / 200) & \
          (np.abs(x - waves[2]) > 8.0 / 200) & (np.abs(x - 0.5) > 8.0 / 200)
    sel = plateau & far
    assert sel.sum() > 100 and (np.abs(rho - ex)[sel] / ex[sel]).max() < 2e-2


def _decay_rate(o, U0, comp_fn, steps, dt):
    a0 = comp_fn(U0)
    U, _, _ = o.run(U0, steps, dt_fixed=dt)
    return -math.log(comp_fn(U) / a0) / (steps * dt)


def test_shear_wave_decay_teno_viscous():
    # v = A sin(k x) on a periodic 2D box at rest decays at nu k^2: the
    # 6th-order face derivative and interpolation carry the viscous term
    n, mu = 32, 0.02
    case = _teno(W.Case(name="shear", ndim=2, n=(n, 4, 1), lo=(0, 0, 0),
                        hi=(2 * math.pi, 1, 1), gamma=1.4, R=1.0, Pr=0.7, visc_law="power",
                        mu_ref=mu, T_ref=1.0, visc_param=0.0, bc=("periodic",) * 6))
    o = Oracle(case)
    x = (np.arange(n) + 0.5) * 2 * math.pi / n
    P = np.zeros((5, 1, 4, n))
    P[0] = 1.0
    P[4] = 1.0
    ref = np.broadcast_to(np.sin(x), (1, 4, n))
    P[2] = 1e-4 * ref
    amp = lambda U: float(np.sum(U[2] / U[0] * ref) / np.sum(ref * ref))  # noqa: E731
    rate = _decay_rate(o, o.cons(P), amp, 40, 5e-3)
    assert abs(rate - mu) < 2e-3 * mu, (rate, mu)


def test_cross_derivative_terms_teno():
    # u = A cos x sin y, v = -A sin x cos y (divergence free), rho = p = 1 on
    # a periodic box: at t = 0 the x-momentum right-hand side is
    # A^2 sin x cos x - 2 mu A cos x sin y.  Its viscous part comes from the
    # normal derivative of u and the tangential derivative of v at x faces
    # (tau_xx), while tau_xy = mu (u_y + v_x) vanishes only when the normal
    # and tangential derivatives at y faces agree.  Against the continuous
    # value the point-value sampling limits the rate to 2nd order; a wrong
    # stencil, metric or sign stalls it.
    A, mu = 1e-3, 0.05
    errs = []
    for n in (16, 32, 64):
        case = _teno(W.Case(name="x", ndim=2, n=(n, n, 1), lo=(0, 0, 0),
                            hi=(2 * math.pi, 2 * math.pi, 1), gamma=1.4, R=1.0, Pr=0.7,
                            visc_law="power", mu_ref=mu, T_ref=1.0, visc_param=0.0,
                            bc=("periodic",) * 6))
        o = Oracle(case)
        x = (np.arange(n) + 0.5) * 2 * math.pi / n
        X, Y = np.meshgrid(x, x)
        P = np.zeros((5, 1, n, n))
        P[0], P[4] = 1.0, 1.0
        P[1, 0] = A * np.cos(X) * np.sin(Y)
        P[2, 0] = -A * np.sin(X) * np.cos(Y)
        R = o.rhs(o.cons(P))
        exact = A * A * np.sin(X) * np.cos(X) - 2.0 * mu * A * np.cos(X) * np.sin(Y)
        errs.append(np.abs(R[1, 0] - exact).max() / np.abs(exact).max())
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5, errs
    assert errs[-1] < 1e-2
