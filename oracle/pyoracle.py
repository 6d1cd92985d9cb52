"""ctypes front end of the CPU oracle (test infrastructure only).

Marshals a ``workloads.Case`` into the oracle's own C struct and calls the
oracle's C entry points.  Nothing in the GPU library imports this module.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_BC = {"periodic": 0, "wall": 1, "porous": 2, "zerograd": 3, "dirichlet": 4, "disturb": 5}
_VISC = {"none": 0, "power": 1, "sutherland": 2}
_STRETCH = {"uniform": 0, "tanh2": 1, "tanh1": 2}
_SRC = {"none": 0, "massflux": 1}
_SCHEME = {"weno5": 0, "teno6a": 1}

_dp = C.POINTER(C.c_double)


class OrcCase(C.Structure):
    _fields_ = [
        ("ndim", C.c_int), ("n", C.c_int * 3), ("lo", C.c_double * 3), ("hi", C.c_double * 3),
        ("stretch", C.c_int * 3), ("beta", C.c_double * 3),
        ("gamma", C.c_double), ("R", C.c_double), ("Pr", C.c_double),
        ("visc_law", C.c_int), ("mu_ref", C.c_double), ("T_ref", C.c_double),
        ("visc_param", C.c_double), ("bc", C.c_int * 6), ("T_wall", C.c_double * 6),
        ("dirichlet", _dp * 6), ("porous_face", C.c_int), ("porous_begin", C.c_int),
        ("porous_end", C.c_int), ("p_inf", C.c_double), ("source", C.c_int),
        ("cost_face", C.c_int), ("scheme", C.c_int),
    ]


_lib = None


def lib():
    global _lib
    if _lib is None:
        path = _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        P = C.POINTER(OrcCase)
        sig = {
            "orc_nk": (C.c_int, [P]),
            "orc_ncells": (C.c_long, [P]),
            "orc_nbox": (C.c_long, [P]),
            "orc_grid": (None, [P, C.c_int, _dp, _dp, _dp, _dp]),
            "orc_weno5": (C.c_double, [C.c_double] * 5),
            "orc_hllc": (None, [_dp, _dp, C.c_double, _dp]),
            "orc_teno6a": (C.c_double, [_dp, _dp, _dp]),
            "orc_teno6a_beta": (None, [_dp, _dp]),
            "orc_central_stencils": (None, [_dp, _dp]),
            "orc_cons_from_prim": (None, [P, _dp, _dp]),
            "orc_prims_halo": (None, [P, _dp, _dp, _dp, _dp]),
            "orc_rhs": (None, [P, _dp, _dp, _dp]),
            "orc_dt": (C.c_double, [P, _dp, C.c_double]),
            "orc_step": (None, [P, _dp, _dp, C.c_double]),
            "orc_run": (C.c_int, [P, _dp, _dp, C.c_int, C.c_double, C.c_double, C.c_double, _dp]),
            "orc_diag": (None, [P, _dp, _dp]),
            "orc_cost_term": (C.c_double, [P, _dp]),
            "orc_cost_term_grad": (None, [P, _dp, _dp]),
            "orc_jvp_step": (None, [P, _dp, _dp, _dp, _dp, C.c_double, _dp, _dp]),
            "orc_vjp_step": (None, [P, _dp, _dp, C.c_double, _dp, _dp, _dp]),
            "orc_gradient": (C.c_double, [P, _dp, _dp, C.c_int, C.c_double, _dp, _dp]),
            "orc_set_threads": (C.c_int, [C.c_int]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def set_threads(n: int = 0) -> int:
    """OpenMP threads of the oracle's loops (n > 0 sets them); returns the
    number in use."""
    return int(lib().orc_set_threads(int(n)))


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_dp)


class Oracle:
    """One case on the CPU oracle.  Arrays are numpy float64, C-contiguous:
    U is [nv][nz][ny][nx]; P (primitives) is [5][nz][ny][nx]."""

    def __init__(self, case, K=None):
        self.case = case
        s = OrcCase()
        s.ndim = case.ndim
        for d in range(3):
            s.n[d] = case.n[d]
            s.lo[d] = case.lo[d]
            s.hi[d] = case.hi[d]
            s.stretch[d] = _STRETCH[case.stretch[d]]
            s.beta[d] = case.beta[d]
        s.gamma, s.R, s.Pr = case.gamma, case.R, case.Pr
        s.visc_law = _VISC[case.visc_law]
        s.mu_ref, s.T_ref, s.visc_param = case.mu_ref, case.T_ref, case.visc_param
        self._keep = []
        for f in range(6):
            s.bc[f] = _BC[case.bc[f]]
            s.T_wall[f] = case.T_wall[f]
            if f in case.dirichlet:
                arr = np.ascontiguousarray(case.dirichlet[f], dtype=np.float64)
                self._keep.append(arr)
                s.dirichlet[f] = _ptr(arr)
        s.porous_face, s.porous_begin, s.porous_end = case.porous_face, case.porous_begin, case.porous_end
        s.p_inf = case.p_inf
        s.source = _SRC[case.source]
        s.cost_face = case.cost_face
        s.scheme = _SCHEME[getattr(case, "scheme", "weno5")]
        self.s = s
        self.L = lib()
        self.nk = self.L.orc_nk(C.byref(s))
        assert self.nk == case.nk
        # boundary parameters: porous coefficients, then (A, kappa) per
        # disturbance face (taken from the case when only K is given)
        th = case.theta(K)
        self.K = np.ascontiguousarray(th if th.size else np.zeros(1), dtype=np.float64)

    # ---- helpers -------------------------------------------------------
    @property
    def shape(self):
        c = self.case
        return (c.nv, c.n[2], c.n[1], c.n[0])

    def box_shape(self):
        c = self.case
        h = [3 if d < c.ndim else 0 for d in range(3)]
        return (c.n[2] + 2 * h[2], c.n[1] + 2 * h[1], c.n[0] + 2 * h[0])

    def grid(self, axis):
        n = self.case.n[axis]
        xf, dx, mc, mf = np.zeros(n + 1), np.zeros(n), np.zeros(n), np.zeros(n + 1)
        self.L.orc_grid(C.byref(self.s), axis, _ptr(xf), _ptr(dx), _ptr(mc), _ptr(mf))
        return xf, dx, mc, mf

    def cons(self, P):
        P = np.ascontiguousarray(P, dtype=np.float64)
        U = np.zeros(self.shape)
        self.L.orc_cons_from_prim(C.byref(self.s), _ptr(P), _ptr(U))
        return U

    def prims_halo(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        bs = self.box_shape()
        Q = np.zeros((6,) + bs)
        mu = np.zeros(bs)
        self.L.orc_prims_halo(C.byref(self.s), _ptr(self.K), _ptr(U), _ptr(Q), _ptr(mu))
        return Q, mu

    def rhs(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        R = np.zeros(self.shape)
        self.L.orc_rhs(C.byref(self.s), _ptr(self.K), _ptr(U), _ptr(R))
        return R

    def dt(self, U, cfl=None):
        U = np.ascontiguousarray(U, dtype=np.float64)
        return self.L.orc_dt(C.byref(self.s), _ptr(U), self.case.cfl if cfl is None else cfl)

    def step(self, U, dt):
        U = np.array(U, dtype=np.float64, order="C", copy=True)
        self.L.orc_step(C.byref(self.s), _ptr(self.K), _ptr(U), float(dt))
        return U

    def run(self, U, max_steps, cfl=None, dt_fixed=0.0, t_end=0.0):
        U = np.array(U, dtype=np.float64, order="C", copy=True)
        t = C.c_double(0.0)
        n = self.L.orc_run(C.byref(self.s), _ptr(self.K), _ptr(U), int(max_steps),
                           self.case.cfl if cfl is None else cfl, float(dt_fixed), float(t_end),
                           C.byref(t))
        return U, n, t.value

    def diag(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        out = np.zeros(8)
        self.L.orc_diag(C.byref(self.s), _ptr(U), _ptr(out))
        return dict(ek=out[0], eps=out[1], mass=out[2], mom=out[3:6].copy(), energy=out[6],
                    vol=out[7])

    def cost_term(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        return self.L.orc_cost_term(C.byref(self.s), _ptr(U))

    def cost_term_grad(self, U):
        U = np.ascontiguousarray(U, dtype=np.float64)
        g = np.zeros(self.shape)
        self.L.orc_cost_term_grad(C.byref(self.s), _ptr(U), _ptr(g))
        return g

    def jvp_step(self, U, dU, dt, dK=None):
        U = np.ascontiguousarray(U, dtype=np.float64)
        dU = np.ascontiguousarray(dU, dtype=np.float64)
        dKa = np.zeros_like(self.K) if dK is None else np.ascontiguousarray(dK, dtype=np.float64)
        U1, dU1 = np.zeros(self.shape), np.zeros(self.shape)
        self.L.orc_jvp_step(C.byref(self.s), _ptr(self.K), _ptr(dKa), _ptr(U), _ptr(dU), float(dt),
                            _ptr(U1), _ptr(dU1))
        return U1, dU1

    def vjp_step(self, U, lam, dt):
        U = np.ascontiguousarray(U, dtype=np.float64)
        lam = np.ascontiguousarray(lam, dtype=np.float64)
        lu = np.zeros(self.shape)
        lk = np.zeros(max(self.nk, 1))
        self.L.orc_vjp_step(C.byref(self.s), _ptr(self.K), _ptr(U), float(dt), _ptr(lam), _ptr(lu),
                            _ptr(lk))
        return lu, lk[: self.nk]

    def gradient(self, U0, nsteps, dt):
        U0 = np.ascontiguousarray(U0, dtype=np.float64)
        gk = np.zeros(max(self.nk, 1))
        gu = np.zeros(self.shape)
        J = self.L.orc_gradient(C.byref(self.s), _ptr(self.K), _ptr(U0), int(nsteps), float(dt),
                                _ptr(gk), _ptr(gu))
        return J, gk[: self.nk], gu


def weno5(a, b, c, d, e):
    return lib().orc_weno5(a, b, c, d, e)


def teno6a(v):
    """(value, C_T, weights) of the TENO6-A reconstruction at the right face
    of the third of six cells."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    ct = C.c_double()
    w = np.zeros(4)
    y = lib().orc_teno6a(_ptr(v), C.byref(ct), _ptr(w))
    return y, ct.value, w


def teno6a_beta(v):
    """(beta0, beta1, beta2, beta3, beta6) of TENO6-A on six cells."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    b = np.zeros(5)
    lib().orc_teno6a_beta(_ptr(v), _ptr(b))
    return b


def central_stencils(v):
    """(face value, face derivative, cell derivative) at 6th then 4th order
    from point values at offsets -3 .. 3."""
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = np.zeros(6)
    lib().orc_central_stencils(_ptr(v), _ptr(out))
    return out


def hllc(qL, qR, gamma=1.4):
    qL = np.ascontiguousarray(qL, dtype=np.float64)
    qR = np.ascontiguousarray(qR, dtype=np.float64)
    F = np.zeros(5)
    lib().orc_hllc(_ptr(qL), _ptr(qR), gamma, _ptr(F))
    return F
