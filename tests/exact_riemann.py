"""Exact solution of the Riemann problem for the 1D Euler equations of an ideal
gas (Toro, "Riemann Solvers and Numerical Methods for Fluid Dynamics", 3rd
ed., Chapter 4: pressure function, Newton iteration for p*, wave-pattern
sampling).  Independent of the oracle; used to pin it on the Sod problem."""
import math

import numpy as np


def _f_and_df(p, rho, pK, cK, g):
    if p > pK:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pK
        sq = math.sqrt(A / (p + B))
        f = (p - pK) * sq
        df = sq * (1.0 - 0.5 * (p - pK) / (B + p))
    else:  # rarefaction
        f = 2.0 * cK / (g - 1.0) * ((p / pK) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * cK) * (p / pK) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def star_state(rL, uL, pL, rR, uR, pR, g=1.4):
    """p*, u*, rho*_L, rho*_R."""
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    p = max(1e-12, 0.5 * (pL + pR) - 0.125 * (uR - uL) * (rL + rR) * (cL + cR))
    for _ in range(100):
        fL, dfL = _f_and_df(p, rL, pL, cL, g)
        fR, dfR = _f_and_df(p, rR, pR, cR, g)
        dp = (fL + fR + uR - uL) / (dfL + dfR)
        pn = max(1e-14, p - dp)
        if abs(pn - p) < 1e-15 * (pn + p):
            p = pn
            break
        p = pn
    fL, _ = _f_and_df(p, rL, pL, cL, g)
    fR, _ = _f_and_df(p, rR, pR, cR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)

    def rho_star(rK, pK):
        if p > pK:
            r = p / pK
            q = (g - 1.0) / (g + 1.0)
            return rK * (r + q) / (q * r + 1.0)
        return rK * (p / pK) ** (1.0 / g)

    return p, u, rho_star(rL, pL), rho_star(rR, pR)


def sample(x, t, x0, left, right, g=1.4):
    """(rho, u, p) at positions x and time t for the interface at x0."""
    rL, uL, pL = left
    rR, uR, pR = right
    ps, us, rsL, rsR = star_state(rL, uL, pL, rR, uR, pR, g)
    cL = math.sqrt(g * pL / rL)
    cR = math.sqrt(g * pR / rR)
    out = np.zeros((3, len(x)))
    for n, xi in enumerate(x):
        s = (xi - x0) / t
        if s <= us:  # left of contact
            if ps > pL:  # left shock
                SL = uL - cL * math.sqrt((g + 1) / (2 * g) * ps / pL + (g - 1) / (2 * g))
                w = (rL, uL, pL) if s <= SL else (rsL, us, ps)
            else:  # left rarefaction
                cs = cL * (ps / pL) ** ((g - 1) / (2 * g))
                head, tail = uL - cL, us - cs
                if s <= head:
                    w = (rL, uL, pL)
                elif s >= tail:
                    w = (rsL, us, ps)
                else:
                    u = 2 / (g + 1) * (cL + (g - 1) / 2 * uL + s)
                    c = 2 / (g + 1) * (cL + (g - 1) / 2 * (uL - s))
                    rho = rL * (c / cL) ** (2 / (g - 1))
                    w = (rho, u, pL * (c / cL) ** (2 * g / (g - 1)))
        else:
            if ps > pR:
                SR = uR + cR * math.sqrt((g + 1) / (2 * g) * ps / pR + (g - 1) / (2 * g))
                w = (rR, uR, pR) if s >= SR else (rsR, us, ps)
            else:
                cs = cR * (ps / pR) ** ((g - 1) / (2 * g))
                head, tail = uR + cR, us + cs
                if s >= head:
                    w = (rR, uR, pR)
                elif s <= tail:
                    w = (rsR, us, ps)
                else:
                    u = 2 / (g + 1) * (-cR + (g - 1) / 2 * uR + s)
                    c = 2 / (g + 1) * (cR - (g - 1) / 2 * (uR - s))
                    rho = rR * (c / cR) ** (2 / (g - 1))
                    w = (rho, u, pR * (c / cR) ** (2 * g / (g - 1)))
        out[:, n] = w
    return out


def cell_average(n, t, x0=0.5, left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), g=1.4, sub=64):
    """Cell averages of the exact solution over n uniform cells of [0, 1]."""
    xs = (np.arange(n * sub) + 0.5) / (n * sub)
    w = sample(xs, t, x0, left, right, g)
    return w.reshape(3, n, sub).mean(axis=2)
