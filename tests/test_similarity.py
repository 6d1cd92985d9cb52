"""Pins of the compressible boundary-layer similarity solution used for the
inflow profiles and for the laminar boundary-layer validation (Section 3.2,
Eq. (7)).  The solver is a generic BVP solve, so it is pinned to relations
that hold exactly for the similarity equations."""
import math

import numpy as np

from paper_2406_19494_amd import workloads as W


def test_crocco_busemann_relation_at_unit_prandtl_number():
    # For Pr = 1 and zero pressure gradient the energy equation has the exact
    # integral g = g_w + (1 - g_w) f' + (gamma-1)/2 Ma^2 f' (1 - f') for any
    # viscosity law; at an adiabatic wall g_w = 1 + (gamma-1)/2 Ma^2.
    Ma, gamma = 2.25, 1.4
    r = 0.5 * (gamma - 1.0) * Ma * Ma
    eta, f, fp, g = W.similarity_profile(Ma, 1.0, gamma, None, 110.4 / 169.44)
    assert abs(g[0] - (1.0 + r)) < 1e-6
    assert np.abs(g - (1.0 + r * (1.0 - fp ** 2))).max() < 1e-6
    # isothermal wall at g_w = 2
    eta, f, fp, g = W.similarity_profile(Ma, 1.0, gamma, 2.0, 110.4 / 169.44)
    assert np.abs(g - (2.0 - fp + r * fp * (1.0 - fp))).max() < 1e-6


def test_adiabatic_recovery_factor_near_sqrt_prandtl():
    # Laminar recovery factor r = (g_aw - 1)/((gamma-1)/2 Ma^2) ~ Pr^(1/2).
    Ma, gamma, Pr = 2.25, 1.4, 0.72
    eta, f, fp, g = W.similarity_profile(Ma, Pr, gamma, None, 110.4 / 169.44)
    rec = (g[0] - 1.0) / (0.5 * (gamma - 1.0) * Ma * Ma)
    assert abs(rec - math.sqrt(Pr)) < 0.01 * math.sqrt(Pr)


def test_incompressible_limit_is_blasius():
    # Ma -> 0 with g_w = 1: the momentum equation is Blasius' f''' + f f'' = 0
    # in eta, with f''(0) = 0.4696 (eta = y sqrt(u/(2 nu x)) scaling).
    eta, f, fp, g = W.similarity_profile(1e-3, 0.72, 1.4, 1.0, 1.0)
    fpp0 = (-3 * fp[0] + 4 * fp[1] - fp[2]) / (2 * (eta[1] - eta[0]))
    assert abs(fpp0 - 0.46960) < 2e-4
