"""Pins of the Sedov-Taylor solution (oracle/sedov.py) used to grade the
Sedov test (Sect. 4.3).

* The shock constant xi0 of R = xi0 (E t^2 / rho0)^(1/5): 1.0328 for gamma =
  7/5 and 1.1517 for gamma = 5/3 (the tabulated values, e.g. Kamm & Timmes
  2007, alpha = xi0^-5 = 0.851072 and 0.49365).
* Mass: the shocked sphere holds all the swept-up gas, 3 int_0^1 G l^2 = 1.
* Energy flux: with the energy inside every self-similar sphere l R(t)
  constant, (G V^2/2 + P/(gamma-1)) (l - V) = P V at every l -- an
  algebraic identity of the exact solution that the integrated equations
  (which use the entropy equation, not the energy equation) must satisfy.
* The profile function: undisturbed medium outside R, jump values at R.
"""
import math

import numpy as np
import pytest

from oracle.sedov import Sedov


@pytest.mark.parametrize("gamma,xi0", [(1.4, 1.0328), (5.0 / 3.0, 1.1517)])
def test_shock_constant(gamma, xi0):
    assert abs(Sedov(gamma).xi0 - xi0) < 1e-4


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0, 1.2])
def test_swept_mass(gamma):
    s = Sedov(gamma)
    assert abs(3.0 * np.trapezoid(s.G * s.lam ** 2, s.lam) - 1.0) < 1e-5


@pytest.mark.parametrize("gamma", [1.4, 5.0 / 3.0, 1.2])
def test_energy_flux_identity(gamma):
    s = Sedov(gamma)
    # the integration near the singular centre loses digits as lambda^-2
    # (1e-8 at lambda = 1e-3); the graded profiles start far outside it
    m = s.lam > 0.05
    lhs = (0.5 * s.G * s.V ** 2 + s.P / (gamma - 1.0)) * (s.lam - s.V)
    rhs = s.P * s.V
    assert np.max(np.abs(lhs - rhs)[m]) < 1e-10 * np.max(np.abs(rhs))


def test_profile_outside_and_at_the_shock():
    g = 5.0 / 3.0
    s = Sedov(g)
    E, rho0, t = 1.0, 1.0, 0.1
    R = s.shock_radius(E, rho0, t)
    assert abs(R - 1.1517 * 0.01 ** 0.2) < 1e-4
    rho, v, p = s.profile(np.array([1.01 * R, 2 * R]), E, rho0, t)
    np.testing.assert_array_equal(rho, [1.0, 1.0])
    np.testing.assert_array_equal(v, [0.0, 0.0])
    rho, v, p = s.profile(np.array([R * (1 - 1e-12)]), E, rho0, t)
    Rdot = 0.4 * R / t
    assert abs(rho[0] - (g + 1) / (g - 1)) < 1e-6
    assert abs(v[0] - 2 * Rdot / (g + 1)) < 1e-6 * Rdot
    assert abs(p[0] - 2 * Rdot ** 2 / (g + 1)) < 1e-6 * Rdot ** 2
