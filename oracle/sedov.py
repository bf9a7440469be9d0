"""Sedov-Taylor point explosion in a uniform medium (the analytic comparison
of the Sedov test, Sect. 4.3): the self-similar solution, by integrating its
ordinary differential equations.

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).

A point energy E released at t = 0 in gas of density rho0 at rest with zero
pressure drives a strong spherical shock at R(t) = xi0 (E t^2 / rho0)^(1/5).
With lambda = r / R and Rdot = dR/dt = (2/5) R / t, the flow behind the
shock is v = Rdot V(lambda), rho = rho0 G(lambda), p = rho0 Rdot^2 P(lambda);
the spherical Euler equations with adiabatic flow become

    (V - l) G' + G V' = -2 G V / l                      (mass)
    (V - l) V' + P' / G = (3/2) V                        (momentum; R'' R / Rdot^2 = -3/2)
    (V - l) (P'/P - gamma G'/G) = 3                      (entropy along flow lines)

with the strong-shock jump conditions G(1) = (gamma+1)/(gamma-1),
V(1) = P(1) = 2/(gamma+1), integrated inward from lambda = 1.  The total
energy fixes xi0: E = (16 pi / 25) rho0 xi0^5 (E/rho0) I with
I = int_0^1 (G V^2 / 2 + P / (gamma-1)) lambda^2 dlambda.

Pinned by tests/test_oracle_sedov.py: the textbook shock constants (xi0 =
1.033 for gamma = 7/5 and 1.152 for gamma = 5/3), the swept-up mass
(int G lambda^2 = 1/3), the centre asymptotics (V -> lambda/gamma,
G ~ lambda^(3/(gamma-1))), and the jump conditions.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import solve_ivp


def _rhs(lam, y, gamma):
    G, V, P = y
    d = V - lam
    q = P / G
    dV = (1.5 * V * d - q * (3.0 - 2.0 * gamma * V / lam)) / (d * d - gamma * q)
    dG = -G * (dV + 2.0 * V / lam) / d
    dP = P * (3.0 / d + gamma * dG / G)
    return [dG, dV, dP]


class Sedov:
    """The similarity profiles for one gamma, on a fine grid of lambda."""

    def __init__(self, gamma: float, lam_min: float = 1e-4, n: int = 4001):
        g = float(gamma)
        self.gamma = g
        y1 = [(g + 1.0) / (g - 1.0), 2.0 / (g + 1.0), 2.0 / (g + 1.0)]
        lam = np.concatenate([np.geomspace(lam_min, 0.05, 800, endpoint=False),
                              np.linspace(0.05, 1.0, n)])[::-1]
        sol = solve_ivp(_rhs, (1.0, lam_min), y1, args=(g,), t_eval=lam, method="DOP853",
                        rtol=1e-12, atol=1e-14)
        if not sol.success:
            raise RuntimeError(sol.message)
        self.lam = sol.t[::-1]
        self.G, self.V, self.P = (sol.y[k][::-1] for k in range(3))
        integrand = (0.5 * self.G * self.V ** 2 + self.P / (g - 1.0)) * self.lam ** 2
        self.I = float(np.trapezoid(integrand, self.lam))
        self.xi0 = (25.0 / (16.0 * math.pi * self.I)) ** 0.2

    def shock_radius(self, E: float, rho0: float, t: float) -> float:
        return self.xi0 * (E * t * t / rho0) ** 0.2

    def profile(self, r, E: float, rho0: float, t: float):
        """rho, v_r, P at radii r (arrays) and time t; undisturbed outside R."""
        r = np.asarray(r, dtype=np.float64)
        R = self.shock_radius(E, rho0, t)
        Rdot = 0.4 * R / t
        lam = r / R
        inside = lam < 1.0
        li = np.clip(lam, self.lam[0], 1.0)
        G = np.interp(li, self.lam, self.G)
        V = np.interp(li, self.lam, self.V)
        P = np.interp(li, self.lam, self.P)
        rho = np.where(inside, rho0 * G, rho0)
        v = np.where(inside, Rdot * V, 0.0)
        p = np.where(inside, rho0 * Rdot * Rdot * P, 0.0)
        return rho, v, p
