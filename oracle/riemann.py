"""Exact solution of the 1D Riemann problem for an ideal gas.

TEST INFRASTRUCTURE ONLY (part of the oracle).  Used to grade the shock-tube
workload of the paper's Sect. 4 (Sod test) against its analytic solution; the
paper extracted the exact solution with an external plotting tool, so this is
written here from the standard textbook construction (Toro, "Riemann Solvers
and Numerical Methods for Fluid Dynamics", ch. 4): the star-region pressure is
the root of f_L(p) + f_R(p) + (u_R - u_L) = 0, with the shock branch
(Rankine-Hugoniot) for p > p_K and the rarefaction branch (isentropic) for
p <= p_K; the root is bracketed and found with scipy's brentq.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.optimize import brentq


def _fK(p, rho, pk, gamma):
    c = math.sqrt(gamma * pk / rho)
    if p > pk:  # shock
        A = 2.0 / ((gamma + 1.0) * rho)
        B = (gamma - 1.0) / (gamma + 1.0) * pk
        return (p - pk) * math.sqrt(A / (p + B))
    return 2.0 * c / (gamma - 1.0) * ((p / pk) ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)


def star_state(left, right, gamma):
    """Star region of the Riemann problem.

    left, right: (rho, u, p).  Returns dict with p_star, u_star, rho_star_L,
    rho_star_R and the wave speeds (head/tail of a rarefaction or the shock
    speed) on each side.
    """
    rL, uL, pL = map(float, left)
    rR, uR, pR = map(float, right)
    g = float(gamma)

    def f(p):
        return _fK(p, rL, pL, g) + _fK(p, rR, pR, g) + (uR - uL)

    lo, hi = 1e-14, max(pL, pR)
    while f(hi) < 0.0:
        hi *= 2.0
    p = brentq(f, lo, hi, xtol=1e-15, rtol=4 * np.finfo(float).eps, maxiter=500)
    u = 0.5 * (uL + uR) + 0.5 * (_fK(p, rR, pR, g) - _fK(p, rL, pL, g))
    gm = (g - 1.0) / (g + 1.0)
    cL, cR = math.sqrt(g * pL / rL), math.sqrt(g * pR / rR)
    out = dict(p_star=p, u_star=u)
    if p > pL:
        out["rho_star_L"] = rL * (p / pL + gm) / (gm * p / pL + 1.0)
        out["S_L"] = uL - cL * math.sqrt((g + 1.0) / (2 * g) * p / pL + (g - 1.0) / (2 * g))
        out["left_wave"] = "shock"
    else:
        out["rho_star_L"] = rL * (p / pL) ** (1.0 / g)
        cs = cL * (p / pL) ** ((g - 1.0) / (2 * g))
        out["S_HL"] = uL - cL
        out["S_TL"] = u - cs
        out["left_wave"] = "rarefaction"
    if p > pR:
        out["rho_star_R"] = rR * (p / pR + gm) / (gm * p / pR + 1.0)
        out["S_R"] = uR + cR * math.sqrt((g + 1.0) / (2 * g) * p / pR + (g - 1.0) / (2 * g))
        out["right_wave"] = "shock"
    else:
        out["rho_star_R"] = rR * (p / pR) ** (1.0 / g)
        cs = cR * (p / pR) ** ((g - 1.0) / (2 * g))
        out["S_HR"] = uR + cR
        out["S_TR"] = u + cs
        out["right_wave"] = "rarefaction"
    return out


def sample(xi, left, right, gamma):
    """(rho, u, p) at similarity coordinates xi = (x - x0)/t (array)."""
    st = star_state(left, right, gamma)
    rL, uL, pL = map(float, left)
    rR, uR, pR = map(float, right)
    g = float(gamma)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    cL, cR = math.sqrt(g * pL / rL), math.sqrt(g * pR / rR)
    us, ps = st["u_star"], st["p_star"]
    for k, s in np.ndenumerate(xi):
        if s <= us:  # left of the contact
            if st["left_wave"] == "shock":
                if s <= st["S_L"]:
                    val = (rL, uL, pL)
                else:
                    val = (st["rho_star_L"], us, ps)
            else:
                if s <= st["S_HL"]:
                    val = (rL, uL, pL)
                elif s >= st["S_TL"]:
                    val = (st["rho_star_L"], us, ps)
                else:  # inside the left fan
                    c = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * (uL - s))
                    uu = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * uL + s)
                    rr = rL * (c / cL) ** (2.0 / (g - 1.0))
                    val = (rr, uu, pL * (c / cL) ** (2.0 * g / (g - 1.0)))
        else:
            if st["right_wave"] == "shock":
                if s >= st["S_R"]:
                    val = (rR, uR, pR)
                else:
                    val = (st["rho_star_R"], us, ps)
            else:
                if s >= st["S_HR"]:
                    val = (rR, uR, pR)
                elif s <= st["S_TR"]:
                    val = (st["rho_star_R"], us, ps)
                else:
                    c = 2.0 / (g + 1.0) * (cR - 0.5 * (g - 1.0) * (uR - s))
                    uu = 2.0 / (g + 1.0) * (-cR + 0.5 * (g - 1.0) * uR + s)
                    rr = rR * (c / cR) ** (2.0 / (g - 1.0))
                    val = (rr, uu, pR * (c / cR) ** (2.0 * g / (g - 1.0)))
        rho[k], u[k], p[k] = val
    return rho, u, p
