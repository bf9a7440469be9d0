"""Reference gradients of the SPH evaluation and of leapfrog rollouts.

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle``: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
use it.

The forward equations of Sect. 2.2-2.6 (density sums, grad-h term, equation
of state, momentum and energy equations with viscosity and conductivity) and
of the leapfrog (Sect. 2.4, eq:predict_pos, eq:predict_vel, eq:correct_vel)
are written out in plain PyTorch float64 CPU operations, and torch.autograd
differentiates them.  Three things are held fixed, as the adjoint does:

* the neighbour sets: those of the FP64 C oracle at the forward's smoothing
  lengths (a pair that enters or leaves a set has W = F = 0 there, so the
  loss is continuous across such events);
* the step dt (the Courant minimum is not smooth);
* the switches of the viscosity (approaching pairs, w < 0).

The smoothing length is the root of f(h) = S0(h) - m (hfact/h)^3 (Sect. 2.2).
Its value is the C oracle's root; its derivative is the implicit one,
dh = -(df/dx) dx / (df/dh), carried by adding -f/f' (value zero at the root,
gradient -(df/dx)/f' with f' held constant) to the root.

The functions here are pinned by tests/test_oracle_adjoint.py: the kernel
polynomials against the C oracle, the forward values against the C oracle's
evaluation and step, and the gradients against central finite differences of
the C oracle's rollout (which re-solves h and re-finds the neighbours).
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import density, make_params, neighbours

M4, M6, WENDLAND_C6 = 0, 1, 2
SUPPORT = {M4: 2.0, M6: 3.0, WENDLAND_C6: 2.0}
NORM = {M4: 1.0 / math.pi, M6: 1.0 / (120.0 * math.pi), WENDLAND_C6: 1365.0 / (512.0 * math.pi)}


def _pos(t):
    return torch.clamp(t, min=0.0)


def kernel_f(kind: int, q):
    """Dimensionless kernel shape f(q), W = C f(r/h) / h^3 (Sect. 2.3)."""
    if kind == M6:
        return _pos(3.0 - q) ** 5 - 6.0 * _pos(2.0 - q) ** 5 + 15.0 * _pos(1.0 - q) ** 5
    if kind == WENDLAND_C6:
        s = _pos(1.0 - 0.5 * q)
        return s ** 8 * (((4.0 * q + 6.25) * q + 4.0) * q + 1.0)
    inner = 1.0 - 1.5 * q * q + 0.75 * q ** 3
    outer = 0.25 * _pos(2.0 - q) ** 3
    return torch.where(q < 1.0, inner, outer)


def kernel_df(kind: int, q):
    """df/dq, written out (pinned against autograd of kernel_f)."""
    if kind == M6:
        return -5.0 * _pos(3.0 - q) ** 4 + 30.0 * _pos(2.0 - q) ** 4 - 75.0 * _pos(1.0 - q) ** 4
    if kind == WENDLAND_C6:
        s = _pos(1.0 - 0.5 * q)
        g = ((4.0 * q + 6.25) * q + 4.0) * q + 1.0
        dg = (12.0 * q + 12.5) * q + 4.0
        return s ** 7 * (-4.0 * g + s * dg)
    inner = -3.0 * q + 2.25 * q * q
    outer = -0.75 * _pos(2.0 - q) ** 2
    return torch.where(q < 1.0, inner, outer)


def kernel_w(kind, r, h):
    return NORM[kind] * kernel_f(kind, r / h) / h ** 3


def kernel_F(kind, r, h):
    """dW/dr."""
    return NORM[kind] * kernel_df(kind, r / h) / h ** 4


def kernel_dwdh(kind, r, h):
    q = r / h
    return -NORM[kind] * (3.0 * kernel_f(kind, q) + q * kernel_df(kind, q)) / h ** 4


def _fold(d, length, periodic):
    if not periodic:
        return d
    half = 0.5 * length
    return torch.where(d > half, d - length, torch.where(d < -half, d + length, d))


def _wrap(x, lo, length, periodic):
    if not periodic:
        return x
    return torch.where(x >= lo + length, x - length, torch.where(x < lo, x + length, x))


def _pairs(off, idx, drop_self):
    off = np.asarray(off)
    I = np.repeat(np.arange(off.size - 1), np.diff(off))
    J = np.asarray(idx)
    if drop_self:
        keep = I != J
        I, J = I[keep], J[keep]
    return torch.from_numpy(I.astype(np.int64)), torch.from_numpy(J.astype(np.int64))


class Frozen:
    """What the forward fixes for one evaluation: the root h and the two
    neighbour sets at that h, found by the C oracle."""

    def __init__(self, cfg, params, x, y, z, m, h_start):
        arr = [np.ascontiguousarray(t.detach().numpy()) for t in (x, y, z)]
        d = density(arr[0], arr[1], arr[2], m, h_start, params)
        self.h = d["h"]
        off, idx = neighbours(arr[0], arr[1], arr[2], self.h, params, mode=0)
        self.dI, self.dJ = _pairs(off, idx, drop_self=True)
        off, idx = neighbours(arr[0], arr[1], arr[2], self.h, params, mode=1)
        self.fI, self.fJ = _pairs(off, idx, drop_self=False)


def _sep(cfg, I, J, x, y, z):
    L, per = cfg["box_len"], cfg["periodic"]
    dx = _fold(x[I] - x[J], L[0], per[0])
    dy = _fold(y[I] - y[J], L[1], per[1])
    dz = _fold(z[I] - z[J], L[2], per[2])
    return dx, dy, dz


def _density_sums(kind, cfg, fr, x, y, z, m, h):
    """S0_i = sum_j m_j W(r_ij, h_i), S1_i = sum_j m_j dW/dh (r_ij, h_i),
    j over the density set (self included: r = 0)."""
    n = m.shape[0]
    I, J = fr.dI, fr.dJ
    dx, dy, dz = _sep(cfg, I, J, x, y, z)
    r = torch.sqrt(dx * dx + dy * dy + dz * dz)
    hi = h[I]
    zero = torch.zeros(n, dtype=torch.float64)
    S0 = m * kernel_w(kind, zero, h) + zero.index_add(0, I, m[J] * kernel_w(kind, r, hi))
    S1 = m * kernel_dwdh(kind, zero, h) + zero.index_add(0, I, m[J] * kernel_dwdh(kind, r, hi))
    return S0, S1


def evaluate(cfg, params, state, fr=None, kind=None):
    """One evaluation (density at the root h, EOS, force) as a differentiable
    function of the tensors state['x','y','z','vx','vy','vz','u'].

    Returns dict of tensors ax, ay, az, dudt, h, rho, omega, P, cs and the
    Frozen record used.
    """
    kind = cfg.get("kernel", 0) if kind is None else kind
    x, y, z = state["x"], state["y"], state["z"]
    vx, vy, vz, u = state["vx"], state["vy"], state["vz"], state["u"]
    m = torch.as_tensor(np.asarray(cfg["m"], dtype=np.float64))
    if fr is None:
        fr = Frozen(cfg, params, x, y, z, np.asarray(cfg["m"], dtype=np.float64),
                    np.asarray(state["h_start"], dtype=np.float64))
    hfact = float(cfg["hfact"])
    hs = torch.from_numpy(fr.h.copy())
    # implicit derivative of the root
    S0, S1 = _density_sums(kind, cfg, fr, x, y, z, m, hs)
    rho_h = m * (hfact / hs) ** 3
    f = S0 - rho_h
    fp = (S1 + 3.0 * rho_h / hs).detach()
    delta = -f / fp
    h = hs + (delta - delta.detach())
    S0, S1 = _density_sums(kind, cfg, fr, x, y, z, m, h)
    rho = S0
    omega = 1.0 + h * S1 / (3.0 * rho)
    gm1, gamma = float(cfg["gamma_minus_1"]), float(cfg["gamma"])
    P = gm1 * rho * u
    cs = torch.sqrt(gamma * gm1 * u)
    al, be, au = float(cfg["alpha_av"]), float(cfg["beta_av"]), float(cfg["alpha_u"])

    I, J = fr.fI, fr.fJ
    dx, dy, dz = _sep(cfg, I, J, x, y, z)
    r = torch.sqrt(dx * dx + dy * dy + dz * dz)
    ex, ey, ez = dx / r, dy / r, dz / r
    w = (vx[I] - vx[J]) * ex + (vy[I] - vy[J]) * ey + (vz[I] - vz[J]) * ez
    Fi = kernel_F(kind, r, h[I])
    Fj = kernel_F(kind, r, h[J])
    appr = w < 0.0  # the viscosity switch, held fixed
    zero_p = torch.zeros_like(w)
    vsi = torch.where(appr, al * cs[I] + be * torch.abs(w), zero_p)
    vsj = torch.where(appr, al * cs[J] + be * torch.abs(w), zero_p)
    qi = -0.5 * rho[I] * vsi * w
    qj = -0.5 * rho[J] * vsj * w
    ti = (P[I] + qi) / (rho[I] * rho[I] * omega[I]) * Fi
    tj = (P[J] + qj) / (rho[J] * rho[J] * omega[J]) * Fj
    pa = m[J] * (ti + tj)
    gi = P[I] / (rho[I] * rho[I] * omega[I])
    ki = 1.0 / (omega[I] * rho[I])
    kj = 1.0 / (omega[J] * rho[J])
    e1 = gi * m[J] * w * Fi
    e2 = -ki * m[J] * vsi * 0.5 * w * w * Fi
    rbar = 0.5 * (rho[I] + rho[J])
    dP = torch.abs(P[I] - P[J])
    # sqrt has no derivative at 0: where P_i = P_j the term's derivative is
    # taken as zero (the subgradient the GPU adjoint uses as well)
    safe = dP > 0.0
    vu = torch.where(safe, torch.sqrt(torch.where(safe, dP, torch.ones_like(dP)) / rbar), zero_p)
    e3 = m[J] * au * vu * (u[I] - u[J]) * 0.5 * (Fi * ki + Fj * kj)
    n = m.shape[0]
    zero = torch.zeros(n, dtype=torch.float64)
    ax = -zero.index_add(0, I, pa * ex)
    ay = -zero.index_add(0, I, pa * ey)
    az = -zero.index_add(0, I, pa * ez)
    du = zero.index_add(0, I, e1 + e2 + e3)
    return dict(ax=ax, ay=ay, az=az, dudt=du, h=h, rho=rho, omega=omega, P=P, cs=cs, frozen=fr)


def _leaf(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), requires_grad=True)


def rollout(cfg, dt, K, kind=None):
    """Initial evaluation and K leapfrog steps of fixed dt from cfg's state,
    built as one autograd graph.  Returns (inputs, outputs): inputs are leaf
    tensors x, y, z, vx, vy, vz, u; outputs the final state tensors x, y, z,
    vx, vy, vz, u, ax, ay, az, dudt, in the input particle order."""
    params = make_params(cfg)
    L, lo, per = cfg["box_len"], cfg["box_lo"], cfg["periodic"]
    inp = {k: _leaf(cfg[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "u")}
    s = dict(inp)
    s["h_start"] = np.asarray(cfg["h"], dtype=np.float64)
    e = evaluate(cfg, params, s, kind=kind)
    a = {k: e[k] for k in ("ax", "ay", "az", "dudt")}
    h = e["frozen"].h
    for _ in range(K):
        # predictor (eq:predict_pos, eq:predict_vel; u likewise)
        p = {}
        for ax_i, (c, v, acc) in enumerate((("x", "vx", "ax"), ("y", "vy", "ay"),
                                            ("z", "vz", "az"))):
            p[c] = _wrap(s[c] + (s[v] * dt + (0.5 * dt * dt) * a[acc]), lo[ax_i], L[ax_i],
                         per[ax_i])
            p[v] = s[v] + a[acc] * dt
        p["u"] = s["u"] + a["dudt"] * dt
        p["h_start"] = h
        e = evaluate(cfg, params, p, kind=kind)
        h = e["frozen"].h
        # corrector (eq:correct_vel; u likewise)
        hdt = 0.5 * dt
        nxt = {c: p[c] for c in ("x", "y", "z")}
        for v, acc in (("vx", "ax"), ("vy", "ay"), ("vz", "az"), ("u", "dudt")):
            nxt[v] = p[v] + (e[acc] - a[acc]) * hdt
        a = {k: e[k] for k in ("ax", "ay", "az", "dudt")}
        s = nxt
    out = {k: s[k] for k in ("x", "y", "z", "vx", "vy", "vz", "u")}
    out.update(a)
    return inp, out


def loss_of(cfg, out):
    """sum m |a|^2 at the final state plus the final kinetic energy."""
    m = torch.as_tensor(np.asarray(cfg["m"], dtype=np.float64))
    acc = out["ax"] ** 2 + out["ay"] ** 2 + out["az"] ** 2
    ke = 0.5 * (out["vx"] ** 2 + out["vy"] ** 2 + out["vz"] ** 2)
    return torch.sum(m * acc) + torch.sum(m * ke)


def rollout_grad(cfg, dt, K, kind=None):
    """Gradient of loss_of after K steps w.r.t. the initial x, y, z, vx, vy,
    vz, u (numpy arrays, input particle order), and the loss."""
    inp, out = rollout(cfg, dt, K, kind=kind)
    L = loss_of(cfg, out)
    keys = ("x", "y", "z", "vx", "vy", "vz", "u")
    g = torch.autograd.grad(L, [inp[k] for k in keys])
    return {k: gi.numpy() for k, gi in zip(keys, g)}, float(L.detach())


def eval_vjp(cfg, cot, kind=None):
    """Cotangents of one evaluation's inputs (x, y, z, vx, vy, vz, u) for
    the cotangents ``cot`` of its outputs ax, ay, az, dudt."""
    params = make_params(cfg)
    inp = {k: _leaf(cfg[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "u")}
    s = dict(inp)
    s["h_start"] = np.asarray(cfg["h"], dtype=np.float64)
    e = evaluate(cfg, params, s, kind=kind)
    outs = [e[k] for k in ("ax", "ay", "az", "dudt")]
    gos = [torch.as_tensor(np.asarray(cot[k], dtype=np.float64)) for k in ("ax", "ay", "az", "dudt")]
    keys = ("x", "y", "z", "vx", "vy", "vz", "u")
    g = torch.autograd.grad(outs, [inp[k] for k in keys], grad_outputs=gos)
    return {k: gi.numpy() for k, gi in zip(keys, g)}, {k: e[k].detach().numpy() for k in
                                                      ("ax", "ay", "az", "dudt", "h", "rho")}
