"""Seeded synthetic particle sets for the SPH hydro step.

This module only lays particles out (lattices, jitter, velocity fields) and
fills in the run parameters; it contains none of the SPH arithmetic.  Both the
GPU library's tests/benchmark and the CPU oracle take their inputs from here.

The paper built its initial conditions with another code's setup programs
(Sect. 4); those are not available, so these generators stand in for them with
the paper's shapes and contrasts:

* ``lattice``          -- periodic unit cube, jittered cubic lattice, uniform
                          density (plain-method workload, 32^3 by default);
* ``sod``              -- 3D shock tube of Sect. 4 (left [rho,P]=[1,1], right
                          [0.125,0.1]; density set by a lattice spacing ratio 2);
* ``kelvin_helmholtz`` -- shear layer of Sect. 4 (dense band |y-1/2|<1/4
                          moving at +0.5, the rest at -0.5, P=2.5), density
                          contrast by a particle-mass ratio on one lattice;
* ``turbulent_box``    -- periodic cube with a Gaussian random solenoidal
                          velocity field, P(k) ~ k^-4 on 1 <= |k| <= 8.

Seeds are 1909 + 10*workload + variant (PCG64).  Every array is float64 in
the order the particles were laid out; ``id`` is 0..n-1.
"""
from __future__ import annotations

import math

import numpy as np

DEFAULTS = dict(
    gamma=5.0 / 3.0,
    gamma_minus_1=2.0 / 3.0,
    hfact=1.2,
    alpha_av=1.0,
    beta_av=2.0,
    alpha_u=1.0,
    c_cour=0.3,
    n_leaf=16,  # the paper's timing runs (Sect. 4.6)
    n_group=8,
    kernel=0,  # M4 cubic spline
)

# Smoothing kernels of Sect. 2.3 and the h_fact each is run with (the paper
# gives none): M4 with support 2h at 1.2 (about 58 neighbours), the M6 quintic
# with support 3h at 1.0 (about 113) and Wendland C6 with support 2h at 1.6
# (about 137).
KERNELS = {"m4": 0, "m6": 1, "wc6": 2}
KERNEL_HFACT = {0: 1.2, 1: 1.0, 2: 1.6}


def with_kernel(cfg: dict, kernel) -> dict:
    """A copy of workload ``cfg`` run with another smoothing kernel: the
    kernel's h_fact, and start values of h scaled by the h_fact ratio."""
    kind = KERNELS[kernel] if isinstance(kernel, str) else int(kernel)
    out = dict(cfg)
    hf = KERNEL_HFACT[kind]
    out["h"] = np.ascontiguousarray(cfg["h"] * (hf / cfg["hfact"]))
    out["hfact"] = hf
    out["kernel"] = kind
    out["workload"] = cfg["workload"] + ("" if kind == 0 else {1: "_m6", 2: "_wc6"}[kind])
    return out


def _rng(workload: int, variant: int = 0) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(1909 + 10 * workload + variant))


def _wrap(v: np.ndarray, lo: float, length: float) -> np.ndarray:
    v = lo + np.mod(v - lo, length)
    v[v >= lo + length] -= length
    v[v < lo] += length
    return v


def _grid(nx: int, ny: int, nz: int):
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    return (i.ravel().astype(np.float64), j.ravel().astype(np.float64),
            k.ravel().astype(np.float64))


def _finish(cfg: dict, arrays: dict) -> dict:
    n = arrays["x"].size
    out = dict(DEFAULTS)
    out.update(cfg)
    for k in ("x", "y", "z", "vx", "vy", "vz", "m", "u", "h"):
        out[k] = np.ascontiguousarray(arrays[k], dtype=np.float64)
    for k in ("ax", "ay", "az", "dudt"):
        out[k] = np.zeros(n)
    out["id"] = np.arange(n, dtype=np.int64)
    out["n"] = n
    return out


def lattice(n_side: int = 32, jitter: float = 0.05, velocities: bool = False,
            seed_variant: int = 0) -> dict:
    """Jittered cubic lattice in the periodic unit cube, total mass 1, u=1.

    Site (i,j,k) sits at ((i+1/2)/n, ...) plus a uniform offset in
    [-jitter, jitter] lattice spacings per coordinate.  With ``velocities``
    each velocity component is uniform in +-0.1 of the sound speed at u=1 and
    u = 1 + U(-0.1, 0.1), which switches on viscosity and conductivity.
    """
    rng = _rng(1, seed_variant + (1 if velocities else 0))
    n = n_side ** 3
    dx = 1.0 / n_side
    i, j, k = _grid(n_side, n_side, n_side)
    pos = [(c + 0.5) * dx + rng.uniform(-jitter, jitter, n) * dx for c in (i, j, k)]
    pos = [_wrap(p, 0.0, 1.0) for p in pos]
    cfg = dict(box_lo=(0.0, 0.0, 0.0), box_len=(1.0, 1.0, 1.0), periodic=(1, 1, 1),
               workload=f"lattice{n_side}" + ("v" if velocities else ""), dx=dx)
    g = DEFAULTS["gamma"]
    if velocities:
        c0 = math.sqrt(g * (g - 1.0) * 1.0)
        v = [rng.uniform(-0.1, 0.1, n) * c0 for _ in range(3)]
        u = 1.0 + rng.uniform(-0.1, 0.1, n)
    else:
        v = [np.zeros(n) for _ in range(3)]
        u = np.ones(n)
    arrays = dict(x=pos[0], y=pos[1], z=pos[2], vx=v[0], vy=v[1], vz=v[2],
                  m=np.full(n, 1.0 / n), u=u, h=np.full(n, DEFAULTS["hfact"] * dx))
    return _finish(cfg, arrays)


def adjoint_lattice(n_side: int = 64) -> dict:
    """Workload of the rollout gradient: the jittered lattice (+-0.05
    spacings) with seeded velocities (each component uniform in +-0.1 of the
    sound speed) and u on two levels, 1 and 1.2, at random.  At v = 0 every
    pair would sit on the viscosity switch (w = 0), where the loss has no
    derivative in v; with u on two levels the conductivity's sqrt|P_i - P_j|
    is far from its kink wherever u_i != u_j."""
    cfg = lattice(n_side, jitter=0.05, velocities=True)
    rng = _rng(4, 0)
    cfg["u"] = np.where(rng.random(cfg["n"]) < 0.5, 1.0, 1.2)
    cfg["workload"] = f"adjoint_lattice{n_side}"
    return cfg


def sod(dx_left: float = 1.0 / 512, width: float = 1.0 / 16, gamma: float = 5.0 / 3.0) -> dict:
    """Shock tube on [-1/2,1/2] x [-w/2,w/2]^2, periodic on all axes.

    Left (x<0): rho=1, P=1 on a lattice of spacing dx_left.  Right: rho=0.125,
    P=0.1 on spacing 2*dx_left.  Equal particle masses rho_L dx_left^3.  With
    the defaults: 256x32x32 + 128x16x16 = 294,912 particles.
    """
    dl, dr = dx_left, 2.0 * dx_left
    gm1 = gamma - 1.0
    nxl, nyl = int(round(0.5 / dl)), int(round(width / dl))
    nxr, nyr = int(round(0.5 / dr)), int(round(width / dr))
    il, jl, kl = _grid(nxl, nyl, nyl)
    ir, jr, kr = _grid(nxr, nyr, nyr)
    x = np.concatenate([-0.5 + (il + 0.5) * dl, (ir + 0.5) * dr])
    y = np.concatenate([-0.5 * width + (jl + 0.5) * dl, -0.5 * width + (jr + 0.5) * dr])
    z = np.concatenate([-0.5 * width + (kl + 0.5) * dl, -0.5 * width + (kr + 0.5) * dr])
    nl, nr = il.size, ir.size
    m = 1.0 * dl ** 3
    u = np.concatenate([np.full(nl, 1.0 / (gm1 * 1.0)), np.full(nr, 0.1 / (gm1 * 0.125))])
    h = np.concatenate([np.full(nl, DEFAULTS["hfact"] * dl), np.full(nr, DEFAULTS["hfact"] * dr)])
    n = nl + nr
    cfg = dict(box_lo=(-0.5, -0.5 * width, -0.5 * width), box_len=(1.0, width, width),
               periodic=(1, 1, 1), gamma=gamma, gamma_minus_1=gm1,
               workload=f"sod_dx{int(round(1 / dl))}_w{int(round(1 / width))}",
               left=(1.0, 0.0, 1.0), right=(0.125, 0.0, 0.1), n_left=nl, n_right=nr)
    arrays = dict(x=x, y=y, z=z, vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n),
                  m=np.full(n, m), u=u, h=h)
    return _finish(cfg, arrays)


def blast_wave(dx: float = 1.0 / 800, half_length: float = 1.0, n_cross: int = 12,
               gamma: float = 1.4) -> dict:
    """Blast-wave tube (Sect. 4.2): [rho, P] = [1, 1000] for x <= 0 and
    [1, 0.1] for x > 0, gamma = 7/5, both states on one cubic lattice of
    spacing dx (equal densities), n_cross x n_cross particles across.

    The box is [-half_length, half_length] x [-w/2, w/2]^2 (w = n_cross dx),
    periodic on all axes: the periodic copy of the interface at x = +-half_length
    starts a mirrored Riemann problem whose waves, with the default
    half_length = 1, stay clear of |x| < 0.5 until after t = 0.01 (the
    rarefaction heads move at c_L = 37.4).  With the defaults: 1600 x 12 x 12
    = 230,400 particles, 400 per unit length as in the paper.
    """
    gm1 = gamma - 1.0
    nx = int(round(2.0 * half_length / dx))
    i, j, k = _grid(nx, n_cross, n_cross)
    w = n_cross * dx
    x = -half_length + (i + 0.5) * dx
    y = -0.5 * w + (j + 0.5) * dx
    z = -0.5 * w + (k + 0.5) * dx
    n = x.size
    left = x <= 0.0
    u = np.where(left, 1000.0 / gm1, 0.1 / gm1)
    cfg = dict(box_lo=(-half_length, -0.5 * w, -0.5 * w), box_len=(2.0 * half_length, w, w),
               periodic=(1, 1, 1), gamma=gamma, gamma_minus_1=gm1,
               workload=f"blast_dx{int(round(1 / dx))}",
               left=(1.0, 0.0, 1000.0), right=(1.0, 0.0, 0.1), dx=dx)
    arrays = dict(x=x, y=y, z=z, vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n),
                  m=np.full(n, dx ** 3), u=u, h=np.full(n, DEFAULTS["hfact"] * dx))
    return _finish(cfg, arrays)


def sedov(n_side: int = 100, energy: float = 1.0, r_inject: float = 2.0,
          u_ambient: float = 1e-6, gamma: float = 5.0 / 3.0) -> dict:
    """Sedov-Taylor blast (Sect. 4.3): a uniform periodic unit cube (rho = 1)
    on an n_side^3 cubic lattice, at rest, with the energy ``energy`` shared
    equally (as u) by the particles within r_inject lattice spacings of the
    centre; every other particle has u = u_ambient (a pressure 10^-6 of the
    post-shock pressure at t = 0.1, so the shock stays strong).  With the
    defaults the shock reaches R = 1.1517 (E t^2)^(1/5) = 0.458 at t = 0.1,
    inside the box."""
    gm1 = gamma - 1.0
    dx = 1.0 / n_side
    i, j, k = _grid(n_side, n_side, n_side)
    x, y, z = (i + 0.5) * dx, (j + 0.5) * dx, (k + 0.5) * dx
    n = x.size
    m = np.full(n, dx ** 3)
    r = np.sqrt((x - 0.5) ** 2 + (y - 0.5) ** 2 + (z - 0.5) ** 2)
    hot = r < r_inject * dx
    u = np.full(n, u_ambient)
    u[hot] = energy / (m[hot].sum())
    cfg = dict(box_lo=(0.0, 0.0, 0.0), box_len=(1.0, 1.0, 1.0), periodic=(1, 1, 1),
               gamma=gamma, gamma_minus_1=gm1, workload=f"sedov{n_side}", dx=dx,
               energy=energy, centre=(0.5, 0.5, 0.5), n_hot=int(hot.sum()))
    arrays = dict(x=x, y=y, z=z, vx=np.zeros(n), vy=np.zeros(n), vz=np.zeros(n), m=m, u=u,
                  h=np.full(n, DEFAULTS["hfact"] * dx))
    return _finish(cfg, arrays)


def kelvin_helmholtz(n_side: int = 100, jitter: float = 0.02) -> dict:
    """Shear layer in the periodic unit cube.

    One jittered lattice (n_side^3).  Sites with |y_site - 1/2| < 1/4 carry
    mass 2/N and move at v_x=+0.5 (rho=2); the rest carry 1/N at v_x=-0.5
    (rho=1).  P=2.5 everywhere; v_y = 0.01 sin(4 pi x).
    """
    rng = _rng(3)
    n = n_side ** 3
    dx = 1.0 / n_side
    i, j, k = _grid(n_side, n_side, n_side)
    sites = [(c + 0.5) * dx for c in (i, j, k)]
    pos = [_wrap(s + rng.uniform(-jitter, jitter, n) * dx, 0.0, 1.0) for s in sites]
    band = np.abs(sites[1] - 0.5) < 0.25
    g = DEFAULTS["gamma"]
    rho = np.where(band, 2.0, 1.0)
    m = np.where(band, 2.0 / n, 1.0 / n)
    vx = np.where(band, 0.5, -0.5)
    vy = 0.01 * np.sin(4.0 * np.pi * pos[0])
    u = 2.5 / ((g - 1.0) * rho)
    cfg = dict(box_lo=(0.0, 0.0, 0.0), box_len=(1.0, 1.0, 1.0), periodic=(1, 1, 1),
               workload=f"kh{n_side}", dx=dx)
    arrays = dict(x=pos[0], y=pos[1], z=pos[2], vx=vx, vy=vy, vz=np.zeros(n), m=m, u=u,
                  h=np.full(n, DEFAULTS["hfact"] * dx))
    return _finish(cfg, arrays)


def turbulent_box(n_side: int = 256, jitter: float = 0.05, kmin: float = 1.0,
                  kmax: float = 8.0, mach: float = 1.0, gamma: float = 1.0001,
                  gamma_minus_1: float = 1e-4) -> dict:
    """Periodic unit cube, rho=1, Gaussian random solenoidal velocity.

    Fourier amplitudes |v(k)|^2 ~ k^-4 for kmin <= |k| L / 2pi <= kmax, random
    phases, projected onto k.v = 0, real by Hermitian symmetry (irfftn),
    sampled at each particle's lattice site and scaled to rms |v| = mach
    (sound speed 1, so u = 1/(gamma (gamma-1))).
    """
    rng = _rng(5)
    n = n_side ** 3
    dx = 1.0 / n_side
    kf = np.fft.fftfreq(n_side, d=1.0 / n_side)
    kz = np.fft.rfftfreq(n_side, d=1.0 / n_side)
    KX, KY, KZ = np.meshgrid(kf, kf, kz, indexing="ij")
    K2 = KX ** 2 + KY ** 2 + KZ ** 2
    kk = np.sqrt(K2)
    shell = (kk >= kmin) & (kk <= kmax)
    amp = np.zeros_like(kk)
    amp[shell] = kk[shell] ** -2.0  # |v_k| ~ k^-2  ->  |v_k|^2 ~ k^-4
    comps = []
    for _ in range(3):
        re = rng.standard_normal(kk.shape)
        im = rng.standard_normal(kk.shape)
        comps.append((re + 1j * im) * amp)
    K2s = np.where(K2 > 0, K2, 1.0)
    dot = (comps[0] * KX + comps[1] * KY + comps[2] * KZ) / K2s
    comps = [comps[0] - dot * KX, comps[1] - dot * KY, comps[2] - dot * KZ]
    del dot, K2s, KX, KY, KZ, K2, kk, shell, amp
    vel = [np.fft.irfftn(c, s=(n_side, n_side, n_side), axes=(0, 1, 2)).ravel() for c in comps]
    del comps
    rms = math.sqrt(float(np.mean(vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)))
    vel = [v * (mach / rms) for v in vel]
    i, j, k = _grid(n_side, n_side, n_side)
    pos = [_wrap((c + 0.5) * dx + rng.uniform(-jitter, jitter, n) * dx, 0.0, 1.0)
           for c in (i, j, k)]
    u = np.full(n, 1.0 / (gamma * gamma_minus_1))
    cfg = dict(box_lo=(0.0, 0.0, 0.0), box_len=(1.0, 1.0, 1.0), periodic=(1, 1, 1),
               gamma=gamma, gamma_minus_1=gamma_minus_1, workload=f"turb{n_side}", dx=dx)
    arrays = dict(x=pos[0], y=pos[1], z=pos[2], vx=vel[0], vy=vel[1], vz=vel[2],
                  m=np.full(n, 1.0 / n), u=u, h=np.full(n, DEFAULTS["hfact"] * dx))
    return _finish(cfg, arrays)


def subset_params(cfg: dict) -> dict:
    """Only the run parameters of a workload dict (no arrays)."""
    return {k: v for k, v in cfg.items() if not isinstance(v, np.ndarray)}
