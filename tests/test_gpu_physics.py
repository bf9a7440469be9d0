"""Whole-step behaviour on the GPU: the shock tube against its exact Riemann
solution (Sect. 4, Sod test), total energy and momentum over the run
(Sect. 4.5, eq:energy_error), and several leapfrog steps against the oracle.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import riemann
from paper_1909_07439_amd import inputs, sph

from gpu_util import say, to_orig

pytestmark = pytest.mark.gpu


def sod_exact_periodic(x, t, gamma):
    L, R = (1.0, 0.0, 1.0), (0.125, 0.0, 0.1)
    xm = np.where(x > 0.25, x - 0.5, np.where(x < -0.25, x + 0.5, x))
    mirror = np.abs(x) > 0.25
    xi = np.where(mirror, -xm, xm) / t
    r, u, p = riemann.sample(xi, L, R, gamma)
    return r, np.where(mirror, -u, u), p


def run_to(cfg, precision, t_end):
    p = sph.make_params(cfg, precision)
    parts = sph.Particles(cfg)
    ctx = sph.Context(p, cfg["n"])
    sph.sph_build_tree(ctx, parts)
    sph.sph_density(ctx, parts, want_iters=True)
    dt = sph.sph_force(ctx, parts, want_dt=True)
    e0 = sph.sph_reduce(ctx, parts)
    t, steps = 0.0, 0
    while t < t_end - 1e-12:
        dt = min(dt, t_end - t)
        dt_next = sph.sph_step(ctx, parts, dt, want_dt=True)
        t += dt
        steps += 1
        dt = dt_next
    e1 = sph.sph_reduce(ctx, parts)
    return to_orig(parts.numpy()), e0, e1, steps


@pytest.mark.parametrize("precision", [sph.SPH_PREC_MIXED, sph.SPH_PREC_FP64])
def test_shock_tube_against_exact_solution(precision):
    cfg = inputs.sod()
    g, e0, e1, steps = run_to(cfg, precision, 0.1)
    x = g["x"]
    r, u, pr = sod_exact_periodic(x, 0.1, cfg["gamma"])
    regions = {"fan": (x > -0.11) & (x < -0.04), "post": (x > 0.10) & (x < 0.17),
               "left_star": (x > 0.0) & (x < 0.06), "far": (np.abs(x) > 0.2) & (np.abs(x) < 0.3),
               "all": np.abs(x) < 0.3}
    err = {}
    for name, m in regions.items():
        err[name] = (np.abs(g["rho"][m] - r[m]).mean(), np.abs(g["vx"][m] - u[m]).mean(),
                     np.abs(g["P"][m] - pr[m]).mean())
        say(f"  {name}: L1 rho {err[name][0]:.4f} v {err[name][1]:.4f} P {err[name][2]:.4f}")
    de = (e0[0] - e1[0]) / e0[0]
    say(f"  steps {steps}, dE = {de:.3e}, momentum {e1[3:6]}")
    mv = np.sum(g["m"] * np.sqrt(g["vx"] ** 2 + g["vy"] ** 2 + g["vz"] ** 2))
    say(f"  |momentum| / sum m|v| = {np.abs(e1[3:6]).max() / mv:.2e}")
    assert abs(de) < 2e-5
    assert np.abs(e1[3:6]).max() <= (1e-12 if precision == sph.SPH_PREC_FP64 else 1e-6) * mv
    # Bounds from the measured full-resolution runs (dx_L = 1/512), with a
    # margin: the undisturbed states and the right star state (post-shock)
    # follow the exact solution closely; the fan and the left star state
    # carry the resolution-independent offset of the M4 kernel on a lattice
    # stretched along x only (also shown by the oracle at dx_L = 1/128).
    assert err["far"][0] < 0.003 and err["far"][2] < 0.003
    assert err["post"][0] < 0.01 and err["post"][2] < 0.02 and err["post"][1] < 0.05
    assert err["fan"][0] < 0.03 and err["fan"][1] < 0.07 and err["fan"][2] < 0.04
    assert err["left_star"][0] < 0.08 and err["left_star"][2] < 0.09
    assert err["all"][0] < 0.025


def test_several_steps_fp64_match_oracle():
    cfg = inputs.sod(dx_left=1.0 / 64, width=0.25)
    op = oracle.make_params(cfg)
    s = oracle.evaluate(cfg, op)
    p = sph.make_params(cfg, sph.SPH_PREC_FP64)
    state = dict(cfg)
    for k in ("ax", "ay", "az", "dudt", "h"):
        state[k] = s[k]
    parts = sph.Particles(state)
    ctx = sph.Context(p, cfg["n"])
    dt = s["dt_next"]
    for step in range(8):
        s = oracle.step(s, dt, op)
        dtg = sph.sph_step(ctx, parts, dt, want_dt=True)
        assert abs(dtg - s["dt_next"]) <= 1e-11 * s["dt_next"]
        dt = s["dt_next"]
    g = to_orig(parts.numpy())
    for k in ("x", "y", "z", "vx", "u", "rho", "h"):
        e = np.abs(g[k] - s[k]).max() / max(np.abs(s[k]).max(), 1e-300)
        say(f"  after 8 steps {k}: {e:.2e}")
        assert e < 1e-10, k
