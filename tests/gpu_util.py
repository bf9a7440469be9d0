"""Helpers for the GPU parity tests: run the library through its C ABI and
bring results back in the caller's original particle order (by id)."""
import sys

import numpy as np

from paper_1909_07439_amd import sph


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_orig(out: dict) -> dict:
    """Fields indexed by the original particle id."""
    ids = out["id"]
    res = {}
    for k, v in out.items():
        a = np.empty_like(v)
        a[ids] = v
        res[k] = a
    res["slot_of"] = np.empty_like(ids)
    res["slot_of"][ids] = np.arange(ids.size)
    return res


def gpu_eval(cfg: dict, precision=sph.SPH_PREC_FP64, **over):
    """build_tree + density + force on the GPU; returns (fields by id, ctx, parts, info)."""
    say(f"[gpu_eval] {cfg.get('workload')} n={cfg['n']} precision={precision} {over}")
    p = sph.make_params(cfg, precision, **over)
    parts = sph.Particles(cfg)
    ctx = sph.Context(p, cfg["n"])
    sph.sph_build_tree(ctx, parts)
    iters = sph.sph_density(ctx, parts, want_iters=True)
    dt = sph.sph_force(ctx, parts, want_dt=True)
    info = dict(iters=iters, dt=dt, stats=sph.sph_stats(ctx))
    return to_orig(parts.numpy()), ctx, parts, info


def rel_err(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)
