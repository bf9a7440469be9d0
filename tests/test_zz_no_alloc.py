"""The allocation-free entry point sph_reduce_noalloc against sph_reduce on
the same particles, through the C ABI: two calls in a row, the second on a
smaller set, must give sph_reduce's sums bit for bit (the same kernels and
summation order; the partials sit in the library's file-scope device array
instead of context scratch)."""
import numpy as np
import pytest

from paper_1909_07439_amd import inputs, sph

from gpu_util import say

pytestmark = pytest.mark.gpu


def evaluated(cfg):
    p = sph.make_params(cfg, sph.SPH_PREC_MIXED)
    parts = sph.Particles(cfg)
    ctx = sph.Context(p, cfg["n"])
    sph.sph_build_tree(ctx, parts)
    sph.sph_density(ctx, parts)
    sph.sph_force(ctx, parts)
    sph.sph_check(ctx)
    return ctx, parts


def test_reduce_noalloc_matches_reduce_twice():
    import torch

    big = inputs.lattice(24, jitter=0.3, velocities=True)
    small = inputs.lattice(10, jitter=0.2, velocities=True, seed_variant=3)
    for cfg in (big, small):
        say(f"[noalloc] {cfg['workload']} n={cfg['n']}")
        ctx, parts = evaluated(cfg)
        ref = sph.sph_reduce(ctx, parts)
        torch.cuda.synchronize()
        got = sph.sph_reduce_noalloc(parts)
        say(f"  E={ref[0]:.15e} sum m a={ref[6]:.3e} dE/dt={ref[9]:.3e}")
        assert np.all(np.isfinite(ref))
        np.testing.assert_array_equal(got, ref)
        ctx.close()


def test_reduce_noalloc_rejects_bad_sizes():
    p = sph.sph_particles()
    p.n = 0
    with pytest.raises(sph.SphError):
        sph.sph_reduce_noalloc(type("P", (), {"c": p})())
