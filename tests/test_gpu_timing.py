"""Phase timings (sph_timings) and their sampling over sph_step calls
(sph_set_timing)."""
import pytest

from paper_1909_07439_amd import inputs, sph

pytestmark = pytest.mark.gpu


def test_phase_events_are_sampled_and_can_be_switched_off():
    cfg = inputs.lattice(16, jitter=0.1, velocities=True)
    p = sph.make_params(cfg, sph.SPH_PREC_MIXED)
    parts = sph.Particles(cfg)
    ctx = sph.Context(p, cfg["n"])
    try:
        sph.sph_build_tree(ctx, parts)
        sph.sph_density(ctx, parts)
        sph.sph_force(ctx, parts)
        sph.sph_set_timing(ctx, 4)
        sph.sph_timings(ctx)  # drop what the set-up recorded
        for _ in range(8):
            sph.sph_step(ctx, parts, 0.0)
        t = sph.sph_timings(ctx)
        for k in ("keys_sort", "tree", "lists", "density", "force", "integrate", "step"):
            assert t[k] > 0.0, k
        assert t["step"] >= t["lists"] + t["density"] + t["force"]
        # switched off: sph_step records nothing
        sph.sph_set_timing(ctx, 0)
        for _ in range(3):
            sph.sph_step(ctx, parts, 0.0)
        assert all(v == 0.0 for v in sph.sph_timings(ctx).values())
        # every call again, and the other entry points record whenever on
        sph.sph_set_timing(ctx, 1)
        sph.sph_density(ctx, parts)
        assert sph.sph_timings(ctx)["density"] > 0.0
        with pytest.raises(sph.SphError):
            sph.sph_set_timing(ctx, -1)
    finally:
        ctx.close()
