"""MI355X-native SPH hydrodynamics step (Bonsai-SPH, arXiv:1909.07439).

The compute path lives in ``csrc/`` (HIP kernels for gfx950 behind a C ABI,
declared in ``include/sph.h``); ``sph`` is the thin ctypes binding and
``inputs`` the seeded workload generators.  Importing this package loads
nothing; ``sph.load()`` opens the shared library and fails loudly if it has
not been built.
"""
__all__ = ["inputs", "sph"]
