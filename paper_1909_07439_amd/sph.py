"""Thin ctypes binding of ``libsph.so`` (the C ABI in include/sph.h).

The functions carry the ABI's names and only marshal arguments: torch tensors
give device pointers and the current HIP stream, every computation runs in the
library's gfx950 kernels.  There is no fallback: ``load()`` raises if the
library has not been built (``python -m paper_1909_07439_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

SPH_OK = 0
SPH_E_ARG = -1
SPH_E_NOMEM = -2
SPH_E_HIP = -3
SPH_E_NOCONV = -4
SPH_E_OVERFLOW = -5
SPH_E_DOMAIN = -6
SPH_E_NONFINITE = -7
SPH_PREC_FP64 = 0
SPH_PREC_MIXED = 1

STATUS_NAMES = {0: "SPH_OK", -1: "SPH_E_ARG", -2: "SPH_E_NOMEM", -3: "SPH_E_HIP",
                -4: "SPH_E_NOCONV", -5: "SPH_E_OVERFLOW", -6: "SPH_E_DOMAIN",
                -7: "SPH_E_NONFINITE"}

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "m", "u", "h", "ax", "ay", "az", "dudt", "rho",
          "omega", "P", "cs", "vsig_dt")


class SphError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class sph_params(ctypes.Structure):
    _fields_ = [
        ("box_lo", ctypes.c_double * 3),
        ("box_len", ctypes.c_double * 3),
        ("periodic", ctypes.c_int32 * 3),
        ("gamma", ctypes.c_double),
        ("gamma_minus_1", ctypes.c_double),
        ("hfact", ctypes.c_double),
        ("alpha_av", ctypes.c_double),
        ("beta_av", ctypes.c_double),
        ("alpha_u", ctypes.c_double),
        ("c_cour", ctypes.c_double),
        ("kernel", ctypes.c_int32),
        ("n_leaf", ctypes.c_int32),
        ("n_group", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("h_tol", ctypes.c_double),
        ("max_h_iter", ctypes.c_int32),
        ("reserved0", ctypes.c_int32),
        ("h_margin", ctypes.c_double),
    ]


class sph_particles(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("id", ctypes.c_void_p)] + \
        [(f, ctypes.c_void_p) for f in FIELDS]


COT_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "u", "ax", "ay", "az", "dudt")


class sph_cotangents(ctypes.Structure):
    _fields_ = [(f, ctypes.c_void_p) for f in COT_FIELDS]


_lock = threading.Lock()
_lib = None


def load() -> ctypes.CDLL:
    """Open libsph.so; raises if it is missing (no CPU fallback exists)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_1909_07439_amd.build`")
        # torch brings its own HIP runtime; importing it first makes the
        # library bind to that same runtime instead of loading a second one
        # (two runtimes in one process cannot both open the device)
        import torch  # noqa: F401

        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, i64, d = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        P = ctypes.POINTER
        lib.sph_create.argtypes = [P(sph_params), i64, vp, P(vp)]
        lib.sph_destroy.argtypes = [vp]
        lib.sph_destroy.restype = None
        lib.sph_build_tree.argtypes = [vp, P(sph_particles)]
        lib.sph_density.argtypes = [vp, P(sph_particles), P(i32)]
        lib.sph_force.argtypes = [vp, P(sph_particles), P(d)]
        lib.sph_step.argtypes = [vp, P(sph_particles), d, P(d)]
        lib.sph_reduce.argtypes = [vp, P(sph_particles), P(d)]
        lib.sph_reduce_noalloc.argtypes = [P(sph_particles), vp, P(d)]
        lib.sph_check.argtypes = [vp]
        lib.sph_get_keys.argtypes = [vp, vp, vp]
        lib.sph_get_tree.argtypes = [vp, P(i64), vp, vp, vp, vp, vp, vp]
        lib.sph_get_groups.argtypes = [vp, P(i64), vp, vp]
        lib.sph_neighbours.argtypes = [vp, P(sph_particles), i32, vp, vp, i64]
        lib.sph_list_pairs.argtypes = [vp, P(sph_particles), i32, vp, vp, i64]
        lib.sph_timings.argtypes = [vp, P(d)]
        lib.sph_set_timing.argtypes = [vp, i32]
        lib.sph_stats.argtypes = [vp, P(i64)]
        lib.sph_eval_adjoint.argtypes = [vp, P(sph_particles), P(sph_cotangents)]
        lib.sph_step_adjoint.argtypes = [vp, P(sph_particles), d, P(sph_cotangents)]
        lib.sph_last_error.argtypes = [vp]
        lib.sph_last_error.restype = ctypes.c_char_p
        for name in ("sph_create", "sph_build_tree", "sph_density", "sph_force", "sph_step",
                     "sph_reduce", "sph_reduce_noalloc", "sph_check", "sph_get_keys",
                     "sph_get_tree",
                     "sph_get_groups", "sph_neighbours", "sph_list_pairs", "sph_timings",
                     "sph_set_timing",
                     "sph_stats",
                     "sph_eval_adjoint", "sph_step_adjoint"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
        return lib


def make_params(cfg: dict, precision: int = SPH_PREC_FP64, **over) -> sph_params:
    """sph_params from a workload dict (keys as in paper_1909_07439_amd.inputs)."""
    c = dict(cfg)
    c.update(over)
    p = sph_params()
    for a in range(3):
        p.box_lo[a] = float(c["box_lo"][a])
        p.box_len[a] = float(c["box_len"][a])
        p.periodic[a] = int(c["periodic"][a])
    p.gamma = float(c["gamma"])
    p.gamma_minus_1 = float(c["gamma_minus_1"])
    p.hfact = float(c["hfact"])
    p.alpha_av = float(c["alpha_av"])
    p.beta_av = float(c["beta_av"])
    p.alpha_u = float(c["alpha_u"])
    p.c_cour = float(c["c_cour"])
    p.kernel = int(c.get("kernel", 0))
    p.n_leaf = int(c["n_leaf"])
    p.n_group = int(c["n_group"])
    p.precision = int(c.get("precision", precision))
    p.h_tol = float(c.get("h_tol", 0.0))
    p.max_h_iter = int(c.get("max_h_iter", 0))
    p.h_margin = float(c.get("h_margin", 0.0))
    return p


def _check(ctx, st: int, what: str):
    if st != SPH_OK:
        msg = load().sph_last_error(ctx) if ctx else b""
        raise SphError(st, f"{what}: {msg.decode() if msg else ''}")


class Particles:
    """Device-resident SoA particle set (torch float64 tensors) + its C view."""

    def __init__(self, arrays: dict, device="cuda"):
        import torch

        n = int(arrays["x"].shape[0])
        self.n = n
        self.t = {}
        for f in FIELDS:
            src = arrays.get(f)
            if src is None:
                self.t[f] = torch.zeros(n, dtype=torch.float64, device=device)
            else:
                self.t[f] = torch.as_tensor(np.ascontiguousarray(src, dtype=np.float64)).to(device)
        ids = arrays.get("id", np.arange(n, dtype=np.int64))
        self.t["id"] = torch.as_tensor(np.ascontiguousarray(ids, dtype=np.int64)).to(device)
        self.c = sph_particles()
        self.c.n = n
        self.c.id = self.t["id"].data_ptr()
        for f in FIELDS:
            setattr(self.c, f, self.t[f].data_ptr())

    @classmethod
    def from_tensors(cls, tensors: dict) -> "Particles":
        """A particle set holding copies of the given device tensors (missing
        fields are zero; missing ids are 0..n-1)."""
        import torch

        self = cls.__new__(cls)
        ref = tensors["x"]
        n = int(ref.shape[0])
        self.n = n
        self.t = {}
        for f in FIELDS:
            src = tensors.get(f)
            self.t[f] = (torch.zeros(n, dtype=torch.float64, device=ref.device) if src is None
                         else src.detach().to(torch.float64).contiguous().clone())
        ids = tensors.get("id")
        self.t["id"] = (torch.arange(n, dtype=torch.int64, device=ref.device) if ids is None
                        else ids.detach().to(torch.int64).contiguous().clone())
        self.c = sph_particles()
        self.c.n = n
        self.c.id = self.t["id"].data_ptr()
        for f in FIELDS:
            setattr(self.c, f, self.t[f].data_ptr())
        return self

    def numpy(self, *names) -> dict:
        names = names or (FIELDS + ("id",))
        return {k: self.t[k].detach().cpu().numpy() for k in names}


class Context:
    """Owns one sph_ctx on the current device and torch's current stream."""

    def __init__(self, params: sph_params, n_max: int, stream=None):
        import torch

        lib = load()
        self.lib = lib
        self.params = params
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.stream = stream
        h = ctypes.c_void_p()
        st = lib.sph_create(ctypes.byref(params), int(n_max), ctypes.c_void_p(stream),
                            ctypes.byref(h))
        if st != SPH_OK:
            msg = lib.sph_last_error(None)
            raise SphError(st, msg.decode() if msg else "sph_create")
        self.h = h

    def close(self):
        if self.h:
            self.lib.sph_destroy(self.h)
            self.h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sph_create(params: sph_params, n_max: int, stream=None) -> Context:
    return Context(params, n_max, stream)


def sph_destroy(ctx: Context) -> None:
    ctx.close()


def sph_build_tree(ctx: Context, p: Particles) -> None:
    _check(ctx.h, ctx.lib.sph_build_tree(ctx.h, ctypes.byref(p.c)), "sph_build_tree")


def sph_density(ctx: Context, p: Particles, want_iters: bool = False):
    it = ctypes.c_int32(0)
    _check(ctx.h, ctx.lib.sph_density(ctx.h, ctypes.byref(p.c),
                                      ctypes.byref(it) if want_iters else None), "sph_density")
    return int(it.value) if want_iters else None


def sph_force(ctx: Context, p: Particles, want_dt: bool = False):
    dt = ctypes.c_double(0.0)
    _check(ctx.h, ctx.lib.sph_force(ctx.h, ctypes.byref(p.c),
                                    ctypes.byref(dt) if want_dt else None), "sph_force")
    return float(dt.value) if want_dt else None


def sph_step(ctx: Context, p: Particles, dt: float = 0.0, want_dt: bool = False):
    dn = ctypes.c_double(0.0)
    _check(ctx.h, ctx.lib.sph_step(ctx.h, ctypes.byref(p.c), float(dt),
                                   ctypes.byref(dn) if want_dt else None), "sph_step")
    return float(dn.value) if want_dt else None


def sph_reduce(ctx: Context, p: Particles) -> np.ndarray:
    out = (ctypes.c_double * 12)()
    _check(ctx.h, ctx.lib.sph_reduce(ctx.h, ctypes.byref(p.c), out), "sph_reduce")
    return np.array(out[:])


def sph_reduce_noalloc(p: Particles, stream=None) -> np.ndarray:
    """sph_reduce without a context (the library's allocation-free entry
    point); on the current torch stream unless one is given."""
    import torch

    lib = load()
    s = torch.cuda.current_stream() if stream is None else stream
    out = (ctypes.c_double * 12)()
    st = lib.sph_reduce_noalloc(ctypes.byref(p.c), ctypes.c_void_p(s.cuda_stream), out)
    if st != 0:
        msg = lib.sph_last_error(None)
        raise SphError(st, f"sph_reduce_noalloc: {msg.decode() if msg else ''}")
    return np.array(out[:])


def sph_check(ctx: Context) -> None:
    _check(ctx.h, ctx.lib.sph_check(ctx.h), "sph_check")


def sph_get_keys(ctx: Context, n: int):
    keys = np.empty(n, np.uint64)
    perm = np.empty(n, np.int64)
    _check(ctx.h, ctx.lib.sph_get_keys(ctx.h, keys.ctypes.data, perm.ctypes.data), "sph_get_keys")
    return keys, perm


def sph_get_tree(ctx: Context) -> dict:
    nn = ctypes.c_int64(0)
    _check(ctx.h, ctx.lib.sph_get_tree(ctx.h, ctypes.byref(nn), None, None, None, None, None,
                                       None), "sph_get_tree")
    n = nn.value
    out = dict(level=np.empty(n, np.int32), prefix=np.empty(n, np.uint64),
               first=np.empty(n, np.int64), count=np.empty(n, np.int64),
               child_first=np.empty(n, np.int64), n_child=np.empty(n, np.int32))
    _check(ctx.h, ctx.lib.sph_get_tree(ctx.h, ctypes.byref(nn), *[out[k].ctypes.data for k in (
        "level", "prefix", "first", "count", "child_first", "n_child")]), "sph_get_tree")
    return out


def sph_get_groups(ctx: Context) -> dict:
    ng = ctypes.c_int64(0)
    _check(ctx.h, ctx.lib.sph_get_groups(ctx.h, ctypes.byref(ng), None, None), "sph_get_groups")
    first = np.empty(ng.value, np.int64)
    count = np.empty(ng.value, np.int64)
    _check(ctx.h, ctx.lib.sph_get_groups(ctx.h, ctypes.byref(ng), first.ctypes.data,
                                         count.ctypes.data), "sph_get_groups")
    return dict(first=first, count=count)


def sph_neighbours(ctx: Context, p: Particles, mode: int):
    off = np.empty(p.n + 1, np.int64)
    _check(ctx.h, ctx.lib.sph_neighbours(ctx.h, ctypes.byref(p.c), int(mode), off.ctypes.data,
                                         None, 0), "sph_neighbours")
    total = int(off[-1])
    idx = np.empty(max(total, 1), np.int32)
    _check(ctx.h, ctx.lib.sph_neighbours(ctx.h, ctypes.byref(p.c), int(mode), off.ctypes.data,
                                         idx.ctypes.data, total), "sph_neighbours")
    return off, idx[:total]


def sph_list_pairs(ctx: Context, p: Particles, mode: int):
    """Pairs the hot path's density (0) or force (1) kernel accepts, as
    (offsets, indices) over the current particle order."""
    off = np.empty(p.n + 1, np.int64)
    _check(ctx.h, ctx.lib.sph_list_pairs(ctx.h, ctypes.byref(p.c), int(mode), off.ctypes.data,
                                         None, 0), "sph_list_pairs")
    total = int(off[-1])
    idx = np.empty(max(total, 1), np.int32)
    _check(ctx.h, ctx.lib.sph_list_pairs(ctx.h, ctypes.byref(p.c), int(mode), off.ctypes.data,
                                         idx.ctypes.data, total), "sph_list_pairs")
    return off, idx[:total]


class Cotangents:
    """The eleven cotangent arrays of the adjoint (device float64 tensors of
    n entries, indexed by particle id), and their C view."""

    def __init__(self, n: int, device="cuda", tensors: dict | None = None):
        import torch

        self.t = {}
        for f in COT_FIELDS:
            src = None if tensors is None else tensors.get(f)
            self.t[f] = (torch.zeros(n, dtype=torch.float64, device=device) if src is None
                         else src.detach().to(torch.float64).contiguous().clone())
        self.c = sph_cotangents()
        for f in COT_FIELDS:
            setattr(self.c, f, self.t[f].data_ptr())


def sph_eval_adjoint(ctx: Context, p: Particles, g: Cotangents) -> None:
    _check(ctx.h, ctx.lib.sph_eval_adjoint(ctx.h, ctypes.byref(p.c), ctypes.byref(g.c)),
           "sph_eval_adjoint")


def sph_step_adjoint(ctx: Context, p: Particles, dt: float, g: Cotangents) -> None:
    _check(ctx.h, ctx.lib.sph_step_adjoint(ctx.h, ctypes.byref(p.c), float(dt),
                                           ctypes.byref(g.c)), "sph_step_adjoint")


STEP_FIELDS = ("x", "y", "z", "vx", "vy", "vz", "m", "u", "h", "ax", "ay", "az", "dudt")
ROLLOUT_IN = ("x", "y", "z", "vx", "vy", "vz", "u")
ROLLOUT_OUT = COT_FIELDS


def _original_order(p: Particles, names):
    """Fields of p scattered back to the callers' order (by id)."""
    import torch

    ids = p.t["id"]
    out = []
    for k in names:
        o = torch.empty_like(p.t[k])
        o[ids] = p.t[k]
        out.append(o)
    return out


def _rollout_autograd():
    import torch

    class Rollout(torch.autograd.Function):
        """Initial evaluation and K leapfrog steps of fixed dt as one
        differentiable function of the initial x, y, z, vx, vy, vz, u (device
        float64 tensors in the callers' order).  Returns the final x, y, z,
        vx, vy, vz, u, ax, ay, az, dudt in the same order.  The forward keeps
        the state at the start of every step (checkpoints); the backward
        replays each step in reverse through sph_step_adjoint and ends with
        sph_eval_adjoint of the initial evaluation."""

        @staticmethod
        def forward(fctx, spec, *inp):
            ctx, m, h0, dt, K = spec
            state = dict(zip(ROLLOUT_IN, inp))
            state.update(m=m, h=h0)
            p = Particles.from_tensors(state)
            sph_build_tree(ctx, p)
            sph_density(ctx, p)
            sph_force(ctx, p)
            ckpt = []
            for _ in range(K):
                ckpt.append({k: p.t[k].clone() for k in STEP_FIELDS + ("id",)})
                sph_step(ctx, p, dt)
            fctx.spec = spec
            fctx.ckpt = ckpt
            fctx.save_for_backward(*inp)
            return tuple(_original_order(p, ROLLOUT_OUT))

        @staticmethod
        def backward(fctx, *gout):
            ctx, m, h0, dt, K = fctx.spec
            inp = fctx.saved_tensors
            n = inp[0].shape[0]
            g = Cotangents(n, device=inp[0].device,
                           tensors={k: v for k, v in zip(ROLLOUT_OUT, gout) if v is not None})
            for s in reversed(range(K)):
                p = Particles.from_tensors(fctx.ckpt[s])
                sph_step_adjoint(ctx, p, dt, g)
            state = dict(zip(ROLLOUT_IN, inp))
            state.update(m=m, h=h0)
            p = Particles.from_tensors(state)
            sph_build_tree(ctx, p)
            sph_density(ctx, p)
            sph_force(ctx, p)
            sph_eval_adjoint(ctx, p, g)
            return (None,) + tuple(g.t[k] for k in ROLLOUT_IN)

    return Rollout


_ROLLOUT = None


def rollout(ctx: Context, state: dict, dt: float, K: int) -> dict:
    """Differentiable K-step rollout (see Rollout).  ``state`` holds device
    float64 tensors x, y, z, vx, vy, vz, u (may require grad), m and h (the
    smoothing-length start values)."""
    global _ROLLOUT
    if _ROLLOUT is None:
        _ROLLOUT = _rollout_autograd()
    spec = (ctx, state["m"], state["h"], float(dt), int(K))
    out = _ROLLOUT.apply(spec, *[state[k] for k in ROLLOUT_IN])
    return dict(zip(ROLLOUT_OUT, out))


PHASES = ("keys_sort", "permute", "tree", "density", "force", "integrate", "step",
          "lists", "density_fallback", "force_fallback", "adjoint", "adjoint_force")


def sph_set_timing(ctx: Context, every: int) -> None:
    """Record the phase events on one sph_step call in ``every`` (0: none)."""
    _check(ctx.h, ctx.lib.sph_set_timing(ctx.h, int(every)), "sph_set_timing")


def sph_timings(ctx: Context) -> dict:
    out = (ctypes.c_double * 12)()
    _check(ctx.h, ctx.lib.sph_timings(ctx.h, out), "sph_timings")
    return {k: float(out[i]) for i, k in enumerate(PHASES)}


STATS = ("n_nodes", "n_groups", "max_density_sums", "density_pairs", "force_pairs",
         "density_pair_sums", "density_candidates", "force_candidates", "density_walks",
         "error_word", "total_density_pair_sums", "total_force_pairs", "density_launches",
         "force_launches", "groups_rows_overflow", "groups_h_outgrew",
         "total_list_candidates", "lists_launches")


def sph_stats(ctx: Context) -> dict:
    out = (ctypes.c_int64 * len(STATS))()
    _check(ctx.h, ctx.lib.sph_stats(ctx.h, out), "sph_stats")
    return {k: int(out[i]) for i, k in enumerate(STATS)}
