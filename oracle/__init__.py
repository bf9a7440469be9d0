"""FP64 CPU oracle for the SPH hydrodynamics step of Bonsai-SPH
(Bedorf & Portegies Zwart, arXiv:1909.07439).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the HIP library: the arithmetic lives in ``sph_oracle.c`` (plain
C, FP64, ``-ffp-contract=off``) and in ``riemann.py`` (textbook exact Riemann
solver); this module only marshals numpy arrays through ctypes and composes
the C steps into an evaluation and a leapfrog step.

Which passage each function follows is stated in ``sph_oracle.c``.  Every
function here is pinned by ``tests/test_oracle_*.py`` against something other
than itself (library routines, closed forms, finite differences, brute force,
conservation laws, textbook values).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sph_oracle.c")
_SO = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

OK = 0
E_ARG = -1
E_NOMEM = -2
E_NOCONV = -4
E_OVERFLOW = -5


def build(force: bool = True) -> str:
    """Compile ``sph_oracle.c`` into ``liboracle.so`` (gcc, OpenMP, no FP contraction)."""
    if not force and os.path.exists(_SO):
        return _SO
    tmp = _SO + ".tmp"
    cmd = ["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _SO)
    return _SO


class Params(ctypes.Structure):
    _fields_ = [
        ("box_lo", ctypes.c_double * 3),
        ("box_len", ctypes.c_double * 3),
        ("periodic", ctypes.c_int * 3),
        ("gamma", ctypes.c_double),
        ("gamma_minus_1", ctypes.c_double),
        ("hfact", ctypes.c_double),
        ("alpha_av", ctypes.c_double),
        ("beta_av", ctypes.c_double),
        ("alpha_u", ctypes.c_double),
        ("c_cour", ctypes.c_double),
        ("n_leaf", ctypes.c_int),
        ("n_group", ctypes.c_int),
        ("h_tol", ctypes.c_double),
        ("max_h_iter", ctypes.c_int),
        ("kernel", ctypes.c_int),
    ]


def make_params(cfg: dict) -> Params:
    """Build the C parameter block from a plain dict (keys as in ``Params``)."""
    p = Params()
    for d in range(3):
        p.box_lo[d] = float(cfg["box_lo"][d])
        p.box_len[d] = float(cfg["box_len"][d])
        p.periodic[d] = int(cfg["periodic"][d])
    p.gamma = float(cfg["gamma"])
    p.gamma_minus_1 = float(cfg["gamma_minus_1"])
    p.hfact = float(cfg["hfact"])
    p.alpha_av = float(cfg["alpha_av"])
    p.beta_av = float(cfg["beta_av"])
    p.alpha_u = float(cfg["alpha_u"])
    p.c_cour = float(cfg["c_cour"])
    p.n_leaf = int(cfg["n_leaf"])
    p.n_group = int(cfg["n_group"])
    p.h_tol = float(cfg.get("h_tol_oracle", 1e-10))
    p.max_h_iter = int(cfg.get("max_h_iter", 30))
    p.kernel = int(cfg.get("kernel", 0))
    return p


_D = ctypes.POINTER(ctypes.c_double)
_I64 = ctypes.POINTER(ctypes.c_int64)
_U64 = ctypes.POINTER(ctypes.c_uint64)
_I32 = ctypes.POINTER(ctypes.c_int32)
_P = ctypes.POINTER(Params)


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(_SO):
            build(force=False)
        lib = ctypes.CDLL(_SO)
        lib.orc_kernel_m4.argtypes = [ctypes.c_int64, _D, _D, _D, _D, _D]
        lib.orc_kernel.argtypes = [ctypes.c_int, ctypes.c_int64, _D, _D, _D, _D, _D]
        lib.orc_kernel_support.argtypes = [ctypes.c_int]
        lib.orc_kernel_support.restype = ctypes.c_double
        lib.orc_keys.argtypes = [ctypes.c_int64, _D, _D, _D, _P, _U64]
        lib.orc_sort.argtypes = [ctypes.c_int64, _U64, _I64]
        lib.orc_tree.argtypes = [ctypes.c_int64, _U64, ctypes.c_int, ctypes.c_int64,
                                 _I32, _U64, _I64, _I64, _I64, _I32]
        lib.orc_tree.restype = ctypes.c_int64
        lib.orc_groups.argtypes = [ctypes.c_int64, _U64, ctypes.c_int, ctypes.c_int64, _I64, _I64]
        lib.orc_groups.restype = ctypes.c_int64
        lib.orc_neighbours.argtypes = [ctypes.c_int64, _D, _D, _D, _D, _P, ctypes.c_int,
                                       ctypes.c_int, _I64, _I64, ctypes.c_int64]
        lib.orc_neighbours.restype = ctypes.c_int64
        lib.orc_neighbours_sel.argtypes = [ctypes.c_int64, _D, _D, _D, _D, _P, ctypes.c_int,
                                           ctypes.c_int, _I64, ctypes.c_int64, _I64, _I64,
                                           ctypes.c_int64]
        lib.orc_neighbours_sel.restype = ctypes.c_int64
        lib.orc_density.argtypes = [ctypes.c_int64, _D, _D, _D, _D, _D, _P, _D, _D, _D, _I64, _I32]
        lib.orc_density.restype = ctypes.c_int
        lib.orc_density_sel.argtypes = [ctypes.c_int64, _D, _D, _D, _D, _D, _P, _I64,
                                        ctypes.c_int64, _D, _D, _D, _I64, _I32]
        lib.orc_density_sel.restype = ctypes.c_int
        lib.orc_force_sel.argtypes = [ctypes.c_int64] + [_D] * 13 + [_P, _I64, ctypes.c_int64] + \
            [_D] * 7 + [_I64]
        lib.orc_force_sel.restype = ctypes.c_int
        lib.orc_eos.argtypes = [ctypes.c_int64, _D, _D, _P, _D, _D]
        lib.orc_force.argtypes = [ctypes.c_int64] + [_D] * 13 + [_P] + [_D] * 7 + [_I64]
        lib.orc_force.restype = ctypes.c_int
        lib.orc_courant_dt.argtypes = [ctypes.c_int64, _D, _D, _P]
        lib.orc_courant_dt.restype = ctypes.c_double
        lib.orc_predict.argtypes = [ctypes.c_int64] + [_D] * 11 + [ctypes.c_double, _P]
        lib.orc_correct.argtypes = [ctypes.c_int64] + [_D] * 12 + [ctypes.c_double]
        lib.orc_reduce.argtypes = [ctypes.c_int64] + [_D] * 9 + [_D]
        lib.orc_num_threads.restype = ctypes.c_int
        lib.orc_set_num_threads.argtypes = [ctypes.c_int]
        lib.orc_set_num_threads.restype = None
        _lib = lib
        return lib


def _dptr(a):
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(_D)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def num_threads() -> int:
    return int(_load().orc_num_threads())


def set_num_threads(k: int) -> None:
    """Threads of the oracle's parallel loops from now on."""
    _load().orc_set_num_threads(int(k))


def kernel_m4(r, h):
    """W(r,h), F(r,h)=dW/dr and dW/dh of the 3D M4 spline, elementwise."""
    r = _f64(r).ravel()
    h = _f64(np.broadcast_to(h, r.shape)).copy()
    w, F, dh = np.empty_like(r), np.empty_like(r), np.empty_like(r)
    _load().orc_kernel_m4(r.size, _dptr(r), _dptr(h), _dptr(w), _dptr(F), _dptr(dh))
    return w, F, dh


M4, M6, WENDLAND_C6 = 0, 1, 2


def kernel(kind: int, r, h):
    """W(r,h), F(r,h)=dW/dr and dW/dh of kernel ``kind`` (M4, M6 or
    WENDLAND_C6), elementwise."""
    r = _f64(r).ravel()
    h = _f64(np.broadcast_to(h, r.shape)).copy()
    w, F, dh = np.empty_like(r), np.empty_like(r), np.empty_like(r)
    _load().orc_kernel(int(kind), r.size, _dptr(r), _dptr(h), _dptr(w), _dptr(F), _dptr(dh))
    return w, F, dh


def kernel_support(kind: int) -> float:
    """Support radius of kernel ``kind`` in units of h."""
    return float(_load().orc_kernel_support(int(kind)))


def keys(x, y, z, params: Params) -> np.ndarray:
    x, y, z = _f64(x), _f64(y), _f64(z)
    k = np.empty(x.size, dtype=np.uint64)
    _load().orc_keys(x.size, _dptr(x), _dptr(y), _dptr(z), ctypes.byref(params),
                     k.ctypes.data_as(_U64))
    return k


def sort(k: np.ndarray) -> np.ndarray:
    """Stable ascending order of the keys (ties keep input order)."""
    k = np.ascontiguousarray(k, dtype=np.uint64)
    perm = np.empty(k.size, dtype=np.int64)
    _load().orc_sort(k.size, k.ctypes.data_as(_U64), perm.ctypes.data_as(_I64))
    return perm


def tree(sorted_keys: np.ndarray, n_leaf: int) -> dict:
    sk = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    n = sk.size
    cap = 2 * n + 64
    level = np.empty(cap, np.int32)
    prefix = np.empty(cap, np.uint64)
    first = np.empty(cap, np.int64)
    count = np.empty(cap, np.int64)
    child_first = np.empty(cap, np.int64)
    n_child = np.empty(cap, np.int32)
    nn = _load().orc_tree(n, sk.ctypes.data_as(_U64), int(n_leaf), cap,
                          level.ctypes.data_as(_I32), prefix.ctypes.data_as(_U64),
                          first.ctypes.data_as(_I64), count.ctypes.data_as(_I64),
                          child_first.ctypes.data_as(_I64), n_child.ctypes.data_as(_I32))
    if nn < 0:
        raise RuntimeError(f"orc_tree failed: {nn}")
    return dict(level=level[:nn], prefix=prefix[:nn], first=first[:nn], count=count[:nn],
                child_first=child_first[:nn], n_child=n_child[:nn])


def groups(sorted_keys: np.ndarray, n_group: int) -> dict:
    sk = np.ascontiguousarray(sorted_keys, dtype=np.uint64)
    n = sk.size
    cap = n + 1
    first = np.empty(cap, np.int64)
    count = np.empty(cap, np.int64)
    ng = _load().orc_groups(n, sk.ctypes.data_as(_U64), int(n_group), cap,
                            first.ctypes.data_as(_I64), count.ctypes.data_as(_I64))
    if ng < 0:
        raise RuntimeError(f"orc_groups failed: {ng}")
    return dict(first=first[:ng], count=count[:ng])


def neighbours(x, y, z, h, params: Params, mode: int = 0, brute: bool = False, sel=None):
    """CSR (offsets, idx) of neighbour sets, ascending indices.

    mode 0: density set, r_ij < 2 h_i, self included.
    mode 1: force set, j != i and r_ij < 2 max(h_i, h_j).
    sel: only these particles (row k is particle sel[k]); default all.
    """
    x, y, z, h = _f64(x), _f64(y), _f64(z), _f64(h)
    n = x.size
    if sel is None:
        selp, nsel = None, n
    else:
        sel = np.ascontiguousarray(sel, dtype=np.int64)
        selp, nsel = sel.ctypes.data_as(_I64), sel.size
    off = np.empty(nsel + 1, np.int64)
    lib = _load()
    args = (n, _dptr(x), _dptr(y), _dptr(z), _dptr(h), ctypes.byref(params), int(mode),
            int(bool(brute)), selp, nsel, off.ctypes.data_as(_I64))
    tot = lib.orc_neighbours_sel(*args, None, 0)
    if tot not in (E_OVERFLOW,) and tot < 0:
        raise RuntimeError(f"orc_neighbours failed: {tot}")
    total = int(off[nsel])
    idx = np.empty(max(total, 1), np.int64)
    tot = lib.orc_neighbours_sel(*args, idx.ctypes.data_as(_I64), total)
    if tot < 0:
        raise RuntimeError(f"orc_neighbours failed: {tot}")
    return off, idx[:total]


def density(x, y, z, m, h, params: Params) -> dict:
    """Smoothing length root, density, Omega, neighbour count, NR sum evaluations."""
    x, y, z, m, h = _f64(x), _f64(y), _f64(z), _f64(m), _f64(h)
    n = x.size
    ho, rho, om = np.empty(n), np.empty(n), np.empty(n)
    nn = np.empty(n, np.int64)
    it = np.empty(n, np.int32)
    st = _load().orc_density(n, _dptr(x), _dptr(y), _dptr(z), _dptr(m), _dptr(h),
                             ctypes.byref(params), _dptr(ho), _dptr(rho), _dptr(om),
                             nn.ctypes.data_as(_I64), it.ctypes.data_as(_I32))
    if st != OK:
        raise RuntimeError(f"orc_density failed: {st}")
    return dict(h=ho, rho=rho, omega=om, nneigh=nn, iters=it)


def eos(rho, u, params: Params):
    rho, u = _f64(rho), _f64(u)
    P, cs = np.empty_like(rho), np.empty_like(rho)
    _load().orc_eos(rho.size, _dptr(rho), _dptr(u), ctypes.byref(params), _dptr(P), _dptr(cs))
    return P, cs


def force(s: dict, params: Params) -> dict:
    """Acceleration, du/dt, signal speed for dt, and per-particle normalisers."""
    a = {k: _f64(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "u", "h", "rho",
                                  "omega", "P", "cs")}
    n = a["x"].size
    out = {k: np.empty(n) for k in ("ax", "ay", "az", "dudt", "vsig_dt", "anorm", "unorm")}
    nn = np.empty(n, np.int64)
    st = _load().orc_force(n, *[_dptr(a[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m",
                                                       "u", "h", "rho", "omega", "P", "cs")],
                           ctypes.byref(params),
                           *[_dptr(out[k]) for k in ("ax", "ay", "az", "dudt", "vsig_dt",
                                                     "anorm", "unorm")],
                           nn.ctypes.data_as(_I64))
    if st != OK:
        raise RuntimeError(f"orc_force failed: {st}")
    out["nneigh_force"] = nn
    return out


def evaluate_subset(s: dict, params: Params, sel) -> dict:
    """Density (root h), EOS and force for the particles ``sel`` only.

    Every particle's fields are inputs (the neighbours of a selected particle
    are found among all of them, and the force needs each neighbour's rho,
    Omega, P, c_s: these are solved for the neighbours too).  Outputs are
    arrays over ``sel`` in its order.  The arithmetic is that of
    ``evaluate``; only the particle loops are restricted.
    """
    a = {k: _f64(s[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "u", "h")}
    n = a["x"].size
    sel = np.ascontiguousarray(sel, dtype=np.int64)
    lib = _load()
    # particles whose rho, Omega, P, c_s the force on sel needs: sel and all
    # force neighbours of sel at the start h grown by a safe factor
    grow = a["h"] * 1.6
    off, idx = neighbours(a["x"], a["y"], a["z"], grow, params, mode=1, sel=sel)
    need = np.unique(np.concatenate([sel, idx]))
    m = need.size
    ho, rho, om = np.empty(m), np.empty(m), np.empty(m)
    nn = np.empty(m, np.int64)
    it = np.empty(m, np.int32)
    st = lib.orc_density_sel(n, _dptr(a["x"]), _dptr(a["y"]), _dptr(a["z"]), _dptr(a["m"]),
                             _dptr(a["h"]), ctypes.byref(params), need.ctypes.data_as(_I64), m,
                             _dptr(ho), _dptr(rho), _dptr(om), nn.ctypes.data_as(_I64),
                             it.ctypes.data_as(_I32))
    if st != OK:
        raise RuntimeError(f"orc_density_sel failed: {st}")
    full = {k: np.full(n, np.nan) for k in ("h", "rho", "omega")}
    full["h"] = a["h"].copy()
    full["h"][need], full["rho"][need], full["omega"][need] = ho, rho, om
    P, cs = np.full(n, np.nan), np.full(n, np.nan)
    P[need], cs[need] = eos(rho, a["u"][need], params)
    # a neighbour of sel outside `need` would leave a NaN in the sums: checked
    k = sel.size
    out = {q: np.empty(k) for q in ("ax", "ay", "az", "dudt", "vsig_dt", "anorm", "unorm")}
    nnf = np.empty(k, np.int64)
    st = lib.orc_force_sel(n, *[_dptr(v) for v in (a["x"], a["y"], a["z"], a["vx"], a["vy"],
                                                   a["vz"], a["m"], a["u"], full["h"],
                                                   full["rho"], full["omega"], P, cs)],
                           ctypes.byref(params), sel.ctypes.data_as(_I64), k,
                           *[_dptr(out[q]) for q in ("ax", "ay", "az", "dudt", "vsig_dt",
                                                      "anorm", "unorm")],
                           nnf.ctypes.data_as(_I64))
    if st != OK:
        raise RuntimeError(f"orc_force_sel failed: {st}")
    pos = np.searchsorted(need, sel)
    out.update(h=ho[pos], rho=rho[pos], omega=om[pos], nneigh=nn[pos], P=P[sel], cs=cs[sel],
               nneigh_force=nnf)
    for q in ("ax", "dudt"):
        if not np.all(np.isfinite(out[q])):
            raise RuntimeError("a neighbour of a selected particle was not solved for")
    return out


def courant_dt(h, vsig_dt, params: Params) -> float:
    h, v = _f64(h), _f64(vsig_dt)
    return float(_load().orc_courant_dt(h.size, _dptr(h), _dptr(v), ctypes.byref(params)))


def evaluate(s: dict, params: Params) -> dict:
    """One hydro evaluation: density (NR to the root), EOS, force.

    Returns a new dict with the input fields plus h, rho, omega, P, cs, ax, ay,
    az, dudt, vsig_dt, anorm, unorm, nneigh, iters and dt_next.
    """
    o = {k: _f64(v).copy() for k, v in s.items() if isinstance(v, np.ndarray)}
    d = density(o["x"], o["y"], o["z"], o["m"], o["h"], params)
    o.update(h=d["h"], rho=d["rho"], omega=d["omega"], nneigh=d["nneigh"], iters=d["iters"])
    o["P"], o["cs"] = eos(o["rho"], o["u"], params)
    o.update(force(o, params))
    o["dt_next"] = courant_dt(o["h"], o["vsig_dt"], params)
    return o


def step(s: dict, dt: float, params: Params) -> dict:
    """Leapfrog predictor, evaluation at the predicted state, corrector.

    ``s`` must hold x,y,z,vx,vy,vz,m,u,h and the previous ax,ay,az,dudt.
    """
    o = {k: _f64(v).copy() for k, v in s.items() if isinstance(v, np.ndarray)}
    n = o["x"].size
    lib = _load()
    lib.orc_predict(n, *[_dptr(o[k]) for k in ("x", "y", "z", "vx", "vy", "vz", "u", "ax", "ay",
                                               "az", "dudt")], float(dt), ctypes.byref(params))
    e = evaluate({k: o[k] for k in ("x", "y", "z", "vx", "vy", "vz", "m", "u", "h")}, params)
    a0 = {k: o[k] for k in ("ax", "ay", "az", "dudt")}
    lib.orc_correct(n, *[_dptr(o[k]) for k in ("vx", "vy", "vz", "u")],
                    *[_dptr(a0[k]) for k in ("ax", "ay", "az", "dudt")],
                    *[_dptr(e[k]) for k in ("ax", "ay", "az", "dudt")], float(dt))
    for k in ("h", "rho", "omega", "P", "cs", "vsig_dt", "anorm", "unorm", "nneigh", "iters",
              "nneigh_force"):
        o[k] = e[k]
    o["ax"], o["ay"], o["az"], o["dudt"] = a0["ax"], a0["ay"], a0["az"], a0["dudt"]
    o["dt_next"] = e["dt_next"]
    return o


def reduce(s: dict) -> np.ndarray:
    """{E, E_kin, E_th, p_x, p_y, p_z, sum m a (3), dE/dt, sum m|a|, sum m(|v.a|+|du|)}"""
    a = [_f64(s[k]) for k in ("vx", "vy", "vz", "m", "u", "ax", "ay", "az", "dudt")]
    out = np.zeros(12)
    _load().orc_reduce(a[0].size, *[_dptr(v) for v in a], _dptr(out))
    return out
