"""Host-side checks of libsph.so that need no GPU: it loads, exports every
entry point include/sph.h declares, its structs have the layout the binding
assumes, and sph_create rejects bad parameters before touching the device."""
import ctypes
import os
import re
import subprocess

import pytest

from paper_1909_07439_amd import sph

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "sph.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(sph.LIB_PATH):
        from paper_1909_07439_amd import build

        build.build()
    return sph.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", text)))


def test_exports_every_declared_symbol(lib):
    names = declared_functions()
    assert "sph_build_tree" in names and "sph_step" in names and len(names) >= 14
    for name in names:
        assert hasattr(lib, name), name


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    src.write_text(r'''
#include <stddef.h>
#include <stdio.h>
#include "sph.h"
int main(void) {
  printf("%zu %zu %zu %zu %zu %zu\n", sizeof(sph_params), offsetof(sph_params, gamma),
         offsetof(sph_params, kernel), offsetof(sph_params, h_tol),
         offsetof(sph_params, h_margin), sizeof(sph_particles));
  printf("%zu %zu\n", offsetof(sph_particles, x), offsetof(sph_particles, vsig_dt));
  printf("%zu %zu %zu\n", sizeof(sph_cotangents), offsetof(sph_cotangents, u),
         offsetof(sph_cotangents, dudt));
  return 0;
}
''')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)],
                   check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()
    P, Q = sph.sph_params, sph.sph_particles
    assert int(out[0]) == ctypes.sizeof(P)
    assert int(out[1]) == P.gamma.offset
    assert int(out[2]) == P.kernel.offset
    assert int(out[3]) == P.h_tol.offset
    assert int(out[4]) == P.h_margin.offset
    assert int(out[5]) == ctypes.sizeof(Q)
    assert int(out[6]) == Q.x.offset
    assert int(out[7]) == Q.vsig_dt.offset
    G = sph.sph_cotangents
    assert int(out[8]) == ctypes.sizeof(G)
    assert int(out[9]) == G.u.offset
    assert int(out[10]) == G.dudt.offset


def _params(**kw):
    from paper_1909_07439_amd import inputs

    cfg = dict(inputs.DEFAULTS, box_lo=(0, 0, 0), box_len=(1, 1, 1), periodic=(1, 1, 1))
    cfg.update(kw)
    return sph.make_params(cfg)


@pytest.mark.parametrize("bad", [dict(n_group=6), dict(n_leaf=0), dict(n_leaf=65),
                                 dict(box_len=(1, 0, 1)), dict(hfact=0.0),
                                 dict(gamma_minus_1=0.0), dict(precision=3), dict(kernel=3),
                                 dict(kernel=-1)])
def test_create_rejects_bad_parameters(lib, bad):
    p = _params(**bad)
    h = ctypes.c_void_p()
    st = lib.sph_create(ctypes.byref(p), 1000, None, ctypes.byref(h))
    assert st == sph.SPH_E_ARG
    assert not h.value
    # the reason is kept for the calling thread
    assert lib.sph_last_error(None).startswith(b"sph_create: ")


def test_create_rejects_bad_sizes(lib):
    p = _params()
    h = ctypes.c_void_p()
    assert lib.sph_create(ctypes.byref(p), 0, None, ctypes.byref(h)) == sph.SPH_E_ARG
    assert lib.sph_create(ctypes.byref(p), 1 << 40, None, ctypes.byref(h)) == sph.SPH_E_ARG
    assert lib.sph_create(None, 10, None, ctypes.byref(h)) == sph.SPH_E_ARG


def test_null_context_is_an_argument_error(lib):
    assert lib.sph_build_tree(None, None) == sph.SPH_E_ARG
    assert lib.sph_check(None) == sph.SPH_E_ARG
    assert lib.sph_eval_adjoint(None, None, None) == sph.SPH_E_ARG
    assert lib.sph_step_adjoint(None, None, 1.0, None) == sph.SPH_E_ARG
    assert lib.sph_set_timing(None, 1) == sph.SPH_E_ARG
    assert isinstance(lib.sph_last_error(None), bytes)
    lib.sph_destroy(None)
