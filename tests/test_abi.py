"""C-ABI library checks that need no GPU: it builds, loads and exports every
symbol include/sph.h declares, and the host-side argument checks run before
any device work."""
import ctypes as C
import os
import re

import pytest

from paper_1809_08013_amd import sph as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sph.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sph_[a-z_]+)\s*\(", txt)))


def _lib():
    if not os.path.exists(S.LIB_PATH):
        from paper_1809_08013_amd import build
        build.build()
    return S.load()


def test_header_declares_the_hot_path_calls():
    names = _declared()
    for n in ("sph_build_cells", "sph_find_neighbors", "sph_density", "sph_eos",
              "sph_momentum_energy", "sph_integrate", "sph_timestep"):
        assert n in names


def test_library_exports_every_declared_symbol():
    L = _lib()
    missing = [n for n in _declared() if not hasattr(L, n)]
    assert not missing, missing


def test_status_strings_and_null_checks():
    L = _lib()
    assert L.sph_status_string(S.SPH_OK) == b"ok"
    assert L.sph_status_string(S.SPH_E_CAPACITY).startswith(b"neighbour")
    assert L.sph_status_string(99) == b"unknown status"
    # NULL out-pointer and bad sizes are rejected on the host, before any HIP call
    assert L.sph_ctx_create(None, 10, 10, None) == S.SPH_E_INVALID
    h = C.c_void_p()
    assert L.sph_ctx_create(C.byref(h), 0, 10, None) == S.SPH_E_INVALID
    assert L.sph_ctx_create(C.byref(h), 10, 0, None) == S.SPH_E_INVALID
    assert L.sph_ctx_create(C.byref(h), 10, 5000, None) == S.SPH_E_INVALID
    assert b"max_nb" in L.sph_last_error(None)
    for fn in ("sph_ctx_check", "sph_build_cells", "sph_find_neighbors", "sph_density",
               "sph_eos", "sph_momentum_energy", "sph_integrate", "sph_timestep"):
        f = getattr(L, fn)
        nargs = len(f.argtypes)
        args = [None] * nargs
        if fn == "sph_build_cells":
            args[3] = 1.0
        if fn == "sph_integrate":
            args[3] = 0
        assert f(*args) == S.SPH_E_INVALID, fn
