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
               "sph_eos", "sph_momentum_energy", "sph_integrate", "sph_timestep",
               "sph_gravity_direct", "sph_volume_weights", "sph_gravity_tree"):
        f = getattr(L, fn)
        nargs = len(f.argtypes)
        args = [None] * nargs
        if fn == "sph_build_cells":
            args[3] = 1.0
        if fn == "sph_integrate":
            args[3] = 0
        if fn == "sph_gravity_direct":
            args[2] = 0.01
        if fn == "sph_volume_weights":
            args[3] = 0.7
        if fn == "sph_gravity_tree":
            args[2], args[3], args[4] = 0.01, 0.5, 16
        assert f(*args) == S.SPH_E_INVALID, fn
    # the captured step: a NULL context is refused before any HIP call
    assert L.sph_step_capture(None, None, None, 1.0, None, None, None, None, None,
                              None) == S.SPH_E_INVALID
    assert L.sph_step_replay(None) == S.SPH_E_INVALID


def test_ensemble_host_checks():
    """sph_ens_*: configuration and request checks run on the host before any
    device work."""
    L = _lib()
    h = C.c_void_p()
    assert L.sph_ens_create(None, None) == S.SPH_E_INVALID
    for cfg in (S.EnsConfig(0, 7, 128, 4, 1 << 30, 1000),     # precision
                S.EnsConfig(0, 0, 0, 4, 1 << 30, 1000),       # max_nb
                S.EnsConfig(0, 0, 128, 0, 1 << 30, 1000),     # max_slots
                S.EnsConfig(0, 0, 128, 512, 1 << 30, 1000),
                S.EnsConfig(0, 0, 128, 4, 1 << 30, 0),        # max_n_per_run
                S.EnsConfig(0, 0, 128, 4, 1 << 20, 1000)):    # budget below one run
        assert L.sph_ens_create(C.byref(h), C.byref(cfg)) == S.SPH_E_INVALID
    assert b"budget" in L.sph_ens_last_error(None)
    t = C.c_uint64()
    assert L.sph_ens_submit(None, None, C.byref(t)) == S.SPH_E_INVALID
    assert L.sph_ens_poll(None, 1, None) == S.SPH_E_INVALID
    assert L.sph_ens_wait(None, 1, None) == S.SPH_E_INVALID
    assert L.sph_ens_stats(None, None) == S.SPH_E_INVALID
    assert L.sph_ens_destroy(None) == S.SPH_E_INVALID
    a = L.sph_ens_clock()
    b = L.sph_ens_clock()
    assert 0 < a <= b


def test_ensemble_structs_match_header():
    """ctypes mirrors of the ensemble structs, sph_params and sph_particles
    have the C sizes and offsets."""
    import subprocess
    import tempfile
    src = r'''
#include <stddef.h>
#include <stdio.h>
#include "sph.h"
int main(void) {
    printf("%zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu %zu\n",
           sizeof(sph_ens_config), sizeof(sph_run_request), sizeof(sph_run_result),
           sizeof(sph_ens_counters), offsetof(sph_run_request, rho_ref),
           offsetof(sph_run_result, status), offsetof(sph_ens_counters, busy_seconds),
           sizeof(sph_params), offsetof(sph_params, kernel), offsetof(sph_params, sinc_n),
           offsetof(sph_params, volume), offsetof(sph_params, volume_p),
           sizeof(sph_particles), offsetof(sph_particles, xw));
    return 0;
}
'''
    with tempfile.TemporaryDirectory() as d:
        c = os.path.join(d, "t.c")
        exe = os.path.join(d, "t")
        open(c, "w").write(src)
        subprocess.check_call(["gcc", "-I", os.path.join(ROOT, "include"), c, "-o", exe])
        got = [int(v) for v in subprocess.check_output([exe]).split()]
    want = [C.sizeof(S.EnsConfig), C.sizeof(S.RunRequest), C.sizeof(S.RunResult),
            C.sizeof(S.EnsCounters), S.RunRequest.rho_ref.offset, S.RunResult.status.offset,
            S.EnsCounters.busy_seconds.offset, C.sizeof(S.Params), S.Params.kernel.offset,
            S.Params.sinc_n.offset, S.Params.volume.offset, S.Params.volume_p.offset,
            C.sizeof(S.Particles), S.Particles.xw.offset]
    assert got == want


def test_smoothing_length_host_checks():
    L = _lib()
    it = C.c_int32(0)
    assert L.sph_smoothing_length(None, None, None, 100.0, 95, 105, 10, None,
                                  C.byref(it)) == S.SPH_E_INVALID
    assert L.sph_step_blocks(None, None, None, 1.0, None, None, None, None, 2, None, None,
                             None, C.byref(it)) == S.SPH_E_INVALID


def test_density_noalloc_host_checks():
    """The entry point that allocates nothing rejects sizes beyond its static
    scratch (SPH_E_CAPACITY) and malformed arguments on the host, before any
    HIP call."""
    L = _lib()
    box = S.make_box((0.0,) * 3, (1.0,) * 3, (0, 0, 0))
    prm = S.Params()
    nb = S.Nbrs(128, None, None)
    p = S.Particles(S.SPH_DENSITY_NOALLOC_MAX_N + 1)
    assert L.sph_density_noalloc(C.byref(p), C.byref(box), C.byref(nb), C.byref(prm), None,
                                 None) == S.SPH_E_CAPACITY
    assert b"static scratch" in L.sph_last_error(None)
    p = S.Particles(10)
    assert L.sph_density_noalloc(None, C.byref(box), C.byref(nb), C.byref(prm), None,
                                 None) == S.SPH_E_INVALID
    assert L.sph_density_noalloc(C.byref(p), C.byref(box), C.byref(nb), C.byref(prm), None,
                                 None) == S.SPH_E_INVALID
    assert b"count and idx" in L.sph_last_error(None)
    p0 = S.Particles(0)
    assert L.sph_density_noalloc(C.byref(p0), C.byref(box), C.byref(nb), C.byref(prm), None,
                                 None) == S.SPH_OK

