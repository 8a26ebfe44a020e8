"""Python binding of libsph (include/sph.h): argument marshalling only.

Every step of the SPH path runs in the HIP kernels of libsph.so; this module
only turns torch device tensors into the plain pointers and structs of the C
ABI and raises SphError on a non-zero status. torch provides device memory
and streams. There is no CPU fallback: if the library is missing, loading it
raises.

The functions carry the C names (sph_build_cells, sph_find_neighbors,
sph_density, sph_eos, sph_momentum_energy, sph_integrate, sph_timestep,
sph_init_forces, sph_step, sph_ctx_check, sph_export_neighbors). `SphState`
holds one run's device arrays.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

SPH_OK, SPH_E_INVALID, SPH_E_CAPACITY, SPH_E_HIP = 0, 1, 2, 3
SPH_E_DOMAIN, SPH_E_NOMEM, SPH_E_AGAIN, SPH_E_NONFINITE = 4, 5, 6, 7
SPH_FP64, SPH_FP32_PAIR = 0, 1
SPH_EOS_TAIT, SPH_EOS_IDEAL = 0, 1
SPH_KICK_DRIFT, SPH_KICK = 0, 1

_VP = C.c_void_p


class SphError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


class Particles(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, _VP) for k in (
        "x", "y", "z", "vx", "vy", "vz", "u", "h", "m", "rho_ref", "p_bg",
        "gx", "gy", "gz", "id")]


class Box(C.Structure):
    _fields_ = [("lo", C.c_double * 3), ("hi", C.c_double * 3),
                ("periodic", C.c_int32 * 3)]


class Nbrs(C.Structure):
    _fields_ = [("max_nb", C.c_int32), ("count", _VP), ("idx", _VP)]


class Fields(C.Structure):
    _fields_ = [(k, _VP) for k in ("rho", "p", "c", "pr2")]


class Accel(C.Structure):
    _fields_ = [(k, _VP) for k in ("ax", "ay", "az", "dudt", "mumax")]


class Params(C.Structure):
    _fields_ = [("precision", C.c_int32), ("eos", C.c_int32)] + [
        (k, C.c_double) for k in ("rho0", "c0", "gamma_tait", "gamma_gas", "alpha",
                                  "beta", "eta2", "c_cfl", "c_force")]


_lib = None
_lock = threading.Lock()


def load():
    """Load libsph.so (after torch, so both share one HIP runtime)."""
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        import torch  # noqa: F401  (loads the HIP runtime libsph links against)
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with paper_1809_08013_amd.build.build()")
        L = C.CDLL(LIB_PATH)
        P, B, N = C.POINTER(Particles), C.POINTER(Box), C.POINTER(Nbrs)
        F, A, M = C.POINTER(Fields), C.POINTER(Accel), C.POINTER(Params)
        sig = {
            "sph_status_string": (C.c_char_p, [C.c_int32]),
            "sph_last_error": (C.c_char_p, [_VP]),
            "sph_version": (C.c_char_p, []),
            "sph_ctx_create": (C.c_int32, [C.POINTER(_VP), C.c_int64, C.c_int32, _VP]),
            "sph_ctx_destroy": (C.c_int32, [_VP]),
            "sph_ctx_check": (C.c_int32, [_VP]),
            "sph_ctx_scratch_bytes": (C.c_int64, [_VP]),
            "sph_build_cells": (C.c_int32, [_VP, P, B, C.c_double]),
            "sph_find_neighbors": (C.c_int32, [_VP, P, B, N]),
            "sph_density": (C.c_int32, [_VP, P, B, N, M, _VP]),
            "sph_eos": (C.c_int32, [_VP, P, M, F]),
            "sph_momentum_energy": (C.c_int32, [_VP, P, B, N, M, F, A]),
            "sph_integrate": (C.c_int32, [_VP, P, B, C.c_int32, _VP, A]),
            "sph_timestep": (C.c_int32, [_VP, P, M, F, A, _VP, _VP]),
            "sph_init_forces": (C.c_int32, [_VP, P, B, C.c_double, N, M, F, A, C.c_int32,
                                            _VP, _VP]),
            "sph_step": (C.c_int32, [_VP, P, B, C.c_double, N, M, F, A, _VP, _VP]),
            "sph_export_neighbors": (C.c_int32, [_VP, P, N, _VP, _VP, C.c_int64,
                                                 C.POINTER(C.c_int64)]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        return L


def _ptr(t):
    return None if t is None else _VP(t.data_ptr())


class Context:
    """Owns one sph_ctx (scratch for up to n_max particles)."""

    def __init__(self, n_max: int, max_nb: int, stream=None):
        import torch
        self.lib = load()
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = _VP()
        s = self.lib.sph_ctx_create(C.byref(h), int(n_max), int(max_nb),
                                    _VP(stream.cuda_stream))
        if s != SPH_OK:
            raise SphError(s, self.lib.sph_last_error(None).decode())
        self.h = h
        self.n_max, self.max_nb = int(n_max), int(max_nb)

    def close(self):
        if self.h:
            self.lib.sph_ctx_destroy(self.h)
            self.h = _VP()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def raise_on(self, s: int):
        if s != SPH_OK:
            raise SphError(s, self.lib.sph_last_error(self.h).decode())

    @property
    def scratch_bytes(self) -> int:
        return int(self.lib.sph_ctx_scratch_bytes(self.h))


def make_params(p, precision: int = SPH_FP64) -> Params:
    """Params struct from an inputs.SphParams-like object."""
    return Params(int(precision), int(p.eos), float(p.rho0), float(p.c0),
                  float(p.gamma_tait), float(p.gamma_gas), float(p.alpha),
                  float(p.beta), float(p.eta2), float(p.c_cfl), float(p.c_force))


def make_box(lo, hi, periodic) -> Box:
    return Box((C.c_double * 3)(*map(float, lo)), (C.c_double * 3)(*map(float, hi)),
               (C.c_int32 * 3)(*map(int, periodic)))


class SphState:
    """Device arrays of one run (torch tensors), in the library's cell order.

    Fields mirror the C structs: particle arrays, neighbour lists, fields,
    accelerations, dt_dev (1 double) and diag (8 doubles).
    """

    PARTICLE_KEYS = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m", "rho_ref", "p_bg")

    def __init__(self, ic, max_nb: int, device="cuda", rho_ref=None, g=None):
        import torch
        self.device = torch.device(device)
        dev = self.device
        n = ic.n
        self.n = n
        self.max_nb = int(max_nb)
        f64 = dict(dtype=torch.float64, device=dev)
        arrs = ic.arrays()
        self.t = {}
        for k in self.PARTICLE_KEYS:
            if k == "rho_ref":
                src = rho_ref if rho_ref is not None else np.ones(n)
            else:
                src = arrs[k]
            self.t[k] = torch.as_tensor(np.ascontiguousarray(src, dtype=np.float64)).to(**f64)
        self.t["id"] = torch.as_tensor(np.ascontiguousarray(ic.id, dtype=np.int32)).to(dev)
        if g is not None:
            for k, a in zip(("gx", "gy", "gz"), g):
                self.t[k] = torch.as_tensor(np.ascontiguousarray(a, dtype=np.float64)).to(**f64)
        for k in ("rho", "p", "c", "pr2", "ax", "ay", "az", "dudt", "mumax"):
            self.t[k] = torch.zeros(max(n, 1), **f64)
        self.t["count"] = torch.zeros(max(n, 1), dtype=torch.int32, device=dev)
        self.t["idx"] = torch.zeros(max(n, 1) * self.max_nb, dtype=torch.int32, device=dev)
        self.t["dt"] = torch.zeros(1, **f64)
        self.t["diag"] = torch.zeros(8, **f64)
        self.box = make_box(ic.lo, ic.hi, ic.periodic)
        self.box_tuple = (tuple(ic.lo), tuple(ic.hi), tuple(ic.periodic))
        self.h_max = float(np.max(ic.h)) if n else 1.0
        self._refresh()

    def _refresh(self):
        t = self.t
        self.particles = Particles(self.n, *[_ptr(t.get(k)) for k in (
            "x", "y", "z", "vx", "vy", "vz", "u", "h", "m", "rho_ref", "p_bg",
            "gx", "gy", "gz", "id")])
        self.nbrs = Nbrs(self.max_nb, _ptr(t["count"]), _ptr(t["idx"]))
        self.fields = Fields(*[_ptr(t[k]) for k in ("rho", "p", "c", "pr2")])
        self.accel = Accel(*[_ptr(t[k]) for k in ("ax", "ay", "az", "dudt", "mumax")])

    def host(self, keys=None, original_order=True) -> dict:
        """Copy arrays to numpy; by default reordered to original ids."""
        keys = keys or [k for k in self.t if k not in ("idx", "dt", "diag")]
        ids = self.t["id"][: self.n].cpu().numpy()
        inv = np.empty(self.n, dtype=np.int64)
        inv[ids] = np.arange(self.n)
        out = {}
        for k in keys:
            if k not in self.t:
                continue
            a = self.t[k][: self.n].cpu().numpy()
            out[k] = a[inv] if original_order else a
        return out

    @property
    def dt(self) -> float:
        return float(self.t["dt"].item())

    @property
    def diag(self) -> np.ndarray:
        return self.t["diag"].cpu().numpy()


# ----------------------------------------------------------------- C names --

def sph_ctx_check(ctx: Context) -> int:
    """Synchronise and return the device status (raises on error)."""
    s = ctx.lib.sph_ctx_check(ctx.h)
    ctx.raise_on(s)
    return s


def sph_build_cells(ctx: Context, st: SphState, h_max: float | None = None):
    ctx.raise_on(ctx.lib.sph_build_cells(ctx.h, C.byref(st.particles), C.byref(st.box),
                                         float(h_max if h_max is not None else st.h_max)))


def sph_find_neighbors(ctx: Context, st: SphState):
    ctx.raise_on(ctx.lib.sph_find_neighbors(ctx.h, C.byref(st.particles), C.byref(st.box),
                                            C.byref(st.nbrs)))


def sph_density(ctx: Context, st: SphState, prm: Params):
    ctx.raise_on(ctx.lib.sph_density(ctx.h, C.byref(st.particles), C.byref(st.box),
                                     C.byref(st.nbrs), C.byref(prm), _ptr(st.t["rho"])))


def sph_eos(ctx: Context, st: SphState, prm: Params):
    ctx.raise_on(ctx.lib.sph_eos(ctx.h, C.byref(st.particles), C.byref(prm),
                                 C.byref(st.fields)))


def sph_momentum_energy(ctx: Context, st: SphState, prm: Params):
    ctx.raise_on(ctx.lib.sph_momentum_energy(ctx.h, C.byref(st.particles), C.byref(st.box),
                                             C.byref(st.nbrs), C.byref(prm),
                                             C.byref(st.fields), C.byref(st.accel)))


def sph_integrate(ctx: Context, st: SphState, stage: int):
    ctx.raise_on(ctx.lib.sph_integrate(ctx.h, C.byref(st.particles), C.byref(st.box),
                                       int(stage), _ptr(st.t["dt"]), C.byref(st.accel)))


def sph_timestep(ctx: Context, st: SphState, prm: Params, diag: bool = True):
    ctx.raise_on(ctx.lib.sph_timestep(ctx.h, C.byref(st.particles), C.byref(prm),
                                      C.byref(st.fields), C.byref(st.accel),
                                      _ptr(st.t["dt"]), _ptr(st.t["diag"]) if diag else None))


def sph_init_forces(ctx: Context, st: SphState, prm: Params, set_rho_ref: bool = True,
                    h_max: float | None = None):
    ctx.raise_on(ctx.lib.sph_init_forces(
        ctx.h, C.byref(st.particles), C.byref(st.box),
        float(h_max if h_max is not None else st.h_max), C.byref(st.nbrs), C.byref(prm),
        C.byref(st.fields), C.byref(st.accel), int(bool(set_rho_ref)), _ptr(st.t["dt"]),
        _ptr(st.t["diag"])))


def sph_step(ctx: Context, st: SphState, prm: Params, h_max: float | None = None,
             diag: bool = True):
    ctx.raise_on(ctx.lib.sph_step(
        ctx.h, C.byref(st.particles), C.byref(st.box),
        float(h_max if h_max is not None else st.h_max), C.byref(st.nbrs), C.byref(prm),
        C.byref(st.fields), C.byref(st.accel), _ptr(st.t["dt"]),
        _ptr(st.t["diag"]) if diag else None))


def sph_export_neighbors(ctx: Context, st: SphState):
    """Neighbour sets as (offsets int64[n+1], ids int32[]) in original ids."""
    n = st.n
    off = np.zeros(n + 1, dtype=np.int64)
    cap = int(n) * st.max_nb
    ids = np.zeros(max(cap, 1), dtype=np.int32)
    tot = C.c_int64(0)
    ctx.raise_on(ctx.lib.sph_export_neighbors(
        ctx.h, C.byref(st.particles), C.byref(st.nbrs), _VP(off.ctypes.data),
        _VP(ids.ctypes.data), cap, C.byref(tot)))
    return off, ids[: tot.value].copy()


def version() -> str:
    return load().sph_version().decode()
