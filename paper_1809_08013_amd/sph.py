"""Python binding of libsph (include/sph.h): argument marshalling only.

Every step of the SPH path runs in the HIP kernels of libsph.so; this module
only turns torch device tensors into the plain pointers and structs of the C
ABI and raises SphError on a non-zero status. torch provides device memory
and streams. There is no CPU fallback: if the library is missing, loading it
raises.

The functions carry the C names (sph_build_cells, sph_find_neighbors,
sph_density, sph_eos, sph_momentum_energy, sph_integrate, sph_timestep,
sph_init_forces, sph_step, sph_ctx_check, sph_export_neighbors). `SphState`
holds one run's device arrays. `Ensemble` wraps the serving engine
(sph_ens_create, sph_ens_submit, sph_ens_poll, sph_ens_wait, sph_ens_stats,
sph_ens_destroy).
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
SPH_KERNEL_M4, SPH_KERNEL_WENDLAND_C2, SPH_KERNEL_SINC = 0, 1, 2
SPH_GRAD_KERNEL, SPH_GRAD_IAD = 0, 1
SPH_VOLUME_STANDARD, SPH_VOLUME_GENERALISED = 0, 1
SPH_DENSITY_NOALLOC_MAX_N = 1 << 20  # the static scratch of sph_density_noalloc

_VP = C.c_void_p


class SphError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"[{status}] {message}")
        self.status = status


class Particles(C.Structure):
    _fields_ = [("n", C.c_int64)] + [(k, _VP) for k in (
        "x", "y", "z", "vx", "vy", "vz", "u", "h", "m", "rho_ref", "p_bg",
        "gx", "gy", "gz", "id", "xw")]


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
                                  "beta", "eta2", "c_cfl", "c_force")] + [
        ("kernel", C.c_int32), ("sinc_n", C.c_int32), ("gradient", C.c_int32),
        ("volume", C.c_int32), ("volume_p", C.c_double)]


class EnsConfig(C.Structure):
    _fields_ = [("device", C.c_int32), ("precision", C.c_int32), ("max_nb", C.c_int32),
                ("max_slots", C.c_int32), ("hbm_budget_bytes", C.c_int64),
                ("max_n_per_run", C.c_int64), ("pinned_submit_bytes", C.c_int64)]


_REQ_ARRAYS = ("x", "y", "z", "vx", "vy", "vz", "u", "h", "m", "p_bg", "rho_ref", "id")
_RES_ARRAYS = ("x", "y", "z", "vx", "vy", "vz", "u", "rho")


class RunRequest(C.Structure):
    _fields_ = [("n", C.c_int64), ("n_steps", C.c_int32), ("set_rho_ref", C.c_int32),
                ("params", Params), ("box", Box), ("h_max", C.c_double)] + [
        (k, _VP) for k in _REQ_ARRAYS]


class RunResult(C.Structure):
    _fields_ = [(k, _VP) for k in _RES_ARRAYS] + [
        ("diag", C.c_double * 8), ("dt", C.c_double), ("t_submit", C.c_double),
        ("t_admit", C.c_double), ("t_done", C.c_double), ("steps_done", C.c_int32),
        ("status", C.c_int32)]


class EnsCounters(C.Structure):
    _fields_ = [(k, C.c_int64) for k in (
        "submitted", "completed", "queued", "running", "steps", "particle_steps",
        "capacity_particles", "capacity_cells", "bytes_per_particle", "bytes_allocated",
        "peak_particles")] + [("peak_runs", C.c_int32), ("max_slots", C.c_int32),
                              ("busy_seconds", C.c_double)]


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
            "sph_ctx_timing": (C.c_int32, [_VP, C.c_int32]),
            "sph_ctx_kernel_time": (C.c_int32, [_VP, C.c_char_p, C.POINTER(C.c_double),
                                                C.POINTER(C.c_int64)]),
            "sph_build_cells": (C.c_int32, [_VP, P, B, C.c_double]),
            "sph_find_neighbors": (C.c_int32, [_VP, P, B, N]),
            "sph_density": (C.c_int32, [_VP, P, B, N, M, _VP]),
            "sph_density_noalloc": (C.c_int32, [P, B, N, M, _VP, _VP]),
            "sph_eos": (C.c_int32, [_VP, P, M, F]),
            "sph_gravity_direct": (C.c_int32, [_VP, P, C.c_double, _VP, _VP, _VP]),
            "sph_volume_weights": (C.c_int32, [_VP, P, _VP, C.c_double]),
            "sph_gravity_tree": (C.c_int32, [_VP, P, C.c_double, C.c_double, C.c_int32, _VP,
                                             _VP, _VP]),
            "sph_momentum_energy": (C.c_int32, [_VP, P, B, N, M, F, A]),
            "sph_integrate": (C.c_int32, [_VP, P, B, C.c_int32, _VP, A]),
            "sph_timestep": (C.c_int32, [_VP, P, M, F, A, _VP, _VP]),
            "sph_init_forces": (C.c_int32, [_VP, P, B, C.c_double, N, M, F, A, C.c_int32,
                                            _VP, _VP]),
            "sph_step": (C.c_int32, [_VP, P, B, C.c_double, N, M, F, A, _VP, _VP]),
            "sph_step_capture": (C.c_int32, [_VP, P, B, C.c_double, N, M, F, A, _VP, _VP]),
            "sph_step_replay": (C.c_int32, [_VP]),
            "sph_step_blocks": (C.c_int32, [_VP, P, B, C.c_double, N, M, F, A, C.c_int32, _VP,
                                            _VP, _VP, C.POINTER(C.c_int32)]),
            "sph_export_neighbors": (C.c_int32, [_VP, P, N, _VP, _VP, C.c_int64,
                                                 C.POINTER(C.c_int64)]),
            "sph_smoothing_length": (C.c_int32, [_VP, P, B, C.c_double, C.c_int32, C.c_int32,
                                                 C.c_int32, _VP, C.POINTER(C.c_int32)]),
            "sph_ens_create": (C.c_int32, [C.POINTER(_VP), C.POINTER(EnsConfig)]),
            "sph_ens_submit": (C.c_int32, [_VP, C.POINTER(RunRequest),
                                           C.POINTER(C.c_uint64)]),
            "sph_ens_poll": (C.c_int32, [_VP, C.c_uint64, C.POINTER(RunResult)]),
            "sph_ens_wait": (C.c_int32, [_VP, C.c_uint64, C.POINTER(RunResult)]),
            "sph_ens_stats": (C.c_int32, [_VP, C.POINTER(EnsCounters)]),
            "sph_ens_destroy": (C.c_int32, [_VP]),
            "sph_ens_last_error": (C.c_char_p, [_VP]),
            "sph_ens_clock": (C.c_double, []),
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

    def timing(self, enable: bool):
        """sph_ctx_timing: HIP events around the timed kernels' launches."""
        self.raise_on(self.lib.sph_ctx_timing(self.h, 1 if enable else 0))

    def kernel_time(self, kernel: str):
        """sph_ctx_kernel_time: (mean ms per launch, launches) of a timed
        kernel since timing was enabled."""
        ms, k = C.c_double(), C.c_int64()
        self.raise_on(self.lib.sph_ctx_kernel_time(self.h, kernel.encode(), C.byref(ms),
                                                   C.byref(k)))
        return float(ms.value), int(k.value)


def make_params(p, precision: int = SPH_FP64) -> Params:
    """Params struct from an inputs.SphParams-like object."""
    return Params(int(precision), int(p.eos), float(p.rho0), float(p.c0),
                  float(p.gamma_tait), float(p.gamma_gas), float(p.alpha),
                  float(p.beta), float(p.eta2), float(p.c_cfl), float(p.c_force),
                  int(getattr(p, "kernel", SPH_KERNEL_M4)), int(getattr(p, "sinc_n", 5)),
                  int(getattr(p, "gradient", SPH_GRAD_KERNEL)),
                  int(getattr(p, "volume", SPH_VOLUME_STANDARD)),
                  float(getattr(p, "volume_p", 0.7)))


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
        if getattr(ic.params, "volume", SPH_VOLUME_STANDARD) == SPH_VOLUME_GENERALISED:
            # weights of generalised volume elements, permuted with the state
            self.t["xw"] = torch.as_tensor(np.ascontiguousarray(ic.m, dtype=np.float64)).to(**f64)
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
            "gx", "gy", "gz", "id", "xw")])
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


def sph_density_noalloc(st: SphState, prm: Params, rho, stream=None):
    """The density through the entry point that allocates nothing (no
    context; static device scratch): rho is a float64 device tensor of at
    least st.n entries; st must hold lists from sph_find_neighbors."""
    import torch
    lib = load()
    if stream is None:
        stream = torch.cuda.current_stream()
    s = lib.sph_density_noalloc(C.byref(st.particles), C.byref(st.box), C.byref(st.nbrs),
                                C.byref(prm), _ptr(rho), _VP(stream.cuda_stream))
    if s != SPH_OK:
        raise SphError(s, lib.sph_last_error(None).decode())


def sph_gravity_direct(ctx: Context, st: SphState, eps: float = 0.01):
    """Direct-sum self-gravity into st.t["gx"/"gy"/"gz"] (current order). The
    arrays are created if the state has none; from then on the integration
    adds them as the external acceleration."""
    import torch
    if "gx" not in st.t:
        for k in ("gx", "gy", "gz"):
            st.t[k] = torch.zeros(max(st.n, 1), dtype=torch.float64, device=st.device)
        st._refresh()
    ctx.raise_on(ctx.lib.sph_gravity_direct(ctx.h, C.byref(st.particles), float(eps),
                                            _ptr(st.t["gx"]), _ptr(st.t["gy"]),
                                            _ptr(st.t["gz"])))


def sph_gravity_tree(ctx: Context, st: SphState, eps: float = 0.01, theta: float = 0.5,
                     leaf_size: int = 16):
    """Octree (quadrupole) self-gravity into st.t["gx"/"gy"/"gz"] (current
    order), created if the state has none, like sph_gravity_direct."""
    import torch
    if "gx" not in st.t:
        for k in ("gx", "gy", "gz"):
            st.t[k] = torch.zeros(max(st.n, 1), dtype=torch.float64, device=st.device)
        st._refresh()
    ctx.raise_on(ctx.lib.sph_gravity_tree(ctx.h, C.byref(st.particles), float(eps),
                                          float(theta), int(leaf_size), _ptr(st.t["gx"]),
                                          _ptr(st.t["gy"]), _ptr(st.t["gz"])))


def sph_volume_weights(ctx: Context, st: SphState, exponent: float, rho=None):
    """st.t["xw"] = (m / rho)^exponent, rho defaulting to the state's density."""
    import torch
    if "xw" not in st.t:
        st.t["xw"] = torch.zeros(max(st.n, 1), dtype=torch.float64, device=st.device)
        st._refresh()
    r = st.t["rho"] if rho is None else rho
    ctx.raise_on(ctx.lib.sph_volume_weights(ctx.h, C.byref(st.particles), _ptr(r),
                                            float(exponent)))


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


def sph_step_capture(ctx: Context, st: SphState, prm: Params, h_max: float | None = None,
                     diag: bool = True):
    """Record one sph_step on st into the context's HIP graph (kept with
    ctx; st's tensors must stay allocated); sph_step_replay runs it."""
    ctx._captured = (st, prm)  # keep the arguments' memory alive
    ctx.raise_on(ctx.lib.sph_step_capture(
        ctx.h, C.byref(st.particles), C.byref(st.box),
        float(h_max if h_max is not None else st.h_max), C.byref(st.nbrs), C.byref(prm),
        C.byref(st.fields), C.byref(st.accel), _ptr(st.t["dt"]),
        _ptr(st.t["diag"]) if diag else None))


def sph_step_replay(ctx: Context):
    ctx.raise_on(ctx.lib.sph_step_replay(ctx.h))


def sph_step_blocks(ctx: Context, st: SphState, prm: Params, max_bin: int,
                    h_max: float | None = None, diag: bool = True) -> int:
    """One step with individual time steps (bins in st.t["bin"], created on
    first use); st.t["dt"] receives the step D. Returns the substep count."""
    import torch
    if "bin" not in st.t:
        st.t["bin"] = torch.zeros(max(st.n, 1), dtype=torch.float64, device=st.device)
    subs = C.c_int32(0)
    ctx.raise_on(ctx.lib.sph_step_blocks(
        ctx.h, C.byref(st.particles), C.byref(st.box),
        float(h_max if h_max is not None else st.h_max), C.byref(st.nbrs), C.byref(prm),
        C.byref(st.fields), C.byref(st.accel), int(max_bin), _ptr(st.t["bin"]),
        _ptr(st.t["dt"]), _ptr(st.t["diag"]) if diag else None, C.byref(subs)))
    return int(subs.value)


def sph_smoothing_length(ctx: Context, st: SphState, n_target: float = 100.0,
                         lo_count: int = 95, hi_count: int = 105, max_iter: int = 10) -> int:
    """Count-based h iteration on the GPU; gather counts land in st.t["count"]
    (current order) and st.h_max is updated. Returns the last iteration."""
    it = C.c_int32(0)
    ctx.raise_on(ctx.lib.sph_smoothing_length(
        ctx.h, C.byref(st.particles), C.byref(st.box), float(n_target), int(lo_count),
        int(hi_count), int(max_iter), _ptr(st.t["count"]), C.byref(it)))
    st.h_max = float(st.t["h"][: st.n].max().item()) if st.n else st.h_max
    return int(it.value)


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


# ---------------------------------------------------------------- serving --

class Ensemble:
    """The serving engine (include/sph.h, sph_ens_*): runs are submitted as
    host arrays, advanced together on the GPU, and collected by ticket."""

    def __init__(self, budget_bytes: int, max_slots: int = 64, max_n_per_run: int = 262144,
                 precision: int = SPH_FP64, max_nb: int = 128, device: int | None = None,
                 pinned_submit_bytes: int = 0):
        import torch
        self.lib = load()
        if device is None:
            device = torch.cuda.current_device()
        cfg = EnsConfig(int(device), int(precision), int(max_nb), int(max_slots),
                        int(budget_bytes), int(max_n_per_run), int(pinned_submit_bytes))
        h = _VP()
        s = self.lib.sph_ens_create(C.byref(h), C.byref(cfg))
        if s != SPH_OK:
            raise SphError(s, self.lib.sph_ens_last_error(None).decode())
        self.h = h

    def _raise(self, s: int):
        if s != SPH_OK:
            raise SphError(s, self.lib.sph_ens_last_error(self.h).decode())

    def submit(self, ic, n_steps: int, set_rho_ref: bool = True, h_max: float | None = None,
               rho_ref=None) -> int:
        """Queue a run of the initial state `ic` (inputs.SphIC); returns the ticket."""
        arrs = ic.arrays()
        keep = {}
        for k in _REQ_ARRAYS:
            if k == "rho_ref":
                src = rho_ref
            else:
                src = arrs[k]
            if src is None:
                keep[k] = None
                continue
            dt = np.int32 if k == "id" else np.float64
            keep[k] = np.ascontiguousarray(src, dtype=dt)
        req = RunRequest(int(ic.n), int(n_steps), int(bool(set_rho_ref)),
                         make_params(ic.params, SPH_FP64), make_box(ic.lo, ic.hi, ic.periodic),
                         float(h_max if h_max is not None else np.max(ic.h)),
                         *[None if keep[k] is None else _VP(keep[k].ctypes.data)
                           for k in _REQ_ARRAYS])
        t = C.c_uint64(0)
        self._raise(self.lib.sph_ens_submit(self.h, C.byref(req), C.byref(t)))
        return int(t.value)

    def _result(self, fn, ticket: int, n: int, arrays: bool = True):
        out = {k: np.empty(n) for k in _RES_ARRAYS} if arrays else {}
        res = RunResult(*[_VP(out[k].ctypes.data) if arrays else None for k in _RES_ARRAYS])
        s = fn(self.h, C.c_uint64(ticket), C.byref(res))
        if s == SPH_E_AGAIN:
            return None
        self._raise(s)
        out.update(diag=np.array(res.diag[:]), dt=res.dt, t_submit=res.t_submit,
                   t_admit=res.t_admit, t_done=res.t_done, steps_done=res.steps_done,
                   status=res.status)
        return out

    def poll(self, ticket: int, n: int, arrays: bool = True):
        """Result dict (arrays in id order unless arrays=False), or None while
        the run is not done."""
        return self._result(self.lib.sph_ens_poll, ticket, n, arrays)

    def wait(self, ticket: int, n: int, arrays: bool = True):
        return self._result(self.lib.sph_ens_wait, ticket, n, arrays)

    def stats(self) -> dict:
        c = EnsCounters()
        self._raise(self.lib.sph_ens_stats(self.h, C.byref(c)))
        return {k: getattr(c, k) for k, _ in EnsCounters._fields_}

    def close(self):
        if self.h:
            s = self.lib.sph_ens_destroy(self.h)
            self.h = _VP()
            self._raise(s)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def ens_clock() -> float:
    return float(load().sph_ens_clock())
