#!/usr/bin/env python3
"""Benchmark: SPH hydro steps of the 1,000,000-particle rotating square patch
on one MI355X, through the C ABI of libsph.

One step = kick-drift, cell build (Morton radix sort + reorder), neighbour
search, density, EOS, momentum/energy with artificial viscosity, kick, and
the global time-step with the FP64 conserved totals, all on the GPU. Inputs
are resident in HBM before the timed region; the t = 0 force evaluation is
untimed. Prints ONE JSON line.

    python bench.py [--gpus 1] [--steps 50] [--warmup 5]

value = pair-interactions/s of the plain FP64 form (directed neighbour pairs
per step / wall time per step of the call-by-call launches). The same step
captured in a HIP graph (sph_step_capture) is replayed afterwards and its
step time reported beside it. The FP32-pair form (FP32 pair arithmetic,
FP64 state, integration and reductions) is timed on the same GPU and
reported beside it. The CPU baseline is the FP64 oracle on the host cores.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
FP64_VECTOR_PEAK_TFLOPS = 78.6  # MI355X FP64 vector
FP32_VECTOR_PEAK_TFLOPS = 157.3

CALLS = ("integrate_kd", "build_cells", "find_neighbors", "density", "eos",
         "momentum_energy", "integrate_k", "timestep")


def log(msg: str) -> None:
    """Progress on stderr (stdout carries only the JSON line)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def stencil_candidates(ic) -> float:
    """Candidates a cell-list search tests: for every particle, the particles
    of the 27 cells around its own (cells of side >= 2 h_max, the grid the
    library builds for this box, at most 1024 per axis), summed exactly from
    the cell occupancy."""
    import numpy as np
    lo, hi, per = np.array(ic.lo), np.array(ic.hi), ic.periodic
    want = 2.0 * float(np.max(ic.h)) * (1.0 + 1e-9)
    nc = np.clip(np.floor((hi - lo) / want), 1, 1024).astype(int)
    idx = []
    for a, v in enumerate((ic.x, ic.y, ic.z)):
        c = np.floor((v - lo[a]) * (nc[a] / (hi[a] - lo[a])))
        idx.append(np.clip(c, 0, nc[a] - 1).astype(int))
    cnt = np.zeros(nc, dtype=np.int64)
    np.add.at(cnt, tuple(idx), 1)
    tot = np.zeros_like(cnt)
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dz in (-1, 0, 1):
                sh = cnt
                for a, d in enumerate((dx, dy, dz)):
                    if d == 0:
                        continue
                    if per[a]:
                        sh = np.roll(sh, -d, axis=a)
                    else:
                        sh = np.roll(sh, -d, axis=a)
                        sl = [slice(None)] * 3
                        sl[a] = slice(nc[a] - 1, nc[a]) if d > 0 else slice(0, 1)
                        sh = sh.copy()
                        sh[tuple(sl)] = 0
                tot += sh
    return float(np.sum(cnt * tot))


def kernel_model(n: int, pairs: float, candidates: float, precision: int) -> dict:
    """Algorithmic HBM bytes and FP64-equivalent flops per launch of each call.

    Bytes: compulsory traffic with each particle's own arrays read or written
    once, neighbour-list entries 4 B each, neighbour (j) data served from
    cache, the reorder counted in place (read + write of every field once).
    Flops (FMA = 2): the search tests every stencil candidate (3 differences,
    r^2 with one multiply and two FMAs: 8); density ~20 and momentum ~75 per
    directed pair.
    """
    nb = pairs / max(n, 1)
    own_pair = 88 if precision == 0 else 68
    per_particle_bytes = {
        "integrate_kd": 144,
        "build_cells": 40 + 3 * 16 + 2 * 92 + 32,
        "find_neighbors": 40 + 4 * nb,
        "density": 52 + 4 * nb,
        "eos": 48,
        "momentum_energy": own_pair + 44 + 4 * nb,
        "integrate_k": 120,
        "timestep": 112,
    }
    flops = {"find_neighbors": 8.0 * candidates, "density": 20.0 * pairs,
             "momentum_energy": 75.0 * pairs}
    return {k: (per_particle_bytes[k] * n, flops.get(k, 0.0)) for k in CALLS}


# the timed kernels (sph_ctx_kernel_time) and the call each belongs to
TIMED_KERNELS = ("find_neighbors_kernel", "fallback_kernel", "density_kernel", "iad_kernel",
                 "momentum_kernel")
CALL_OF_KERNEL = {"find_neighbors_kernel": "find_neighbors", "fallback_kernel": "find_neighbors",
                  "density_kernel": "density", "iad_kernel": "momentum_energy",
                  "momentum_kernel": "momentum_energy"}
# non-packed lane-instructions per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
VALU_LANE_INSTS_PER_S = 256 * 4 * 16 * 2.4e9


def recorded_counters(kernel: str, workload: str) -> dict:
    """Counter figures per launch of `kernel` from the committed summary
    (profiles/<kernel>_<workload>_counters.md): HBM bytes (traffic) and
    SQ_INSTS_VALU (valu_insts, wave-instructions); empty when there is none or
    the kernel source changed since the counters were taken."""
    import hashlib
    import re
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_counters.md")
    if not os.path.exists(path):
        return {}
    txt = open(path).read()
    h = re.search(r"source_sha256:\s*([0-9a-f]{64})\s+(\S+)", txt)
    if not h:
        return {}
    src = os.path.join(ROOT, h.group(2))
    if not os.path.exists(src):
        return {}
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != h.group(1):
        return {}
    out = {}
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    if m:
        out["traffic"] = float(m.group(1))
    m = re.search(r"valu_insts_per_launch:\s*([0-9.eE+]+)", txt)
    if m:
        out["valu_insts"] = float(m.group(1))
    return out


def run_gpu(ic, precision: int, steps: int, warmup: int, max_nb: int = 128, g=None,
            iterate_h: bool = False, self_gravity=None, graph: bool = False) -> dict:
    """Three legs from the same state (a snapshot taken after the t = 0
    evaluation, restored before each): `steps` steps call by call with no
    instrumentation, whose wall time is ms_per_step; the same steps with a
    HIP event between calls and the library's kernel timer on (per-call and
    per-kernel times, which the events themselves slow slightly); with
    graph=True, sph_step captured into a HIP graph after the warm-up and
    `steps` replays timed (graph_ms_per_step). Each leg runs `warmup` steps
    first."""
    import numpy as np
    import torch

    from paper_1809_08013_amd import sph as S

    log(f"run n={ic.n} precision={precision} steps={steps} warmup={warmup}")
    ctx = S.Context(ic.n, max_nb)
    st = S.SphState(ic, max_nb, g=g)
    prm = S.make_params(ic.params, precision)
    h_iter = None
    if iterate_h:
        # count-based smoothing-length iteration on the GPU (setup, untimed in
        # the step rate; its own time is reported)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        it = S.sph_smoothing_length(ctx, st)
        torch.cuda.synchronize()
        h_iter = {"iterations": it, "ms": (time.perf_counter() - t0) * 1e3,
                  "gather_count_min": int(st.t["count"][: ic.n].min().item()),
                  "gather_count_max": int(st.t["count"][: ic.n].max().item())}
    S.sph_init_forces(ctx, st, prm, set_rho_ref=ic.params.eos == S.SPH_EOS_TAIT)
    S.sph_ctx_check(ctx)
    diag0 = st.diag.tolist()

    calls = [
        lambda: S.sph_integrate(ctx, st, S.SPH_KICK_DRIFT),
        lambda: S.sph_build_cells(ctx, st),
        lambda: S.sph_find_neighbors(ctx, st),
        lambda: S.sph_density(ctx, st, prm),
        lambda: S.sph_eos(ctx, st, prm),
        lambda: S.sph_momentum_energy(ctx, st, prm),
        lambda: S.sph_integrate(ctx, st, S.SPH_KICK),
        lambda: S.sph_timestep(ctx, st, prm),
    ]
    names = list(CALLS)
    if self_gravity is not None:
        # Alg. 1 step 4 in the loop: octree gravity at the drifted positions,
        # before the closing kick (which adds g)
        eps, theta, leaf = self_gravity
        S.sph_gravity_tree(ctx, st, eps, theta, leaf)
        calls.insert(6, lambda: S.sph_gravity_tree(ctx, st, eps, theta, leaf))
        names.insert(6, "gravity_tree")
    stream = ctx.stream
    # the state every leg starts from (the lists are rebuilt by every step
    # before they are read)
    snap = {k: v.clone() for k, v in st.t.items() if k not in ("idx", "count")}

    def restore():
        for k, v in snap.items():
            st.t[k].copy_(v)

    def step(evs=None):
        for k, c in enumerate(calls):
            if evs is not None:
                evs[k].record(stream)
            c()
        if evs is not None:
            evs[len(calls)].record(stream)

    for _ in range(warmup):
        step()
    S.sph_ctx_check(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        step()
    torch.cuda.synchronize()
    eager_ms = (time.perf_counter() - t0) * 1e3 / steps
    S.sph_ctx_check(ctx)
    pairs = float(st.t["count"][: ic.n].sum().item())
    diag = st.diag
    dt = st.dt
    max_count = int(st.t["count"][: ic.n].max().item())
    restore()
    for _ in range(warmup):
        step()
    S.sph_ctx_check(ctx)
    events = [[torch.cuda.Event(enable_timing=True) for _ in range(len(calls) + 1)]
              for _ in range(steps)]
    ctx.timing(True)  # HIP events around the hot kernels, on the library's stream
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        step(events[s])
    torch.cuda.synchronize()
    ctx.timing(False)
    kernel_ms = {}
    for k in TIMED_KERNELS:
        ms, launches = ctx.kernel_time(k)
        if launches:
            kernel_ms[k] = {"avg_ms": round(ms, 5), "launches": launches}
    S.sph_ctx_check(ctx)
    per_call = {k: 0.0 for k in names}
    for evs in events:
        for k, name in enumerate(names):
            per_call[name] += evs[k].elapsed_time(evs[k + 1])
    per_call = {k: v / steps for k, v in per_call.items()}  # ms per launch
    # hipEvent time from the first call to the last of each step, median over
    # the timed steps after the first
    step_ev = sorted(evs[0].elapsed_time(evs[len(calls)]) for evs in events[1:]) or [0.0]
    step_median = step_ev[len(step_ev) // 2]
    graph_ms = None
    if graph and self_gravity is None:
        restore()
        for _ in range(warmup - 1):
            step()
        S.sph_step_capture(ctx, st, prm)
        S.sph_step_replay(ctx)  # first replay (graph upload): the last warm-up step
        S.sph_ctx_check(ctx)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(steps):
            S.sph_step_replay(ctx)
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) * 1e3 / steps
        S.sph_ctx_check(ctx)
    return dict(ms_per_step=eager_ms, graph_ms_per_step=graph_ms,
                step_ms_median_events=step_median,
                per_call_ms=per_call, kernel_ms=kernel_ms,
                candidates=stencil_candidates(ic),
                pairs_per_step=pairs, dt=dt, diag=diag.tolist(), diag0=diag0,
                max_count=max_count, scratch_bytes=ctx.scratch_bytes, h_iteration=h_iter)


def roofline(n: int, r: dict, precision: int, workload: str | None = None,
             copy_gbs: float | None = None) -> dict:
    """HBM roofline of the dominant kernel: the timed kernel with the longest
    mean duration per launch (HIP events around its launches on the library's
    stream, over the timed steps). achieved = its call's algorithmic bytes per
    launch (kernel_model: compulsory traffic, neighbour data from cache) / that
    duration, against the 8 TB/s HBM peak. Beside it: the same kernel's share
    of VALU issue from the committed SQ_INSTS_VALU counter (lane-instructions
    per launch / duration / the chip's 39.3e12 non-packed lane-instructions
    per second), and the counter traffic, both null when the kernel source has
    changed since the counters were taken."""
    model = kernel_model(n, r["pairs_per_step"], r["candidates"], precision)
    km = r["kernel_ms"]
    # kernel time per call; the dominant call's largest kernel is reported
    # alone when it takes >= 95% of the call's kernel time (else the call's
    # kernels together, e.g. the search's two kernels on the Evrard sphere)
    per_call = {}
    for k, v in km.items():
        per_call.setdefault(CALL_OF_KERNEL[k], []).append(k)
    call = max(per_call, key=lambda c: sum(km[k]["avg_ms"] for k in per_call[c]))
    ks = sorted(per_call[call], key=lambda k: -km[k]["avg_ms"])
    tot = sum(km[k]["avg_ms"] for k in ks)
    if km[ks[0]]["avg_ms"] >= 0.95 * tot:
        ks = ks[:1]
    kern = "+".join(ks)
    b, fl = model[call]
    t = sum(km[k]["avg_ms"] for k in ks) * 1e-3
    gbs = b / t / 1e9
    rec = (recorded_counters(kern, workload)
           if (workload and precision == 0 and len(ks) == 1) else {})
    valu = rec.get("valu_insts")
    out = dict(kernel=kern, call=call, bound="hbm", achieved=round(gbs, 1),
               peak=HBM_PEAK_GBS, unit="GB/s", frac=round(gbs / HBM_PEAK_GBS, 4),
               traffic=rec.get("traffic"), ms_per_launch=round(t * 1e3, 5),
               launches=km[ks[0]]["launches"], algorithmic_bytes=b,
               valu_issue_frac=(round(valu * 64 / t / VALU_LANE_INSTS_PER_S, 4)
                                if valu else None),
               call_ms_per_launch=round(r["per_call_ms"][call], 5))
    if copy_gbs:
        out["copy_ceiling_gbs"] = round(copy_gbs, 1)
        out["frac_of_copy"] = round(gbs / copy_gbs, 4)
    return out


def copy_ceiling() -> float:
    """A device-to-device copy of 1 GiB (read + written), best of 5: the HBM
    rate a plain streaming kernel reaches on this GPU, beside the 8 TB/s
    specification."""
    import torch
    a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    best = 0.0
    for _ in range(5):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        best = max(best, 2.0 * a.numel() * 8 / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    return best


def pair_rates(r: dict) -> dict:
    """Directed pairs per second of the density and momentum kernels alone
    (live kernel times)."""
    km, p = r["kernel_ms"], r["pairs_per_step"]
    return {k: p / (km[f"{k}_kernel"]["avg_ms"] * 1e-3)
            for k in ("density", "momentum") if f"{k}_kernel" in km}


def step_hbm(n: int, r: dict, precision: int) -> dict:
    """Whole-step algorithmic bytes against HBM peak."""
    model = kernel_model(n, r["pairs_per_step"], r["candidates"], precision)
    b = sum(v[0] for v in model.values())
    gbs = b / (r["ms_per_step"] * 1e-3) / 1e9
    return {"bytes_per_step": b, "gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
            "ms_at_peak": b / (HBM_PEAK_GBS * 1e9) * 1e3}


def run_evrard(steps: int, warmup: int, n: int = 1_000_000) -> dict:
    """Evrard-like sphere, hydro step only, FP64 and FP32-pair.

    h starts from the analytic estimate for ~100 gather neighbours under the
    1/r profile and is iterated on the GPU (sph_smoothing_length) until every
    gather count is in [95, 105]. The self-gravity of the t = 0 particles is
    summed directly on the GPU (sph_gravity_direct, Plummer eps = 0.01; its
    time is reported) and held fixed as an external acceleration over the
    timed hydro steps: gravity is outside the timed path. The octree gravity
    (sph_gravity_tree, theta = 0.5, leaves of 16) is timed on the same state
    and checked against the direct sum, a third run takes individual time
    steps (sph_step_blocks, max_bin = 5) with the fixed field and compares the
    wall time over the same simulated interval with the global step's, and a
    fourth
    recomputes the octree gravity inside every step (the Evrard collapse with
    self-gravity, Alg. 1 step 4).
    """
    import numpy as np
    import torch

    from paper_1809_08013_amd import inputs as I
    from paper_1809_08013_amd import sph as S
    log(f"generating Evrard sphere n={n}")
    ic = I.evrard(n, seed=0)
    log("direct-sum self-gravity")
    ctx = S.Context(n, 64)
    st = S.SphState(ic, 64)
    S.sph_gravity_direct(ctx, st, 0.01)  # first call: code load
    S.sph_ctx_check(ctx)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S.sph_gravity_direct(ctx, st, 0.01)
    S.sph_ctx_check(ctx)
    t_grav = time.perf_counter() - t0
    gh = st.host(["gx", "gy", "gz"])
    g = (gh["gx"], gh["gy"], gh["gz"])
    log("octree self-gravity")
    S.sph_gravity_tree(ctx, st, 0.01, 0.5, 16)  # first call: buffers, code load
    reps = 10
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        S.sph_gravity_tree(ctx, st, 0.01, 0.5, 16)
    t_tree = (time.perf_counter() - t0) / reps
    th = st.host(["gx", "gy", "gz"])
    gd = np.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
    # |g| -> 0 at the centre, so errors are given in units of the mean |g|
    et = np.sqrt((th["gx"] - g[0]) ** 2 + (th["gy"] - g[1]) ** 2
                 + (th["gz"] - g[2]) ** 2) / float(np.mean(gd))
    tree = {"ms": t_tree * 1e3, "eps": 0.01, "theta": 0.5, "leaf_size": 16,
            "err_vs_direct_in_mean_g_median": float(np.median(et)),
            "err_vs_direct_in_mean_g_p99": float(np.percentile(et, 99)),
            "err_vs_direct_in_mean_g_max": float(et.max()),
            "speedup_vs_direct": t_grav / t_tree}
    del ctx, st
    out = {"workload": f"Evrard-like sphere, {n:,} particles, rho ~ 1/r, ideal gas gamma=5/3, "
                       "h iterated on the GPU to 95-105 gather neighbours, direct-sum "
                       "self-gravity of the initial state as a fixed external g",
           "gravity_direct": {"ms": t_grav * 1e3, "eps": 0.01,
                              "pair_interactions_per_s": float(n) * (n - 1) / t_grav},
           "gravity_tree": tree}
    for name, prec in (("fp64", S.SPH_FP64), ("fp32_pair", S.SPH_FP32_PAIR)):
        res = run_gpu(ic, prec, steps, warmup, max_nb=512, g=g, iterate_h=True)
        out[name] = {"value": res["pairs_per_step"] / (res["ms_per_step"] * 1e-3),
                     "ms_per_step": res["ms_per_step"],
                     "per_call_ms": {k: round(v, 4) for k, v in res["per_call_ms"].items()},
                     "kernel_ms": res["kernel_ms"],
                     "roofline": roofline(n, res, prec),
                     "step_hbm": step_hbm(n, res, prec),
                     "mean_neighbours": res["pairs_per_step"] / n,
                     "max_neighbours": res["max_count"],
                     "h_iteration": res["h_iteration"]}
    out["fp64_individual_time_steps"] = run_blocks(ic, g, max(2, steps // 10), 5)
    res = run_gpu(ic, S.SPH_FP64, steps, warmup, max_nb=512, g=g, iterate_h=True,
                  self_gravity=(0.01, 0.5, 16))
    out["fp64_self_gravity"] = {
        "note": "hydro step plus octree self-gravity recomputed every step",
        "ms_per_step": res["ms_per_step"],
        "per_call_ms": {k: round(v, 4) for k, v in res["per_call_ms"].items()}}
    return out


def run_blocks(ic, g, steps: int, max_bin: int, max_nb: int = 512) -> dict:
    """Individual time steps (sph_step_blocks) against the global step over
    the same simulated interval, from the same state (h iterated, t = 0
    forces): `steps` block steps advance T; global steps (sph_step) then run
    from the same start until they pass T. Reports both wall times."""
    import torch

    from paper_1809_08013_amd import sph as S
    log(f"individual time steps n={ic.n} max_bin={max_bin}")
    prm = S.make_params(ic.params)

    def start():
        ctx = S.Context(ic.n, max_nb)
        st = S.SphState(ic, max_nb, g=g)
        S.sph_smoothing_length(ctx, st)
        S.sph_init_forces(ctx, st, prm, set_rho_ref=False)
        S.sph_ctx_check(ctx)
        torch.cuda.synchronize()
        return ctx, st

    ctx, st = start()
    t_sim, subs = 0.0, []
    t0 = time.perf_counter()
    for _ in range(steps):
        subs.append(S.sph_step_blocks(ctx, st, prm, max_bin))
        t_sim += st.dt
    torch.cuda.synchronize()
    wall_blk = time.perf_counter() - t0
    S.sph_ctx_check(ctx)
    bins = st.host(["bin"])["bin"].astype(int)
    del ctx, st
    ctx, st = start()
    t_glob, n_glob = 0.0, 0
    t0 = time.perf_counter()
    while t_glob < t_sim:
        dt = st.dt  # the dt the next step takes (synchronises)
        S.sph_step(ctx, st, prm, diag=False)
        t_glob += dt
        n_glob += 1
    torch.cuda.synchronize()
    wall_glob = time.perf_counter() - t0
    S.sph_ctx_check(ctx)
    return {"max_bin": max_bin, "steps": steps, "simulated_interval": t_sim,
            "ms_per_step": wall_blk * 1e3 / steps, "mean_substeps": float(sum(subs)) / steps,
            "wall_s": wall_blk, "global_steps": n_glob, "global_wall_s": wall_glob,
            "global_simulated_interval": t_glob, "speedup_vs_global_step": wall_glob / wall_blk,
            "bin_counts_last_step": {int(k): int((bins == k).sum())
                                     for k in sorted(set(bins.tolist()))}}


def drift(r: dict) -> dict:
    """Relative change of total energy and of L_z (|L| for an open box) over
    all steps taken (warm-up included), from the FP64 on-device totals."""
    d0, d1 = r["diag0"], r["diag"]
    de = abs(d1[7] - d0[7]) / max(abs(d0[7]), 1e-300)
    dl = abs(d1[6] - d0[6]) / max(abs(d0[6]), 1e-300)
    return {"energy": de, "angular_momentum_z": dl}


def run_large(n_side: int, steps: int, warmup: int) -> dict:
    """Large rotating square patch (n_side^3 particles), FP32-pair and FP64."""
    from paper_1809_08013_amd import inputs as I
    from paper_1809_08013_amd import sph as S
    log(f"generating square patch {n_side}^3")
    ic = I.square_patch(n_side, seed=0)
    n = ic.n
    out = {"workload": f"rotating square patch, {n_side}^3 = {n:,} particles, same physics "
                       "as the 1M case", "steps": steps, "warmup": warmup}
    finals = {}
    for name, prec in (("fp32_pair", S.SPH_FP32_PAIR), ("fp64", S.SPH_FP64)):
        res = run_gpu(ic, prec, steps, warmup)
        finals[name] = res["diag"]
        out[name] = {"value": res["pairs_per_step"] / (res["ms_per_step"] * 1e-3),
                     "ms_per_step": res["ms_per_step"],
                     "per_call_ms": {k: round(v, 4) for k, v in res["per_call_ms"].items()},
                     "kernel_ms": res["kernel_ms"],
                     "roofline": roofline(n, res, prec),
                     "step_hbm": step_hbm(n, res, prec),
                     "drift": drift(res),
                     "mean_neighbours": res["pairs_per_step"] / n,
                     "scratch_bytes": res["scratch_bytes"]}
    # after the same steps from the same state: FP32-pair totals against FP64
    d32, d64 = finals["fp32_pair"], finals["fp64"]
    out["fp32_vs_fp64"] = {"energy_rel": abs(d32[7] - d64[7]) / abs(d64[7]),
                           "lz_rel": abs(d32[6] - d64[6]) / abs(d64[6])}
    return out


def serving_workload(runs: int, seed: int = 0):
    """Ensemble requests: n log-uniform in [4096, 262144] rounded to a cube
    n_side^3 (n_side in [16, 64]), omega ~ U[2, 8], 50 steps each; each run
    is a seeded rotating square patch. ICs are made before the clock starts
    (a client prepares them before it submits)."""
    import numpy as np
    from concurrent.futures import ThreadPoolExecutor

    from paper_1809_08013_amd import inputs as I
    rng = np.random.default_rng(seed)
    n = np.exp(rng.uniform(np.log(4096), np.log(262144), runs))
    sides = np.clip(np.rint(np.cbrt(n)), 16, 64).astype(int)
    omegas = rng.uniform(2.0, 8.0, runs)
    gaps = rng.exponential(1.0, runs)  # unit-rate Poisson gaps, scaled per rate
    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        ics = list(ex.map(lambda k: I.square_patch(int(sides[k]), omega=float(omegas[k]),
                                                    seed=1000 + k), range(runs)))
    return ics, gaps


def serve(ics, gaps, steps: int, budget: int, max_slots: int, rate: float | None) -> dict:
    """Submit every run (all at once, or at Poisson arrival times of the
    given rate from a client thread), wait for all; latency = done - submit."""
    import threading

    import numpy as np

    from paper_1809_08013_amd import sph as S
    ens = S.Ensemble(budget, max_slots=max_slots, max_n_per_run=max(ic.n for ic in ics))
    tickets = [None] * len(ics)
    try:
        t0 = S.ens_clock()
        if rate is None:
            for k, ic in enumerate(ics):
                tickets[k] = ens.submit(ic, steps)
        else:
            arrive = t0 + np.cumsum(gaps) / rate

            def client():
                for k, ic in enumerate(ics):
                    d = arrive[k] - S.ens_clock()
                    if d > 0:
                        time.sleep(d)
                    tickets[k] = ens.submit(ic, steps)
            th = threading.Thread(target=client)
            th.start()
        res = []
        for k, ic in enumerate(ics):
            while tickets[k] is None:
                time.sleep(0.0005)
            r = ens.wait(tickets[k], ic.n, arrays=False)
            if r["status"] != S.SPH_OK:
                raise RuntimeError(f"run {k} ended with status {r['status']}")
            res.append(r)
        if rate is not None:
            th.join()
        st = ens.stats()
    finally:
        ens.close()
    lat = np.array([r["t_done"] - r["t_submit"] for r in res])
    svc = np.array([r["t_done"] - r["t_admit"] for r in res])
    t_first = min(r["t_submit"] for r in res)
    span = max(r["t_done"] for r in res) - t_first
    pst = float(sum(ic.n for ic in ics)) * steps
    return {"runs_per_s": len(ics) / span, "particle_steps_per_s": pst / span,
            "makespan_s": span, "p50_latency_s": float(np.percentile(lat, 50)),
            "p99_latency_s": float(np.percentile(lat, 99)),
            "p50_service_s": float(np.percentile(svc, 50)),
            "p99_service_s": float(np.percentile(svc, 99)),
            "peak_runs": st["peak_runs"], "peak_particles": st["peak_particles"],
            "batched_steps": st["steps"], "capacity_particles": st["capacity_particles"],
            "bytes_per_particle": st["bytes_per_particle"]}


def run_serving(runs: int, steps: int = 50, budget_gib: float = 8.0) -> dict:
    budget = int(budget_gib * (1 << 30))
    log(f"serving: generating {runs} runs")
    ics, gaps = serving_workload(runs)
    tot = sum(ic.n for ic in ics)
    out = {"workload": f"{runs} rotating square patch runs, n = n_side^3 log-uniform in "
                       f"[4096, 262144] (n_side in [16, 64]), omega ~ U[2, 8], {steps} steps "
                       f"each, HBM budget {budget_gib:g} GiB, FP64, Poisson arrivals",
           "total_particles": tot, "steps_per_run": steps}
    log("serving: saturated (all submitted at once)")
    sat = serve(ics, gaps, steps, budget, 511, None)
    out["saturated"] = sat
    mu = sat["runs_per_s"]
    out["poisson"] = []
    for f in (0.5, 0.8, 1.0):
        log(f"serving: Poisson arrivals at {f} x saturated rate")
        r = serve(ics, gaps, steps, budget, 511, f * mu)
        r["load_fraction"] = f
        r["arrival_rate_runs_per_s"] = f * mu
        out["poisson"].append(r)
    # the baseline engine holds one run: its budget (and so its launch grids)
    # is sized for the largest run, not for the batch
    one_budget = (16 << 20) + int(sat["bytes_per_particle"]) * max(ic.n for ic in ics) * 11 // 10
    log("serving: one run at a time (same engine and kernels, one slot)")
    one = serve(ics, gaps, steps, one_budget, 1, None)
    one["budget_bytes"] = one_budget
    out["one_at_a_time"] = one
    out["throughput_speedup_vs_one_at_a_time"] = sat["runs_per_s"] / one["runs_per_s"]
    return out


def run_kernels(ic, steps: int, warmup: int) -> dict:
    """The interchangeable kernels (M4, Wendland C2, sinc n = 5), the IAD
    gradients and the generalised volume elements (both with M4) on the same
    neighbour lists: time per sph_density and per sph_momentum_energy call
    (IAD: including its matrix pass), FP64, and the pair rate of the two
    together."""
    import dataclasses

    import torch

    from paper_1809_08013_amd import sph as S

    log("kernel families")
    ctx = S.Context(ic.n, 128)
    st = S.SphState(ic, 128)
    S.sph_init_forces(ctx, st, S.make_params(ic.params), set_rho_ref=True)
    S.sph_ctx_check(ctx)
    pairs = float(st.t["count"][: ic.n].sum().item())
    out = {"workload": "rotating square patch 100^3, the same lists; density and "
                       "momentum/energy calls only", "pairs": pairs}
    stream = ctx.stream
    G0, VS, VG = S.SPH_GRAD_KERNEL, S.SPH_VOLUME_STANDARD, S.SPH_VOLUME_GENERALISED
    for name, fam, n, grad, vol in (("m4", S.SPH_KERNEL_M4, 5, G0, VS),
                                    ("wendland_c2", S.SPH_KERNEL_WENDLAND_C2, 5, G0, VS),
                                    ("sinc_5", S.SPH_KERNEL_SINC, 5, G0, VS),
                                    ("m4_iad", S.SPH_KERNEL_M4, 5, S.SPH_GRAD_IAD, VS),
                                    ("m4_gve", S.SPH_KERNEL_M4, 5, G0, VG)):
        prm = S.make_params(dataclasses.replace(ic.params, kernel=fam, sinc_n=n, gradient=grad,
                                                volume=vol))
        if vol == VG:
            S.sph_volume_weights(ctx, st, 0.7)  # weights from the standard density
        for _ in range(warmup):
            S.sph_density(ctx, st, prm)
            S.sph_eos(ctx, st, prm)
            S.sph_momentum_energy(ctx, st, prm)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        dens = mom = 0.0
        for _ in range(steps):
            ev[0].record(stream)
            S.sph_density(ctx, st, prm)
            ev[1].record(stream)
            S.sph_eos(ctx, st, prm)
            S.sph_momentum_energy(ctx, st, prm)
            ev[2].record(stream)
            torch.cuda.synchronize()
            dens += ev[0].elapsed_time(ev[1])
            mom += ev[1].elapsed_time(ev[2])
        S.sph_ctx_check(ctx)
        d, m = dens / steps, mom / steps
        out[name] = {"density_ms": round(d, 4), "eos_plus_momentum_ms": round(m, 4),
                     "pair_rate_both": 2 * pairs / ((d + m) * 1e-3)}
    return out


def gpu_trajectories(ic, steps: int) -> dict:
    """The GPU half of the trajectory comparison: FP64 and FP32-pair runs of
    `steps` KDK steps from the t = 0 state (rho_ref = rho(t = 0)); returns
    each form's final fields (original order), dt and on-device totals."""
    from paper_1809_08013_amd import sph as S
    out = {}
    for name, prec in (("fp64", S.SPH_FP64), ("fp32_pair", S.SPH_FP32_PAIR)):
        log(f"trajectory: GPU {name}, {steps} steps")
        ctx = S.Context(ic.n, 128)
        st = S.SphState(ic, 128)
        prm = S.make_params(ic.params, prec)
        S.sph_init_forces(ctx, st, prm, set_rho_ref=True)
        d0 = st.diag.copy()
        for _ in range(steps):
            S.sph_step(ctx, st, prm)
        S.sph_ctx_check(ctx)
        out[name] = {"fields": st.host(["x", "y", "z", "vx", "vy", "vz", "u", "rho"]),
                     "dt": st.dt, "diag0": d0, "diag": st.diag.copy()}
        del ctx, st
    return out


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_other_configs(threads: int) -> dict:
    """The oracle (all host threads) on the parity-sized patch (20^3, 10 KDK
    steps) and one step of the 1M Evrard sphere (its analytic h, no external
    field: the step's cost, not its physics), each after an untimed t = 0
    force evaluation."""
    import oracle as O
    from paper_1809_08013_amd import inputs as I
    out = {}
    for name, ic, steps in (("square_patch_20", I.square_patch(20, seed=0), 10),
                            ("evrard_1M", I.evrard(1_000_000, seed=0), 1)):
        log(f"CPU oracle: {name}, {steps} steps on {threads} threads")
        run = O.OracleRun(ic).init()
        t0 = time.perf_counter()
        pairs = 0
        for _ in range(steps):
            run.step()
            pairs += run.n_pairs
        t = time.perf_counter() - t0
        out[name] = {"value": pairs / t, "unit": "pair-interactions/s",
                     "ms_per_step": t * 1e3 / steps, "steps": steps, "cores": threads}
    return out


def cpu_leg(ic, traj_steps: int, gpu_traj: dict | None) -> tuple:
    """The CPU baseline leg, the only part of this script that runs the
    oracle: the FP64 oracle (OpenMP over particles, all host threads) takes
    `traj_steps` full KDK steps of the 1M input after an untimed t = 0 force
    evaluation; their rate is cpu_baseline.value. One more step on one thread
    gives the one-core rate. The oracle's final state is the reference for the
    per-field errors of the GPU trajectories (positions, velocities, u, rho:
    max and RMS absolute error, max relative to the field's RMS) and of dt;
    totals drift comes from the FP64 on-device reductions."""
    import numpy as np

    import oracle as O
    threads = O.num_threads()
    log(f"CPU oracle: {traj_steps} steps on {threads} threads")
    run = O.OracleRun(ic).init()
    t0 = time.perf_counter()
    pairs = 0
    for _ in range(traj_steps):
        run.step()
        pairs += run.n_pairs
    t = time.perf_counter() - t0
    base = dict(value=pairs / t, unit="pair-interactions/s", cores=threads,
                kind="oracle", ms_per_step=t * 1e3 / traj_steps, cpu_model=cpu_model(),
                sample=f"{traj_steps} full KDK steps of the same 1,000,000-particle input "
                       "(after an untimed t=0 force evaluation), FP64 oracle, OpenMP over "
                       "particles; one_core: one more step on one thread")
    # copies: the oracle integrates its state arrays in place
    refs = {k: v.copy() for k, v in run.s.items()}
    refs["rho"] = run.rho.copy()
    ref_dt = run.dt
    log("CPU oracle: one step on one thread")
    O.num_threads(1)
    try:
        t0 = time.perf_counter()
        run.step()
        t1 = time.perf_counter() - t0
    finally:
        O.num_threads(threads)
    base["one_core"] = {"value": run.n_pairs / t1, "ms_per_step": t1 * 1e3, "cores": 1}
    base["other_configs"] = cpu_other_configs(threads)
    traj = None
    if gpu_traj is not None:
        traj = {"workload": f"rotating square patch, {ic.n:,} particles, {traj_steps} steps "
                            "from the t = 0 state, GPU against the FP64 oracle",
                "steps": traj_steps}
        for name, g in gpu_traj.items():
            err = {}
            for k in ("x", "y", "z", "vx", "vy", "vz", "u", "rho"):
                d = g["fields"][k] - refs[k]
                scale = float(np.sqrt(np.mean(refs[k] ** 2))) or 1.0
                err[k] = {"max_abs": float(np.max(np.abs(d))),
                          "rms_abs": float(np.sqrt(np.mean(d * d))),
                          "max_rel_to_rms": float(np.max(np.abs(d))) / scale}
            d0, d1 = g["diag0"], g["diag"]
            traj[name] = {"errors": err, "dt_rel": abs(g["dt"] - ref_dt) / ref_dt,
                          "energy_drift": abs(d1[7] - d0[7]) / abs(d0[7]),
                          "lz_drift": abs(d1[6] - d0[6]) / abs(d0[6]),
                          "px_drift_abs": abs(d1[1] - d0[1]),
                          "py_drift_abs": abs(d1[2] - d0[2])}
    return base, traj


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-side", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the CPU oracle leg (and with it the trajectory errors)")
    ap.add_argument("--no-fp32", action="store_true")
    ap.add_argument("--no-evrard", action="store_true",
                    help="skip the 1,000,000-particle Evrard-like sphere leg")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one 1 GiB device-to-device copy (a known-size "
                         "reference for hardware byte counters)")
    ap.add_argument("--trajectory", type=int, default=50, metavar="STEPS",
                    help="FP64 and FP32-pair GPU runs of STEPS steps compared with the "
                         "oracle's (the CPU leg runs the oracle for as many steps; 0: the "
                         "CPU leg times 3 steps and no trajectory is compared)")
    ap.add_argument("--serve-runs", type=int, default=512,
                    help="ensemble serving requests (0 skips the serving leg)")
    ap.add_argument("--no-kernels", action="store_true",
                    help="skip the timing of the Wendland C2 and sinc kernels")
    ap.add_argument("--large", type=int, default=400, metavar="N_SIDE",
                    help="the large square patch of N_SIDE^3 particles (400 gives "
                         "64,000,000), 20 steps after 2 warm-up steps; 0 skips it")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not built)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1809_08013_amd import inputs as I
    from paper_1809_08013_amd import sph as S
    if not os.path.exists(S.LIB_PATH):
        from paper_1809_08013_amd import build
        build.build()
    torch.cuda.set_device(0)
    if args.calibrate_copy:
        a = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    copy_gbs = copy_ceiling()
    ic = I.square_patch(args.n_side, seed=0)
    n = ic.n
    r64 = run_gpu(ic, S.SPH_FP64, args.steps, args.warmup, graph=True)
    r32 = None if args.no_fp32 else run_gpu(ic, S.SPH_FP32_PAIR, args.steps, args.warmup,
                                            graph=True)
    value = r64["pairs_per_step"] / (r64["ms_per_step"] * 1e-3)
    line = {
        "metric": "SPH pair-interactions/s & step time @1M; p50/p99 ensemble-request latency",
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r64["ms_per_step"],
        "graph_ms_per_step": r64["graph_ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"rotating square patch, {args.n_side}^3 = {n:,} particles, "
                        "periodic z, h = 1.5 spacing, cubic spline, Tait EOS, Monaghan AV "
                        "alpha=1 beta=2, KDK with global Courant dt, FP64",
            "n_particles": n,
            "pairs_per_step": r64["pairs_per_step"],
            "mean_neighbours": r64["pairs_per_step"] / n,
            "max_neighbours": r64["max_count"],
        },
        "step_ms_median_events": r64["step_ms_median_events"],
        "per_call_ms": {k: round(v, 4) for k, v in r64["per_call_ms"].items()},
        "kernel_ms": r64["kernel_ms"],
        "pair_rates": pair_rates(r64),
        "roofline": roofline(n, r64, 0, f"square_patch_{args.n_side}", copy_gbs),
        "step_hbm": step_hbm(n, r64, 0),
        "drift": drift(r64),
    }
    if r32 is not None:
        v32 = r32["pairs_per_step"] / (r32["ms_per_step"] * 1e-3)
        line["fp32_pair"] = {
            "value": v32, "ms_per_step": r32["ms_per_step"],
            "graph_ms_per_step": r32["graph_ms_per_step"],
            "speedup_vs_fp64": r64["ms_per_step"] / r32["ms_per_step"],
            "per_call_ms": {k: round(v, 4) for k, v in r32["per_call_ms"].items()},
            "step_ms_median_events": r32["step_ms_median_events"],
            "kernel_ms": r32["kernel_ms"],
            "pair_rates": pair_rates(r32),
            "roofline": roofline(n, r32, 1, None, copy_gbs),
            "step_hbm": step_hbm(n, r32, 1),
        }
    if not args.no_kernels:
        line["kernels"] = run_kernels(ic, min(args.steps, 20), 2)
    traj = None
    if args.trajectory > 0 and not args.no_cpu_baseline:
        traj = gpu_trajectories(ic, args.trajectory)
    if args.serve_runs > 0:
        line["serving"] = run_serving(args.serve_runs)
    if not args.no_evrard:
        line["evrard"] = run_evrard(args.steps, args.warmup)
    if args.large:
        line["large"] = run_large(args.large, 20, 2)
    if not args.no_cpu_baseline:
        base, terr = cpu_leg(ic, args.trajectory if args.trajectory > 0 else 3, traj)
        line["cpu_baseline"] = base
        if terr is not None:
            line["trajectory"] = terr
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
