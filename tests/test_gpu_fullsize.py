"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (the single-run calls, one context sized for the run).

* Rotating square patch 100^3 (1,000,000 particles): every particle's
  neighbour set bit-exact, and rho, a, du/dt against the FP64 oracle within
  the FP64 and FP32-pair tolerances; the same for the kernel options the
  bench times on these lists (Wendland C2, sinc, IAD, generalised volume
  elements).
* Evrard-like sphere, 1,000,000 particles (analytic h, dense centre): the
  same, covering the dense-cell and per-lane search paths at full size.
* Rotating square patch 400^3 (64,000,000 particles): a random sample of
  10^4 particles per call against the oracle's subset evaluator (neighbour
  sets bit-exact; rho, a, du/dt in FP64 and FP32-pair, on identical input
  snapshots), which runs the 64-bit record offsets of the pair kernels (the
  records exceed 4 GiB); and properties that hold at any size: linear
  momentum of the pairwise forces to round-off, neighbour counts within the
  lattice bounds, and L_z and total energy after steps.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_1809_08013_amd import inputs as I  # noqa: E402
from paper_1809_08013_amd import sph as S  # noqa: E402
from gpu_helpers import field_errors, gpu_forces, oracle_forces  # noqa: E402

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

FP64_TOL = 1e-12
FP32_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.load()
    torch.cuda.set_device(0)


def _check(ic, ref, max_nb, label):
    got, _, ctx = gpu_forces(ic, ref["rho_ref"], S.SPH_FP64, max_nb=max_nb, rho_in=ref["rho"])
    assert np.array_equal(got["off"], ref["off"]), label
    assert np.array_equal(got["ids"], ref["ids"]), label
    e = field_errors(ref, got)
    print(label, "fp64", e, flush=True)
    assert e["rho"] <= FP64_TOL and e["a"] <= FP64_TOL and e["du"] <= FP64_TOL
    assert e["dt"] <= 1e-14
    got32, _, _ = gpu_forces(ic, ref["rho_ref"], S.SPH_FP32_PAIR, max_nb=max_nb,
                             rho_in=ref["rho"], export=False, ctx=ctx)
    e32 = field_errors(ref, got32)
    print(label, "fp32-pair", e32, flush=True)
    assert e32["rho"] <= FP32_TOL and e32["a"] <= FP32_TOL and e32["du"] <= FP32_TOL
    assert e32["dt"] <= FP32_TOL


def test_square_patch_1M_every_particle():
    ic = I.square_patch(100, seed=0)
    print("case square patch 100^3", flush=True)
    ref = oracle_forces(ic)
    _check(ic, ref, 128, "patch 1M")


@pytest.mark.parametrize("option", ["wendland_c2", "sinc_5", "m4_iad", "m4_gve"])
def test_square_patch_1M_kernel_options(option):
    """The kernel options the bench times on the 1M patch lists, every
    particle against the full FP64 oracle with the same option: Wendland C2,
    sinc n = 5, IAD gradients, generalised volume elements (X = (m/rho)^0.7
    from the oracle's standard density)."""
    import dataclasses
    import oracle as O
    ic = I.square_patch(100, seed=0)
    print(f"case square patch 100^3, {option}", flush=True)
    lo, hi, per = ic.lo, ic.hi, ic.periodic
    xw = None
    if option == "m4_gve":
        ic.params = dataclasses.replace(ic.params, volume=S.SPH_VOLUME_GENERALISED,
                                        volume_p=0.7)
        off, ids = O.neighbors(ic.x, ic.y, ic.z, ic.h, lo, hi, per)
        rho0 = O.density(ic.x, ic.y, ic.z, ic.h, ic.m, lo, hi, per, off, ids)
        xw = O.volume_weights(ic.m, rho0, 0.7)
        rho = O.density(ic.x, ic.y, ic.z, ic.h, ic.m, lo, hi, per, off, ids, X=xw)
        p, c, pr2 = O.eos(ic.params, rho, ic.u, rho0, ic.p_bg)
        acc = O.momentum_energy(ic.x, ic.y, ic.z, ic.vx, ic.vy, ic.vz, ic.h, ic.m, rho, c,
                                pr2, lo, hi, per, off, ids, ic.params, scales=True, X=xw)
        dt = O.timestep(ic.h, c, acc["mumax"], acc["ax"], acc["ay"], acc["az"], ic.params)
        ref = dict(off=off, ids=ids, rho=rho, rho_ref=rho0, dt=dt, **acc)
    else:
        family = {"wendland_c2": S.SPH_KERNEL_WENDLAND_C2, "sinc_5": S.SPH_KERNEL_SINC,
                  "m4_iad": S.SPH_KERNEL_M4}[option]
        grad = S.SPH_GRAD_IAD if option == "m4_iad" else S.SPH_GRAD_KERNEL
        ic.params = dataclasses.replace(ic.params, kernel=family, sinc_n=5, gradient=grad)
        O.set_kernel(family, 5)
        O.set_gradient(O.GRADIENT_IAD if option == "m4_iad" else O.GRADIENT_KERNEL)
        try:
            ref = oracle_forces(ic)
        finally:
            O.set_kernel(O.KERNEL_M4)
            O.set_gradient(O.GRADIENT_KERNEL)
    got, _, ctx = gpu_forces(ic, ref["rho_ref"], S.SPH_FP64, max_nb=128, rho_in=ref["rho"],
                             xw=xw)
    assert np.array_equal(got["off"], ref["off"]) and np.array_equal(got["ids"], ref["ids"])
    e = field_errors(ref, got)
    print(option, "fp64", e, flush=True)
    assert e["rho"] <= FP64_TOL and e["a"] <= FP64_TOL and e["du"] <= FP64_TOL
    assert e["dt"] <= 1e-13
    got32, _, _ = gpu_forces(ic, ref["rho_ref"], S.SPH_FP32_PAIR, max_nb=128,
                             rho_in=ref["rho"], xw=xw, export=False, ctx=ctx)
    e32 = field_errors(ref, got32)
    print(option, "fp32-pair", e32, flush=True)
    assert e32["rho"] <= FP32_TOL and e32["a"] <= FP32_TOL and e32["du"] <= FP32_TOL


def test_evrard_1M_every_particle():
    ic = I.evrard(1_000_000, seed=0)
    print("case Evrard 1M", flush=True)
    ref = oracle_forces(ic, rho_ref=np.ones(ic.n))
    max_nb = int(np.diff(ref["off"]).max()) + 8
    _check(ic, ref, max_nb, "evrard 1M")


def test_evrard_1M_gpu_iterated_h():
    """The Evrard sphere in the state the bench times: h from the GPU's own
    count iteration (sph_smoothing_length), whose largest h sets coarser
    cells than the analytic guess, so the dense centre takes the dense-union
    walk with more candidates. Every particle's set bit-exact, fields within
    the FP64 and FP32-pair tolerances."""
    ic = I.evrard(1_000_000, seed=0)
    print("case Evrard 1M, GPU-iterated h", flush=True)
    ctx = S.Context(ic.n, 64)
    st = S.SphState(ic, 64)
    S.sph_smoothing_length(ctx, st)
    ic.h = st.host(["h"])["h"]
    del ctx, st
    ref = oracle_forces(ic, rho_ref=np.ones(ic.n))
    max_nb = int(np.diff(ref["off"]).max()) + 8
    _check(ic, ref, max_nb, "evrard 1M iterated h")


def test_evrard_1M_smoothing_length_bitwise():
    """The GPU h iteration at full size equals the oracle's bit for bit."""
    import oracle as O
    ic = I.evrard(1_000_000, seed=0)
    print("case Evrard 1M h iteration", flush=True)
    h_ref, cnt_ref, it_ref = O.smoothing_length(ic.x, ic.y, ic.z, ic.h, ic.lo, ic.hi,
                                                ic.periodic)
    ctx = S.Context(ic.n, 64)
    st = S.SphState(ic, 64)
    it = S.sph_smoothing_length(ctx, st)
    got = st.host(["h", "count"])
    print("iterations", it, it_ref, flush=True)
    assert it == it_ref
    assert np.array_equal(got["count"], cnt_ref)
    assert np.array_equal(got["h"], h_ref)


def _sampled_parity(ctx, st, ic, prm, precision, sel, ref, label):
    """One density and one EOS + momentum call of the given precision on the
    state's current lists, checked on the sampled particles against the
    oracle's subset results ref (computed on the same FP64 snapshot). The
    momentum call gets the FP64 density the oracle used."""
    import torch as T
    n = ic.n
    p = S.make_params(ic.params, precision)
    S.sph_density(ctx, st, p)
    S.sph_ctx_check(ctx)
    rho = st.t["rho"][:n][T.as_tensor(sel, device=st.device)].cpu().numpy()
    er = float(np.max(np.abs(rho - ref["rho"]) / ref["rho"]))
    st.t["rho"][:n].copy_(T.as_tensor(ref["rho_all"], device=st.device))
    S.sph_eos(ctx, st, p)
    S.sph_momentum_energy(ctx, st, p)
    S.sph_ctx_check(ctx)
    sl = T.as_tensor(sel, device=st.device)
    g = {k: st.t[k][:n][sl].cpu().numpy() for k in ("ax", "ay", "az", "dudt")}
    da = np.sqrt((g["ax"] - ref["ax"]) ** 2 + (g["ay"] - ref["ay"]) ** 2
                 + (g["az"] - ref["az"]) ** 2)
    ea = float(np.max(da / np.where(ref["sa"] > 0, ref["sa"], 1.0)))
    eu = float(np.max(np.abs(g["dudt"] - ref["dudt"]) / np.where(ref["su"] > 0, ref["su"], 1.0)))
    print(label, "sampled errors rho", er, "a", ea, "du", eu, flush=True)
    return er, ea, eu


def test_square_patch_64M_sampled_and_invariants():
    import oracle as O
    ic = I.square_patch(400, seed=0)
    n = ic.n
    print("case square patch 400^3", flush=True)
    ctx = S.Context(n, 128)
    st = S.SphState(ic, 128)
    prm = S.make_params(ic.params)
    S.sph_init_forces(ctx, st, prm, set_rho_ref=True)
    S.sph_ctx_check(ctx)
    t = st.t
    # sampled parity per call, on the state after the t = 0 evaluation (the
    # lists, density, pressure and sound speed of this state; GPU order)
    keys = ("x", "y", "z", "vx", "vy", "vz", "h", "m", "rho", "c", "pr2", "count")
    H = {k: t[k][:n].cpu().numpy() for k in keys}
    sel = np.sort(np.random.default_rng(7).choice(n, 10_000, replace=False))
    box = (ic.lo, ic.hi, ic.periodic)
    so, si = O.neighbors_subset(H["x"], H["y"], H["z"], H["h"], *box, sel)
    rows = t["idx"][: 128 * n].view(128, n)[:, torch.as_tensor(sel, device=st.device)]
    rows = rows.cpu().numpy()
    for q in range(len(sel)):
        c = int(H["count"][sel[q]])
        assert c == so[q + 1] - so[q], q
        assert np.array_equal(rows[:c, q], si[so[q]:so[q + 1]]), q
    ref = {"rho": O.density_subset(H["x"], H["y"], H["z"], H["h"], H["m"], *box, sel, so, si),
           "rho_all": H["rho"]}
    ref.update(O.momentum_energy_subset(H["x"], H["y"], H["z"], H["vx"], H["vy"], H["vz"],
                                        H["h"], H["m"], H["rho"], H["c"], H["pr2"], *box, sel,
                                        so, si, ic.params))
    del H
    er, ea, eu = _sampled_parity(ctx, st, ic, prm, S.SPH_FP64, sel, ref, "64M fp64")
    assert er <= FP64_TOL and ea <= FP64_TOL and eu <= FP64_TOL
    er, ea, eu = _sampled_parity(ctx, st, ic, prm, S.SPH_FP32_PAIR, sel, ref, "64M fp32-pair")
    assert er <= FP32_TOL and ea <= FP32_TOL and eu <= FP32_TOL
    # back to the FP64 state for the invariants
    S.sph_density(ctx, st, prm)
    S.sph_eos(ctx, st, prm)
    S.sph_momentum_energy(ctx, st, prm)
    S.sph_timestep(ctx, st, prm)
    S.sph_ctx_check(ctx)
    cnt = t["count"][:n]
    # interior lattice particles have 92..122 neighbours, none more than 128
    assert int(cnt.max().item()) <= 128 and int(cnt.min().item()) >= 20
    # pairwise antisymmetric forces: sum m a = 0 to round-off (periodic z only
    # adds exact images, so this holds in every component)
    m = t["m"][:n]
    tot = [float(torch.sum(m * t[k][:n]).item()) for k in ("ax", "ay", "az")]
    scale = float(torch.sum(m * torch.sqrt(t["ax"][:n] ** 2 + t["ay"][:n] ** 2
                                           + t["az"][:n] ** 2)).item())
    print("sum m a", tot, "scale", scale, flush=True)
    assert max(abs(v) for v in tot) < 1e-10 * scale
    d0 = st.diag.copy()
    for _ in range(3):
        S.sph_step(ctx, st, prm)
    S.sph_ctx_check(ctx)
    d1 = st.diag
    print("totals before", d0, "after", d1, flush=True)
    assert abs(d1[6] - d0[6]) <= 1e-12 * abs(d0[6])     # L_z
    assert abs(d1[7] - d0[7]) <= 1e-6 * abs(d0[7])      # energy over 3 steps
    assert abs(d1[1] - d0[1]) < 1e-12 and abs(d1[2] - d0[2]) < 1e-12  # P_x, P_y


def test_evrard_1M_gravity_sampled():
    """Direct-sum self-gravity on the 1M Evrard sphere: 2,000 sampled
    particles against the oracle's sum over all 10^6 (errors in units of the
    sum of the absolute pair terms)."""
    import oracle as O
    ic = I.evrard(1_000_000, seed=0)
    print("case Evrard 1M gravity", flush=True)
    ctx = S.Context(ic.n, 64)
    st = S.SphState(ic, 64)
    S.sph_gravity_direct(ctx, st, 0.01)
    S.sph_ctx_check(ctx)
    got = st.host(["gx", "gy", "gz"])
    sel = np.random.default_rng(7).choice(ic.n, 2000, replace=False)
    gx, gy, gz, sg = O.gravity_direct_subset(ic.x, ic.y, ic.z, ic.m, sel, eps=0.01)
    d = np.sqrt((got["gx"][sel] - gx) ** 2 + (got["gy"][sel] - gy) ** 2
                + (got["gz"][sel] - gz) ** 2)
    e = float(np.max(d / sg))
    print("gravity 1M sampled error", e, flush=True)
    assert e <= 1e-12


def test_evrard_1M_gravity_tree():
    """Octree gravity at the bench's size (1M Evrard sphere, theta = 0.5,
    leaves of 16), every particle against the oracle's octree within 1e-12
    of its term-magnitude sum."""
    import oracle as O
    ic = I.evrard(1_000_000, seed=0)
    print("case tree evrard_1M", flush=True)
    gx, gy, gz, sc, st = O.gravity_tree(ic.x, ic.y, ic.z, ic.m, 0.01, 0.5, 16)
    ctx = S.Context(ic.n, 64)
    s = S.SphState(ic, 64)
    S.sph_gravity_tree(ctx, s, 0.01, 0.5, 16)
    S.sph_ctx_check(ctx)
    got = s.host(["gx", "gy", "gz"])
    err = np.sqrt((got["gx"] - gx) ** 2 + (got["gy"] - gy) ** 2 + (got["gz"] - gz) ** 2)
    rel = float(np.max(err / sc))
    print("evrard 1M tree max err / scale", rel, st, flush=True)
    assert rel <= 1e-12


def test_evrard_1M_individual_time_steps():
    """One step with individual time steps (max_bin = 4) at the bench's size:
    the 1M Evrard sphere (analytic h) with the oracle's octree field held
    fixed; D, every bin and the state against the oracle."""
    import oracle as O
    ic = I.evrard(1_000_000, seed=0)
    print("case Evrard 1M individual time steps", flush=True)
    g = O.gravity_tree(ic.x, ic.y, ic.z, ic.m, 0.01, 0.5, 16)[:3]
    ref = O.OracleRun(ic, g=g).init()
    max_nb = int(np.diff(ref.off).max()) + 64
    ctx = S.Context(ic.n, max_nb)
    st = S.SphState(ic, max_nb, g=g)
    prm = S.make_params(ic.params)
    S.sph_init_forces(ctx, st, prm, set_rho_ref=False)
    subs = S.sph_step_blocks(ctx, st, prm, 4)
    D, b, rsubs = ref.step_blocks(4)
    S.sph_ctx_check(ctx)
    got = st.host(["bin", "x", "y", "z", "vx", "vy", "vz", "u"])
    print("D", st.dt, D, "substeps", subs, rsubs, flush=True)
    assert subs == rsubs and abs(st.dt - D) <= 1e-14 * D
    assert np.array_equal(got["bin"].astype(np.int64), b)
    err = {k: float(np.max(np.abs(got[k] - ref.s[k]))) for k in ("x", "y", "z", "vx", "vy",
                                                                   "vz", "u")}
    print("evrard 1M blocks max errors", err, flush=True)
    assert max(err[k] for k in ("x", "y", "z")) <= 1e-12
    assert max(err[k] for k in ("vx", "vy", "vz", "u")) <= 1e-10
