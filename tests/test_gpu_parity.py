"""Parity of the HIP path (through the C ABI) with the FP64 oracle, element
by element on identical seeded inputs: neighbour sets bit-exact as sorted
original-id sets; rho, a, du/dt, dt within 1e-12 (FP64 form) or 1e-5
(FP32-pair form) in the metrics of tests/gpu_helpers.field_errors."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle as O  # noqa: E402
from paper_1809_08013_amd import inputs as I  # noqa: E402
from paper_1809_08013_amd import sph as S  # noqa: E402
from gpu_helpers import field_errors, gpu_forces, oracle_forces  # noqa: E402

pytestmark = pytest.mark.gpu

FP64_TOL = 1e-12
FP32_TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    S.load()  # fails loudly if libsph.so is missing
    torch.cuda.set_device(0)


def _moving_lattice(seed=0):
    lat = I.lattice_periodic(16, spacing=2.0 ** -4)
    rng = np.random.default_rng(seed)
    lat.vx, lat.vy, lat.vz = (rng.uniform(-1, 1, lat.n) for _ in range(3))
    lat.p_bg = rng.uniform(-0.5, 0.5, lat.n)
    return lat


def _cases():
    return {
        "tie_lattice": (_moving_lattice, 128),
        "cloud_open": (lambda: I.random_cloud(4096, seed=1, h_min=0.03, h_max=0.07), 256),
        "cloud_pz": (lambda: I.random_cloud(3000, seed=2, h_min=0.05, h_max=0.05,
                                            periodic=(0, 0, 1)), 256),
        "cloud_pxyz": (lambda: I.random_cloud(2049, seed=3, h_min=0.04, h_max=0.09,
                                              periodic=(1, 1, 1)), 512),
        "square_patch_c0": (lambda: I.square_patch(20), 128),
        "clump_across_open_faces": (lambda: _clump_cloud(0.95), 256),
        "clump_outside_open_box": (lambda: _clump_cloud(1.10), 256),
    }


def _clump_cloud(c0):
    """A dense clump of 4000 particles (h = 0.0077, ~60 neighbours) in the
    cube [c0, c0 + 0.1] on the open x and z axes of a unit box (partly or
    wholly outside it, so clamped into the border cells), next to 600 sparse
    particles with h up to 0.08 in x < 0.6. The cells (side 2 h_max = 0.16)
    then hold the whole clump in one or two cells: its tiles take the
    dense-union walk, whose windows must keep the clamped particles."""
    ic = I.random_cloud(4600, seed=11, h_min=0.07, h_max=0.08)
    rng = np.random.default_rng(12)
    nc = 4000
    ic.x[:nc] = rng.uniform(c0, c0 + 0.1, nc)
    ic.y[:nc] = rng.uniform(0.45, 0.55, nc)
    ic.z[:nc] = rng.uniform(c0, c0 + 0.1, nc)
    ic.h[:nc] = 0.0077
    ic.x[nc:] *= 0.6
    return ic


@pytest.mark.parametrize("name", list(_cases()))
def test_neighbors_and_fields_fp64(name):
    make, max_nb = _cases()[name]
    ic = make()
    print(f"case {name} n={ic.n}", flush=True)
    ref = oracle_forces(ic)
    got, st, ctx = gpu_forces(ic, ref["rho_ref"], S.SPH_FP64, max_nb=max_nb, rho_in=ref["rho"])
    assert np.array_equal(got["off"], ref["off"])
    assert np.array_equal(got["ids"], ref["ids"])
    e = field_errors(ref, got)
    print(name, e)
    assert e["rho"] <= FP64_TOL and e["a"] <= FP64_TOL and e["du"] <= FP64_TOL
    assert e["dt"] <= 1e-14
    # |mu| = hbar |v.r| / (r^2 + eta2 hbar^2) <= |v_ij| / (2 sqrt(eta2)) = 5 |v_ij|:
    # the scale of mu's rounding error (mu is pure rounding noise under rigid rotation)
    vmax = np.sqrt(ic.vx ** 2 + ic.vy ** 2 + ic.vz ** 2).max()
    assert np.max(np.abs(got["mumax"] - ref["mumax"])) <= 1e-12 * 10 * max(vmax, 1e-300)
    # EOS on identical density: P to rounding of its largest term
    B = ic.params.rho0 * ic.params.c0 ** 2 / ic.params.gamma_tait
    pscale = np.abs(ic.p_bg) + (B * (ref["rho"] / ref["rho_ref"]) ** 7 if ic.params.eos == 0
                                else np.abs(ref["p"]))
    assert np.max(np.abs(got["p"] - ref["p"]) / pscale) <= 1e-14
    assert np.max(np.abs(got["c"] / ref["c"] - 1)) <= 1e-14


def test_tie_lattice_counts_92():
    lat = I.lattice_periodic(16, spacing=2.0 ** -4)
    ref = oracle_forces(lat)
    got, _, _ = gpu_forces(lat, ref["rho_ref"])
    assert (np.diff(got["off"]) == 92).all()
    assert np.abs(got["rho"] - 1.001794705350405).max() < 1e-13


@pytest.mark.parametrize("name", ["square_patch_c0", "cloud_open", "cloud_pxyz"])
def test_fp32_pair_form(name):
    make, max_nb = _cases()[name]
    ic = make()
    ref = oracle_forces(ic)
    # density in the FP32-pair form
    got_d, _, _ = gpu_forces(ic, ref["rho_ref"], S.SPH_FP32_PAIR, max_nb=max_nb)
    assert np.array_equal(got_d["ids"], ref["ids"])  # the relation stays FP64
    e_d = field_errors(ref, got_d)
    # momentum/energy pair kernel on FP64 density (identical inputs)
    got_m, _, _ = gpu_forces(ic, ref["rho_ref"], S.SPH_FP32_PAIR, max_nb=max_nb,
                             rho_in=ref["rho"], export=False)
    e_m = field_errors(ref, got_m)
    print(name, "density-form", e_d, "pair-form", e_m)
    assert e_d["rho"] <= FP32_TOL
    assert e_m["a"] <= FP32_TOL and e_m["du"] <= FP32_TOL and e_m["dt"] <= FP32_TOL


@pytest.mark.parametrize("n", [1, 2, 63, 65, 2047, 2048, 2049, 5000])
def test_ragged_sizes(n):
    ic = I.random_cloud(n, seed=100 + n, h_min=0.06, h_max=0.1, periodic=(0, 1, 0))
    ref = oracle_forces(ic)
    got, _, _ = gpu_forces(ic, ref["rho_ref"], max_nb=512, rho_in=ref["rho"])
    assert np.array_equal(got["off"], ref["off"]) and np.array_equal(got["ids"], ref["ids"])
    e = field_errors(ref, got)
    assert e["rho"] <= FP64_TOL and e["a"] <= FP64_TOL and e["du"] <= FP64_TOL


def test_empty_input():
    ic = I.random_cloud(5, seed=0).take(np.arange(0))
    ctx = S.Context(16, 8)
    st = S.SphState(ic, 8)
    prm = S.make_params(ic.params)
    S.sph_build_cells(ctx, st, h_max=0.1)
    S.sph_find_neighbors(ctx, st)
    S.sph_density(ctx, st, prm)
    S.sph_eos(ctx, st, prm)
    S.sph_momentum_energy(ctx, st, prm)
    S.sph_timestep(ctx, st, prm)
    S.sph_ctx_check(ctx)
    assert st.dt == float("inf")
    assert (st.diag == 0).all()


def test_capacity_overflow_raises_and_counts_exact():
    ic = I.square_patch(12)
    ref = oracle_forces(ic)
    ctx = S.Context(ic.n, 32)
    st = S.SphState(ic, 32, rho_ref=ref["rho_ref"])
    S.sph_build_cells(ctx, st)
    S.sph_find_neighbors(ctx, st)
    with pytest.raises(S.SphError) as ei:
        S.sph_ctx_check(ctx)
    assert ei.value.status == S.SPH_E_CAPACITY
    cnt = st.host(["count"])["count"]
    assert np.array_equal(cnt, np.diff(ref["off"]))
    S.sph_ctx_check(ctx)  # the status word was cleared


def test_domain_error_on_h_above_h_max():
    ic = I.square_patch(10)
    ctx = S.Context(ic.n, 128)
    st = S.SphState(ic, 128)
    S.sph_build_cells(ctx, st, h_max=0.5 * float(ic.h.max()))
    with pytest.raises(S.SphError) as ei:
        S.sph_ctx_check(ctx)
    assert ei.value.status == S.SPH_E_DOMAIN


def test_host_argument_errors():
    ic = I.square_patch(8)
    ctx = S.Context(ic.n, 128)
    st = S.SphState(ic, 128)
    with pytest.raises(S.SphError) as ei:
        S.sph_find_neighbors(ctx, st)  # no build yet
    assert ei.value.status == S.SPH_E_INVALID
    with pytest.raises(S.SphError) as ei:
        S.sph_build_cells(ctx, st, h_max=0.3)  # periodic z shorter than 4 h_max
    assert ei.value.status == S.SPH_E_DOMAIN
    small = S.Context(10, 128)
    with pytest.raises(S.SphError) as ei:
        S.sph_build_cells(small, st)
    assert ei.value.status == S.SPH_E_INVALID


def test_deterministic_bitwise():
    ic = I.random_cloud(4000, seed=9, h_min=0.04, h_max=0.06)
    a, _, _ = gpu_forces(ic, np.ones(ic.n), export=False)
    b, _, _ = gpu_forces(ic, np.ones(ic.n), export=False)
    for k in ("rho", "ax", "ay", "az", "dudt", "mumax"):
        assert np.array_equal(a[k], b[k]), k
    assert a["dt"] == b["dt"] and np.array_equal(a["diag"], b["diag"])


def test_diagnostics_and_integrate_match_oracle():
    ic = I.square_patch(14, seed=4)
    ref = oracle_forces(ic)
    got, st, ctx = gpu_forces(ic, ref["rho_ref"], export=False, rho_in=ref["rho"])
    d_ref = O.diagnostics(ic.x, ic.y, ic.z, ic.vx, ic.vy, ic.vz, ic.u, ic.m)
    assert np.allclose(got["diag"], d_ref, rtol=1e-13, atol=1e-16)
    # one kick-drift on both sides with the GPU's dt
    S.sph_integrate(ctx, st, S.SPH_KICK_DRIFT)
    S.sph_ctx_check(ctx)
    s = {k: np.array(getattr(ic, k), dtype=np.float64) for k in
         ("x", "y", "z", "vx", "vy", "vz", "u")}
    O.integrate(s, 0, got["dt"], ref, ic.lo, ic.hi, ic.periodic)
    h = st.host(["x", "y", "z", "vx", "vy", "vz", "u"])
    for k in s:
        assert np.max(np.abs(h[k] - s[k])) <= 1e-13 * max(1.0, np.abs(s[k]).max()), k


def test_trajectory_square_patch_c0():
    """configs[0]: 20^3 patch, 10 KDK steps, FP64; the GPU and oracle runs
    (each with its own rho_ref = rho(t = 0)) stay together to round-off
    growth, and linear momentum and L_z are conserved."""
    ic = I.square_patch(20)
    ref = O.OracleRun(ic).init()
    ctx = S.Context(ic.n, 128)
    st = S.SphState(ic, 128)
    prm = S.make_params(ic.params)
    S.sph_init_forces(ctx, st, prm, set_rho_ref=True)
    d0 = st.diag.copy()
    for _ in range(10):
        S.sph_step(ctx, st, prm)
        ref.step()
    S.sph_ctx_check(ctx)
    got = st.host(["x", "y", "z", "vx", "vy", "vz", "u", "rho"])
    err = {k: float(np.max(np.abs(got[k] - ref.s[k]))) for k in ("x", "y", "z", "vx", "vy", "vz", "u")}
    err["rho"] = float(np.max(np.abs(got["rho"] / ref.rho - 1)))
    print("trajectory max errors after 10 steps", err)
    assert max(err[k] for k in ("x", "y", "z")) < 1e-12
    assert max(err[k] for k in ("vx", "vy", "vz")) < 1e-10
    assert err["rho"] < 1e-11
    d1 = st.diag
    assert abs(d1[1] - d0[1]) < 1e-15 and abs(d1[2] - d0[2]) < 1e-15
    assert abs(d1[6] - d0[6]) < 1e-13
    assert abs(st.dt - ref.dt) / ref.dt < 1e-10


def test_evrard_variable_h():
    ic = I.evrard(20000, seed=3)
    h, cnt, _ = O.smoothing_length(ic.x, ic.y, ic.z, ic.h, ic.lo, ic.hi, ic.periodic)
    ic.h = h
    ref = oracle_forces(ic, rho_ref=np.ones(ic.n))
    max_nb = int(np.diff(ref["off"]).max()) + 8
    got, _, _ = gpu_forces(ic, np.ones(ic.n), max_nb=max_nb, rho_in=ref["rho"])
    assert np.array_equal(got["off"], ref["off"]) and np.array_equal(got["ids"], ref["ids"])
    e = field_errors(ref, got)
    print("evrard fp64", e, "max count", max_nb - 8)
    assert e["rho"] <= FP64_TOL and e["a"] <= FP64_TOL and e["du"] <= FP64_TOL
    got32, _, _ = gpu_forces(ic, np.ones(ic.n), S.SPH_FP32_PAIR, max_nb=max_nb,
                             rho_in=ref["rho"], export=False)
    e32 = field_errors(ref, got32)
    print("evrard fp32-pair", e32)
    assert e32["rho"] <= FP32_TOL and e32["a"] <= FP32_TOL and e32["du"] <= FP32_TOL


def _cluster_isolated():
    """A cube of 4,000 particles whose h is near its converged value, and 24
    isolated particles around it with h far too small: from the second sweep
    on, the isolated ones are the few particles to recount in their waves
    (the lane-group counts), and their doubling h outgrows the cells there,
    several times, before the tenth sweep ends the iteration."""
    ic = I.random_cloud(4024, seed=8, h_min=0.016, h_max=0.020, periodic=(0, 0, 0))
    rng = np.random.default_rng(9)
    P = rng.uniform(0.4, 0.6, size=(4000, 3))
    iso = []
    while len(iso) < 24:
        q = rng.uniform(0.0, 1.0, size=3)
        if np.max(np.abs(q - 0.5)) > 0.2:
            iso.append(q)
    P = np.vstack([P, np.array(iso)])
    ic.x[:], ic.y[:], ic.z[:] = P[:, 0], P[:, 1], P[:, 2]
    ic.h[4000:] = 0.004
    return ic


@pytest.mark.parametrize("case", ["evrard_20k", "cloud_periodic", "cloud_tiny_h",
                                  "cloud_tiny_h_pz", "cluster_isolated"])
def test_smoothing_length_iteration_bitwise(case):
    """sph_smoothing_length reproduces the oracle's count-based h iteration
    bit for bit: same iterations, same final gather counts, same h. The
    tiny-h clouds start far below the target (every count 0, h doubling), so
    h outgrows the cells the device sweeps started on (two cells of reach)
    and the host rebuilds them mid-iteration."""
    if case == "evrard_20k":
        ic = I.evrard(20000, seed=3)
    elif case == "cloud_periodic":
        ic = I.random_cloud(5000, seed=4, h_min=0.02, h_max=0.08, periodic=(1, 1, 1))
    elif case == "cloud_tiny_h":
        ic = I.random_cloud(4000, seed=6, h_min=0.002, h_max=0.004, periodic=(0, 0, 0))
    elif case == "cluster_isolated":
        ic = _cluster_isolated()
    else:
        ic = I.random_cloud(4000, seed=7, h_min=0.002, h_max=0.004, periodic=(0, 0, 1))
    print("case", case, flush=True)
    h_ref, cnt_ref, it_ref = O.smoothing_length(ic.x, ic.y, ic.z, ic.h, ic.lo, ic.hi,
                                                ic.periodic)
    ctx = S.Context(ic.n, 64)
    st = S.SphState(ic, 64)
    it = S.sph_smoothing_length(ctx, st)
    got = st.host(["h", "count"])
    print(case, "iterations", it, it_ref, "count range", cnt_ref.min(), cnt_ref.max(), flush=True)
    assert it == it_ref
    assert np.array_equal(got["count"], cnt_ref)
    assert np.array_equal(got["h"], h_ref)


KERNEL_CASES = [(S.SPH_KERNEL_WENDLAND_C2, 5), (S.SPH_KERNEL_SINC, 5), (S.SPH_KERNEL_SINC, 3)]


@pytest.mark.parametrize("family,n", KERNEL_CASES)
@pytest.mark.parametrize("name", ["square_patch_c0", "cloud_open", "cloud_pxyz"])
def test_other_kernels(family, n, name):
    """The mini-app's interchangeable kernels (Wendland C2, sinc): density and
    momentum/energy against the oracle with the same kernel, uniform h (the
    square patch) and variable h with all image cases."""
    import dataclasses
    make, max_nb = _cases()[name]
    ic = make()
    ic.params = dataclasses.replace(ic.params, kernel=family, sinc_n=n)
    print(f"case {name} kernel {family} n {n}", flush=True)
    O.set_kernel(family, n)
    try:
        ref = oracle_forces(ic)
    finally:
        O.set_kernel(O.KERNEL_M4)
    got, _, ctx = gpu_forces(ic, ref["rho_ref"], S.SPH_FP64, max_nb=max_nb, rho_in=ref["rho"])
    assert np.array_equal(got["off"], ref["off"]) and np.array_equal(got["ids"], ref["ids"])
    e = field_errors(ref, got)
    print(name, "fp64", e, flush=True)
    assert e["rho"] <= FP64_TOL and e["a"] <= FP64_TOL and e["du"] <= FP64_TOL
    assert e["dt"] <= 1e-13
    got32, _, _ = gpu_forces(ic, ref["rho_ref"], S.SPH_FP32_PAIR, max_nb=max_nb,
                             rho_in=ref["rho"], export=False, ctx=ctx)
    e32 = field_errors(ref, got32)
    print(name, "fp32-pair", e32, flush=True)
    assert e32["rho"] <= FP32_TOL and e32["a"] <= FP32_TOL and e32["du"] <= FP32_TOL


def test_kernel_choice_rejected():
    import dataclasses
    ic = I.square_patch(10)
    ctx = S.Context(ic.n, 128)
    st = S.SphState(ic, 128)
    S.sph_build_cells(ctx, st)
    S.sph_find_neighbors(ctx, st)
    for kernel, n in ((7, 5), (S.SPH_KERNEL_SINC, 2), (S.SPH_KERNEL_SINC, 13)):
        prm = S.make_params(dataclasses.replace(ic.params, kernel=kernel, sinc_n=n))
        with pytest.raises(S.SphError) as e:
            S.sph_density(ctx, st, prm)
        assert e.value.status == S.SPH_E_INVALID
    S.sph_ctx_check(ctx)


def _gravity_errors(got, ref):
    """max_i |g_gpu - g_ref| / S^g_i, S^g the sum of the absolute pair terms."""
    gx, gy, gz, sg = ref
    d = np.sqrt((got[0] - gx) ** 2 + (got[1] - gy) ** 2 + (got[2] - gz) ** 2)
    return float(np.max(d / sg))


@pytest.mark.parametrize("case", ["evrard_20k", "cloud_eps0", "ragged"])
def test_gravity_direct(case):
    """Direct-sum self-gravity (Alg. 1 step 4) against the oracle's, every
    particle; errors in units of the sum of the absolute pair terms."""
    if case == "evrard_20k":
        ic, eps = I.evrard(20_000, seed=0), 0.01
    elif case == "cloud_eps0":
        ic, eps = I.random_cloud(3000, seed=4, h_min=0.03, h_max=0.05), 0.0
    else:
        ic, eps = I.random_cloud(7, seed=5, h_min=0.03, h_max=0.05), 0.02
    print(f"case gravity {case} n={ic.n} eps={eps}", flush=True)
    ctx = S.Context(ic.n, 64)
    st = S.SphState(ic, 64)
    S.sph_gravity_direct(ctx, st, eps)
    S.sph_ctx_check(ctx)
    got = st.host(["gx", "gy", "gz"])
    ref = O.gravity_direct_subset(ic.x, ic.y, ic.z, ic.m, np.arange(ic.n), eps=eps)
    e = _gravity_errors((got["gx"], got["gy"], got["gz"]), ref)
    print(case, "gravity error", e, flush=True)
    assert e <= 1e-12


def _iad_case(name):
    """Inputs for IAD: the square patch (free surfaces on x and y), the
    Evrard sphere and a periodic cloud with h from the oracle's count
    iteration (about 100 gather neighbours each), and raw clouds in open,
    periodic-z and periodic boxes with h ~ U[0.02, 0.08], where about one
    particle in seven has fewer than a handful of particles inside its own
    2 h_i, so its tau_i is close to singular or exactly zero: there the
    conditioning rule (isotropic form below det / (tr / 3)^3 = 0.01, zero
    without a neighbour inside 2 h_i) decides c_i on both sides."""
    if name == "square_patch_c0":
        return I.square_patch(20), 128
    if name.startswith("cloud_raw"):
        per = {"cloud_raw_open": (0, 0, 0), "cloud_raw_z": (0, 0, 1),
               "cloud_raw_xyz": (1, 1, 1)}[name]
        return I.random_cloud(5000, seed=4, h_min=0.02, h_max=0.08, periodic=per), 256
    if name == "evrard_iter":
        ic = I.evrard(20000, seed=3)
    else:
        ic = I.random_cloud(5000, seed=4, h_min=0.02, h_max=0.08, periodic=(1, 1, 1))
    ic.h, _, _ = O.smoothing_length(ic.x, ic.y, ic.z, ic.h, ic.lo, ic.hi, ic.periodic)
    return ic, 256


@pytest.mark.parametrize("family", [S.SPH_KERNEL_M4, S.SPH_KERNEL_WENDLAND_C2, S.SPH_KERNEL_SINC])
@pytest.mark.parametrize("name", ["square_patch_c0", "evrard_iter", "cloud_iter",
                                  "cloud_raw_open", "cloud_raw_z", "cloud_raw_xyz"])
def test_iad_gradients(family, name):
    """Integral approach to derivatives (the SPHYNX gradients of Table 1):
    momentum and energy against the oracle with the same gradient and
    kernel, FP64 and FP32-pair."""
    import dataclasses
    ic, max_nb = _iad_case(name)
    ic.params = dataclasses.replace(ic.params, kernel=family, sinc_n=5,
                                    gradient=S.SPH_GRAD_IAD)
    print(f"case {name} IAD kernel {family}", flush=True)
    O.set_kernel(family, 5)
    O.set_gradient(O.GRADIENT_IAD)
    try:
        ref = oracle_forces(ic)
    finally:
        O.set_kernel(O.KERNEL_M4)
        O.set_gradient(O.GRADIENT_KERNEL)
    got, _, ctx = gpu_forces(ic, ref["rho_ref"], S.SPH_FP64, max_nb=max_nb, rho_in=ref["rho"])
    assert np.array_equal(got["off"], ref["off"]) and np.array_equal(got["ids"], ref["ids"])
    e = field_errors(ref, got)
    print(name, "IAD fp64", e, flush=True)
    assert e["a"] <= FP64_TOL and e["du"] <= FP64_TOL and e["dt"] <= 1e-13
    got32, _, _ = gpu_forces(ic, ref["rho_ref"], S.SPH_FP32_PAIR, max_nb=max_nb,
                             rho_in=ref["rho"], export=False, ctx=ctx)
    e32 = field_errors(ref, got32)
    print(name, "IAD fp32-pair", e32, flush=True)
    assert e32["a"] <= FP32_TOL and e32["du"] <= FP32_TOL


def _gve_case(name):
    """Generalised volume elements with X = (m / rho)^0.7: the 20^3 patch and
    a periodic-z cloud with masses varying by a factor three, with h from the
    oracle's count iteration ("cloud") and raw ("cloud_raw", h ~ U[0.03,
    0.07], where the IAD conditioning rule decides the sparse particles)."""
    import dataclasses
    if name == "square_patch_c0":
        ic = I.square_patch(20)
    else:
        ic = I.random_cloud(4000, seed=17, h_min=0.03, h_max=0.07, velocity=2.0,
                            periodic=(0, 0, 1))
        ic.m = ic.m * np.random.default_rng(5).uniform(0.5, 1.5, ic.n)
        if name == "cloud":
            ic.h, _, _ = O.smoothing_length(ic.x, ic.y, ic.z, ic.h, ic.lo, ic.hi,
                                            ic.periodic)
    ic.params = dataclasses.replace(ic.params, volume=S.SPH_VOLUME_GENERALISED, volume_p=0.7)
    return ic


@pytest.mark.parametrize("name", ["square_patch_c0", "cloud"])
def test_gve_volume_weights(name):
    """sph_volume_weights: X = (m / rho)^p against the oracle on the same rho
    (each side's own pow, so a few ulp)."""
    import torch
    ic = _gve_case(name)
    off, ids = O.neighbors(ic.x, ic.y, ic.z, ic.h, ic.lo, ic.hi, ic.periodic)
    rho = O.density(ic.x, ic.y, ic.z, ic.h, ic.m, ic.lo, ic.hi, ic.periodic, off, ids)
    X = O.volume_weights(ic.m, rho, 0.7)
    ctx = S.Context(ic.n, 128)
    st = S.SphState(ic, 128)
    S.sph_volume_weights(ctx, st, 0.7, rho=torch.as_tensor(rho).to(st.device))
    S.sph_ctx_check(ctx)
    got = st.host(["xw"])["xw"]
    err = float(np.max(np.abs(got / X - 1)))
    print(name, "volume weights max rel", err, flush=True)
    assert err <= 1e-15


@pytest.mark.parametrize("gradient", [S.SPH_GRAD_KERNEL, S.SPH_GRAD_IAD])
@pytest.mark.parametrize("name", ["square_patch_c0", "cloud", "cloud_raw"])
def test_gve_forces(name, gradient):
    """Generalised volume elements (SPHYNX, Table 1): density and
    momentum/energy against the oracle on the same weights, with kernel
    derivatives and with IAD, FP64 and FP32-pair."""
    import dataclasses
    ic = _gve_case(name)
    ic.params = dataclasses.replace(ic.params, gradient=gradient)
    print(f"case {name} GVE gradient {gradient}", flush=True)
    lo, hi, per = ic.lo, ic.hi, ic.periodic
    off, ids = O.neighbors(ic.x, ic.y, ic.z, ic.h, lo, hi, per)
    max_nb = int(np.diff(off).max()) + 8
    rho0 = O.density(ic.x, ic.y, ic.z, ic.h, ic.m, lo, hi, per, off, ids)
    X = O.volume_weights(ic.m, rho0, 0.7)
    rho = O.density(ic.x, ic.y, ic.z, ic.h, ic.m, lo, hi, per, off, ids, X=X)
    p, c, pr2 = O.eos(ic.params, rho, ic.u, rho, ic.p_bg)
    O.set_gradient(gradient)
    try:
        acc = O.momentum_energy(ic.x, ic.y, ic.z, ic.vx, ic.vy, ic.vz, ic.h, ic.m, rho, c,
                                pr2, lo, hi, per, off, ids, ic.params, scales=True, X=X)
    finally:
        O.set_gradient(O.GRADIENT_KERNEL)
    dt = O.timestep(ic.h, c, acc["mumax"], acc["ax"], acc["ay"], acc["az"], ic.params)
    ref = dict(off=off, ids=ids, rho=rho, dt=dt, **acc)
    got, _, ctx = gpu_forces(ic, rho, S.SPH_FP64, max_nb=max_nb, rho_in=rho, xw=X)
    assert np.array_equal(got["off"], off) and np.array_equal(got["ids"], ids)
    e = field_errors(ref, got)
    print(name, "GVE fp64", e, flush=True)
    assert e["rho"] <= FP64_TOL and e["a"] <= FP64_TOL and e["du"] <= FP64_TOL
    assert e["dt"] <= 1e-13
    got32, _, _ = gpu_forces(ic, rho, S.SPH_FP32_PAIR, max_nb=max_nb, rho_in=rho, xw=X,
                             export=False, ctx=ctx)
    e32 = field_errors(ref, got32)
    print(name, "GVE fp32-pair", e32, flush=True)
    assert e32["rho"] <= FP32_TOL and e32["a"] <= FP32_TOL and e32["du"] <= FP32_TOL


def test_gve_trajectory_square_patch_c0():
    """Generalised volume elements through sph_init_forces and sph_step (the
    weights taken from the previous density before each step, from a standard
    density at t = 0) against the oracle run doing the same: 5 steps."""
    ic = _gve_case("square_patch_c0")
    ref = O.OracleRun(ic).init()
    ctx = S.Context(ic.n, 128)
    st = S.SphState(ic, 128)
    prm = S.make_params(ic.params)
    S.sph_init_forces(ctx, st, prm, set_rho_ref=True)
    for _ in range(5):
        S.sph_step(ctx, st, prm)
        ref.step()
    S.sph_ctx_check(ctx)
    got = st.host(["x", "y", "z", "vx", "vy", "vz", "rho", "xw"])
    err = {k: float(np.max(np.abs(got[k] - ref.s[k]))) for k in ("x", "y", "z", "vx", "vy", "vz")}
    err["rho"] = float(np.max(np.abs(got["rho"] / ref.rho - 1)))
    err["xw"] = float(np.max(np.abs(got["xw"] / ref.X - 1)))
    print("GVE trajectory max errors after 5 steps", err, flush=True)
    assert max(err[k] for k in ("x", "y", "z")) < 1e-12
    assert max(err[k] for k in ("vx", "vy", "vz")) < 1e-10
    assert err["rho"] < 1e-11 and err["xw"] < 1e-11
    assert abs(st.dt - ref.dt) / ref.dt < 1e-10


def _tree_case(name):
    if name == "evrard_20k":
        ic = I.evrard(20000, seed=3)
        return ic, 0.01
    if name == "cloud_eps0":
        ic = I.random_cloud(3000, seed=8, h_min=0.03, h_max=0.06, periodic=(0, 0, 0))
        ic.m = ic.m * np.random.default_rng(6).uniform(0.5, 1.5, ic.n)
        return ic, 0.0
    if name == "two_groups":
        return I.random_cloud(65, seed=12, h_min=0.05, h_max=0.08, periodic=(0, 0, 0)), 0.02
    if name == "clump":
        # 300 particles inside one finest-level cell (a leaf of more than 64,
        # cut into runs of 64) next to a sparse cloud
        ic = I.random_cloud(700, seed=14, h_min=0.05, h_max=0.08, periodic=(0, 0, 0))
        rng = np.random.default_rng(15)
        for a in ("x", "y", "z"):
            getattr(ic, a)[:300] = 0.5 + 1e-7 * rng.random(300)
        return ic, 0.01
    return I.random_cloud(7, seed=13, h_min=0.05, h_max=0.08, periodic=(0, 0, 0)), 0.02


@pytest.mark.parametrize("theta", [0.5, 0.8])
@pytest.mark.parametrize("name", ["evrard_20k", "cloud_eps0", "two_groups", "ragged", "clump"])
def test_gravity_tree(name, theta):
    """Octree gravity (sph_gravity_tree) against the oracle's octree with the
    same keys, nodes, moments and acceptance test: every particle within
    1e-12 of the sum of its term magnitudes; the particles are first put
    through a cell build, so the GPU's order differs from the oracle's."""
    ic, eps = _tree_case(name)
    print(f"case tree {name} n={ic.n} eps={eps} theta={theta}", flush=True)
    gx, gy, gz, sc, st = O.gravity_tree(ic.x, ic.y, ic.z, ic.m, eps, theta, 16)
    ctx = S.Context(ic.n, 64)
    s = S.SphState(ic, 64)
    S.sph_build_cells(ctx, s)
    S.sph_gravity_tree(ctx, s, eps, theta, 16)
    S.sph_ctx_check(ctx)
    got = s.host(["gx", "gy", "gz"])
    err = np.sqrt((got["gx"] - gx) ** 2 + (got["gy"] - gy) ** 2 + (got["gz"] - gz) ** 2)
    rel = float(np.max(err / sc))
    print(name, theta, "tree max err / scale", rel, st, flush=True)
    assert rel <= 1e-12


def test_blocks_zero_is_sph_step():
    """sph_step_blocks with max_bin = 0 is sph_step, bit for bit, over 3 steps."""
    ic = I.square_patch(12)
    prm = S.make_params(ic.params)
    out = []
    for blocks in (False, True):
        ctx = S.Context(ic.n, 128)
        st = S.SphState(ic, 128)
        S.sph_init_forces(ctx, st, prm, set_rho_ref=True)
        for _ in range(3):
            if blocks:
                assert S.sph_step_blocks(ctx, st, prm, 0) == 1
            else:
                S.sph_step(ctx, st, prm)
        S.sph_ctx_check(ctx)
        out.append(st.host(["x", "y", "z", "vx", "vy", "vz", "u", "rho"]))
    for k in out[0]:
        assert np.array_equal(out[0][k], out[1][k]), k


def _blocks_case(name):
    if name == "isolated":
        import importlib
        pins = importlib.import_module("test_oracle_pins")
        ic, g = pins._isolated()
        return ic, g, 4, 16
    if name == "square_patch_c0":
        return I.square_patch(20), None, 3, 128
    if name == "square_patch_gve":
        import dataclasses
        ic = I.square_patch(20)
        ic.params = dataclasses.replace(ic.params, volume=S.SPH_VOLUME_GENERALISED)
        return ic, None, 3, 128
    ic = I.evrard(20000, seed=3)
    ic.h, _, _ = O.smoothing_length(ic.x, ic.y, ic.z, ic.h, ic.lo, ic.hi, ic.periodic)
    g = O.gravity_direct(ic.x, ic.y, ic.z, ic.m, 0.01)
    return ic, g, 5, 256


@pytest.mark.parametrize("name", ["isolated", "square_patch_c0", "square_patch_gve",
                                  "evrard_iter"])
def test_blocks_against_oracle(name):
    """Individual time steps (sph_step_blocks) against the oracle's: the step
    D, every particle's bin and, after two steps, the state."""
    ic, g, max_bin, max_nb = _blocks_case(name)
    print(f"case blocks {name} n={ic.n} max_bin={max_bin}", flush=True)
    ref = O.OracleRun(ic, g=g).init()
    ctx = S.Context(ic.n, max_nb)
    st = S.SphState(ic, max_nb, g=g)
    prm = S.make_params(ic.params)
    S.sph_init_forces(ctx, st, prm, set_rho_ref=True)
    for k in range(2):
        subs = S.sph_step_blocks(ctx, st, prm, max_bin)
        D, b, rsubs = ref.step_blocks(max_bin)
        S.sph_ctx_check(ctx)
        got_bin = st.host(["bin"])["bin"]
        print(name, "step", k, "D", D, st.dt, "substeps", subs, rsubs, flush=True)
        assert subs == rsubs and abs(st.dt - D) <= 1e-14 * D
        assert np.array_equal(got_bin.astype(np.int64), b)
    got = st.host(["x", "y", "z", "vx", "vy", "vz", "u"])
    err = {k: float(np.max(np.abs(got[k] - ref.s[k]))) for k in got}
    scale = {k: float(np.max(np.abs(ref.s[k]))) + 1e-300 for k in got}
    print(name, "blocks max errors", err, flush=True)
    for k in ("x", "y", "z"):
        assert err[k] <= 1e-12 * max(1.0, scale[k])
    for k in ("vx", "vy", "vz", "u"):
        assert err[k] <= 1e-10 * max(1.0, scale[k])


@pytest.mark.parametrize("name,precision", [("square_patch_c0", S.SPH_FP64),
                                            ("cloud_pxyz", S.SPH_FP32_PAIR)])
def test_step_graph_replay_is_sph_step(name, precision):
    """sph_step_capture + sph_step_replay against eager sph_step, bit for bit:
    four replays, each followed by an eager step of a twin run and a
    synchronisation, every replay compared with the eager state."""
    make, max_nb = _cases()[name]
    ic = make()
    print(f"case graph {name} n={ic.n} precision={precision}", flush=True)
    prm = S.make_params(ic.params, precision)
    keys = ["x", "y", "z", "vx", "vy", "vz", "u", "rho", "ax", "ay", "az", "dudt"]
    runs = []
    for _ in range(2):
        ctx = S.Context(ic.n, max_nb)
        st = S.SphState(ic, max_nb)
        S.sph_init_forces(ctx, st, prm, set_rho_ref=True)
        runs.append((ctx, st))
    (cg, sg), (ce, se) = runs
    with pytest.raises(S.SphError) as ei:
        S.sph_step_replay(cg)
    assert ei.value.status == S.SPH_E_INVALID
    before = sg.host(keys)
    S.sph_step_capture(cg, sg, prm)
    torch.cuda.synchronize()
    after = sg.host(keys)
    for k in keys:  # capturing runs nothing
        assert np.array_equal(before[k], after[k]), k
    for r in range(4):
        S.sph_step_replay(cg)
        S.sph_step(ce, se, prm)
        S.sph_ctx_check(cg)
        S.sph_ctx_check(ce)
        g, e = sg.host(keys), se.host(keys)
        for k in keys:
            assert np.array_equal(g[k], e[k]), (r, k)
        assert sg.dt == se.dt and np.array_equal(sg.diag, se.diag), r
